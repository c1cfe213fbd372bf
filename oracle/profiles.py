"""Power-Doppler profile (PDfP, Sec. IV-A) and power-delay profile (PDP, Sec. IV-B).
TEST INFRASTRUCTURE ONLY.

Both are incoherent power sums over bins.  A sample is one (ray, instant) pair of
extrapolate(): its power is |a|^2, the squared modulus of the field coefficient at the
carrier (unit transmitted power, isotropic antennas), its Doppler shift is f_D and its delay
tau = L / c.  Instants are grouped into time bins of `steps_per_bin` consecutive instants
(instant j belongs to bin j // steps_per_bin).  A sample is counted when its chain is
consistent and, with `in_bounds_only`, when the validity monitor finds it in bounds.  Each
counted sample adds its power to

  pdfp[b, k]  k = floor((f_D - dop_lo) / dop_step),     if 0 <= k < n_dop,
  pdp[b, k]   k = floor((tau - delay_lo) / delay_step), if 0 <= k < n_delay,
  total[b]    whether or not it falls in a bin,

b being its time bin.  The paper's profile uses 200 ms x 14.34 Hz bins (Sec. IV-A); its PDP
is a map of power over simulation time and delay (Sec. IV-B).
"""
import numpy as np

from .drt import extrapolate


def bin_index(x, lo, step, n):
    """floor((x - lo) / step) where that lies in [0, n), else -1."""
    with np.errstate(invalid="ignore"):
        k = np.floor((np.asarray(x, dtype=np.float64) - lo) / step)
    return np.where((k >= 0) & (k < n), k, -1).astype(np.int64)


def bin_samples(ex, j, bins):
    """Profiles of the extrapolate() outputs `ex` at the grid instants j (its columns).

    bins: dict with steps_per_bin, n_dop, dop_lo, dop_step, n_delay, delay_lo, delay_step
    and in_bounds_only.  Returns dict with pdfp (n_tb, n_dop), pdp (n_tb, n_delay) and
    total (n_tb,) for time bins 0 .. max(j) // steps_per_bin, and the samples behind them:
    power, dop, tau, counted, bounds_margin (R, len(j)) and tbin (len(j),)."""
    j = np.atleast_1d(np.asarray(j, dtype=np.int64))
    spb = int(bins["steps_per_bin"])
    n_tb = int(j.max()) // spb + 1
    tb = j // spb
    power = np.abs(ex["gain"]) ** 2
    counted = ex["valid"].copy()
    if bins.get("in_bounds_only", 0):
        counted &= ex["in_bounds"]
    out = {"pdfp": np.zeros((n_tb, int(bins["n_dop"]))),
           "pdp": np.zeros((n_tb, int(bins["n_delay"]))),
           "total": np.zeros(n_tb)}
    r, c = np.nonzero(counted)
    b, p = tb[c], power[r, c]
    np.add.at(out["total"], b, p)
    kd = bin_index(ex["dop"][r, c], bins["dop_lo"], bins["dop_step"], int(bins["n_dop"]))
    m = kd >= 0
    np.add.at(out["pdfp"], (b[m], kd[m]), p[m])
    kt = bin_index(ex["tau"][r, c], bins["delay_lo"], bins["delay_step"], int(bins["n_delay"]))
    m = kt >= 0
    np.add.at(out["pdp"], (b[m], kt[m]), p[m])
    out.update(power=power, dop=ex["dop"], tau=ex["tau"], counted=counted,
               bounds_margin=ex["bounds_margin"], tbin=tb)
    return out


def power_profiles(scene, j, dt, f_c, bins, rays=None):
    """Profiles over the instants t = j * dt (j: integer indices into the time grid): the
    samples of extrapolate() binned by bin_samples()."""
    j = np.atleast_1d(np.asarray(j, dtype=np.int64))
    return bin_samples(extrapolate(scene, j * dt, f_c, rays=rays), j, bins)


def edge_distance(x, lo, step):
    """Distance from x to the nearest bin edge lo + k step, in units of x."""
    u = (np.asarray(x, dtype=np.float64) - lo) / step
    return np.abs(u - np.round(u)) * step

