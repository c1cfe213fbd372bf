"""Pins of the diffracted-ray field coefficient as the oracle assembles it in `extrapolate`
(Sec. III-B: the UTD coefficient of the updated geometry, ref. [UTD]): the wedge angles from
the (image) source and receiver, the distance parameter L_d = s s' sin^2(beta0) / (s + s'),
the spreading sqrt(s' / (s (s + s'))) / s' and, for chains with reflections, the Fresnel
factors of the walls before and after the edge.

Three independent references:

* the exact Sommerfeld solution of a perfectly conducting half-plane (n = 2) lit by a plane
  wave, at normal and oblique incidence, written here with Fresnel integrals (scipy); the
  oracle sees a point source so far away that its wave is plane over the observation region;
* continuity of the total field (line of sight + 0-face reflection + diffraction) across the
  incidence and reflection shadow boundaries of a right-angle wedge (n = 1.5) for a point
  source at oblique incidence: the diffracted field must cancel the jump of the geometrical
  optics field exactly, which fixes its amplitude and its distance parameter;
* a chain with reflections before or after the edge equals the unfolded single-edge ray from
  the image source or receiver times the reflection coefficients, taken at the incidence
  angles measured on the unfolded geometry.
"""
import math

import numpy as np
import pytest
from scipy.special import fresnel

import oracle
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_R, KIND_D, POL_PERP, POL_PAR

C0 = 299_792_458.0


def _tail(x):
    """int_x^inf exp(-j tau^2) d tau for real x (either sign), from scipy's Fresnel integrals
    S(u), C(u) = int_0^u sin, cos(pi t^2 / 2) dt with tau = sqrt(pi/2) t."""
    u = np.asarray(x, dtype=np.float64) * math.sqrt(2.0 / math.pi)
    S, C = fresnel(u)
    return math.sqrt(math.pi / 2.0) * ((0.5 - C) - 1j * (0.5 - S))


def _sommerfeld_half_plane(rho, phi, phi_p, kt, soft):
    """Exact total field of a perfectly conducting half-plane (the +x half of the plane
    y = 0, edge on the z axis) for the unit plane wave exp(j kt rho cos(phi - phi_p)) with
    time factor e^{+j w t}: U(phi - phi_p) -/+ U(phi + phi_p) (minus for the soft, Dirichlet
    problem), U(b) = exp(j kt rho cos b) (e^{j pi/4}/sqrt(pi)) int_{-sqrt(2 kt rho) cos(b/2)}^inf
    exp(-j tau^2) d tau."""
    def U(b):
        return (np.exp(1j * kt * rho * np.cos(b)) * np.exp(1j * math.pi / 4) / math.sqrt(math.pi)
                * _tail(-math.sqrt(2.0 * kt * rho) * np.cos(b / 2.0)))
    return U(phi - phi_p) - U(phi + phi_p) if soft else U(phi - phi_p) + U(phi + phi_p)


def _wedge_scene(tx, rx, n, pol, extra_planes=(), sig="L,R,D"):
    """A perfectly conducting wedge whose edge is the z axis and whose 0-face is the +x half
    of the plane y = 0 (outward normal +y); exterior angle n pi.  Rays by signature letters:
    L line of sight, R reflection on the 0-face plane, D diffraction at the edge.  With
    `extra_planes` (body-0 PEC walls given as (point, normal)), letters G and W refer to
    them in order."""
    b = SceneBuilder()
    pec = b.add_material(1.0, 0.0, True)
    face = b.add_plane(0, pec, (0, 0, 0), (0, 1, 0))
    edge = b.add_edge(0, (0, 0, 0), (0, 0, 1), (1, 0, 0), (0, 1, 0), n)
    walls = [b.add_plane(0, pec, p, nn) for p, nn in extra_planes]
    names = {"G": 0, "W": 1}
    for ray in sig.split(","):
        kinds, prims, pols = [], [], []
        for ch in ray:
            if ch == "L":
                break
            if ch == "R":
                kinds.append(KIND_R), prims.append(face), pols.append(pol)
            elif ch == "D":
                kinds.append(KIND_D), prims.append(edge), pols.append(pol)
            else:
                kinds.append(KIND_R), prims.append(walls[names[ch]]), pols.append(pol)
        b.add_ray(kinds, prims, pols)
    return b.build(tx_p=tx, rx_p=rx)


def _fields(scene, f_c):
    """Per-ray complex field a_r exp(-j k L_r) at the carrier and the validity flags."""
    out = oracle.extrapolate(scene, np.zeros(1), f_c)
    k = 2.0 * math.pi * f_c / C0
    return out["gain"][:, 0] * np.exp(-1j * k * out["L"][:, 0]), out["valid"][:, 0], out


# ------------------------------------------------------------------ half-plane, exact solution

@pytest.mark.parametrize("beta0_deg", [90.0, 62.0, 121.0])
@pytest.mark.parametrize("pol", [POL_PERP, POL_PAR])
def test_half_plane_matches_sommerfeld(beta0_deg, pol):
    """n = 2 (a screen): line of sight where lit, 0-face reflection where it exists, plus the
    diffracted ray, against the exact solution at oblique incidence (the 3D field is the 2D
    solution with kt = k sin beta0 times exp(-j k z cos beta0)).  The Kouyoumjian-Pathak
    coefficient reproduces the plane-wave half-plane solution exactly, so what is left is the
    curvature of a wave from a source 1e8 m away (< 1e-5)."""
    f_c = 3e9
    lam = C0 / f_c
    k = 2.0 * math.pi / lam
    b0 = math.radians(beta0_deg)
    kt = k * math.sin(b0)
    s0 = 1e8
    phi_p = math.radians(57.0)
    khat = np.array([-math.sin(b0) * math.cos(phi_p), -math.sin(b0) * math.sin(phi_p), math.cos(b0)])
    tx = -s0 * khat                      # the wave travels along khat through the origin
    rho = 2.3
    # a sweep over the exterior plus points close to both shadow boundaries
    phis = list(np.linspace(0.08, 2 * math.pi - 0.08, 23))
    for bnd in (math.pi - phi_p, math.pi + phi_p):
        phis += [bnd + d for d in (-3e-3, -2e-4, 2e-4, 3e-3)]
    worst = 0.0
    for phi in phis:
        for zr in (-0.7, 0.0, 1.9):
            rx = np.array([rho * math.cos(phi), rho * math.sin(phi), zr])
            s = _wedge_scene(tx, rx, 2.0, pol)
            E, valid, _ = _fields(s, f_c)
            assert valid[2]
            lit = phi < math.pi + phi_p
            refl = phi < math.pi - phi_p
            assert valid[1] == refl or not refl       # the formal reflection exists where GO has it
            tot = (E[0] if lit else 0) + (E[1] if refl else 0) + E[2]
            tot *= 4.0 * math.pi * s0 / lam * np.exp(1j * k * s0)     # unit plane wave at the origin
            ref = (_sommerfeld_half_plane(rho, phi, phi_p, kt, pol == POL_PERP)
                   * np.exp(-1j * k * zr * math.cos(b0)))
            worst = max(worst, abs(tot - ref))
            assert abs(tot - ref) < 2e-5, (phi, zr, abs(tot - ref), abs(ref))
    assert worst > 0.0


def test_half_plane_diffracted_part_alone():
    """Deep in the shadow (no GO field) the exact field is the diffracted one alone, of order
    1/sqrt(kt rho): checks the diffracted amplitude away from the transition regions."""
    f_c = 3e9
    lam = C0 / f_c
    k = 2.0 * math.pi / lam
    s0 = 1e8
    phi_p = math.radians(40.0)
    b0 = math.radians(70.0)
    khat = np.array([-math.sin(b0) * math.cos(phi_p), -math.sin(b0) * math.sin(phi_p), math.cos(b0)])
    tx = -s0 * khat
    for rho in (0.5, 4.0, 30.0):
        for phi in (math.pi + phi_p + 0.6, 2 * math.pi - 0.3):
            rx = np.array([rho * math.cos(phi), rho * math.sin(phi), 0.4])
            E, valid, _ = _fields(_wedge_scene(tx, rx, 2.0, POL_PAR), f_c)
            d = E[2] * 4.0 * math.pi * s0 / lam * np.exp(1j * k * s0)
            ref = (_sommerfeld_half_plane(rho, phi, phi_p, k * math.sin(b0), False)
                   * np.exp(-1j * k * 0.4 * math.cos(b0)))
            assert abs(ref) > 1e-3
            assert abs(d - ref) < 2e-5 * max(1.0, rho / 4.0), (rho, phi, abs(d - ref), abs(ref))


# ------------------------------------------------------------------ wedge, shadow boundaries

@pytest.mark.parametrize("pol", [POL_PERP, POL_PAR])
@pytest.mark.parametrize("zs", [(6.0, -1.5), (-4.0, 2.5), (0.0, 0.0)])
def test_wedge_total_field_continuous_through_extrapolate(pol, zs):
    """A right-angle wedge (n = 1.5) and a point source 9 m from the edge at oblique
    incidence.  Crossing the incidence (phi = pi + phi') and reflection (phi = pi - phi')
    shadow boundaries, the geometrical-optics field jumps by the line-of-sight or reflected
    field; the diffracted ray assembled by the oracle must cancel the jump (residual after
    removing the linear variation below 1e-6 of the jump)."""
    f_c = 28e9
    z_tx, z_rx = zs
    phi_p = math.radians(50.0)
    tx = np.array([9.0 * math.cos(phi_p), 9.0 * math.sin(phi_p), z_tx])
    rho = 5.0

    def total(phi, diffracted=True):
        rx = np.array([rho * math.cos(phi), rho * math.sin(phi), z_rx])
        E, valid, _ = _fields(_wedge_scene(tx, rx, 1.5, pol), f_c)
        U = (E[0] if phi < math.pi + phi_p else 0) + (E[1] if phi < math.pi - phi_p else 0)
        return U + (E[2] if diffracted else 0)

    for bnd in (math.pi + phi_p, math.pi - phi_p):
        d = 2e-7
        U = [total(bnd + m * d) for m in (-3, -1, 1, 3)]
        jump = (U[2] - U[1]) - 0.5 * ((U[3] - U[2]) + (U[1] - U[0]))
        go = abs(total(bnd + d, False) - total(bnd - d, False))
        assert go > 2e-5                      # about lambda / (4 pi L) at L ~ 14-17 m
        assert abs(jump) < 1e-5 * go, (bnd, abs(jump), go)


def test_wedge_diffracted_field_jumps_by_the_go_field():
    """Across a shadow boundary the diffracted field alone jumps by exactly the GO field that
    switches off there (same path length at the boundary), whatever the obliquity: with
    E_d and E_go taken 1e-6 rad on either side, (E_d(+) - E_d(-)) / E_go = 1."""
    f_c = 28e9
    for z_tx, z_rx in ((6.0, -1.5), (-3.0, 4.0)):
        phi_p = math.radians(35.0)
        tx = np.array([7.0 * math.cos(phi_p), 7.0 * math.sin(phi_p), z_tx])
        for which, bnd in ((0, math.pi + phi_p), (1, math.pi - phi_p)):
            for pol in (POL_PERP, POL_PAR):
                E = []
                for side in (-1, 1):
                    phi = bnd + side * 1e-6
                    rx = np.array([3.0 * math.cos(phi), 3.0 * math.sin(phi), z_rx])
                    E.append(_fields(_wedge_scene(tx, rx, 1.5, pol), f_c)[0])
                ratio = (E[1][2] - E[0][2]) / E[0][which]
                assert abs(ratio - 1.0) < 1e-4, (which, pol, ratio)


# ------------------------------------------------------------------ chains vs unfolded

def _mirror(X, p, n):
    X, p, n = (np.asarray(v, float) for v in (X, p, n))
    return X - 2.0 * np.dot(X - p, n) * n


@pytest.mark.parametrize("sig", ["GD", "DG", "GWD", "WGD", "DWG", "GDW"])
@pytest.mark.parametrize("pol", [POL_PERP, POL_PAR])
def test_chain_equals_unfolded_single_edge(sig, pol):
    """A ground plane z = 0 and an overhanging wall (normal (1, 0, -0.5), through
    (-6, 0, 0); the two mirrors do not commute), both PEC, around a vertical edge: the
    chain's coefficient is that of the single edge seen from the image source (walls before
    the edge, mirrored in order) and the image receiver (walls after, mirrored from the last
    one back), times -1 (soft) or +1 (hard) per wall; the path lengths agree."""
    ground = ((0, 0, 0), (0, 0, 1))
    wall = ((-6, 0, 0), tuple(np.array([1.0, 0.0, -0.5]) / math.sqrt(1.25)))
    planes = {"G": ground, "W": wall}
    f_c = 28e9
    rng = np.random.default_rng(sum(map(ord, sig)) + 7 * pol)
    d = sig.index("D")
    checked = 0
    for _ in range(400):
        if checked >= 8:
            break
        tx = np.array([rng.uniform(-5.9, 15), rng.uniform(-15, 15), rng.uniform(0.1, 15)])
        rx = np.array([rng.uniform(-5.9, 15), rng.uniform(-15, 15), rng.uniform(0.1, 15)])
        s = _wedge_scene(tx, rx, 1.5, pol, extra_planes=(ground, wall), sig=sig)
        out = oracle.extrapolate(s, np.zeros(1), f_c)
        if not out["valid"][0, 0]:
            continue
        A = tx
        for ch in sig[:d]:
            A = _mirror(A, *planes[ch])
        B = rx
        for ch in reversed(sig[d + 1:]):
            B = _mirror(B, *planes[ch])
        u = _wedge_scene(A, B, 1.5, pol, sig="D")
        ou = oracle.extrapolate(u, np.zeros(1), f_c)
        assert ou["valid"][0, 0]
        gam = (-1.0 if pol == POL_PERP else 1.0) ** (len(sig) - 1)
        assert abs(out["L"][0, 0] - ou["L"][0, 0]) < 1e-12 * ou["L"][0, 0]
        a, au = out["gain"][0, 0], ou["gain"][0, 0]
        assert abs(a - gam * au) < 1e-12 * abs(au), (a, gam * au)
        checked += 1
    assert checked >= 5


@pytest.mark.parametrize("sig", ["GD", "DG"])
def test_chain_dielectric_wall_uses_unfolded_incidence_angle(sig):
    """As above with a lossy dielectric ground: the factor is the Fresnel coefficient at the
    incidence angle of the unfolded ray where it crosses the ground plane."""
    f_c = 28e9
    lam = C0 / f_c
    eps_r, sigma = 5.0, 0.3
    rng = np.random.default_rng(11 if sig == "GD" else 12)
    checked = 0
    for _ in range(30):
        phi_p, phi = rng.uniform(0.3, 1.2), rng.uniform(1.9, 4.3)
        tx = np.array([6 * math.cos(phi_p), 6 * math.sin(phi_p), rng.uniform(0.5, 5)])
        rx = np.array([5 * math.cos(phi), 5 * math.sin(phi), rng.uniform(0.5, 5)])
        for pol in (POL_PERP, POL_PAR):
            b = SceneBuilder()
            pec = b.add_material(1.0, 0.0, True)
            gm = b.add_material(eps_r, sigma)
            g = b.add_plane(0, gm, (0, 0, 0), (0, 0, 1))
            e = b.add_edge(0, (0, 0, 0), (0, 0, 1), (1, 0, 0), (0, 1, 0), 1.5)
            kinds = [KIND_R, KIND_D] if sig == "GD" else [KIND_D, KIND_R]
            prims = [g, e] if sig == "GD" else [e, g]
            b.add_ray(kinds, prims, [pol, pol])
            s = b.build(tx_p=tx, rx_p=rx)
            out = oracle.extrapolate(s, np.zeros(1), f_c)
            if not out["valid"][0, 0]:
                continue
            A = _mirror(tx, (0, 0, 0), (0, 0, 1)) if sig == "GD" else tx
            B = rx if sig == "GD" else _mirror(rx, (0, 0, 0), (0, 0, 1))
            ou = oracle.extrapolate(_wedge_scene(A, B, 1.5, pol, sig="D"), np.zeros(1), f_c)
            # the unfolded ray A -> Q_D -> B: the leg that crosses z = 0 and its direction
            QD = np.array([0.0, 0.0, 0.0])
            QD[2] = B[2] + math.hypot(B[0], B[1]) * (A[2] - B[2]) / (math.hypot(A[0], A[1]) + math.hypot(B[0], B[1]))
            leg = QD - A if sig == "GD" else B - QD
            cos_t = abs(leg[2]) / np.linalg.norm(leg)
            root = np.sqrt(eps_r - 1j * 60 * sigma * lam - (1 - cos_t ** 2))
            epsc = eps_r - 1j * 60 * sigma * lam
            gam = ((cos_t - root) / (cos_t + root) if pol == POL_PERP
                   else (epsc * cos_t - root) / (epsc * cos_t + root))
            assert abs(out["gain"][0, 0] - gam * ou["gain"][0, 0]) < 1e-12 * abs(ou["gain"][0, 0])
            checked += 1
    assert checked >= 10
