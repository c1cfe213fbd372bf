"""Pins of the oracle's transfer function H(t, f) = sum_r a_r exp(-j 2 pi f tau_r)
(Sec. II: the time-variant channel transfer function of the extrapolated multipath)."""
import math

import numpy as np

import oracle
from paper_2205_00237_amd import scenes

C0 = 299_792_458.0


def test_single_ray_magnitude_group_delay_and_impulse_peak():
    rng = np.random.default_rng(0)
    K, B, fc = 4096, 400e6, 28e9
    f = oracle.freq_axis(fc, B, K)
    for _ in range(20):
        L = rng.uniform(5, 600)
        a = complex(rng.normal(), rng.normal()) * 1e-5
        H = oracle.cfr(np.array([[L]]), np.array([[a]]), f)[0]
        assert np.abs(np.abs(H) - abs(a)).max() < 1e-15 * 1e3
        ph = np.unwrap(np.angle(H))
        slope = np.polyfit(f - fc, ph, 1)[0]
        assert abs(slope + 2 * math.pi * L / C0) < 1e-9 * 2 * math.pi * L / C0
        # the inverse DFT over the band peaks at the delay bin (modulo the band's alias)
        h = np.fft.ifft(H * np.exp(2j * math.pi * f[0] * L / C0))
        peak = np.argmax(np.abs(h))
        assert abs(((L / C0) * B - peak + K / 2) % K - K / 2) <= 1


def test_two_ray_closed_form():
    rng = np.random.default_rng(1)
    f = oracle.freq_axis(60e9, 2e9, 64)
    for _ in range(20):
        L1, L2 = rng.uniform(5, 300, 2)
        a1, a2 = rng.normal(size=2) + 1j * rng.normal(size=2)
        H = oracle.cfr(np.array([[L1], [L2]]), np.array([[a1], [a2]]), f)[0]
        p = abs(a1) ** 2 + abs(a2) ** 2 + 2 * np.real(a1 * np.conj(a2) * np.exp(-2j * math.pi * f * (L1 - L2) / C0))
        assert np.abs(np.abs(H) ** 2 - p).max() < 1e-9 * p.max()


def test_phase_advance_follows_doppler():
    """arg H(t_{j+1}, f_c) - arg H(t_j, f_c) = 2 pi f_D dt (trapezoid rule) for one ray whose
    coefficient has a constant phase (line of sight, and the front face of the PEC box)."""
    s, tg, fg = scenes.config1()
    kc = fg.n_sub // 2
    for r in (0, 2):
        out1, H1 = oracle.run(s, tg, fg, rays=[r])
        dph = np.angle(H1[1:, kc] * np.conj(H1[:-1, kc]))
        fD = out1["dop"][0]
        mid = 0.5 * (fD[1:] + fD[:-1])
        wrapped = np.angle(np.exp(1j * (dph - 2 * math.pi * mid * tg.dt)))
        assert np.abs(wrapped).max() < 1e-6
