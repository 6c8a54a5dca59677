"""Pins for oracle.sht (spin-0 SHT on McEwen-Wiaux sampling)."""
import math

import numpy as np
import scipy.special as sps

from oracle import sampling, sht
from paper_1511_05578_amd import inputs


def _library_inverse(flm, L):
    th = sampling.mw_theta(L)[:, None]
    ph = sampling.mw_phi(L)[None, :]
    out = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    for l in range(L):
        for m in range(-l, l + 1):
            out += flm[l * l + l + m] * sps.sph_harm_y(l, m, th, ph)
    return out


def test_inverse_matches_library_harmonics():
    L = 10
    flm = inputs.uniform_complex_flm(L, seed=3)
    assert np.abs(sht.inverse(flm, L) - _library_inverse(flm, L)).max() < 1e-13


def test_y00_constant():
    L = 6
    flm = np.zeros(L * L, dtype=np.complex128)
    flm[0] = 1.0
    m = sht.inverse(flm, L)
    assert np.abs(m - 1 / math.sqrt(4 * math.pi)).max() < 1e-15


def test_mw_last_ring_is_south_pole():
    assert abs(sampling.mw_theta(9)[-1] - math.pi) < 1e-15


def test_forward_of_library_harmonic_is_delta():
    L = 9
    th = sampling.mw_theta(L)[:, None]
    ph = sampling.mw_phi(L)[None, :]
    for (l, m) in [(0, 0), (3, -2), (5, 5), (8, 1), (8, -8)]:
        y = sps.sph_harm_y(l, m, th, ph)
        f = sht.forward(y, L)
        exp = np.zeros(L * L, dtype=np.complex128)
        exp[l * l + l + m] = 1.0
        assert np.abs(f - exp).max() < 1e-13, (l, m)


def test_round_trip_complex_and_real():
    for L in (4, 16, 33):
        f = inputs.uniform_complex_flm(L, seed=L)
        assert np.abs(sht.forward(sht.inverse(f, L), L) - f).max() < 1e-12
    L = 24
    f = inputs.gaussian_real_flm(L, seed=0)
    m = sht.inverse(f, L)
    assert np.abs(m.imag).max() < 1e-15
    assert np.abs(sht.forward(m.real, L) - f).max() < 1e-13


def test_real_input_generator_symmetry():
    L = 12
    f = inputs.gaussian_real_flm(L, seed=5)
    for l in range(L):
        assert abs(f[l * l + l].imag) == 0.0
        for m in range(1, l + 1):
            assert f[l * l + l - m] == (-1) ** m * np.conj(f[l * l + l + m])


def test_point_source_flm_library_and_peak():
    # sum_k A_k conj(Y_lm(omega_k)) against the library Y_lm, and the peak of
    # the band-limited source: sum_lm |Y_lm(omega)|^2 = L^2 / (4 pi) (addition
    # theorem), so a single source of amplitude A is A L^2 / (4 pi) at omega.
    L = 12
    th = np.array([0.4, 2.0])
    ph = np.array([1.0, 5.5])
    amp = np.array([1.5, -0.5])
    f = sht.point_source_flm(L, th, ph, amp)
    for l in range(L):
        for m in range(-l, l + 1):
            ref = np.sum(amp * np.conj(sps.sph_harm_y(l, m, th, ph)))
            assert abs(f[sht.lm_index(l, m)] - ref) < 1e-14
    one = sht.point_source_flm(L, th[:1], ph[:1], np.array([2.0]))
    val = sum(one[sht.lm_index(l, m)] * sps.sph_harm_y(l, m, th[0], ph[0])
              for l in range(L) for m in range(-l, l + 1))
    assert abs(val - 2.0 * L * L / (4 * np.pi)) < 1e-12
