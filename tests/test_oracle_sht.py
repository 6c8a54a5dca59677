"""Pins for oracle.sht (spin-0 SHT on McEwen-Wiaux sampling)."""
import math

import numpy as np
import pytest
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


# ---- spin-s transforms (Sec. II-A) ----

def _sY_sum(l, m, s, th, ph):
    # sY_lm from the explicit factorial sum of d (exact, mpmath)
    from oracle import wigner
    return ((-1.0) ** s * math.sqrt((2 * l + 1) / (4 * math.pi))
            * float(wigner.d_sum(l, m, -s, th)) * np.exp(1j * m * ph))


@pytest.mark.parametrize("s", [0, 1, -2, 3])
def test_inverse_spin_against_explicit_sum(s):
    L = 6
    rng = np.random.default_rng(40 + s)
    f = rng.standard_normal(L * L) + 1j * rng.standard_normal(L * L)
    for l in range(abs(s)):
        f[l * l:(l + 1) * (l + 1)] = 0
    m_ = sht.inverse_spin(f, L, s)
    th = sampling.mw_theta(L)
    ph = sampling.mw_phi(L)
    for t in (0, 2, L - 1):
        for p in (0, 3, 2 * L - 2):
            ref = sum(f[sht.lm_index(l, m)] * _sY_sum(l, m, s, th[t], ph[p])
                      for l in range(abs(s), L) for m in range(-l, l + 1))
            assert abs(m_[t, p] - ref) < 1e-13


def test_spin_one_textbook_value():
    # 1Y_10 = sqrt(3/(8 pi)) sin(theta) in the convention of Sec. II-A
    L = 3
    f = np.zeros(L * L, dtype=np.complex128)
    f[sht.lm_index(1, 0)] = 1.0
    m_ = sht.inverse_spin(f, L, 1)
    th = sampling.mw_theta(L)
    assert np.allclose(m_, (math.sqrt(3 / (8 * math.pi)) * np.sin(th))[:, None], atol=1e-15)


def test_spin_ll_closed_form():
    # the closed form of d^l_{l,-s}(theta) the paper writes in its FWHM analysis
    # (Sec. II-B): (-1)^(l+s) sqrt((2l)!/((l-s)!(l+s)!)) sin(theta/2)^(l+s) cos(theta/2)^(l-s)
    L, s, l = 9, 2, 7
    f = np.zeros(L * L, dtype=np.complex128)
    f[sht.lm_index(l, l)] = 1.0
    m_ = sht.inverse_spin(f, L, s)
    th = sampling.mw_theta(L)
    ph = sampling.mw_phi(L)
    d = ((-1.0) ** (l + s) * math.sqrt(math.factorial(2 * l) / (math.factorial(l + s) * math.factorial(l - s)))
         * np.cos(th / 2) ** (l - s) * np.sin(th / 2) ** (l + s))
    ref = (-1.0) ** s * math.sqrt((2 * l + 1) / (4 * math.pi)) * d[:, None] * np.exp(1j * l * ph)[None, :]
    assert np.abs(m_ - ref).max() < 1e-13


@pytest.mark.parametrize("s", [0, 2, -1])
def test_spin_round_trip_and_conjugate_symmetry(s):
    L = 10
    rng = np.random.default_rng(7)
    f = rng.uniform(-1, 1, L * L) + 1j * rng.uniform(-1, 1, L * L)
    for l in range(abs(s)):
        f[l * l:(l + 1) * (l + 1)] = 0
    m_ = sht.inverse_spin(f, L, s)
    assert np.abs(sht.forward_spin(m_, L, s) - f).max() < 1e-12
    # conj(sY_lm) = (-1)^(s+m) (-s)Y_{l,-m}: conj of the spin-s map is the
    # spin -s map of g_lm = (-1)^(s+m) conj(f_{l,-m})
    g = np.zeros_like(f)
    for l in range(L):
        for m in range(-l, l + 1):
            g[sht.lm_index(l, m)] = (-1.0) ** (s + m) * np.conj(f[sht.lm_index(l, -m)])
    assert np.abs(np.conj(m_) - sht.inverse_spin(g, L, -s)).max() < 1e-12
    if s == 0:  # spin 0 agrees with the spin-0 transforms (pinned to library Y_lm)
        assert np.abs(m_ - sht.inverse(f, L)).max() < 1e-13
