"""Pins for oracle.kernels (Sec. II-B, Sec. II-D admissibility)."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sps

from oracle import kernels


def _k_scipy(t, lam):
    # Independent evaluation of k_lambda with adaptive Gauss-Kronrod (QUADPACK).
    def s2(u):
        x = 2 * lam / (lam - 1) * (u - 1 / lam) - 1
        if abs(x) >= 1:
            return 0.0
        return math.exp(-2.0 / (1 - x * x)) / u
    if t <= 1 / lam:
        return 1.0
    if t >= 1:
        return 0.0
    num = si.quad(s2, t, 1, epsabs=0, epsrel=2e-14, limit=400)[0]
    den = si.quad(s2, 1 / lam, 1, epsabs=0, epsrel=2e-14, limit=400)[0]
    return num / den


@pytest.mark.parametrize("lam", [2.0, 1.5, 3.0])
def test_k_lambda_two_quadratures(lam):
    for t in np.linspace(1 / lam + 1e-3, 1 - 1e-3, 13):
        assert abs(kernels.k_lambda(t, lam) - _k_scipy(t, lam)) < 1e-12


def test_k_lambda_limits_and_monotone():
    lam = 2.0
    assert kernels.k_lambda(0.1, lam) == 1.0
    assert kernels.k_lambda(0.5, lam) == 1.0
    assert kernels.k_lambda(1.0, lam) == 0.0
    assert kernels.k_lambda(3.0, lam) == 0.0
    ts = np.linspace(0.5, 1.0, 41)
    ks = [kernels.k_lambda(t, lam) for t in ts]
    assert all(a >= b for a, b in zip(ks, ks[1:]))


@pytest.mark.parametrize("lam", [2.0, 1.5])
def test_kappa_peak_and_support(lam):
    for j in (2, 3, 5):
        peak = lam ** j
        if abs(peak - round(peak)) < 1e-12:
            assert abs(kernels.kappa(j, int(round(peak)), lam) - 1.0) < 1e-14
        for l in range(0, int(lam ** (j + 1)) + 3):
            inside = lam ** (j - 1) < l < lam ** (j + 1)
            if not inside:
                assert kernels.kappa(j, l, lam) == 0.0
            else:
                assert kernels.kappa(j, l, lam) > 0.0


@pytest.mark.parametrize("L,lam,J0", [(64, 2.0, 2), (40, 2.0, 1), (50, 1.5, 3)])
def test_admissibility(L, lam, J0):
    # 4pi/(2l+1)|Phi_l0|^2 + 8pi^2/(2l+1) sum_j sum_n |Psi^(j)_ln|^2 = 1 for every l < L
    J = kernels.num_scales(L, lam)
    P = kernels.psi_table(L, lam, J0, J)
    phi = kernels.phi_table(L, lam, J0)
    for l in range(L):
        tot = 4 * math.pi / (2 * l + 1) * phi[l] ** 2 \
            + 8 * math.pi ** 2 / (2 * l + 1) * np.sum(np.abs(P[:, l, :]) ** 2)
        assert abs(tot - 1.0) < 1e-13, l


def test_zeta_normalisation_closed_form_and_parity():
    L = 40
    Z = kernels.zeta_table(L)
    for l in range(1, L):
        row = Z[l]
        assert abs(np.sum(row ** 2) - 1.0) < 1e-13
        for n in range(-l, l + 1):
            v = row[n + L - 1]
            if n % 2:
                assert abs(v) < 1e-14
            else:
                exp = math.sqrt(2.0) * math.sqrt(math.comb(2 * l, l + n)) / 2.0 ** l
                assert abs(v - exp) < 1e-13


def test_psi_is_real_curvelet():
    # Real curvelet <=> Psi_{l,-n} = (-1)^n conj(Psi_ln) (Sec. II-A conjugate symmetry)
    L = 32
    P = kernels.psi_table(L, 2.0, 2, kernels.num_scales(L, 2.0))
    for n in range(0, L):
        assert np.allclose(P[:, :, L - 1 - n], (-1) ** n * P[:, :, L - 1 + n], atol=1e-16)


def _psi_on_sphere(coeffs, L, theta, phi):
    # psi(theta, phi) = sum_ln coeffs[l, n + L - 1] Y_ln via the library routine
    out = np.zeros(np.broadcast(theta, phi).shape, dtype=np.complex128)
    for l in range(L):
        for n in range(-l, l + 1):
            c = coeffs[l, n + L - 1]
            if c != 0:
                out += c * sps.sph_harm_y(l, n, theta, phi)
    return out


def test_rotated_curvelet_centred_on_north_pole():
    # Rotated curvelets are centred on the North pole; unrotated ones on the
    # -x axis (theta = pi/2, phi = pi) (Sec. II-B).
    L, lam, J0 = 32, 2.0, 2
    J = kernels.num_scales(L, lam)
    P = kernels.psi_table(L, lam, J0, J)
    j = 4
    th = np.linspace(0, math.pi, 61)[:, None]
    ph = np.linspace(0, 2 * math.pi, 120, endpoint=False)[None, :]
    vals = np.abs(_psi_on_sphere(P[j - J0], L, th, ph))
    it, ip = np.unravel_index(np.argmax(vals), vals.shape)
    assert it == 0
    # unrotated: coefficients sqrt((2l+1)/8pi^2) kappa zeta~
    U = np.zeros_like(P[j - J0])
    for l in range(L):
        k = kernels.kappa(j, l, lam) * math.sqrt((2 * l + 1) / (8 * math.pi ** 2))
        for n in (-l, l):
            U[l, n + L - 1] = k * kernels.zeta_tilde(l, n)
    vals = np.abs(_psi_on_sphere(U, L, th, ph))
    it, ip = np.unravel_index(np.argmax(vals), vals.shape)
    assert abs(th[it, 0] - math.pi / 2) < 1e-12 and abs(ph[0, ip] - math.pi) < 1e-12


def test_scale_parameters():
    assert kernels.num_scales(32, 2.0) == 5
    assert kernels.num_scales(256, 2.0) == 8
    assert kernels.num_scales(1024, 2.0) == 10
    assert [kernels.scale_bandlimit(j, 256, 2.0) for j in range(2, 9)] == \
        [8, 16, 32, 64, 128, 256, 256]
    assert kernels.scaling_bandlimit(256, 2.0, 2) == 4


# ---- pins of the integrand of k_lambda (Sec. II-B) by values the definition fixes ----
# s(x) = exp(-1/(1-x^2)) on (-1, 1): s(0) = e^-1, s(1/2) = e^(-4/3), s(+-1) = 0.
# s_lambda(t) = s(2 lambda/(lambda-1) (t - 1/lambda) - 1) maps t = 1/lambda to
# x = -1, t = 1 to x = +1 and the midpoint (1 + 1/lambda)/2 to x = 0.

def test_s_bump_values():
    assert float(kernels.s_bump(0)) == pytest.approx(math.exp(-1.0), rel=1e-15)
    assert float(kernels.s_bump(0.5)) == pytest.approx(math.exp(-4.0 / 3.0), rel=1e-15)
    assert float(kernels.s_bump(-0.5)) == pytest.approx(math.exp(-4.0 / 3.0), rel=1e-15)
    assert float(kernels.s_bump(1)) == 0.0 and float(kernels.s_bump(-1)) == 0.0
    assert float(kernels.s_bump(1.5)) == 0.0


@pytest.mark.parametrize("lam", [1.5, 2.0, 3.0])
def test_s_lambda_values(lam):
    assert float(kernels.s_lambda(1 / lam, lam)) == 0.0
    assert float(kernels.s_lambda(1.0, lam)) == 0.0
    mid = (1 + 1 / lam) / 2
    assert float(kernels.s_lambda(mid, lam)) == pytest.approx(math.exp(-1.0), rel=1e-14)
    # x = +-1/2 at t = 1/lambda + (1 +- 1/2)(lambda-1)/(2 lambda)
    for x in (-0.5, 0.5):
        t = 1 / lam + (x + 1) * (lam - 1) / (2 * lam)
        assert float(kernels.s_lambda(t, lam)) == pytest.approx(math.exp(-4.0 / 3.0), rel=1e-13)
    # zero outside (1/lambda, 1)
    assert float(kernels.s_lambda(0.99 / lam, lam)) == 0.0
    assert float(kernels.s_lambda(1.01, lam)) == 0.0


@pytest.mark.parametrize("lam", [1.5, 2.0, 3.0])
def test_k_lambda_strictly_decreasing_inside(lam):
    ts = np.linspace(1 / lam, 1.0, 23)[1:-1]
    ks = [kernels.k_lambda(t, lam) for t in ts]
    assert all(0.0 < k < 1.0 for k in ks)
    assert all(a > b for a, b in zip(ks, ks[1:]))


@pytest.mark.parametrize("lam", [1.5, 2.0, 3.0])
def test_k_lambda_slope_ratio(lam):
    # k_lambda(t) = int_t^1 g / int_{1/lambda}^1 g with g(u) = s_lambda(u)^2 / u, so
    # k'(t) = -g(t) / D and the ratio of slopes at two points is g(t_a) / g(t_b),
    # which the definition fixes without any quadrature: at the midpoint t_a
    # g = e^-2 / t_a, at x = 1/2 (t_b) g = e^(-8/3) / t_b.  The slopes are taken
    # from the oracle's k_lambda by central differences (error O(h^2)).
    ta = (1 + 1 / lam) / 2
    tb = 1 / lam + 1.5 * (lam - 1) / (2 * lam)
    h = 1e-4 * (1 - 1 / lam)
    slope = lambda t: (kernels.k_lambda(t + h, lam) - kernels.k_lambda(t - h, lam)) / (2 * h)
    ratio = slope(ta) / slope(tb)
    expect = (math.exp(-2.0) / ta) / (math.exp(-8.0 / 3.0) / tb)
    assert ratio == pytest.approx(expect, rel=1e-6)
    assert slope(ta) < 0
