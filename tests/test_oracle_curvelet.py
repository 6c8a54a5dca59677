"""Pins for oracle.curvelet (Sec. II-D analysis / synthesis, Sec. III-C accuracy)."""
import math

import numpy as np
import pytest
import scipy.special as sps

from oracle import curvelet, sampling, so3, wigner
from paper_1511_05578_amd import inputs


def _rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


def _rot_y(b):
    c, s = math.cos(b), math.sin(b)
    return np.array([[c, 0, s], [0, 1.0, 0], [-s, 0, c]])


def _sh_eval(coeff_lm, L, theta, phi):
    out = np.zeros(np.shape(theta), dtype=np.complex128)
    for l in range(L):
        for m in range(-l, l + 1):
            c = coeff_lm(l, m)
            if c != 0:
                out += c * sps.sph_harm_y(l, m, theta, phi)
    return out


def test_analysis_brute_force_rotation_on_sphere():
    # W(rho) = int f(w) (R_rho psi)^*(w) dw, with (R_rho psi)(w) = psi(R^-1 w) and
    # R = Rz(alpha) Ry(beta) Rz(gamma) (zyz: gamma about z, then beta about y, then
    # alpha about z, in the fixed frame), evaluated by exact quadrature on the
    # sphere with library spherical harmonics: independent of every Wigner-D
    # formula in the oracle.
    L, lam, J0 = 7, 2.0, 1
    plan = curvelet.Plan(L, lam, J0)
    flm = inputs.uniform_complex_flm(L, seed=11)
    j = plan.J
    Lj = plan.Lj[j]
    P = plan.psi_j(j, Lj)
    grid = curvelet.analysis_scale(plan, flm, j)
    # quadrature: Gauss-Legendre in cos(theta) x uniform phi; exact for degree <= 2L-2
    x, w = np.polynomial.legendre.leggauss(2 * L)
    th = np.arccos(x)
    ph = 2 * np.pi * np.arange(4 * L) / (4 * L)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    Wq = np.repeat(w[:, None], len(ph), axis=1) * (2 * np.pi / len(ph))
    fvals = _sh_eval(lambda l, m: flm[l * l + l + m], L, TH, PH)
    vec = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    al, be, ga = sampling.so3_alpha(Lj), sampling.so3_beta(Lj), sampling.so3_gamma(Lj)
    for (a, b, g) in [(0, 0, 0), (2, 1, 3), (5, 3, 1), (7, 6, 10), (12, 2, 9)]:
        R = _rot_z(al[a]) @ _rot_y(be[b]) @ _rot_z(ga[g])
        v = vec @ R  # rows: R^T v = R^{-1} v
        th2 = np.arccos(np.clip(v[..., 2], -1, 1))
        ph2 = np.arctan2(v[..., 1], v[..., 0])
        psi = _sh_eval(lambda l, n: P[l, n + Lj - 1] if abs(n) < Lj else 0.0, Lj, th2, ph2)
        brute = np.sum(Wq * fvals * np.conj(psi))
        assert abs(brute - grid[a, b, g]) < 1e-13, (a, b, g, brute, grid[a, b, g])


@pytest.mark.parametrize("L,J0", [(8, 1), (16, 2), (32, 2)])
def test_exact_reconstruction_real(L, J0):
    plan = curvelet.Plan(L, 2.0, J0)
    flm = inputs.gaussian_real_flm(L, seed=0)
    scal, grids = curvelet.analysis(plan, flm)
    for g in grids.values():
        assert np.abs(g.imag).max() <= 1e-14 * max(np.abs(g.real).max(), 1e-300)
    assert np.abs(scal.imag).max() < 1e-15
    rec = curvelet.synthesis(plan, scal, grids)
    assert np.abs(rec - flm).max() < 1e-13


@pytest.mark.parametrize("L", [4, 8, 16])
def test_round_trip_paper_accuracy_experiment(L):
    # Sec. III-C: complex signals with Re, Im ~ U[-1, 1]; error max_lm |f^r - f^o|
    # is close to machine precision.
    plan = curvelet.Plan(L, 2.0, 1)
    for seed in range(3):
        flm = inputs.uniform_complex_flm(L, seed=seed)
        scal, grids = curvelet.analysis(plan, flm)
        rec = curvelet.synthesis(plan, scal, grids)
        assert np.abs(rec - flm).max() < 2e-14 * L


def test_tight_frame_energy():
    # sum|f_lm|^2 = sum|(W^Phi)_lm|^2 + sum_j sum_lmn (2l+1)/(8pi^2) |(W^j)^l_mn|^2
    L = 16
    plan = curvelet.Plan(L, 2.0, 2)
    flm = inputs.gaussian_real_flm(L, seed=4)
    scal, grids = curvelet.analysis(plan, flm)
    e = np.sum(np.abs(curvelet.scaling_flm(plan, flm)) ** 2)
    for j, g in grids.items():
        Lj = plan.Lj[j]
        F = so3.forward(g, Lj, Lj)
        ls = np.arange(Lj)[:, None, None]
        e += np.sum((2 * ls + 1) / (8 * math.pi ** 2) * np.abs(F) ** 2)
    assert abs(e - np.sum(np.abs(flm) ** 2)) < 1e-13 * np.sum(np.abs(flm) ** 2)


def test_inverse_rotation_gives_abs_k_equal_l():
    # Rotating the Wigner coefficients back by rho*' = (0, -theta_j, 0) leaves only
    # |k| = l (Sec. III-A-1): F~^l_mk = sum_n F^l_mn D^{l*}_kn(rho*').
    L = 16
    plan = curvelet.Plan(L, 2.0, 2)
    flm = inputs.gaussian_real_flm(L, seed=7)
    j = plan.J
    Lj = plan.Lj[j]
    F = so3.forward(curvelet.analysis_scale(plan, flm, j), Lj, Lj)
    scale = np.abs(F).max()
    for l in range(2, Lj):
        d = wigner.d_matrix(l, -math.pi / 2)      # D^l_kn(0,-pi/2,0) = d^l_kn(-pi/2), real
        sub = F[l, Lj - 1 - l:Lj + l, Lj - 1 - l:Lj + l]   # [m, n]
        Ft = sub @ d.T                               # [m, k]
        mask = np.ones(2 * l + 1, bool)
        mask[[0, 2 * l]] = False
        assert np.abs(Ft[:, mask]).max() <= 1e-13 * scale, l
