"""Pins for the unrotated curvelet coefficients of the oracle (Sec. III-A-1).

The unrotated curvelets psi~ keep the directional component zeta~ (non-zero
only at |n| = l); their coefficients are W~(rho) = <f, R_rho psi~>.  Since the
rotated curvelets are psi = R_{rho*} psi~ with rho* = (0, pi/2, 0), the two
grids are one function right-translated: W~(rho) = W(rho rho*^-1).
"""
import math

import numpy as np
import pytest
import scipy.special as sps

from oracle import curvelet, sampling, so3
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


class _Sphere:
    """Exact quadrature of band-limited products on the sphere (Gauss-Legendre
    in cos(theta) x uniform phi), with library spherical harmonics only."""

    def __init__(self, L, flm):
        x, w = np.polynomial.legendre.leggauss(2 * L)
        th = np.arccos(x)
        ph = 2 * np.pi * np.arange(4 * L) / (4 * L)
        TH, PH = np.meshgrid(th, ph, indexing="ij")
        self.W = np.repeat(w[:, None], len(ph), axis=1) * (2 * np.pi / len(ph))
        self.f = _sh_eval(lambda l, m: flm[l * l + l + m], L, TH, PH)
        self.vec = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)

    def coefficient(self, R, P, Lj):
        """<f, R psi> with (R psi)(w) = psi(R^-1 w), psi from P[l, n + Lj - 1]."""
        v = self.vec @ R  # rows: R^T v = R^-1 v
        th2 = np.arccos(np.clip(v[..., 2], -1, 1))
        ph2 = np.arctan2(v[..., 1], v[..., 0])
        psi = _sh_eval(lambda l, n: P[l, n + Lj - 1] if abs(n) < Lj else 0.0, Lj, th2, ph2)
        return np.sum(self.W * self.f * np.conj(psi))


def _euler(al, be, ga):
    return _rot_z(al) @ _rot_y(be) @ _rot_z(ga)


POINTS = [(0, 0, 0), (2, 1, 3), (5, 3, 1), (7, 6, 10), (12, 2, 9)]


def test_unrotated_kernel_support_is_abs_n_equal_l():
    plan = curvelet.Plan(16, 2.0, 2, rotated=False)
    L = plan.L
    for jj, j in enumerate(plan.scales):
        P = plan.psi[jj]
        for l in range(L):
            for n in range(-(L - 1), L):
                if abs(n) != l:
                    assert P[l, n + L - 1] == 0.0
        # real curvelet: Psi_{l,-n} = (-1)^n conj(Psi_ln)
        for l in range(1, L):
            assert P[l, -l + L - 1] == pytest.approx((-1) ** l * P[l, l + L - 1], abs=0)


def test_unrotated_analysis_brute_force_on_sphere():
    # W~(rho) = <f, R_rho psi~> by quadrature on the sphere, independent of every
    # Wigner-D formula in the oracle.
    L = 7
    plan = curvelet.Plan(L, 2.0, 1, rotated=False)
    flm = inputs.uniform_complex_flm(L, seed=12)
    sph = _Sphere(L, flm)
    j = plan.J
    Lj = plan.Lj[j]
    grid = curvelet.analysis_scale(plan, flm, j)
    al, be, ga = sampling.so3_alpha(Lj), sampling.so3_beta(Lj), sampling.so3_gamma(Lj)
    for a, b, g in POINTS:
        brute = sph.coefficient(_euler(al[a], be[b], ga[g]), plan.psi_j(j, Lj), Lj)
        assert abs(brute - grid[a, b, g]) < 1e-13, (a, b, g, brute, grid[a, b, g])


def test_right_translation_by_rho_star():
    # W~(rho) = W(rho rho*^-1): the unrotated grid at rho equals the rotated
    # curvelet coefficient for the rotation R(rho) Ry(pi/2)^-1, evaluated on the
    # sphere with the rotated kernel.  The other composition order must fail,
    # so the test sees the side rho* acts on.
    L = 7
    rot = curvelet.Plan(L, 2.0, 1)
    unr = curvelet.Plan(L, 2.0, 1, rotated=False)
    flm = inputs.uniform_complex_flm(L, seed=13)
    sph = _Sphere(L, flm)
    j = rot.J
    Lj = rot.Lj[j]
    grid = curvelet.analysis_scale(unr, flm, j)
    al, be, ga = sampling.so3_alpha(Lj), sampling.so3_beta(Lj), sampling.so3_gamma(Lj)
    Rs_inv = _rot_y(math.pi / 2).T
    worst_wrong = 0.0
    for a, b, g in POINTS:
        R = _euler(al[a], be[b], ga[g])
        w = sph.coefficient(R @ Rs_inv, rot.psi_j(j, Lj), Lj)
        assert abs(w - grid[a, b, g]) < 1e-13, (a, b, g)
        wrong = sph.coefficient(Rs_inv @ R, rot.psi_j(j, Lj), Lj)
        worst_wrong = max(worst_wrong, abs(wrong - grid[a, b, g]))
    assert worst_wrong > 1e-3


def test_unrotated_grid_wigner_support():
    # The Wigner coefficients of every unrotated grid vanish unless |n| = l.
    L = 16
    plan = curvelet.Plan(L, 2.0, 2, rotated=False)
    flm = inputs.gaussian_real_flm(L, seed=8)
    for j in plan.scales:
        Lj = plan.Lj[j]
        F = so3.forward(curvelet.analysis_scale(plan, flm, j), Lj, Lj)
        scale = np.abs(F).max()
        for l in range(Lj):
            row = F[l]  # [m, n]
            mask = np.ones(2 * Lj - 1, bool)
            mask[[Lj - 1 - l, Lj - 1 + l]] = False
            assert np.abs(row[:, mask]).max() <= 1e-13 * scale, (j, l)


@pytest.mark.parametrize("L,J0", [(8, 1), (16, 2), (32, 2)])
def test_unrotated_exact_reconstruction_real(L, J0):
    plan = curvelet.Plan(L, 2.0, J0, rotated=False)
    flm = inputs.gaussian_real_flm(L, seed=1)
    scal, grids = curvelet.analysis(plan, flm)
    for g in grids.values():
        assert np.abs(g.imag).max() <= 1e-14 * max(np.abs(g.real).max(), 1e-300)
    rec = curvelet.synthesis(plan, scal, grids)
    assert np.abs(rec - flm).max() < 1e-13


def test_unrotated_exact_reconstruction_complex():
    L = 8
    plan = curvelet.Plan(L, 2.0, 1, rotated=False)
    flm = inputs.uniform_complex_flm(L, seed=2)
    scal, grids = curvelet.analysis(plan, flm)
    rec = curvelet.synthesis(plan, scal, grids)
    assert np.abs(rec - flm).max() < 2e-14 * L
