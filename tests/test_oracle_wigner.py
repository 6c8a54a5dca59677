"""Pins for oracle.wigner: d^l_mn(beta) (Sec. II-A, factorial-sum expression).

Each test ties the oracle to something other than itself: textbook closed
forms, library Legendre / spherical-harmonic routines, group properties
(unitarity, composition, identity, symmetries) and exact multiprecision sums.
"""
import math

import numpy as np
import pytest
import scipy.special as sps

from oracle import wigner

BETAS = [0.0, 0.37, 1.1, math.pi / 2, 2.3, 3.0, math.pi]


@pytest.mark.parametrize("beta", [0.37, 1.1, 2.3])
def test_d1_textbook(beta):
    # Rank-1 matrix elements in the standard (Condon-Shortley, zyz) convention.
    D = wigner.d_matrix_sum(1, beta)
    c = math.cos(beta)
    s = math.sin(beta)
    exp = np.array([[(1 + c) / 2, s / math.sqrt(2), (1 - c) / 2],
                    [-s / math.sqrt(2), c, s / math.sqrt(2)],
                    [(1 - c) / 2, -s / math.sqrt(2), (1 + c) / 2]])
    # rows are m = -1, 0, 1; columns n = -1, 0, 1
    assert np.allclose(D, exp, atol=1e-15)
    assert np.allclose(wigner.d_matrix(1, beta), exp, atol=1e-15)


@pytest.mark.parametrize("beta", [0.2, 1.3, 2.8])
def test_d_l00_is_legendre(beta):
    for l in range(0, 30):
        D = wigner.d_matrix(l, beta)
        assert abs(D[l, l] - sps.eval_legendre(l, math.cos(beta))) < 1e-13


@pytest.mark.parametrize("theta", [0.25, 1.0, 2.2])
def test_d_m0_matches_library_spherical_harmonics(theta):
    # Y_lm(theta, 0) = sqrt((2l+1)/(4pi)) d^l_{m0}(theta)  (Sec. II-A, spin 0)
    L = 20
    T = wigner.d_m0_table(L, theta)
    for l in range(L):
        for m in range(0, l + 1):
            y = sps.sph_harm_y(l, m, theta, 0.0)
            assert abs(math.sqrt((2 * l + 1) / (4 * math.pi)) * T[l, m] - y.real) < 1e-13
            assert abs(y.imag) < 1e-14


@pytest.mark.parametrize("beta", BETAS)
def test_recurrence_matches_exact_sum(beta):
    for l in range(0, 11):
        A = wigner.d_matrix(l, beta)
        B = wigner.d_matrix_sum(l, beta)
        assert np.abs(A - B).max() < 3e-15, (l, beta)


def test_recurrence_matches_exact_sum_l17():
    A = wigner.d_matrix(17, 0.77)
    B = wigner.d_matrix_sum(17, 0.77)
    assert np.abs(A - B).max() < 3e-15


@pytest.mark.parametrize("beta", [0.05, 0.9, 2.0, 3.1])
def test_unitarity(beta):
    for l, D in wigner.d_iter(64, beta):
        if l in (5, 31, 63):
            S = D[63 - l:63 + l + 1, 63 - l:63 + l + 1]
            assert np.abs(S @ S.T - np.eye(2 * l + 1)).max() < 1e-13


def test_identity_and_pi():
    for l in (3, 12, 40):
        assert np.abs(wigner.d_matrix(l, 0.0) - np.eye(2 * l + 1)).max() == 0.0
        Dp = wigner.d_matrix(l, math.pi)
        exp = np.zeros_like(Dp)
        for m in range(-l, l + 1):
            exp[m + l, -m + l] = (-1) ** (l + m)
        assert np.abs(Dp - exp).max() < 1e-14


def test_composition():
    # d^l(b1 + b2) = d^l(b1) d^l(b2): rotations about y compose additively.
    for l in (7, 25):
        A = wigner.d_matrix(l, 0.4)
        B = wigner.d_matrix(l, 1.3)
        C = wigner.d_matrix(l, 1.7)
        assert np.abs(A @ B - C).max() < 1e-13


def test_symmetries():
    l = 19
    D = wigner.d_matrix(l, 1.234)
    for m in range(-l, l + 1):
        for n in range(-l, l + 1):
            v = D[m + l, n + l]
            assert abs(v - (-1) ** (m - n) * D[n + l, m + l]) < 1e-15
            assert abs(v - D[-n + l, -m + l]) < 1e-15


def test_edge_closed_form_paper():
    # d^l_{l,-s}(theta) = (-1)^(l+s) sqrt((2l)!/((l-s)!(l+s)!)) sin^(l+s)(t/2) cos^(l-s)(t/2)
    th = 1.9
    for l in (4, 15):
        D = wigner.d_matrix(l, th)
        for s in range(-l, l + 1):
            exp = (-1) ** (l + s) * math.sqrt(math.factorial(2 * l)
                                              / (math.factorial(l - s) * math.factorial(l + s))) \
                * math.sin(th / 2) ** (l + s) * math.cos(th / 2) ** (l - s)
            assert abs(D[l + l, -s + l] - exp) < 1e-14


def test_reduced_range_iteration_agrees():
    # Restricting |n| < N must not change the values (N < L path).
    beta = 0.81
    full = {l: D.copy() for l, D in wigner.d_iter(12, beta)}
    for l, D in wigner.d_iter(12, beta, 12, 4):
        assert np.abs(D - full[l][:, 11 - 3:11 + 4]).max() < 1e-15
