"""Pins for oracle.so3 (Wigner transforms on MW-sampled SO(3))."""
import math

import numpy as np
import pytest

from oracle import sampling, so3, wigner


def _random_F(L, N, seed):
    rng = np.random.default_rng(seed)
    F = np.zeros((L, 2 * L - 1, 2 * N - 1), dtype=np.complex128)
    for l in range(L):
        for m in range(-l, l + 1):
            for n in range(-min(l, N - 1), min(l, N - 1) + 1):
                F[l, m + L - 1, n + N - 1] = rng.uniform(-1, 1) + 1j * rng.uniform(-1, 1)
    return F


@pytest.mark.parametrize("l,m,n", [(0, 0, 0), (2, 1, -1), (3, -3, 2), (4, 2, 4)])
def test_single_mode_is_conjugate_wigner_D(l, m, n):
    # F^l'_m'n' = delta  =>  W(rho) = (2l+1)/(8pi^2) D^{l*}_mn(rho),
    # D^l_mn(a,b,g) = e^{-ima} d^l_mn(b) e^{-ing} with d from the exact factorial sum.
    L = N = 5
    F = np.zeros((L, 2 * L - 1, 2 * N - 1), dtype=np.complex128)
    F[l, m + L - 1, n + N - 1] = 1.0
    W = so3.inverse(F, L, N)
    al, be, ga = sampling.so3_alpha(L), sampling.so3_beta(L), sampling.so3_gamma(N)
    for (a, b, g) in [(0, 0, 0), (3, 1, 7), (8, 4, 2), (5, 2, 5)]:
        D = math.e ** 0 * complex(np.exp(-1j * m * al[a]) * float(wigner.d_sum(l, m, n, be[b]))
                                  * np.exp(-1j * n * ga[g]))
        exp = (2 * l + 1) / (8 * math.pi ** 2) * np.conj(D)
        assert abs(W[a, b, g] - exp) < 1e-15


@pytest.mark.parametrize("L,N", [(6, 6), (8, 3), (9, 9)])
def test_round_trip(L, N):
    F = _random_F(L, N, seed=L * 10 + N)
    G = so3.forward(so3.inverse(F, L, N), L, N)
    assert np.abs(G - F).max() < 1e-12


def test_forward_orthogonality_on_exact_D():
    # Forward transform of (2l+1)/(8pi^2) D^{l*}_mn sampled exactly returns delta_{l m n}.
    L = N = 6
    l, m, n = 4, -3, 1
    al, be, ga = sampling.so3_alpha(L), sampling.so3_beta(L), sampling.so3_gamma(N)
    W = np.zeros((2 * L - 1, L, 2 * N - 1), dtype=np.complex128)
    for b in range(L):
        d = float(wigner.d_sum(l, m, n, be[b]))
        W[:, b, :] = (2 * l + 1) / (8 * math.pi ** 2) * np.conj(
            np.exp(-1j * m * al)[:, None] * d * np.exp(-1j * n * ga)[None, :])
    F = so3.forward(W, L, N)
    exp = np.zeros_like(F)
    exp[l, m + L - 1, n + N - 1] = 1.0
    assert np.abs(F - exp).max() < 1e-13
