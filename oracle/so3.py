"""Wigner transforms on SO(3) with McEwen-Wiaux SO(3) sampling, from their definitions.

Test infrastructure (see ``oracle/__init__.py``).

Conventions (Sec. II-A, Sec. II-D): D^l_mn(a, b, g) = e^{-i m a} d^l_mn(b) e^{-i n g};
orthogonality int D^l_mn D^{l'*}_{m'n'} d rho = 8 pi^2/(2l+1) delta delta delta with
d rho = sin(b) da db dg; F^l_mn = <F, D^{l*}_mn>; the inverse transform is
F(rho) = sum_lmn (2l+1)/(8 pi^2) F^l_mn D^{l*}_mn(rho).

Grids are arrays [a][b][g] of shape (2M-1, L, 2N-1) with M = L (alpha
band-limit equal to L); coefficients are dense arrays F[l, m + L - 1, n + N - 1]
(zero where |m| > l or |n| > l).

* ``inverse``: direct evaluation of the sum; for each beta row the l-sum with
  d from ``wigner.d_iter``, then plain Fourier matrices in alpha and gamma.
* ``forward``: alpha/gamma Fourier coefficients of each beta row (exact for a
  band-limited function), exact trigonometric interpolation in beta (extension
  X_mn(2 pi - b) = (-1)^(m+n) X_mn(b)) to L Gauss-Legendre nodes, then
  F^l_mn = (2 pi)^2 sum_q w_q d^l_mn(b_q) X_mn(b_q), exact because
  d^l_mn d^l'_mn is a polynomial in cos(b) of degree l + l' <= 2L-2.
"""
import math

import numpy as np

from . import sampling, sht, wigner


def inverse_rows(L, N, coeff_of_l, rows=None, lmin=0):
    """Grid rows W[a, b, g] for b in ``rows`` (all if None).

    ``coeff_of_l(l)`` returns C^l[m + L - 1, n + N - 1] = (2l+1)/(8pi^2) F^l_mn
    (or None to skip l); W = sum_mn e^{i m a} e^{i n g} sum_l d^l_mn(b) C^l_mn.
    """
    betas = sampling.so3_beta(L)
    if rows is None:
        rows = range(L)
    rows = list(rows)
    Ea = sampling.dft_matrix(np.arange(-(L - 1), L), sampling.so3_alpha(L), +1)  # [a, m]
    Eg = sampling.dft_matrix(np.arange(-(N - 1), N), sampling.so3_gamma(N), +1)  # [g, n]
    out = np.zeros((2 * L - 1, len(rows), 2 * N - 1), dtype=np.complex128)
    for i, b in enumerate(rows):
        T = np.zeros((2 * L - 1, 2 * N - 1), dtype=np.complex128)
        for l, D in wigner.d_iter(L, betas[b], L, N):
            if l < lmin:
                continue
            C = coeff_of_l(l)
            if C is None:
                continue
            T += D * C
        out[:, i, :] = Ea @ T @ Eg.T
    return out


def inverse(F, L, N):
    """Dense inverse Wigner transform of F[l, m + L - 1, n + N - 1]."""
    ls = np.arange(L)
    scale = (2 * ls + 1) / (8 * math.pi ** 2)
    return inverse_rows(L, N, lambda l: scale[l] * F[l])


def gl_rows(grid, L, N):
    """X_q[q, m + L - 1, n + N - 1] = X_mn(b_q) at the L Gauss-Legendre nodes, and weights."""
    grid = np.asarray(grid, dtype=np.complex128)
    Ea = sampling.dft_matrix(np.arange(-(L - 1), L), sampling.so3_alpha(L), -1)  # [a, m]
    Eg = sampling.dft_matrix(np.arange(-(N - 1), N), sampling.so3_gamma(N), -1)  # [g, n]
    norm = 1.0 / ((2 * L - 1) * (2 * N - 1))
    Xb = np.einsum('abg,am,gn->bmn', grid, Ea, Eg, optimize=True) * norm
    nodes, weights = sampling.gauss_legendre_beta(L)
    E1, E2 = sht.theta_interp_matrices(L, nodes)
    ms = np.arange(-(L - 1), L)[:, None]
    ns = np.arange(-(N - 1), N)[None, :]
    sgn = (-1.0) ** np.abs(ms + ns)
    shp = Xb.shape
    flat = Xb.reshape(L, -1)
    Xq = (E1 @ flat).reshape(len(nodes), *shp[1:]) \
        + (E2 @ flat).reshape(len(nodes), *shp[1:]) * sgn[None]
    return nodes, weights, Xq


def forward(grid, L, N):
    """Dense forward Wigner transform: F[l, m + L - 1, n + N - 1]."""
    nodes, weights, Xq = gl_rows(grid, L, N)
    F = np.zeros((L, 2 * L - 1, 2 * N - 1), dtype=np.complex128)
    for q, bq in enumerate(nodes):
        for l, D in wigner.d_iter(L, bq, L, N):
            F[l] += weights[q] * D * Xq[q]
    return F * (2 * math.pi) ** 2
