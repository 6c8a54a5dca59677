"""Spherical harmonic transforms on McEwen-Wiaux sampling (spin 0 and spin s).

Test infrastructure (see ``oracle/__init__.py``).

Conventions (Sec. II-A): Y_lm(theta, phi) = sqrt((2l+1)/(4 pi)) d^l_{m0}(theta) e^{i m phi}
(Condon-Shortley phase carried by d), f_lm = <f, Y_lm>.  Harmonic arrays are
stored flat with index l^2 + l + m.

* ``inverse``: direct summation of f_lm Y_lm at every sample.
* ``forward``: f_lm = 2 pi sqrt((2l+1)/(4pi)) int_0^pi sin(t) d^l_{m0}(t) F_m(t) dt,
  where F_m(theta) is the exact phi-Fourier coefficient of the band-limited map.
  F_m is known at the L MW rings; its extension to [0, 2 pi) by
  F_m(2 pi - t) = (-1)^m F_m(t) is a trigonometric polynomial of degree L-1
  sampled at 2L-1 equispaced points, so plain trigonometric interpolation
  evaluates it exactly at Gauss-Legendre nodes, and L-point Gauss-Legendre in
  cos(theta) integrates the product exactly (polynomial degree <= 2L-2).
* ``inverse_spin`` / ``forward_spin``: the same two routes for a spin-s signal,
  with sY_lm = (-1)^s sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta) e^{i m phi}
  (Sec. II-A) in place of Y_lm: the theta extension of F_m has the parity
  (-1)^{m+s} (d^l_{m,-s}(-t) = (-1)^{m+s} d^l_{m,-s}(t)), and the product of
  two d^l_{m,-s} is still a polynomial in cos(theta) of degree <= 2L-2, so
  the Gauss-Legendre quadrature stays exact.  f_lm = 0 for l < |s|.
"""
import math

import numpy as np

from . import sampling, wigner


def lm_index(l, m):
    return l * l + l + m


def inverse(flm, L):
    """map[t, p] = sum_lm f_lm Y_lm(theta_t, phi_p), complex (L, 2L-1)."""
    flm = np.asarray(flm, dtype=np.complex128)
    thetas = sampling.mw_theta(L)
    phis = sampling.mw_phi(L)
    ms = np.arange(-(L - 1), L)
    Ephi = sampling.dft_matrix(ms, phis, +1)          # [p, m]
    F = np.zeros((L, 2 * L - 1), dtype=np.complex128)  # F[l, m + L - 1]
    for l in range(L):
        for m in range(-l, l + 1):
            F[l, m + L - 1] = flm[lm_index(l, m)] * math.sqrt((2 * l + 1) / (4 * math.pi))
    out = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    for t, th in enumerate(thetas):
        G = np.zeros(2 * L - 1, dtype=np.complex128)
        for l, D in wigner.d_iter(L, th, L, 1):
            G += D[:, 0] * F[l]
        out[t] = Ephi @ G
    return out


def _phi_coeffs(fmap, L):
    """F[t, m + L - 1] = (1/(2L-1)) sum_p map[t, p] e^{-i m phi_p}."""
    phis = sampling.mw_phi(L)
    ms = np.arange(-(L - 1), L)
    E = sampling.dft_matrix(ms, phis, -1)   # [p, m]
    return (np.asarray(fmap, dtype=np.complex128) @ E) / (2 * L - 1)


def theta_interp_matrices(L, nodes):
    """(E1, E2) with F(node_q) = sum_t E1[q,t] F(theta_t) + s * sum_t E2[q,t] F(theta_t)
    for a function whose extension obeys F(2pi - theta) = s F(theta):
    exact trigonometric interpolation through the 2L-1 extended samples."""
    Nt = 2 * L - 1
    th_ext = np.pi * (2 * np.arange(Nt) + 1) / Nt
    ks = np.arange(-(L - 1), L)
    # cardinal functions: C[q, t] = (1/Nt) sum_k e^{i k (node_q - th_t)}
    C = (np.exp(1j * np.outer(nodes, ks)) @ np.exp(-1j * np.outer(ks, th_ext))) / Nt
    E1 = C[:, :L]
    E2 = np.zeros((len(nodes), L), dtype=np.complex128)
    for t in range(L, Nt):
        E2[:, Nt - 1 - t] += C[:, t]
    return E1, E2


def forward(fmap, L):
    """f_lm of a band-limited map sampled on the MW grid (flat, length L^2)."""
    F = _phi_coeffs(fmap, L)                     # [t, m]
    nodes, weights = sampling.gauss_legendre_beta(L)
    E1, E2 = theta_interp_matrices(L, nodes)
    ms = np.arange(-(L - 1), L)
    sgn = (-1.0) ** np.abs(ms)
    Fq = E1 @ F + (E2 @ F) * sgn[None, :]        # [q, m]
    flm = np.zeros(L * L, dtype=np.complex128)
    acc = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    for q, th in enumerate(nodes):
        for l, D in wigner.d_iter(L, th, L, 1):
            acc[l] += weights[q] * D[:, 0] * Fq[q]
    for l in range(L):
        c = 2 * math.pi * math.sqrt((2 * l + 1) / (4 * math.pi))
        for m in range(-l, l + 1):
            flm[lm_index(l, m)] = c * acc[l, m + L - 1]
    return flm


def point_source_flm(L, theta, phi, amp):
    """f_lm = sum_k amp_k conj(Y_lm(theta_k, phi_k)), l < L (flat, length L^2):
    the band-limited point sources of amplitudes amp_k at the given positions
    (the projection of amp_k delta(omega - omega_k) onto Y_lm, Sec. II-A), with
    Y_lm = sqrt((2l+1)/(4pi)) d^l_{m0}(theta) e^{i m phi} from ``wigner.d_iter``."""
    out = np.zeros(L * L, dtype=np.complex128)
    ms = np.arange(-(L - 1), L)
    for th, ph, a in zip(theta, phi, amp):
        e = np.exp(-1j * ms * ph)
        for l, D in wigner.d_iter(L, th, L, 1):
            row = a * math.sqrt((2 * l + 1) / (4 * math.pi)) * D[:, 0] * e
            out[l * l: (l + 1) * (l + 1)] += row[L - 1 - l: L + l]
    return out


def _spin_d_column(L, th, s):
    """Yield (l, v) with v[m + L - 1] = d^l_{m,-s}(th), |m| < L (zero for |m| > l
    or l < |s|), from ``wigner.d_iter`` with n = -s."""
    N = abs(s) + 1
    for l, D in wigner.d_iter(L, th, L, N):
        yield l, D[:, N - 1 - s]


def inverse_spin(flm, L, s):
    """map[t, p] = sum_lm f_lm sY_lm(theta_t, phi_p), complex (L, 2L-1)."""
    flm = np.asarray(flm, dtype=np.complex128)
    thetas = sampling.mw_theta(L)
    phis = sampling.mw_phi(L)
    ms = np.arange(-(L - 1), L)
    Ephi = sampling.dft_matrix(ms, phis, +1)          # [p, m]
    F = np.zeros((L, 2 * L - 1), dtype=np.complex128)  # F[l, m + L - 1]
    for l in range(abs(s), L):
        for m in range(-l, l + 1):
            F[l, m + L - 1] = flm[lm_index(l, m)] * (-1.0) ** s * math.sqrt((2 * l + 1) / (4 * math.pi))
    out = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    for t, th in enumerate(thetas):
        G = np.zeros(2 * L - 1, dtype=np.complex128)
        for l, v in _spin_d_column(L, th, s):
            if l >= abs(s):
                G += v * F[l]
        out[t] = Ephi @ G
    return out


def forward_spin(fmap, L, s):
    """f_lm = <f, sY_lm> of a band-limited spin-s map on the MW grid (flat, L^2)."""
    F = _phi_coeffs(fmap, L)                     # [t, m]
    nodes, weights = sampling.gauss_legendre_beta(L)
    E1, E2 = theta_interp_matrices(L, nodes)
    ms = np.arange(-(L - 1), L)
    sgn = (-1.0) ** np.abs(ms + s)
    Fq = E1 @ F + (E2 @ F) * sgn[None, :]        # [q, m]
    acc = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    for q, th in enumerate(nodes):
        for l, v in _spin_d_column(L, th, s):
            acc[l] += weights[q] * v * Fq[q]
    flm = np.zeros(L * L, dtype=np.complex128)
    for l in range(abs(s), L):
        c = 2 * math.pi * (-1.0) ** s * math.sqrt((2 * l + 1) / (4 * math.pi))
        for m in range(-l, l + 1):
            flm[lm_index(l, m)] = c * acc[l, m + L - 1]
    return flm
