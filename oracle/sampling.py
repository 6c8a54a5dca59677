"""McEwen-Wiaux sample positions on the sphere and on SO(3) (Sec. III-A-2).

Test infrastructure (see ``oracle/__init__.py``).
"""
import numpy as np


def mw_theta(L):
    """theta_t = pi (2t+1) / (2L-1), t = 0..L-1 (the last one is pi)."""
    return np.pi * (2 * np.arange(L) + 1) / (2 * L - 1)


def mw_phi(L):
    """phi_p = 2 pi p / (2L-1), p = 0..2L-2."""
    return 2 * np.pi * np.arange(2 * L - 1) / (2 * L - 1)


def so3_alpha(M):
    """alpha_a = 2 pi a / (2M-1), a = 0..2M-2."""
    return 2 * np.pi * np.arange(2 * M - 1) / (2 * M - 1)


def so3_beta(L):
    """beta_b = pi (2b+1) / (2L-1), b = 0..L-1."""
    return np.pi * (2 * np.arange(L) + 1) / (2 * L - 1)


def so3_gamma(N):
    """gamma_g = 2 pi g / (2N-1), g = 0..2N-2."""
    return 2 * np.pi * np.arange(2 * N - 1) / (2 * N - 1)


def gauss_legendre_beta(n):
    """Nodes beta_q = arccos(x_q) and weights w_q of n-point Gauss-Legendre in
    x = cos(beta): sum_q w_q g(beta_q) = int_0^pi sin(b) g(b) db exactly when g is
    a polynomial in cos(b) of degree <= 2n-1."""
    x, w = np.polynomial.legendre.leggauss(n)
    return np.arccos(x), w


def dft_matrix(ks, xs, sign):
    """E[i, k] = exp(sign * 1j * ks[k] * xs[i]) (plain Fourier matrix)."""
    return np.exp(sign * 1j * np.outer(xs, ks))
