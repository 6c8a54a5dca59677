"""Curvelet kernels, scaling function and curvelet harmonic coefficients (Sec. II-B).

Test infrastructure (see ``oracle/__init__.py``).

* ``s_bump``, ``s_lambda``: the Schwartz bump and its mapped form.
* ``k_lambda``: ratio of two integrals of s_lambda(t)^2 / t, evaluated by
  tanh-sinh quadrature (mpmath) at 30 significant digits.  No closed form
  exists; the tests pin the integrand by values the definition fixes (s and
  s_lambda at the ends, the midpoint and x = +-1/2) and by the ratio of the
  slopes of k_lambda at two points, which equals the ratio of the integrand
  there (k' = -integrand / denominator), plus a second, independent quadrature.
* ``kappa(j, l)`` = kappa_lambda(l / lambda^j),
  kappa_lambda(t) = sqrt(k_lambda(t / lambda) - k_lambda(t)).
* ``phi_l0(l)`` = sqrt((2l+1)/(4 pi)) sqrt(k_lambda(l / lambda^J0)).
* ``zeta_tilde``: the unrotated directional component, 1/sqrt(2) at m = l and,
  for m < 0, (-1)^m / sqrt(2) at m = -l.  The printed condition for m < 0 is
  delta_{l m}, which is identically zero for l > 0; the reading delta_{l,-m}
  is the one under which the curvelet is real, normalised to sum_m |zeta|^2 = 1
  and centred on the -x axis as the text states.
* ``zeta``: zeta_lm = sum_n D^l_mn(rho*) zeta~_ln with rho* = (0, theta_j, 0),
  theta_j = arccos(-s / lambda^j) (= pi/2 for spin 0); D^l_mn(0, b, 0) = d^l_mn(b)
  from ``wigner.d_iter``.
* ``psi(j, l, n)`` = sqrt((2l+1)/(8 pi^2)) kappa^(j)(l) zeta_ln.
"""
import math
from functools import lru_cache

import mpmath as mp
import numpy as np

from . import wigner

_DPS = 30


def s_bump(x):
    """s(x) = exp(-1/(1-x^2)) on (-1, 1), zero outside."""
    x = mp.mpf(x)
    if x <= -1 or x >= 1:
        return mp.mpf(0)
    return mp.exp(-1 / (1 - x * x))


def s_lambda(t, lam):
    """s_lambda(t) = s(2 lambda/(lambda-1) (t - 1/lambda) - 1)."""
    lam = mp.mpf(lam)
    return s_bump(2 * lam / (lam - 1) * (mp.mpf(t) - 1 / lam) - 1)


@lru_cache(maxsize=None)
def _k_num(t_key, lam_key):
    with mp.workdps(_DPS):
        lam = mp.mpf(lam_key)
        t = mp.mpf(t_key)
        f = lambda u: s_lambda(u, lam) ** 2 / u
        return mp.quad(f, [t, 1])


@lru_cache(maxsize=None)
def _k_den(lam_key):
    with mp.workdps(_DPS):
        lam = mp.mpf(lam_key)
        f = lambda u: s_lambda(u, lam) ** 2 / u
        return mp.quad(f, [1 / lam, 1])


def k_lambda(t, lam):
    """k_lambda(t): 1 for t < 1/lambda, 0 for t > 1, else the integral ratio."""
    t = float(t)
    lam = float(lam)
    if t <= 1.0 / lam:
        return 1.0
    if t >= 1.0:
        return 0.0
    with mp.workdps(_DPS):
        return float(_k_num(t, lam) / _k_den(lam))


def kappa_sq(j, l, lam):
    """kappa^(j)(l)^2 = k_lambda(l/lambda^(j+1)) - k_lambda(l/lambda^j)."""
    return k_lambda(l / lam ** (j + 1), lam) - k_lambda(l / lam ** j, lam)


def kappa(j, l, lam):
    """kappa^(j)(l) = kappa_lambda(l / lambda^j)."""
    return math.sqrt(max(kappa_sq(j, l, lam), 0.0))


def phi_l0(l, lam, J0):
    """Phi_l0 = sqrt((2l+1)/(4 pi)) sqrt(k_lambda(l / lambda^J0))."""
    return math.sqrt((2 * l + 1) / (4 * math.pi)) * math.sqrt(k_lambda(l / lam ** J0, lam))


def zeta_tilde(l, m):
    """Unrotated directional component (reading for m < 0: delta_{l,-m})."""
    if l == 0:
        return 1.0 / math.sqrt(2.0) if m == 0 else 0.0
    if m == l:
        return 1.0 / math.sqrt(2.0)
    if m == -l:
        return (-1.0) ** m / math.sqrt(2.0)
    return 0.0


def zeta_table(L, theta_j=math.pi / 2):
    """Z[l, n + L - 1] = zeta_ln = sum_k d^l_nk(theta_j) zeta~_lk (explicit rotation)."""
    Z = np.zeros((L, 2 * L - 1))
    zt = np.zeros(2 * L - 1)
    for l, D in wigner.d_iter(L, theta_j):
        zt[:] = 0.0
        for k in range(-l, l + 1):
            zt[k + L - 1] = zeta_tilde(l, k)
        Z[l] = D @ zt
    return Z


def kappa_table(J0, J, L, lam):
    """K[j - J0, l] = kappa^(j)(l) for J0 <= j <= J, 0 <= l < L."""
    K = np.zeros((J - J0 + 1, L))
    for j in range(J0, J + 1):
        for l in range(L):
            K[j - J0, l] = kappa(j, l, lam)
    return K


def psi_table(L, lam, J0, J, theta_j=math.pi / 2):
    """P[j - J0, l, n + L - 1] = Psi^(j)_ln = sqrt((2l+1)/(8pi^2)) kappa^(j)(l) zeta_ln."""
    Z = zeta_table(L, theta_j)
    K = kappa_table(J0, J, L, lam)
    ls = np.arange(L)
    norm = np.sqrt((2 * ls + 1) / (8 * math.pi ** 2))
    return (norm[None, :, None] * K[:, :, None]) * Z[None, :, :]


def phi_table(L, lam, J0):
    """Phi_l0 for 0 <= l < L."""
    return np.array([phi_l0(l, lam, J0) for l in range(L)])


def num_scales(L, lam):
    """J = ceil(log_lambda L): the smallest J with lambda^J >= L (admissibility
    needs k_lambda(l / lambda^(J+1)) = 1, i.e. l <= lambda^J, for every l < L)."""
    J = 0
    while lam ** J < L:
        J += 1
    return J


def scale_bandlimit(j, L, lam):
    """L_j = min(ceil(lambda^(j+1)), L): kappa^(j) vanishes for l >= lambda^(j+1)."""
    return min(int(math.ceil(lam ** (j + 1) - 1e-9)), L)


def scaling_bandlimit(L, lam, J0):
    """L_Phi = min(ceil(lambda^J0), L): Phi_l0 vanishes for l >= lambda^J0."""
    return min(int(math.ceil(lam ** J0 - 1e-9)), L)
