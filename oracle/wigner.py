"""Wigner small-d functions d^l_mn(beta), zyz convention (Sec. II-A).

Test infrastructure (see ``oracle/__init__.py``).

Two independent evaluations:

* ``d_sum``: the factorial-sum expression of Sec. II-A evaluated term by term in
  exact multiprecision (mpmath).  Ground truth for tiny l.
* ``d_iter``: for one beta, all d^l_mn with |m| < M, |n| < N for l = 0, 1, ...
  by the standard three-term recurrence in l (Varshalovich et al., the Wigner-D
  reference the paper cites) seeded on the edges max(|m|,|n|) = l by the closed
  form of d^l_{l,n} (the same closed form the paper writes for d^l_{l,-s}).

Neither uses Delta = d(pi/2) or any Fourier factorisation.
"""
import math

import mpmath as mp
import numpy as np


def d_sum(l, m, n, beta, dps=50):
    """d^l_mn(beta) from the explicit factorial sum of Sec. II-A, in mpmath.

    d = (-1)^(l-n) sqrt((l+m)!(l-m)!(l+n)!(l-n)!)
        * sum_k (-1)^k sin(b/2)^(2l-m-n-2k) cos(b/2)^(m+n+2k)
                / (k! (l-m-k)! (l-n-k)! (m+n+k)!)
    over every k for which all factorial arguments are non-negative.
    """
    if abs(m) > l or abs(n) > l:
        return mp.mpf(0)
    with mp.workdps(dps):
        b = mp.mpf(beta) if not isinstance(beta, mp.mpf) else beta
        s = mp.sin(b / 2)
        c = mp.cos(b / 2)
        pref = mp.sqrt(mp.factorial(l + m) * mp.factorial(l - m)
                       * mp.factorial(l + n) * mp.factorial(l - n))
        total = mp.mpf(0)
        for k in range(0, 2 * l + 1):
            a1, a2, a3 = l - m - k, l - n - k, m + n + k
            if a1 < 0 or a2 < 0 or a3 < 0:
                continue
            ps = 2 * l - m - n - 2 * k
            pc = m + n + 2 * k
            term = (s ** ps if ps else mp.mpf(1)) * (c ** pc if pc else mp.mpf(1))
            term /= (mp.factorial(k) * mp.factorial(a1) * mp.factorial(a2)
                     * mp.factorial(a3))
            total += (-1) ** k * term
        return (-1) ** (l - n) * pref * total


def d_matrix_sum(l, beta, dps=50):
    """Full (2l+1)x(2l+1) matrix d^l_mn(beta), index [m+l, n+l], via ``d_sum``."""
    out = np.zeros((2 * l + 1, 2 * l + 1))
    for m in range(-l, l + 1):
        for n in range(-l, l + 1):
            out[m + l, n + l] = float(d_sum(l, m, n, beta, dps))
    return out


def _edge_row(l, prev, c, s):
    """R^l_n = d^l_{l,n}(beta) for n = -l..l (closed form of Sec. II-A),

    R^l_n = (-1)^(l-n) sqrt(C(2l, l+n)) cos(b/2)^(l+n) sin(b/2)^(l-n),
    built multiplicatively from R^(l-1) so that nothing overflows:
      n >= 0:  R^l_n = sqrt(2l(2l-1)/((l+n)(l+n-1))) cos^2(b/2) R^(l-1)_(n-1)
      n <  0:  R^l_n = sqrt(2l(2l-1)/((l-n)(l-n-1))) sin^2(b/2) R^(l-1)_(n+1)
    (each ratio follows from the closed form).  ``prev`` is R^(l-1), index n+l-1.
    """
    if l == 0:
        return np.array([1.0])
    if l == 1:
        return np.array([s * s, -math.sqrt(2.0) * c * s, c * c])
    out = np.empty(2 * l + 1)
    n = np.arange(0, l + 1, dtype=np.float64)
    out[l:] = np.sqrt(2.0 * l * (2 * l - 1) / ((l + n) * (l + n - 1))) \
        * (c * c) * prev[l - 2:2 * l - 1]
    n = np.arange(-l, 0, dtype=np.float64)
    out[:l] = np.sqrt(2.0 * l * (2 * l - 1) / ((l - n) * (l - n - 1))) \
        * (s * s) * prev[0:l]
    return out


def d_iter(L, beta, M=None, N=None):
    """Yield (l, D) for l = 0..L-1, D[m+M-1, n+N-1] = d^l_mn(beta), |m|<M, |n|<N.

    Entries with |m| > l or |n| > l are zero.  The returned array is reused
    between iterations: copy it if it must outlive the step.

    Interior entries (max(|m|,|n|) < l) follow the three-term recurrence in l
      (l-1) sqrt((l^2-m^2)(l^2-n^2)) d^l
          = (2l-1)((l-1) l cos(b) - m n) d^(l-1)
            - l sqrt(((l-1)^2-m^2)((l-1)^2-n^2)) d^(l-2);
    edge entries (max(|m|,|n|) = l) come from R^l = d^l_{l,.} and the
    symmetries d^l_mn = (-1)^(m-n) d^l_nm = d^l_{-n,-m}, which give
      d^l_{-l,n} = (-1)^(l+n) R^l_{-n},  d^l_{m,l} = (-1)^(l-m) R^l_m,
      d^l_{m,-l} = R^l_{-m}.
    """
    if M is None:
        M = L
    if N is None:
        N = L
    c = math.cos(beta / 2.0)
    s = math.sin(beta / 2.0)
    cb = math.cos(beta)
    mm = np.arange(-(M - 1), M, dtype=np.float64)[:, None]
    nn = np.arange(-(N - 1), N, dtype=np.float64)[None, :]
    d2 = np.zeros((2 * M - 1, 2 * N - 1))   # d^(l-2)
    d1 = np.zeros((2 * M - 1, 2 * N - 1))   # d^(l-1)
    d0 = np.zeros((2 * M - 1, 2 * N - 1))   # d^l
    R = None
    for l in range(L):
        R = _edge_row(l, R, c, s)
        d0[...] = 0.0
        # interior block |m|,|n| <= l-1 (clipped to the stored ranges)
        km = min(l - 1, M - 1)
        kn = min(l - 1, N - 1)
        if l >= 2 and km >= 0 and kn >= 0:
            sm = slice(M - 1 - km, M + km)
            sn = slice(N - 1 - kn, N + kn)
            m_ = mm[sm]
            n_ = nn[:, sn]
            lhs = (l - 1) * np.sqrt((l * l - m_ * m_) * (l * l - n_ * n_))
            t1 = (2 * l - 1) * ((l - 1) * l * cb - m_ * n_) * d1[sm, sn]
            t2 = l * np.sqrt(np.maximum((l - 1) ** 2 - m_ * m_, 0.0)
                             * np.maximum((l - 1) ** 2 - n_ * n_, 0.0)) * d2[sm, sn]
            d0[sm, sn] = (t1 - t2) / lhs
        elif l == 1:
            d0[M - 1, N - 1] = cb
        # edges max(|m|,|n|) = l
        if l <= M - 1:
            ns = np.arange(-min(l, N - 1), min(l, N - 1) + 1)
            sg = 1.0 - 2.0 * ((l + ns) & 1)
            d0[l + M - 1, ns + N - 1] = R[ns + l]
            d0[-l + M - 1, ns + N - 1] = sg * R[-ns + l]
        if l <= N - 1:
            ms = np.arange(-min(l, M - 1), min(l, M - 1) + 1)
            sg = 1.0 - 2.0 * ((l - ms) & 1)
            d0[ms + M - 1, l + N - 1] = sg * R[ms + l]
            d0[ms + M - 1, -l + N - 1] = R[-ms + l]
        yield l, d0
        d2, d1, d0 = d1, d0, d2


def d_matrix(l, beta):
    """(2l+1)x(2l+1) matrix d^l(beta) from the recurrence, index [m+l, n+l]."""
    for ll, D in d_iter(l + 1, beta, l + 1, l + 1):
        if ll == l:
            return D.copy()
    raise AssertionError


def d_m0_table(L, beta):
    """T[l, m] = d^l_{m,0}(beta) for 0 <= m <= l < L (zero for m > l)."""
    out = np.zeros((L, L))
    for l, D in d_iter(L, beta, L, 1):
        out[l, :] = D[L - 1:, 0]
    return out
