"""Spin-0 curvelet analysis and synthesis straight from their harmonic definitions.

Test infrastructure (see ``oracle/__init__.py``).

Analysis (Sec. II-D-1, harmonic form of the curvelet coefficients):
  W^(j)(rho) = sum_lmn f_lm Psi^(j)*_ln D^{l*}_mn(rho),
i.e. the inverse Wigner transform of (W^(j))^l_mn = 8 pi^2/(2l+1) f_lm Psi^(j)*_ln,
sampled on the MW SO(3) grid of band-limit L_j (N_j = L_j).
Scaling coefficients (same section): (W^Phi)_lm = sqrt(4pi/(2l+1)) f_lm Phi_l0,
returned as a spin-0 MW map of band-limit L_Phi.

Synthesis (Sec. II-D-2, harmonic form of exact reconstruction):
  f_lm = sqrt(4pi/(2l+1)) (W^Phi)_lm Phi_l0 + sum_j sum_n (W^(j))^l_mn Psi^(j)_ln,
with (W^(j))^l_mn the forward Wigner transform of each grid (``so3``).

Unrotated curvelets (Sec. III-A-1): ``Plan(..., rotated=False)`` builds Psi from
zeta~ itself (|n| = l only) instead of its rotation by rho* = (0, pi/2, 0); the
same analysis and synthesis then give W~(rho) = W(rho rho*^-1) and reconstruct
exactly.

Parameters (Sec. II-B and Sec. III-A-3): J = ceil(log_lambda L); per-scale
band-limit L_j = min(ceil(lambda^(j+1)), L); L_Phi = min(ceil(lambda^J0), L).
"""
import math

import numpy as np

from . import kernels, sampling, sht, so3, wigner


class Plan:
    """Kernel tables for one (L, lambda, J0, spin).

    ``rotated`` (default): the curvelets rotated so that they are centred on
    the North pole (Sec. II-B), Psi from zeta = d(theta_j) zeta~ with
    theta_j = arccos(-s / lambda^j) (pi/2 for spin 0; clamped to [0, pi] at
    the scales with lambda^j < |s|).  With rotated=False the unrotated
    curvelets (zeta~ itself, |n| = l only), whose coefficients the fast
    algorithm of Sec. III-A computes: W~(rho) = W(rho rho*^-1) with
    rho* = (0, theta_j, 0).  zeta~, kappa and Phi do not depend on the spin;
    the spin enters through the signal's spin harmonic coefficients and, for
    rotated curvelets, through theta_j."""

    def __init__(self, L, lam=2.0, J0=2, rotated=True, spin=0):
        self.L, self.lam, self.J0 = L, float(lam), J0
        self.rotated = bool(rotated)
        self.spin = int(spin)
        self.J = kernels.num_scales(L, lam)
        if J0 > self.J:
            raise ValueError("J0 must not exceed J = ceil(log_lambda L)")
        self.scales = list(range(J0, self.J + 1))
        self.Lj = {j: kernels.scale_bandlimit(j, L, lam) for j in self.scales}
        self.Lphi = kernels.scaling_bandlimit(L, lam, J0)
        if not rotated:
            self.psi = kernels.psi_table(L, lam, J0, self.J, 0.0)   # [j-J0, l, n+L-1]
        elif self.spin == 0:
            self.psi = kernels.psi_table(L, lam, J0, self.J, math.pi / 2)
        else:
            self.psi = np.stack([kernels.psi_table(L, lam, j, j, self.theta_j(j))[0]
                                 for j in self.scales])
        self.phi = kernels.phi_table(L, lam, J0)                  # [l]

    def theta_j(self, j):
        """Colatitude of the unrotated spin-s curvelet's centre, arccos(-s / lambda^j)."""
        c = -self.spin / self.lam ** j
        return math.acos(min(1.0, max(-1.0, c)))

    def psi_j(self, j, Lj):
        """Psi^(j)_ln restricted to l < Lj, |n| < Lj: [l, n + Lj - 1]."""
        P = self.psi[j - self.J0]
        L = self.L
        return P[:Lj, L - Lj: L + Lj - 1]


def _flm_matrix(flm, Lj):
    """A[l, m + Lj - 1] = f_lm for l < Lj."""
    A = np.zeros((Lj, 2 * Lj - 1), dtype=np.complex128)
    for l in range(Lj):
        for m in range(-l, l + 1):
            A[l, m + Lj - 1] = flm[sht.lm_index(l, m)]
    return A


def scaling_flm(plan, flm):
    """(W^Phi)_lm = sqrt(4pi/(2l+1)) f_lm Phi_l0 for l < L_Phi (flat, length L_Phi^2)."""
    Lp = plan.Lphi
    out = np.zeros(Lp * Lp, dtype=np.complex128)
    for l in range(Lp):
        c = math.sqrt(4 * math.pi / (2 * l + 1)) * plan.phi[l]
        for m in range(-l, l + 1):
            out[sht.lm_index(l, m)] = c * flm[sht.lm_index(l, m)]
    return out


def analysis_scale(plan, flm, j, rows=None):
    """Grid W^(j)[a, b, g] (shape (2L_j-1, len(rows), 2L_j-1)), complex."""
    Lj = plan.Lj[j]
    A = _flm_matrix(flm, Lj)
    P = np.conj(plan.psi_j(j, Lj))

    def coeff(l):
        if not np.any(P[l]):
            return None
        # (2l+1)/(8pi^2) * 8pi^2/(2l+1) f_lm Psi*_ln
        return np.outer(A[l], P[l])

    return so3.inverse_rows(Lj, Lj, coeff, rows=rows)


def analysis(plan, flm):
    """(scaling map (L_Phi, 2L_Phi-1) complex, {j: grid})."""
    scal = sht.inverse(scaling_flm(plan, flm), plan.Lphi)
    grids = {j: analysis_scale(plan, flm, j) for j in plan.scales}
    return scal, grids


def synthesis_scale(plan, grid, j, nodes_subset=None):
    """f^(j)_lm = sum_n (W^(j))^l_mn Psi^(j)_ln as a flat length-L^2 array.

    ``nodes_subset`` restricts the Gauss-Legendre sum to those node indices
    (a partial sum, used only to time a bounded sample)."""
    Lj = plan.Lj[j]
    P = plan.psi_j(j, Lj)
    nodes, weights, Xq = so3.gl_rows(grid, Lj, Lj)
    acc = np.zeros((Lj, 2 * Lj - 1), dtype=np.complex128)
    for q, bq in enumerate(nodes):
        if nodes_subset is not None and q not in nodes_subset:
            continue
        for l, D in wigner.d_iter(Lj, bq, Lj, Lj):
            if not np.any(P[l]):
                continue
            acc[l] += weights[q] * ((D * Xq[q]) @ P[l])
    acc *= (2 * math.pi) ** 2
    out = np.zeros(plan.L * plan.L, dtype=np.complex128)
    for l in range(Lj):
        for m in range(-l, l + 1):
            out[sht.lm_index(l, m)] = acc[l, m + Lj - 1]
    return out


def synthesis(plan, scal_map, grids):
    """Reconstructed f_lm (flat, length L^2)."""
    L = plan.L
    flm = np.zeros(L * L, dtype=np.complex128)
    wphi = sht.forward(scal_map, plan.Lphi)
    for l in range(plan.Lphi):
        c = math.sqrt(4 * math.pi / (2 * l + 1)) * plan.phi[l]
        for m in range(-l, l + 1):
            flm[sht.lm_index(l, m)] += c * wphi[sht.lm_index(l, m)]
    for j in plan.scales:
        flm += synthesis_scale(plan, grids[j], j)
    return flm


def grid_shape(plan, j):
    Lj = plan.Lj[j]
    return (2 * Lj - 1, Lj, 2 * Lj - 1)


def mw_so3_nodes(Lj):
    return sampling.so3_alpha(Lj), sampling.so3_beta(Lj), sampling.so3_gamma(Lj)
