"""Pins for the oracle's spin-s curvelets (Sec. II-B: spin-s curvelets are
centred at colatitude theta_j = arccos(-s / lambda^j) before the rotation
rho* = (0, theta_j, 0) to the North pole; Sec. III-A-1: the inverse rotation
leaves Wigner coefficients at |k| = l only)."""
import math

import numpy as np
import pytest

from oracle import curvelet, kernels, sht, so3, wigner
from paper_1511_05578_amd import inputs


def _zeta_closed(l, n, th):
    # zeta_ln = (d^l_{n,l}(th) + (-1)^l d^l_{n,-l}(th)) / sqrt 2, with the
    # one-term edge cases of the factorial sum of d (Sec. II-A):
    # d^l_{n,l} = sqrt(C(2l, l+n)) sin(th/2)^(l-n) cos(th/2)^(l+n),
    # d^l_{n,-l} = (-1)^(l-n) sqrt(C(2l, l+n)) sin(th/2)^(l+n) cos(th/2)^(l-n)
    s, c = math.sin(th / 2), math.cos(th / 2)
    b = math.sqrt(math.comb(2 * l, l + n))
    return b * (s ** (l - n) * c ** (l + n) + (-1) ** n * s ** (l + n) * c ** (l - n)) / math.sqrt(2)


@pytest.mark.parametrize("s", [1, 2, -3])
def test_spin_zeta_closed_form_normalisation_and_parity(s):
    L, lam, J0 = 24, 2.0, 2
    plan = curvelet.Plan(L, lam, J0, spin=s)
    for jj, j in enumerate(plan.scales):
        th = plan.theta_j(j)
        assert abs(math.cos(th) + s / lam ** j) < 1e-15
        Z = kernels.zeta_table(L, th)
        for l in range(1, L):
            assert abs(np.sum(Z[l] ** 2) - 1.0) < 1e-13
            for n in range(-l, l + 1):
                assert abs(Z[l, n + L - 1] - _zeta_closed(l, n, th)) < 1e-13
                assert abs(Z[l, L - 1 - n] - (-1) ** n * Z[l, n + L - 1]) < 1e-14
        # Psi = sqrt((2l+1)/8pi^2) kappa zeta at this scale's theta_j
        for l in range(L):
            k = kernels.kappa(j, l, lam) * math.sqrt((2 * l + 1) / (8 * math.pi ** 2))
            assert np.allclose(plan.psi[jj, l], k * Z[l], atol=1e-15)
    # spin 0: the spin-0 plan
    assert np.array_equal(curvelet.Plan(L, lam, J0, spin=0).psi, curvelet.Plan(L, lam, J0).psi)


@pytest.mark.parametrize("s,rotated", [(2, True), (-1, True), (3, False)])
def test_spin_exact_reconstruction(s, rotated):
    L, lam, J0 = 16, 2.0, 2
    plan = curvelet.Plan(L, lam, J0, rotated=rotated, spin=s)
    f = inputs.uniform_complex_flm(L, seed=3)
    f[:s * s] = 0
    scal, grids = curvelet.analysis(plan, f)
    rec = curvelet.synthesis(plan, scal, grids)
    assert np.abs(rec - f).max() < 1e-13


@pytest.mark.parametrize("s", [2, -2])
def test_spin_inverse_rotation_gives_abs_k_equal_l(s):
    # F~^l_mk = sum_n F^l_mn D^{l*}_kn(rho*'), rho*' = (0, -theta_j, 0)
    L, lam, J0 = 16, 2.0, 2
    plan = curvelet.Plan(L, lam, J0, spin=s)
    f = inputs.uniform_complex_flm(L, seed=9)
    f[:s * s] = 0
    j = plan.J - 1
    Lj = plan.Lj[j]
    F = so3.forward(curvelet.analysis_scale(plan, f, j), Lj, Lj)
    scale = np.abs(F).max()
    for l in range(3, Lj):
        d = wigner.d_matrix(l, -plan.theta_j(j))
        sub = F[l, Lj - 1 - l:Lj + l, Lj - 1 - l:Lj + l]
        Ft = sub @ d.T
        mask = np.ones(2 * l + 1, bool)
        mask[[0, 2 * l]] = False
        assert np.abs(Ft[:, mask]).max() <= 1e-12 * scale, l


@pytest.mark.parametrize("s", [1, 3])
def test_spin_curvelet_centres(s):
    # The unrotated spin-s curvelet's m = +l part (sY_ll, whose theta factor
    # d^l_{l,-s} the paper shows to peak at arccos(-s/l)) is centred at
    # theta_j = arccos(-s / lambda^j) on the meridian phi = pi, and the
    # rotation by rho* = (0, theta_j, 0) that the plans apply moves it onto
    # the North pole.  (With zeta~ at both m = +-l -- the reading under which
    # a spin-0 curvelet is real -- the m = -l part is the mirror image about
    # the equator, at arccos(s/l).)
    L, lam, j = 64, 2.0, 4
    plan = curvelet.Plan(L, lam, 2, spin=s)
    th_j = plan.theta_j(j)
    up = np.zeros(L * L, dtype=np.complex128)
    rot = np.zeros(L * L, dtype=np.complex128)
    for l in range(abs(s), L):
        k = kernels.kappa(j, l, lam) * math.sqrt((2 * l + 1) / (8 * math.pi ** 2))
        if k == 0:
            continue
        up[l * l + 2 * l] = k * kernels.zeta_tilde(l, l)
        d = wigner.d_matrix(l, th_j)                # D^l_nk(0, theta_j, 0) = d^l_nk(theta_j)
        rot[l * l:(l + 1) * (l + 1)] = k * d[:, 2 * l] * kernels.zeta_tilde(l, l)
    Nt = 2 * L - 1
    for c, expect in ((up, th_j), (rot, 0.0)):
        m = np.abs(sht.inverse_spin(c, L, s))
        t, p = np.unravel_index(np.argmax(m), m.shape)
        th = math.pi * (2 * t + 1) / Nt
        # within two rings: the kernel mixes l in (lambda^(j-1), lambda^(j+1)),
        # whose peaks arccos(-s/l) straddle theta_j (its l = lambda^j)
        assert abs(th - expect) < 4 * math.pi / Nt, (th, expect)
    # the unrotated m = +l part sits on the -x axis side, phi = pi (the sign
    # (-1)^(l+s) of d^l_{l,-s} and e^{i l pi} agree there for every l)
    m = np.abs(sht.inverse_spin(up, L, s))
    t, p = np.unravel_index(np.argmax(m), m.shape)
    assert abs(2 * math.pi * p / Nt - math.pi) < 2 * math.pi / Nt
