"""GPU parity of the unrotated curvelet coefficients (CVL_UNROTATED).

The HIP path (through the C ABI) against the CPU FP64 oracle with
``Plan(..., rotated=False)``: every grid element-wise at small band-limits
(several tiles, ragged and odd L, lambda = 1.5), sampled beta rows at L = 256
and L = 257 (the beta stage as an FFT), exact reconstruction, the
|n| = l support of the grids' Wigner coefficients, and the streaming, batch,
real-grid and determinism properties of the rotated path.

Bars (relative L2 against the oracle): fp64 1e-10, fp32 1e-5, bf16x3 1e-3.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU, skipped
    pytest.skip("no GPU", allow_module_level=True)

from oracle import curvelet as ocurv  # noqa: E402
from oracle import sht as osht  # noqa: E402
from paper_1511_05578_amd import api, inputs  # noqa: E402

BOUND = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(256, 0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("L,lam,J0", [(32, 2.0, 2), (13, 2.0, 1), (20, 1.5, 2), (33, 2.0, 2),
                                      (8, 2.0, 3), (2, 2.0, 1), (3, 2.0, 1), (4, 2.0, 2),
                                      (27, 3.0, 1)])
def test_unrotated_analysis_and_synthesis(ctx, L, lam, J0, prec):
    say("unrotated L=%d lambda=%g J0=%d %s" % (L, lam, J0, prec))
    bound = BOUND[prec]
    plan = ocurv.Plan(L, lam, J0, rotated=False)
    f = inputs.gaussian_real_flm(L, seed=L + 3)
    ref_scal, ref_grids = ocurv.analysis(plan, f)
    fmap = osht.inverse(f, L).real
    scal, grids = ctx.curvelet_analysis(dev(fmap), lam, J0, precision=prec, unrotated=True)
    for s, j in enumerate(plan.scales):
        g = host(grids[s])
        assert g.shape == ref_grids[j].shape
        assert np.all(g.imag == 0)
        e = rel_l2(g, ref_grids[j])
        say("  scale %d (L_j=%d): rel L2 %.2e" % (j, plan.Lj[j], e))
        assert e < bound
    rec = host(ctx.curvelet_synthesis(scal, grids, L, lam, J0, precision=prec, unrotated=True))
    e = rel_l2(rec, fmap)
    say("  round trip rel L2 %.2e" % e)
    assert e < bound
    if prec == "fp64":
        og = [dev(ref_grids[j]) for j in plan.scales]
        rec = host(ctx.curvelet_synthesis(dev(ref_scal.real), og, L, lam, J0, unrotated=True))
        assert rel_l2(rec, fmap) < bound


def test_unrotated_differs_from_rotated(ctx):
    # The flag selects other coefficients (same shapes), not the same ones.
    L, lam, J0 = 32, 2.0, 2
    fmap = osht.inverse(inputs.gaussian_real_flm(L, seed=5), L).real
    _, g_rot = ctx.curvelet_analysis(dev(fmap), lam, J0)
    _, g_unr = ctx.curvelet_analysis(dev(fmap), lam, J0, unrotated=True)
    for a, b in zip(g_rot, g_unr):
        assert a.shape == b.shape
    assert rel_l2(host(g_rot[-1]), host(g_unr[-1])) > 0.1


def test_unrotated_wigner_support(ctx):
    # Wigner coefficients of each GPU grid, by the library's general forward
    # Wigner transform: zero unless |n| = l.
    L, lam, J0 = 32, 2.0, 2
    fmap = osht.inverse(inputs.gaussian_real_flm(L, seed=6), L).real
    _, grids = ctx.curvelet_analysis(dev(fmap), lam, J0, unrotated=True)
    for g in grids:
        Lj = g.shape[1]
        F = host(ctx.wigner_forward(g, Lj, Lj))  # [l, m + Lj - 1, n + Lj - 1]
        scale = np.abs(F).max()
        mask = np.ones(F.shape, bool)
        for l in range(Lj):
            mask[l, :, [Lj - 1 - l, Lj - 1 + l]] = False
        assert np.abs(F[mask]).max() <= 1e-12 * scale


def test_unrotated_streaming_batch_real_grids_deterministic(ctx):
    L, lam, J0 = 64, 2.0, 2
    say("unrotated streaming / batch / real grids L=%d" % L)
    maps = np.stack([osht.inverse(inputs.gaussian_real_flm(L, s), L).real for s in (1, 2)])
    scal_b, grids_b = ctx.curvelet_analysis(dev(maps), lam, J0, unrotated=True)
    scal_1, grids_1 = ctx.curvelet_analysis(dev(maps[1]), lam, J0, unrotated=True)
    assert np.array_equal(host(scal_b[1]), host(scal_1))
    for a, b in zip(grids_b[1], grids_1):
        assert np.array_equal(host(a), host(b))
    _, again = ctx.curvelet_analysis(dev(maps[1]), lam, J0, unrotated=True)
    for a, b in zip(again, grids_1):
        assert np.array_equal(host(a), host(b))
    # real grids hold the same real parts
    _, grids_r = ctx.curvelet_analysis(dev(maps[1]), lam, J0, real_grids=True, unrotated=True)
    for a, b in zip(grids_r, grids_1):
        assert np.array_equal(host(a), host(b).real)
    rec_r = host(ctx.curvelet_synthesis(scal_1, grids_r, L, lam, J0, real_grids=True,
                                        unrotated=True))
    assert rel_l2(rec_r, maps[1]) < 1e-10
    # batch synthesis equals single synthesis
    rec_b = host(ctx.curvelet_synthesis(scal_b, grids_b, L, lam, J0, unrotated=True))
    rec_1 = host(ctx.curvelet_synthesis(scal_1, grids_1, L, lam, J0, unrotated=True))
    assert np.array_equal(rec_b[1], rec_1)
    # one scale at a time: the same grids, the same reconstruction up to rounding
    seen = []
    rec_s, _ = ctx.round_trip_streamed(dev(maps[1]), lam, J0, unrotated=True,
                                       on_grid=lambda j, g: seen.append(host(g).copy()))
    for a, b in zip(seen, grids_1):
        assert np.array_equal(a, host(b))
    assert rel_l2(host(rec_s), maps[1]) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_unrotated_l256_sampled_rows_and_round_trip(ctx, prec):
    # L = 256: the finest scales take the beta stage as an FFT.  Oracle beta
    # rows of the two finest scales, full round trip.
    L, lam, J0 = 256, 2.0, 2
    bound = BOUND[prec]
    plan = ocurv.Plan(L, lam, J0, rotated=False)
    f = inputs.gaussian_real_flm(L, seed=0)
    fmap = osht.inverse(f, L).real
    say("unrotated L=256 %s: GPU analysis" % prec)
    scal, grids = ctx.curvelet_analysis(dev(fmap), lam, J0, precision=prec, unrotated=True)
    rows = [0, 77, 255]
    for s, j in enumerate(plan.scales):
        Lj = plan.Lj[j]
        if Lj < 128:
            continue
        rr = [r for r in rows if r < Lj]
        say("  oracle rows %s of scale %d" % (rr, j))
        ref = ocurv.analysis_scale(plan, f, j, rows=rr)
        assert np.abs(ref).max() > 1e-6
        e = rel_l2(host(grids[s])[:, rr, :], ref)
        say("  scale %d rows rel L2 %.2e" % (j, e))
        assert e < bound
    rec = host(ctx.curvelet_synthesis(scal, grids, L, lam, J0, precision=prec, unrotated=True))
    e = rel_l2(rec, fmap)
    say("  round trip rel L2 %.2e" % e)
    assert e < bound


def test_unrotated_odd_bandlimit_fft_beta():
    # L = 257: odd, FFT beta stage on the unrotated cube (2 L_j rows).
    L, lam, J0 = 257, 2.0, 2
    c = api.Context(L, 0)
    try:
        plan = ocurv.Plan(L, lam, J0, rotated=False)
        f = inputs.gaussian_real_flm(L, seed=9)
        fmap = osht.inverse(f, L).real
        scal, grids = c.curvelet_analysis(dev(fmap), lam, J0, unrotated=True)
        s, j = [(s, j) for s, j in enumerate(plan.scales) if plan.Lj[j] == L][0]
        rows = [0, 100, 256]
        say("unrotated L=257: oracle rows %s of scale %d" % (rows, j))
        ref = ocurv.analysis_scale(plan, f, j, rows=rows)
        e = rel_l2(host(grids[s])[:, rows, :], ref)
        say("  rows rel L2 %.2e" % e)
        assert e < 1e-10
        rec = host(c.curvelet_synthesis(scal, grids, L, lam, J0, unrotated=True))
        e = rel_l2(rec, fmap)
        say("  round trip rel L2 %.2e" % e)
        assert e < 1e-10
    finally:
        torch.cuda.synchronize()
        c.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_unrotated_l512_reduced_precision(prec):
    # L = 512, the reduced-precision configuration's band-limit: oracle beta
    # rows of the finest scale, full round trip, at the precision's bar.
    L, lam, J0 = 512, 2.0, 2
    bound = BOUND[prec]
    c = api.Context(L, 0)
    try:
        plan = ocurv.Plan(L, lam, J0, rotated=False)
        f = inputs.gaussian_real_flm(L, seed=4)
        fmap = osht.inverse(f, L).real
        say("unrotated L=512 %s: GPU analysis" % prec)
        scal, grids = c.curvelet_analysis(dev(fmap), lam, J0, precision=prec, unrotated=True)
        s, j = len(plan.scales) - 1, plan.scales[-1]
        rows = [3, 400]
        say("  oracle rows %s of scale %d" % (rows, j))
        ref = ocurv.analysis_scale(plan, f, j, rows=rows)
        e = rel_l2(host(grids[s])[:, rows, :], ref)
        say("  rows rel L2 %.2e" % e)
        assert e < bound
        rec = host(c.curvelet_synthesis(scal, grids, L, lam, J0, precision=prec, unrotated=True))
        e = rel_l2(rec, fmap)
        say("  round trip rel L2 %.2e" % e)
        assert e < bound
    finally:
        torch.cuda.synchronize()
        c.close()
