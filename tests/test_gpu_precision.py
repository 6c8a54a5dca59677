"""GPU parity of the reduced-precision path against the CPU FP64 oracle.

Reduced precision: complex64 coefficient grids; the two l-contractions on the
matrix cores in FP32 ("fp32") or split bfloat16 ("bf16x3") with FP32
accumulation; the beta stage and the alpha/gamma FFTs in FP32; the Delta
table, the SHTs, the scaling part and the final accumulation of the synthesis
over scales in FP64.

Bars (relative L2 error against the FP64 oracle, on every compared output):
fp32 <= 1e-5, bf16x3 <= 1e-3.  The max-abs error (relative to the largest
magnitude) is printed beside it.
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

BOUND = {"fp32": 1e-5, "bf16x3": 1e-3}
PRECS = ["fp32", "bf16x3"]


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def rel_max(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(256, 0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L,lam,J0", [(32, 2.0, 2), (13, 2.0, 1), (20, 1.5, 2), (64, 2.0, 2)])
def test_analysis_and_synthesis(ctx, prec, L, lam, J0):
    bound = BOUND[prec]
    say("%s curvelet L=%d lambda=%g J0=%d" % (prec, L, lam, J0))
    plan = ocurv.Plan(L, lam, J0)
    f = inputs.gaussian_real_flm(L, seed=L)
    ref_scal, ref_grids = ocurv.analysis(plan, f)
    fmap = osht.inverse(f, L).real
    scal, grids = ctx.curvelet_analysis(dev(fmap), lam, J0, precision=prec)
    assert rel_l2(host(scal), ref_scal.real) < 1e-10  # scaling part stays FP64
    for s, j in enumerate(plan.scales):
        assert grids[s].dtype == torch.complex64
        g = host(grids[s])
        assert g.shape == ref_grids[j].shape
        assert np.all(g.imag == 0)
        e, em = rel_l2(g, ref_grids[j]), rel_max(g, ref_grids[j])
        say("  scale %d (L_j=%d): rel L2 %.2e, max %.2e" % (j, plan.Lj[j], e, em))
        assert e < bound
    # synthesis of the GPU's own grids and of the oracle's grids (rounded to c64)
    rec = host(ctx.curvelet_synthesis(scal, grids, L, lam, J0, precision=prec))
    e = rel_l2(rec, fmap)
    say("  round trip rel L2 %.2e, max %.2e" % (e, rel_max(rec, fmap)))
    assert e < bound
    og = [dev(ref_grids[j], torch.complex64) for j in plan.scales]
    rec2 = host(ctx.curvelet_synthesis(dev(ref_scal.real), og, L, lam, J0, precision=prec))
    e2 = rel_l2(rec2, fmap)
    say("  synthesis of oracle grids rel L2 %.2e" % e2)
    assert e2 < bound


def test_deterministic_and_batch_invariant(ctx):
    L, lam, J0 = 32, 2.0, 2
    maps = np.stack([osht.inverse(inputs.gaussian_real_flm(L, s), L).real for s in range(3)])
    for prec in PRECS:
        say("%s determinism and batch of 3 vs single" % prec)
        s1, g1 = ctx.curvelet_analysis(dev(maps[1]), lam, J0, precision=prec)
        s2, g2 = ctx.curvelet_analysis(dev(maps[1]), lam, J0, precision=prec)
        for a, b in zip(g1, g2):
            assert torch.equal(a, b)
        sb, gb = ctx.curvelet_analysis(dev(maps), lam, J0, precision=prec)
        for a, b in zip(gb[1], g1):
            assert torch.equal(a, b)
        r1 = ctx.curvelet_synthesis(s1, g1, L, lam, J0, precision=prec)
        rb = ctx.curvelet_synthesis(sb, gb, L, lam, J0, precision=prec)
        assert torch.equal(rb[1], r1)


def test_precision_rejects_wrong_grid_type(ctx):
    L = 16
    fmap = dev(osht.inverse(inputs.gaussian_real_flm(L, 0), L).real)
    scal, grids = ctx.curvelet_analysis(fmap, precision="fp64")
    with pytest.raises(AssertionError):
        ctx.curvelet_synthesis(scal, grids, L, precision="fp32")
    p = api.params(L, precision=7)
    n = np.zeros(1, dtype=np.uintp)
    rc = api.lib.cvl_workspace_bytes(p, 1, n.ctypes.data_as(api._c_size_p))
    assert rc == api.CVL_EINVAL


@pytest.mark.parametrize("prec", PRECS)
def test_l256_sampled_rows_and_round_trip(ctx, prec):
    L, lam, J0 = 256, 2.0, 2
    bound = BOUND[prec]
    plan = ocurv.Plan(L, lam, J0)
    f = inputs.gaussian_real_flm(L, seed=0)
    fmap = osht.inverse(f, L).real
    say("%s L=256: GPU analysis" % prec)
    scal, grids = ctx.curvelet_analysis(dev(fmap), lam, J0, precision=prec)
    rows = [0, 77, 128, 255]
    for s, j in enumerate(plan.scales):
        Lj = plan.Lj[j]
        if Lj < 128:
            continue
        rr = [r for r in rows if r < Lj]
        ref = ocurv.analysis_scale(plan, f, j, rows=rr)
        g = host(grids[s])[:, rr, :]
        e = rel_l2(g, ref)
        say("  scale %d rows %s rel L2 %.2e, max %.2e" % (j, rr, e, rel_max(g, ref)))
        assert e < bound
    rec = host(ctx.curvelet_synthesis(scal, grids, L, lam, J0, precision=prec))
    e = rel_l2(rec, fmap)
    say("  round trip rel L2 %.2e" % e)
    assert e < bound


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", [150, 200])
def test_beta_gemm_edge_tiles(ctx, prec, L):
    # Below L_j = 256 both beta stages are the parity-folded GEMM (128-row x
    # 32-k tiles).  L_j = 200: a partial row tile and a partial last K tile;
    # L_j = 150 also a K that is not a multiple of 4 (single-value loads), and
    # an SHT whose phi DFT takes the next FFT size.  Oracle beta rows on both
    # sides of the row-tile edge and the last row (FP64 path and reduced
    # precision), every grid against the library's FP64 path, and the round trip.
    lam, J0 = 2.0, 2
    bound = BOUND[prec]
    plan = ocurv.Plan(L, lam, J0)
    f = inputs.gaussian_real_flm(L, seed=L + 1)
    fmap = osht.inverse(f, L).real
    say("%s L=%d: GPU analysis" % (prec, L))
    scal, grids = ctx.curvelet_analysis(dev(fmap), lam, J0, precision=prec)
    s64, g64 = ctx.curvelet_analysis(dev(fmap), lam, J0)
    for s, j in enumerate(plan.scales):
        ref64 = host(g64[s])
        g = host(grids[s])
        if np.abs(ref64).max() == 0.0:  # a scale whose kernel vanishes below L
            assert np.abs(g).max() == 0.0
            continue
        e = rel_l2(g, ref64)
        say("  scale %d (L_j=%d): vs FP64 path rel L2 %.2e" % (j, plan.Lj[j], e))
        assert e < bound
        if plan.Lj[j] == L:
            rr = [0, 127, 128, L - 1]
            ref = ocurv.analysis_scale(plan, f, j, rows=rr)
            e = rel_l2(ref64[:, rr, :], ref)
            say("  scale %d rows %s FP64 path vs oracle rel L2 %.2e" % (j, rr, e))
            assert e < 1e-10
            e = rel_l2(g[:, rr, :], ref)
            say("  scale %d rows %s vs oracle rel L2 %.2e, max %.2e"
                % (j, rr, e, rel_max(g[:, rr, :], ref)))
            assert e < bound
    rec = host(ctx.curvelet_synthesis(scal, grids, L, lam, J0, precision=prec))
    e = rel_l2(rec, fmap)
    say("  round trip rel L2 %.2e" % e)
    assert e < bound


def test_l512_batch16():
    # 16 real maps at L = 512 in one batched call per precision (the batched
    # precision-path configuration): complex64 grids of all maps resident at
    # once (16 x 9.2 GB); an oracle beta row of one finest scale for the first
    # and of the other for the last map; every map's round trip.
    L, lam, J0, B = 512, 2.0, 2, 16
    free, total = torch.cuda.mem_get_info()
    if free < 180 * 2**30:
        pytest.skip("needs about 160 GB of free device memory")
    c = api.Context(L, 0)
    try:
        plan = ocurv.Plan(L, lam, J0)
        fl = [inputs.gaussian_real_flm(L, seed=100 + i) for i in range(B)]
        maps = torch.stack([c.sht_inverse(dev(f), L) for f in fl]).contiguous()
        refs = {}
        full = [(s, j) for s, j in enumerate(plan.scales) if plan.Lj[j] == L]
        for i, (s, j) in zip((0, B - 1), full):
            say("L=512: oracle row 300 of scale %d, map %d" % (j, i))
            refs[(i, s)] = ocurv.analysis_scale(plan, fl[i], j, rows=[300])
        for prec in PRECS:
            bound = BOUND[prec]
            say("%s L=512 batch %d: analysis" % (prec, B))
            scal, grids = c.curvelet_analysis(maps, lam, J0, precision=prec)
            for (i, s), ref in refs.items():
                g = grids[i][s][:, 300:301, :].cpu().numpy()
                e = rel_l2(g, ref)
                say("  map %d scale %d row rel L2 %.2e, max %.2e" % (i, s, e, rel_max(g, ref)))
                assert e < bound
            say("%s L=512 batch %d: synthesis" % (prec, B))
            rec = c.curvelet_synthesis(scal, grids, L, lam, J0, precision=prec)
            err = ((torch.linalg.norm((rec - maps).reshape(B, -1), dim=1) /
                    torch.linalg.norm(maps.reshape(B, -1), dim=1))).cpu().numpy()
            say("  round trip rel L2 per map: max %.2e, mean %.2e" % (err.max(), err.mean()))
            assert err.max() < bound
            del scal, grids, rec
            torch.cuda.empty_cache()
    finally:
        torch.cuda.synchronize()
        c.close()
        torch.cuda.empty_cache()


@pytest.mark.parametrize("complex_map", [False, True])
def test_line_major_beta_odd_bandlimit(complex_map):
    # Odd L = 515: the finest scales' analysis beta DFT has FFT size 4096 and,
    # in complex64, is written line-major and transposed; at odd L_j the last
    # m row has no odd partner in the paired transform and the W2 plane that
    # then moves to the second cube buffer is larger than the cube.  The
    # complex128 path keeps the direct stores, so FP32 against FP64 on the same
    # map checks the line-major path (every grid within the FP32 bound).
    L, lam, J0 = 515, 2.0, 2
    c = api.Context(L, 0)
    try:
        if complex_map:
            f = inputs.uniform_complex_flm(L, 11)
            m = c.sht_inverse(dev(f), L, complex_map=True)
        else:
            f = inputs.gaussian_real_flm(L, seed=11)
            m = c.sht_inverse(dev(f), L)
        s64, g64 = c.curvelet_analysis(m, lam, J0)
        s32, g32 = c.curvelet_analysis(m, lam, J0, precision="fp32")
        assert g32[-1].shape[1] == L
        checked = 0
        for s_, (a, b) in enumerate(zip(g32, g64)):
            ref = b.abs().max().item()
            if ref == 0.0:  # a scale whose kernel vanishes below L
                assert a.abs().max().item() == 0.0
                continue
            e = (torch.linalg.norm(a.to(b.dtype) - b) / torch.linalg.norm(b)).item()
            mx = (a.to(b.dtype) - b).abs().max().item() / ref
            say("L=515 complex=%s scale %d: FP32 vs FP64 rel L2 %.2e max-abs rel %.2e"
                % (complex_map, s_, e, mx))
            assert e < BOUND["fp32"] and mx < BOUND["fp32"]
            checked += 1
        assert checked >= len(g64) - 1
        rec = c.curvelet_synthesis(s32, g32, L, lam, J0, precision="fp32")
        e = (torch.linalg.norm(rec - m) / torch.linalg.norm(m)).item()
        say("  FP32 round trip rel L2 %.2e" % e)
        assert e < BOUND["fp32"]
    finally:
        torch.cuda.synchronize()
        c.close()
        torch.cuda.empty_cache()
