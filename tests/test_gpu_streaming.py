"""GPU: the streaming (one scale at a time) interface against the all-scales
calls and the oracle, point-source inputs, and the large band-limit in
reduced precision with a single resident grid.

Bars: FP64 1e-10 relative L2 against the oracle; the streamed FP64 path
against the all-scales path bitwise for grids and within 1e-14 for maps;
fp32 1e-5 relative L2.
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


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(128, 0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("L", [32, 45])
def test_streamed_equals_all_scales(ctx, L, prec):
    lam, J0 = 2.0, 2
    say("streamed vs all-scales L=%d %s" % (L, prec))
    fmap = dev(osht.inverse(inputs.gaussian_real_flm(L, 11), L).real)
    scal, grids = ctx.curvelet_analysis(fmap, lam, J0, precision=prec)
    rec = ctx.curvelet_synthesis(scal, grids, L, lam, J0, precision=prec)
    flm = ctx.sht_forward(fmap)
    J = api.num_scales(L, lam, J0)
    for s, j in enumerate(range(J0, J + 1)):
        g = ctx.analysis_scale(flm, L, j, lam, J0, precision=prec)
        assert torch.equal(g, grids[s]), j
    assert torch.equal(ctx.scaling_analysis(flm, L, lam, J0), scal)
    seen = []
    rec2, scal2 = ctx.round_trip_streamed(fmap, lam, J0, precision=prec,
                                          on_grid=lambda j, g: seen.append(j))
    assert seen == list(range(J0, J + 1))
    d = rel_l2(host(rec2), host(rec))
    say("  streamed vs all-scales map rel diff %.2e (bitwise: %s)" % (d, torch.equal(rec, rec2)))
    assert d <= 1e-14


def test_scale_workspace_is_enough_for_the_per_scale_calls(ctx):
    # The per-scale calls run with exactly cvl_scale_workspace_bytes (no side-
    # stream buffers) and give the same grid as with the full workspace; one
    # byte less, or the batched call with that size, is refused before any
    # launch (CVL_ENOMEM, nothing written).
    import ctypes
    L, lam, J0, j = 64, 2.0, 2, 5
    fmap = dev(osht.inverse(inputs.gaussian_real_flm(L, 3), L).real)
    flm = ctx.sht_forward(fmap)
    ref = ctx.analysis_scale(flm, L, j, lam, J0)
    torch.cuda.synchronize()
    n = api.scale_workspace_bytes(L, lam, J0)
    assert n < api.workspace_bytes(L, lam, J0)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    p = api.params(L, lam, J0)
    out = torch.full_like(ref, 7.0)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = api.lib.cvl_curvelet_analysis_scale(ctx.h, ctypes.byref(p), j, flm.data_ptr(),
                                             out.data_ptr(), ws.data_ptr(), n - 1, s)
    assert rc == api.CVL_ENOMEM
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    api._check(api.lib.cvl_curvelet_analysis_scale(ctx.h, ctypes.byref(p), j, flm.data_ptr(),
                                                   out.data_ptr(), ws.data_ptr(), n, s))
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    scal, grids = ctx.alloc_outputs(L, lam, J0)
    arr = (ctypes.c_void_p * len(grids[0]))(*[g.data_ptr() for g in grids[0]])
    rc = api.lib.cvl_curvelet_analysis(ctx.h, ctypes.byref(p), 1, fmap.data_ptr(),
                                       scal.data_ptr(), arr, ws.data_ptr(), n, s)
    assert rc == api.CVL_ENOMEM


def test_point_sources_against_oracle(ctx):
    # Gaussian field plus 64 band-limited point sources (harmonic form, built
    # by the oracle), analysed by both sides.
    L, lam, J0 = 64, 2.0, 2
    say("point sources L=%d" % L)
    f = inputs.gaussian_real_flm(L, 21)
    th, ph, a = inputs.point_sources(64, seed=4)
    f_or = f + osht.point_source_flm(L, th, ph, inputs.source_amplitudes(a, f, L))
    plan = ocurv.Plan(L, lam, J0)
    ref_scal, ref_grids = ocurv.analysis(plan, f_or)
    gmap = ctx.sht_inverse(dev(f_or), L)
    assert rel_l2(host(ctx.sht_forward(gmap)), f_or) < 1e-10
    scal, grids = ctx.curvelet_analysis(gmap, lam, J0)
    for s, j in enumerate(plan.scales):
        e = rel_l2(host(grids[s]), ref_grids[j])
        say("  scale %d rel L2 %.2e" % (j, e))
        assert e < 1e-10
    rec = host(ctx.curvelet_synthesis(scal, grids, L, lam, J0))
    assert rel_l2(rec, host(gmap)) < 1e-10


@pytest.mark.timeout(1200)
def test_l1024_fp32_streamed_point_sources():
    # Band-limit 1024, Gaussian field plus 64 point sources, complex64 grids
    # one scale at a time (a single 34 GB grid buffer), FP32 MFMA contractions,
    # FP64 Delta and final accumulation: one beta row of a finest scale against
    # the oracle, the round trip, the peak device memory; then the same with
    # real (float32) grids, which hold the same real parts in half the memory.
    import l1024_case as case
    L, lam, J0 = case.L, case.LAM, case.J0
    free, total = torch.cuda.mem_get_info()
    if free < 120 * 2**30:
        pytest.skip("needs about 110 GB of free device memory")
    say("L=1024 fp32 streamed: oracle row (background)")
    case.start_oracle_row()
    c = api.Context(L, 0)
    try:
        say("L=1024 fp32 streamed: input")
        fmap = c.sht_inverse(dev(case.flm()), L)
        torch.cuda.reset_peak_memory_stats()
        before = torch.cuda.memory_allocated()
        say("L=1024 fp32 streamed: round trip")
        rows = {}

        def keep_row(j, g):
            if j == case.SCALE:
                rows[j] = g[:, case.ROW, :].cpu().numpy()

        rec, scal = c.round_trip_streamed(fmap, lam, J0, precision="fp32", on_grid=keep_row)
        torch.cuda.synchronize()
        peak = (torch.cuda.max_memory_allocated() - before) / 2**30
        e = (torch.linalg.norm(rec - fmap) / torch.linalg.norm(fmap)).item()
        say("  round trip rel L2 %.2e, peak extra device memory %.1f GiB" % (e, peak))
        assert e < 1e-5
        # one grid (32 GiB) + the FP32 workspace (16 GiB), not all scales'
        # grids (68.5 GiB)
        assert peak < 56
        say("L=1024 fp32 streamed: waiting for the oracle row")
        ref = case.oracle_row()
        g = rows[case.SCALE][:, None, :]
        e = rel_l2(g, ref)
        mx = np.abs(g - ref).max() / np.abs(ref).max()
        say("  scale %d row %d vs oracle: rel L2 %.2e, max-abs rel %.2e" % (case.SCALE, case.ROW, e, mx))
        assert e < 1e-5 and mx < 1e-5
        say("L=1024 fp32 streamed, real grids: round trip")
        torch.cuda.reset_peak_memory_stats()
        before = torch.cuda.memory_allocated()
        rec2, _ = c.round_trip_streamed(fmap, lam, J0, precision="fp32", real_grids=True)
        torch.cuda.synchronize()
        peak2 = (torch.cuda.max_memory_allocated() - before) / 2**30
        say("  bitwise equal: %s, peak extra device memory %.1f GiB" % (torch.equal(rec2, rec), peak2))
        assert torch.equal(rec2, rec)
        assert peak2 < 20  # one float32 grid (16 GiB); the workspace is already held
    finally:
        torch.cuda.synchronize()
        c.close()
        torch.cuda.empty_cache()
