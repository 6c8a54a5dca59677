"""GPU: the allocation-free analysis entry point (static device scratch)
against the workspace entry point, through the C ABI.

Two calls in a row (L = 128, then the smaller L = 32) must each give the same
scaling map and grids as cvl_curvelet_analysis (bitwise: the same kernels on
the same inputs; the side stream only changes when the small scales run).
Calls that do not fit the scratch, or whose tables are not built, or with
per-stage timing on, are refused before anything is written.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU, skipped
    pytest.skip("no GPU", allow_module_level=True)

from paper_1511_05578_amd import api, inputs  # noqa: E402

LAM, J0 = 2.0, 2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _outputs(ctx, L, cplx=False):
    scal, grids = ctx.alloc_outputs(L, LAM, J0, 1, complex_map=cplx)
    scal.fill_(7.0)
    for g in grids[0]:
        g.fill_(7.0)
    flat = grids[0]
    arr = (ctypes.c_void_p * len(flat))(*[g.data_ptr() for g in flat])
    return scal, flat, arr


def _map(ctx, L, seed, cplx=False):
    if cplx:
        f = torch.from_numpy(inputs.uniform_complex_flm(L, seed)).cuda()
        return ctx.sht_inverse(f, L, complex_map=True).contiguous()
    f = torch.from_numpy(inputs.gaussian_real_flm(L, seed)).cuda()
    return ctx.sht_inverse(f, L).contiguous()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_noalloc_matches_workspace_entry_point():
    ctx = api.Context(129, 0)
    try:
        for L in (128, 32, 129):
            ctx.prepare(L, LAM, J0)
        cases = [(128, False), (32, False), (64, True)]
        ctx.prepare(64, LAM, J0)
        for L, cplx in cases:  # two (three) calls in a row, the later ones smaller
            say("noalloc vs workspace entry point: L=%d complex=%s" % (L, cplx))
            fmap = _map(ctx, L, seed=L, cplx=cplx)
            p = api.params(L, LAM, J0, complex_map=cplx)
            s1, g1, a1 = _outputs(ctx, L, cplx)
            nb = api.workspace_bytes(L, LAM, J0, 1, complex_map=cplx)
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
            api._check(api.lib.cvl_curvelet_analysis(ctx.h, ctypes.byref(p), 1, fmap.data_ptr(),
                                                     s1.data_ptr(), a1, ws.data_ptr(), nb,
                                                     _stream()))
            s2, g2, a2 = _outputs(ctx, L, cplx)
            api._check(api.lib.cvl_curvelet_analysis_noalloc(ctx.h, ctypes.byref(p), 1,
                                                             fmap.data_ptr(), s2.data_ptr(), a2,
                                                             _stream()))
            torch.cuda.synchronize()
            assert torch.equal(s1, s2)
            for x, y in zip(g1, g2):
                assert torch.equal(x, y)
            say("  bitwise equal over %d grids" % len(g1))
            del ws
        # does not fit the 80 MiB scratch (L = 129, FP64): refused, nothing written
        p = api.params(129, LAM, J0)
        fmap = _map(ctx, 129, seed=3)
        s3, g3, a3 = _outputs(ctx, 129)
        rc = api.lib.cvl_curvelet_analysis_noalloc(ctx.h, ctypes.byref(p), 1, fmap.data_ptr(),
                                                   s3.data_ptr(), a3, _stream())
        assert rc == api.CVL_ENOMEM
        # tables not built (L = 16 never prepared): refused
        p = api.params(16, LAM, J0)
        fmap = _map(ctx, 16, seed=4)
        s4, g4, a4 = _outputs(ctx, 16)
        rc = api.lib.cvl_curvelet_analysis_noalloc(ctx.h, ctypes.byref(p), 1, fmap.data_ptr(),
                                                   s4.data_ptr(), a4, _stream())
        assert rc == api.CVL_EINVAL
        # per-stage timing on: refused
        ctx.profile_enable(True)
        p = api.params(32, LAM, J0)
        fmap = _map(ctx, 32, seed=5)
        s5, g5, a5 = _outputs(ctx, 32)
        rc = api.lib.cvl_curvelet_analysis_noalloc(ctx.h, ctypes.byref(p), 1, fmap.data_ptr(),
                                                   s5.data_ptr(), a5, _stream())
        ctx.profile_enable(False)
        assert rc == api.CVL_EINVAL
        torch.cuda.synchronize()
        for s_, g_ in ((s3, g3), (s4, g4), (s5, g5)):
            assert bool((s_ == 7.0).all())
            for g in g_:
                assert bool((g == 7.0).all())
    finally:
        torch.cuda.synchronize()
        ctx.close()
