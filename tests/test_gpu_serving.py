"""Serving on the GPU: every request's result is bitwise the same alone and
in the mix (continuous batching across streams, same-L batched calls)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1511_05578_amd import api, serving  # noqa: E402


def test_alone_equals_in_mix():
    Ls = [32, 16, 32, 64, 16, 32, 64, 16, 32, 32]
    arrivals = np.cumsum([0.0, 1e-4, 0, 2e-4, 0, 5e-4, 0, 0, 1e-3, 0])
    srv = serving.CurveletServer(L_max=64, slots=3, max_batch=3, keep_grids=True)
    try:
        srv.prepare(set(Ls))
        reqs = serving.make_requests(srv, len(Ls), Ls, arrivals, seed_base=100)
        done = srv.run(reqs)
        assert len(done) == len(Ls)
        assert all(r.admitted >= r.arrival - 1e-9 and r.done >= r.admitted for r in done)
        assert sum(1 for r in done if r.done_evt is not None) == len(Ls)
        ctx = srv.ctx
        for r in sorted(done, key=lambda r: r.rid):
            scal, grids = ctx.curvelet_analysis(r.fmap)
            rec = ctx.curvelet_synthesis(scal, grids, r.L)
            torch.cuda.synchronize()
            assert torch.equal(rec, r.out), r.rid
            assert torch.equal(scal, r.scal)
            for a, b in zip(grids, r.grids):
                assert torch.equal(a, b)
            err = (torch.linalg.norm(rec - r.fmap) / torch.linalg.norm(r.fmap)).item()
            assert err < 1e-10
    finally:
        srv.close()


def test_budget_serialises_when_tight():
    Ls = [64, 64, 64]
    srv = serving.CurveletServer(L_max=64, slots=3, max_batch=1,
                                 hbm_budget=serving.footprint_bytes(64) + 1)
    try:
        srv.prepare(Ls)
        reqs = serving.make_requests(srv, 3, Ls, np.zeros(3), seed_base=7)
        done = sorted(srv.run(reqs), key=lambda r: r.admitted)
        # one at a time: each is admitted only after the previous one finished
        for a, b in zip(done, done[1:]):
            assert b.admitted >= a.done - 1e-9
    finally:
        srv.close()


def test_unrotated_server_alone_equals_in_mix():
    # A server of unrotated-curvelet coefficients: each request's result is
    # bitwise the library's direct unrotated call, and reconstructs exactly.
    Ls = [32, 16, 32, 16, 64, 32]
    arrivals = np.cumsum([0.0, 1e-4, 0, 3e-4, 0, 1e-3])
    srv = serving.CurveletServer(L_max=64, slots=3, max_batch=2, keep_grids=True,
                                 unrotated=True)
    try:
        srv.prepare(set(Ls))
        reqs = serving.make_requests(srv, len(Ls), Ls, arrivals, seed_base=300)
        done = srv.run(reqs)
        assert len(done) == len(Ls)
        ctx = srv.ctx
        for r in sorted(done, key=lambda r: r.rid):
            scal, grids = ctx.curvelet_analysis(r.fmap, unrotated=True)
            rec = ctx.curvelet_synthesis(scal, grids, r.L, unrotated=True)
            torch.cuda.synchronize()
            assert torch.equal(rec, r.out), r.rid
            for a, b in zip(grids, r.grids):
                assert torch.equal(a, b)
            _, rot = ctx.curvelet_analysis(r.fmap)
            assert not torch.equal(rot[-1], r.grids[-1])
            err = (torch.linalg.norm(rec - r.fmap) / torch.linalg.norm(r.fmap)).item()
            assert err < 1e-10
    finally:
        srv.close()


def test_alone_equals_in_mix_configured_bandlimits():
    # The configured mix {64, 128, 256, 512}, including two L = 512 requests
    # and a batched pair of L = 128: every result (map, scaling map and every
    # grid) bitwise the one-call result.
    Ls = [512, 128, 64, 128, 256, 512, 64, 256]
    arrivals = np.cumsum([0.0, 1e-4, 0, 0, 2e-3, 0, 1e-3, 0])
    srv = serving.CurveletServer(L_max=512, slots=4, max_batch=4, keep_grids=True)
    try:
        srv.prepare(set(Ls))
        reqs = serving.make_requests(srv, len(Ls), Ls, arrivals, seed_base=500)
        done = srv.run(reqs)
        assert len(done) == len(Ls)
        ctx = srv.ctx
        for r in sorted(done, key=lambda r: r.rid):
            print("request %d L=%d admitted %.1f ms after arrival, latency %.1f ms"
                  % (r.rid, r.L, 1e3 * (r.admitted - r.arrival), 1e3 * (r.done - r.arrival)),
                  flush=True)
            scal, grids = ctx.curvelet_analysis(r.fmap)
            rec = ctx.curvelet_synthesis(scal, grids, r.L)
            torch.cuda.synchronize()
            assert torch.equal(rec, r.out), r.rid
            assert torch.equal(scal, r.scal)
            for a, b in zip(grids, r.grids):
                assert torch.equal(a, b)
            err = (torch.linalg.norm(rec - r.fmap) / torch.linalg.norm(r.fmap)).item()
            assert err < 1e-10
            del scal, grids, rec
            r.grids = None
            torch.cuda.empty_cache()
    finally:
        srv.close()
