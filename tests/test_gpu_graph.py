"""GPU: a curvelet round trip captured in a HIP graph.

Once a plan is prepared and the workspace exists, the analysis and synthesis
calls allocate nothing and enqueue only kernels and event records (the side
stream of the smaller scales is forked and joined with events), so they can be
captured.  Each replay, with eager work and synchronisations between replays,
must reproduce the eager results bitwise.
"""
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU, skipped
    pytest.skip("no GPU", allow_module_level=True)

from paper_1511_05578_amd import api, inputs  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L", [32, 256])
def test_graph_replays_equal_eager(L):
    say("graph capture L=%d" % L)
    ctx = api.Context(L, 0)
    try:
        ctx.prepare(L)
        f = torch.from_numpy(inputs.gaussian_real_flm(L, seed=L)).cuda()
        m = ctx.sht_inverse(f, L).unsqueeze(0).contiguous()
        scal, grids = ctx.alloc_outputs(L)
        rec = torch.empty((1, L, 2 * L - 1), dtype=torch.float64, device="cuda")
        ctx.workspace(api.workspace_bytes(L))

        def step():
            ctx.curvelet_analysis(m, out=(scal, grids))
            ctx.curvelet_synthesis(scal, grids, L, out=rec)

        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        ref = rec.clone()
        ref_g = [x.clone() for x in grids[0]]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        torch.cuda.synchronize()
        for r in range(3):
            rec.zero_()
            for x in grids[0]:
                x.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(rec, ref), r
            for a, b in zip(grids[0], ref_g):
                assert torch.equal(a, b), r
            step()  # eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(rec, ref), r
        err = (torch.linalg.norm(ref - m) / torch.linalg.norm(m)).item()
        say("  replays bitwise equal to eager; round trip rel L2 %.2e" % err)
        assert err < 1e-10
        del g
    finally:
        torch.cuda.synchronize()
        ctx.close()
