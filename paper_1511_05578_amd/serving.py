"""Continuous-batching server for curvelet round trips of mixed band-limits.

Requests (a real map of band-limit L) arrive over time.  The server keeps the
Delta table and every (L, lambda, J0) kernel / DFT table resident in one
context, and runs each admitted request's analysis + synthesis on one of
several HIP streams, so work of requests that arrive while others run
overlaps on the device.  A request is admitted when (a) it has arrived,
(b) a stream slot is free and (c) the device-memory footprint of all admitted
requests (grids and maps) stays within the budget; each slot's workspace is
allocated once, before serving starts.  Queued requests
of the same L that can be admitted together are launched as one batched call.

Every request has its own grids and workspace and runs on one stream, so its
result does not depend on what else is in flight (bitwise; tested).

Usage:  python -m paper_1511_05578_amd.serving [--requests 1024] [--loads 0.5 0.7 0.9]
"""
import argparse
import json
import sys
import time
from collections import deque

import numpy as np

from . import api, inputs


def footprint_bytes(L, lam=2.0, J0=2, batch=1):
    """Device bytes one batched call holds until it retires: its grids, its
    scaling maps and its input and output maps.  (Workspaces belong to the
    stream slots and are allocated once.)"""
    grids = 0
    J = api.num_scales(L, lam, J0)
    for j in range(J0, J + 1):
        Lj, Nj = api.scale_shape(L, j, lam, J0)
        grids += (2 * Lj - 1) * Lj * (2 * Nj - 1) * 16  # complex128
    Lp = api.scaling_bandlimit(L, lam, J0)
    maps = 2 * L * (2 * L - 1) * 8 + Lp * (2 * Lp - 1) * 8
    return batch * (grids + maps)


def batch_cap(L, max_batch=4, work_cap=2 * 256 ** 3):
    """Largest batch for band-limit L: the work of a call grows like B L^3, and
    a call that already fills the device gains nothing from batching but
    latency, so B L^3 is capped (L=512: 1, L=256: 2, smaller L: max_batch)."""
    return max(1, min(max_batch, work_cap // (L ** 3)))


def plan_admission(queue_Ls, in_use, budget, free_slots, max_batch, footprint):
    """Admission decisions for one scheduling pass.

    queue_Ls: band-limits of the queued requests in arrival order.  Returns a
    list of groups (lists of queue indices), at most one per free slot; each
    group is the oldest queued request plus younger ones of the same L (up to
    max_batch, an int or a function of L), shrunk until its footprint fits the
    remaining budget.  The pass stops at the first head that does not fit (no overtaking: the oldest
    request is never starved by smaller ones)."""
    groups = []
    taken = set()
    for _ in range(free_slots):
        rest = [i for i in range(len(queue_Ls)) if i not in taken]
        if not rest:
            break
        head = rest[0]
        cap = max_batch(queue_Ls[head]) if callable(max_batch) else max_batch
        group = [head] + [i for i in rest[1:] if queue_Ls[i] == queue_Ls[head]][:cap - 1]
        while len(group) > 1 and in_use + footprint(queue_Ls[head], len(group)) > budget:
            group.pop()
        need = footprint(queue_Ls[head], len(group))
        if in_use + need > budget:
            break
        in_use += need
        taken.update(group)
        groups.append(group)
    return groups


class Request:
    __slots__ = ("rid", "L", "arrival", "fmap", "admitted", "done_evt", "done", "out",
                 "grids", "scal")

    def __init__(self, rid, L, arrival, fmap):
        self.rid, self.L, self.arrival, self.fmap = rid, L, arrival, fmap
        self.admitted = self.done = None
        self.done_evt = self.out = self.grids = self.scal = None


class CurveletServer:
    def __init__(self, L_max=512, lam=2.0, J0=2, slots=4, hbm_budget=None, max_batch=4,
                 keep_grids=False, device=0, unrotated=False):
        """unrotated: every request gets the coefficients of the unrotated
        curvelets (CVL_UNROTATED) instead of the rotated ones."""
        import torch
        self.torch = torch
        self.lam, self.J0 = lam, J0
        self.unrotated = bool(unrotated)
        self.ctx = api.Context(L_max, device)
        self.dev = self.ctx.device
        self.slots = slots
        self.max_batch = max_batch
        self.keep_grids = keep_grids
        self.hbm_budget = hbm_budget
        self.budget = None
        # one stream and one workspace per slot; streams at default priority
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        self.ws = [None] * slots
        self.busy = [None] * slots   # (requests, bytes, buffers) in flight on the slot
        self.in_use = 0

    def cap(self, L):
        return batch_cap(L, self.max_batch)

    def prepare(self, Ls):
        """Build the tables of every band-limit to be served, give each slot a
        workspace large enough for any call, and fix the budget for grids and
        maps (by default 85% of the device memory still free after that)."""
        t = self.torch
        Ls = sorted(set(int(x) for x in Ls))
        for L in Ls:
            self.ctx.prepare(L, self.lam, self.J0)
        nb = max(api.workspace_bytes(L, self.lam, self.J0, self.cap(L), unrotated=self.unrotated)
                 for L in Ls)
        for s in range(self.slots):
            if self.ws[s] is None or self.ws[s].numel() < nb:
                self.ws[s] = None
                self.ws[s] = t.empty(nb, dtype=t.uint8, device=self.dev)
        t.cuda.synchronize()
        # blocks the caching allocator still holds from earlier work (say, large
        # grids of other calls) go back to the device first, so that the budget
        # and the server's allocations start from the same, unfragmented pool
        # (after a 170 GB batched call, capacity had once measured half of it)
        t.cuda.empty_cache()
        free, _ = t.cuda.mem_get_info(self.dev)
        self.budget = self.hbm_budget if self.hbm_budget is not None else int(0.85 * free)

    def _launch(self, slot, reqs):
        t = self.torch
        L = reqs[0].L
        B = len(reqs)
        lam, J0 = self.lam, self.J0
        st = self.streams[slot]
        with t.cuda.stream(st):
            maps = t.stack([r.fmap for r in reqs]).contiguous()
            scal, grids = self.ctx.alloc_outputs(L, lam, J0, B)
            ws = self.ws[slot]
            if ws is None or ws.numel() < api.workspace_bytes(L, lam, J0, B,
                                                              unrotated=self.unrotated):
                raise RuntimeError("band-limit %d was not prepared" % L)
            flat = [g for per in grids for g in per]
            import ctypes
            arr = (ctypes.c_void_p * len(flat))(*[g.data_ptr() for g in flat])
            out = t.empty((B, L, 2 * L - 1), dtype=t.float64, device=self.dev)
            p = api.params(L, lam, J0, unrotated=self.unrotated)
            s = ctypes.c_void_p(st.cuda_stream)
            api._check(api.lib.cvl_curvelet_analysis(self.ctx.h, ctypes.byref(p), B, maps.data_ptr(),
                                                     scal.data_ptr(), arr, ws.data_ptr(), ws.numel(), s))
            api._check(api.lib.cvl_curvelet_synthesis(self.ctx.h, ctypes.byref(p), B, scal.data_ptr(),
                                                      arr, out.data_ptr(), ws.data_ptr(), ws.numel(), s))
            evt = t.cuda.Event()
            evt.record(st)
        for i, r in enumerate(reqs):
            r.done_evt = evt
            r.out = out[i]
            if self.keep_grids:
                r.grids = [g for g in grids[i]]
                r.scal = scal[i]
        self.busy[slot] = (reqs, footprint_bytes(L, lam, J0, B), maps, scal, grids, out)

    def run(self, requests, poll_sleep=0.0):
        """Serve `requests` (sorted by arrival, seconds from start).  Returns them
        with `admitted` / `done` wall times filled in."""
        if self.budget is None:
            raise RuntimeError("call prepare() with the band-limits to serve first")
        queue = deque()
        todo = deque(requests)
        t0 = time.perf_counter()
        finished = []
        while todo or queue or any(b is not None for b in self.busy):
            now = time.perf_counter() - t0
            while todo and todo[0].arrival <= now:
                queue.append(todo.popleft())
            # retire
            for s in range(self.slots):
                b = self.busy[s]
                if b is not None and b[0][0].done_evt.query():
                    tdone = time.perf_counter() - t0
                    for r in b[0]:
                        r.done = tdone
                        finished.append(r)
                    self.in_use -= b[1]
                    self.busy[s] = None
            # admit (continuous batching: same-L requests queued together share a call)
            free = [s for s in range(self.slots) if self.busy[s] is None]
            if free and queue:
                qlist = list(queue)
                fp = lambda L, b: footprint_bytes(L, self.lam, self.J0, b)
                groups = plan_admission([r.L for r in qlist], self.in_use, self.budget,
                                        len(free), self.cap, fp)
                for s, grp in zip(free, groups):
                    reqs = [qlist[i] for i in grp]
                    for r in reqs:
                        queue.remove(r)
                        r.admitted = time.perf_counter() - t0
                    self.in_use += fp(reqs[0].L, len(reqs))
                    self._launch(s, reqs)
            if poll_sleep:
                time.sleep(poll_sleep)
        self.torch.cuda.synchronize()
        return finished

    def close(self):
        self.torch.cuda.synchronize()
        self.ws = [None] * self.slots
        self.ctx.close()


def make_requests(server, n, Ls, arrivals, seed_base=0):
    t = server.torch
    reqs = []
    for i in range(n):
        L = int(Ls[i])
        f = t.from_numpy(inputs.gaussian_real_flm(L, seed=seed_base + i)).to(server.dev)
        fmap = server.ctx.sht_inverse(f, L)
        reqs.append(Request(i, L, float(arrivals[i]), fmap))
    t.cuda.synchronize()
    return reqs


def latency_stats(done):
    lat = np.array([r.done - r.arrival for r in done])
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


def measure_capacity(server, Ls, n=64):
    """Requests/s when every request is queued at t = 0 (closed-loop capacity)."""
    reqs = make_requests(server, n, Ls[:n], np.zeros(n), seed_base=10_000)
    server.run(reqs[:4])  # warm-up (first launches load code objects)
    reqs = make_requests(server, n, Ls[:n], np.zeros(n), seed_base=10_000)
    t0 = time.perf_counter()
    server.run(reqs)
    return n / (time.perf_counter() - t0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=1024)
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5, 0.7, 0.9])
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--bandlimits", type=int, nargs="+", default=[64, 128, 256, 512])
    ap.add_argument("--unrotated", action="store_true",
                    help="serve the coefficients of the unrotated curvelets")
    args = ap.parse_args()
    server = CurveletServer(L_max=max(args.bandlimits), slots=args.slots,
                            unrotated=args.unrotated)
    server.prepare(args.bandlimits)
    _, Ls = inputs.serving_trace(args.requests, tuple(args.bandlimits), 1.0, seed_arrivals=1,
                                 seed_sizes=2)
    cap = measure_capacity(server, Ls)
    print("capacity %.1f req/s" % cap, file=sys.stderr, flush=True)
    out = {"capacity_req_per_s": cap, "slots": args.slots, "budget_bytes": server.budget,
           "bandlimits": args.bandlimits, "unrotated": bool(args.unrotated), "runs": []}
    for rho in args.loads:
        arr, Ls = inputs.serving_trace(args.requests, tuple(args.bandlimits), rho * cap,
                                       seed_arrivals=1, seed_sizes=2)
        reqs = make_requests(server, args.requests, Ls, arr)
        t0 = time.perf_counter()
        done = server.run(reqs)
        wall = time.perf_counter() - t0
        st = latency_stats(done)
        st.update({"load": rho, "offered_req_per_s": rho * cap, "served_req_per_s": len(done) / wall,
                   "requests": len(done)})
        for L in args.bandlimits:
            sel = [r for r in done if r.L == L]
            if sel:
                st["p50_ms_L%d" % L] = latency_stats(sel)["p50_ms"]
                st["p99_ms_L%d" % L] = latency_stats(sel)["p99_ms"]
        out["runs"].append(st)
        print("load %.2f: p50 %.2f ms  p99 %.2f ms" % (rho, st["p50_ms"], st["p99_ms"]),
              file=sys.stderr, flush=True)
        del reqs, done
    server.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
