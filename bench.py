"""Benchmark: spin-0 curvelet analysis + synthesis round trips on one MI355X.

Workload (one step): one real map at L = 256, lambda = 2, J0 = 2 (J = 8, scales
j = 2..8 with L_j = 8, 16, 32, 64, 128, 256, 256), complex128 SO(3) grids,
FP64 throughout: curvelet analysis (map -> scaling map + 7 grids) followed by
curvelet synthesis (-> map).  Inputs are resident in HBM before timing.

Prints ONE JSON line.  `value` is round trips per second.  `roofline` is for
the kernel stage with the largest device time, timed live with HIP events
recorded by the library on the launch stream; `cpu_baseline` is the CPU FP64
oracle timed on a bounded sample of the same workload and extrapolated.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--L 256] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "curvelet fwd+inv transforms/s at L=256,1024; rel-L2 err vs FP64; p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def scale_geoms(L, lam=2.0, J0=2):
    from paper_1511_05578_amd import api
    J = api.num_scales(L, lam, J0)
    kap, _ = api.kernel_tables(L, lam, J0)
    out = []
    for j in range(J0, J + 1):
        Lj = api.scale_shape(L, j, lam, J0)[0]
        nz = [l for l in range(Lj) if kap[j - J0, l] > 0]
        out.append(dict(j=j, L=Lj, Nm=2 * Lj - 1, h=(Lj - 1) // 2, Ne=2 * ((Lj - 1) // 2) + 1,
                        llo=min(nz) if nz else Lj, lhi=max(nz) if nz else Lj - 1))
    return out


def stage_models(L, lam=2.0, J0=2):
    """Algorithmic bytes / flops per round trip of each kernel stage.

    bytes: each stage's input read once and output written once (16 B per
    complex128).  flops: contractions 4 per (l, m, m', n>=0) term of the
    parity-folded sums (complex x real multiply-add); beta GEMMs 2 per
    multiply-add of the L_j x L_j real matrix on the 2*L_j*Ne real columns;
    DFT stages 5 n log2 n per complex line of length n = 2L_j - 1.
    """
    B = 16.0
    m = {}

    def add(name, nbytes, flops):
        b, f = m.get(name, (0.0, 0.0))
        m[name] = (b + nbytes, f + flops)

    for g in scale_geoms(L, lam, J0):
        Lj, Nm, h, Ne = g["L"], g["Nm"], g["h"], g["Ne"]
        terms = sum((l + 1) * (l + 1) * (l // 2 + 1) for l in range(g["llo"], g["lhi"] + 1))
        cube = Lj * Lj * Ne * B
        w2 = Lj * Nm * (h + 1) * B
        grid = Nm * Lj * Nm * B
        v1 = Lj * Nm * Ne * B
        fft = 5.0 * Nm * math.log2(Nm)
        add("contract_inv", cube, 4.0 * terms)
        add("beta_gemm_inv", 2 * cube, 2.0 * Lj * Lj * 2 * Lj * Ne)
        add("alpha_dft_inv", cube + w2, Lj * (h + 1) * fft)
        add("gamma_dft_inv", w2 + grid, Nm * Lj * fft)
        add("gamma_dft_fwd", grid + v1, Nm * Lj * fft)
        add("alpha_dft_fwd", v1 + cube, Lj * Ne * fft)
        add("beta_gemm_fwd", 2 * cube, 2.0 * Lj * Lj * 2 * Lj * Ne)
        add("contract_fwd", cube, 4.0 * terms)
    return m


def grid_bytes(L, lam=2.0, J0=2):
    return sum(g["Nm"] * g["L"] * g["Nm"] * 16.0 for g in scale_geoms(L, lam, J0))


def cpu_baseline(L, lam=2.0, J0=2):
    """Oracle round-trip time at this workload, from a bounded sample: one beta
    row per scale of the analysis and one Gauss-Legendre node per scale of the
    synthesis (plus that scale's full alpha/gamma Fourier step), scaled by the
    rows / nodes each scale has."""
    import numpy as np
    from oracle import curvelet as ocurv
    from oracle import sht as osht
    from paper_1511_05578_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    plan = ocurv.Plan(L, lam, J0)
    f = inputs.gaussian_real_flm(L, seed=0)
    t_an = 0.0
    t_sy = 0.0
    t0 = time.perf_counter()
    for j in plan.scales:
        Lj = plan.Lj[j]
        a = time.perf_counter()
        row = ocurv.analysis_scale(plan, f, j, rows=[Lj // 2])
        t_row = time.perf_counter() - a
        t_an += t_row * Lj
        # synthesis: full alpha/gamma step + one node, scaled to all nodes
        grid = np.zeros((2 * Lj - 1, Lj, 2 * Lj - 1), dtype=np.complex128)
        grid[:, Lj // 2:Lj // 2 + 1, :] = row
        a = time.perf_counter()
        from oracle import so3
        so3.gl_rows(grid, Lj, Lj)
        t_gl = time.perf_counter() - a
        a = time.perf_counter()
        ocurv.synthesis_scale(plan, grid, j, nodes_subset={0})
        t_node = time.perf_counter() - a - t_gl
        t_sy += t_gl + max(t_node, 0.0) * Lj
    a = time.perf_counter()
    osht.forward(osht.inverse(f, L).real, L)
    t_sht = time.perf_counter() - a
    wall = time.perf_counter() - t0
    t_total = t_an + t_sy + 2 * t_sht
    return {"value": 1.0 / t_total, "unit": "transforms/s", "cores": threads, "kind": "oracle",
            "sample": "L=%d: 1 beta row per scale of the analysis and 1 Gauss-Legendre node per "
                      "scale of the synthesis (with its full alpha/gamma step), extrapolated by "
                      "rows/nodes per scale, plus one SHT pair; %.1f s sampled, estimated %.1f s "
                      "per round trip" % (L, wall, t_total)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1511_05578_amd import api, inputs

    L, lam, J0 = args.L, 2.0, 2
    ctx = api.Context(L, 0)
    ctx.prepare(L, lam, J0)
    f = torch.from_numpy(inputs.gaussian_real_flm(L, seed=0)).cuda()
    fmap = ctx.sht_inverse(f, L)
    scal, grids = ctx.alloc_outputs(L, lam, J0, 1)
    rec = torch.empty((1, L, 2 * L - 1), dtype=torch.float64, device="cuda")
    fmap1 = fmap.unsqueeze(0).contiguous()

    def step():
        ctx.curvelet_analysis(fmap1, lam, J0, out=(scal, grids))
        ctx.curvelet_synthesis(scal, grids, L, lam, J0, out=rec)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    err = (torch.linalg.norm(rec[0] - fmap) / torch.linalg.norm(fmap)).item()

    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)

    ms = dt * 1e3 / args.steps
    models = stage_models(L, lam, J0)
    stages = {k: {"launches": v[0], "ms_per_step": v[1] / args.steps} for k, v in prof.items() if v[0]}
    top = max((k for k in stages if k in models), key=lambda k: stages[k]["ms_per_step"])
    t_top = stages[top]["ms_per_step"] * 1e-3 / (stages[top]["launches"] / args.steps)  # s per launch
    nb, nf = models[top]
    launches_per_step = stages[top]["launches"] / args.steps
    bytes_per_launch = nb / launches_per_step
    flops_per_launch = nf / launches_per_step
    ai = nf / max(nb, 1.0)
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if ai < ridge:
        roof = {"bound": "hbm", "achieved": bytes_per_launch / t_top / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": flops_per_launch / t_top / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = top
    roof["algorithmic_per_launch"] = {"bytes": bytes_per_launch, "flops": flops_per_launch}

    out = {
        "metric": METRIC,
        "value": 1e3 / ms,
        "unit": "transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: f_lm ~ N(0,(l+1)^-2) real-map coefficients, seed 0",
        "config": {"workload": "C2: one real spin-0 map, L=%d, lambda=2, J0=2, J=%d, N_j=L_j, "
                               "complex128 grids, analysis+synthesis round trip" % (L, api.num_scales(L)),
                   "L": L, "lambda": lam, "J0": J0, "grid_bytes": grid_bytes(L, lam, J0)},
        "round_trip_rel_l2": err,
        "hbm_roofline_ms": 2 * grid_bytes(L, lam, J0) / (HBM_PEAK_GBS * 1e9) * 1e3,
        "roofline": roof,
        "stages": stages,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(L, lam, J0)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
