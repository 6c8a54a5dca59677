"""Benchmark: spin-0 curvelet analysis + synthesis round trips on one MI355X.

Default workload (one step): one real map at L = 256, lambda = 2, J0 = 2 (J = 8,
scales j = 2..8 with L_j = 8, 16, 32, 64, 128, 256, 256), complex128 SO(3)
grids, FP64 throughout: curvelet analysis (map -> scaling map + 7 grids)
followed by curvelet synthesis (-> map).  Inputs are resident in HBM before
timing.  Other workloads: --L, --batch (maps per call) and --precision
(fp64 | fp32 | bf16x3: complex64 grids, reduced-precision contractions) and
--real-grids (float64 / float32 grids: the real coefficients without the zero
imaginary parts).

Prints ONE JSON line.  `value` is round trips (maps) per second.  Every
launch of the warm-up steps after the first is timed with HIP events (the
per-stage breakdown `stages`, `stages_by_bandlimit`, and the choice of the
dominant kernel: the (stage, L_j) pair with the largest device time).  In the
timed region only that kernel's launches carry events, recorded by the library
on the launch stream, so `ms_per_step` does not pay for events on the other
launches; `roofline` uses their average duration.  `whole_roofline` is the
whole round trip against max(bytes / HBM peak, contraction flops / matrix
peak + DFT flops / vector peak).  `cpu_baseline` is the CPU
FP64 oracle timed on a bounded sample of the same workload and extrapolated.  For
the reduced precisions the grids and the round trip are compared with the
FP64 path (itself held to the oracle by the parity tests).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--L 256] [--batch 1]
                       [--precision fp64] [--stream] [--real-grids] [--graph] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Band-limit from which the analysis beta stage runs as an odd-length DFT
# (even/odd m' line pairs through the Bluestein engine) instead of a GEMM.
BETA_FFT_MIN_L = 256

METRIC = "curvelet fwd+inv transforms/s at L=256,1024; rel-L2 err vs FP64; p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0


def stage_peak(stage, precision):
    """Compute peak (TFLOP/s) of a stage's arithmetic in a given precision."""
    if precision == "fp64":
        return FP64_PEAK_TFLOPS
    if precision == "bf16x3" and stage.startswith("contract"):
        return BF16_MFMA_PEAK_TFLOPS
    return FP32_PEAK_TFLOPS


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


def _unrot_live_lines(Lj):
    """Line pairs (m, column) of the unrotated cube with a non-zero entry:
    row (m, s) holds n of parity (m + s) mod 2 at column c (even n = 2(c - h),
    c <= 2h; odd n = 2(c - floor(L_j/2)) + 1, c < 2 floor(L_j/2)); the entry
    can be non-zero only if m <= |n|."""
    import numpy as np
    h, ho = (Lj - 1) // 2, Lj // 2
    Nc = max(2 * h + 1, 2 * ho)
    c = np.arange(Nc)
    le = np.where(c <= 2 * h, np.abs(2 * (c - h)), -1)       # even-n class
    lo = np.where(c < 2 * ho, np.abs(2 * (c - ho) + 1), -1)  # odd-n class
    m = np.arange(Lj)[:, None]
    # rows (m, 0) and (m, 1) hold the two classes, in an order set by m's parity
    return int(np.count_nonzero((m <= le[None, :]) | (m <= lo[None, :])))


def stage_models(L, lam=2.0, J0=2, B=16.0, GB=None, unrot=False):
    """Algorithmic bytes / flops of each kernel stage per round trip of one
    map, keyed (stage, L_j): one launch per scale, scales of equal L_j summed.

    bytes: each stage's input read once and output written once (B = 16 bytes
    per complex128, 8 per complex64; GB per grid element, B by default, B / 2
    for real grids).
    flops: contractions 4 per (l, m, m', n>=0) term of the parity-folded sums
    (complex x real multiply-add); beta GEMMs 2 per multiply-add of the
    L_j x L_j real matrix on the 2*L_j*Ne real columns; DFT stages
    5 n log2 n per complex line of length n = 2L_j - 1 (from L_j =
    BETA_FFT_MIN_L on, the analysis beta stage is such a DFT stage over
    (L_j + 1) / 2 * Ne line pairs).

    Unrotated curvelets (unrot): only what the method needs is counted.  A
    cube entry (m', m >= 0, n) is non-zero only for m, m' <= l = |n| (nnz of
    them, one contraction term each); the analysis beta DFT transforms the
    line pairs (m, column) holding one (live lines), the alpha DFTs read or
    write the |m| <= |n| entries, and the synthesis beta GEMM needs, for each
    column with m <= |n|, the |n| + 1 outputs m' <= |n| (2 flops per
    multiply-add of the real L_j-long rows on the two real parts).  Below
    BETA_FFT_MIN_L the analysis beta stage is the dense GEMM on the whole cube
    (2 L_j rows of Nc columns per plane, Nc = max(2h + 1, 2 floor(L_j / 2))).
    """
    m = {}
    GB = B if GB is None else GB

    def add(name, Lj, nbytes, flops):
        b, f, n = m.get((name, Lj), (0.0, 0.0, 0))
        m[(name, Lj)] = (b + nbytes, f + flops, n + 1)

    for g in scale_geoms(L, lam, J0):
        Lj, Nm, h, Ne = g["L"], g["Nm"], g["h"], g["Ne"]
        if unrot:
            Nc = max(2 * h + 1, 2 * (Lj // 2))
            terms = sum((l + 1) * (l + 1) * (2 if l else 1)
                        for l in range(g["llo"], g["lhi"] + 1))
            nnz = sum((l + 1) * (l + 1) * (2 if l else 1) for l in range(Lj))
            cols = sum(abs(n) + 1 for n in range(-(Lj - 1), Lj))  # columns with m <= |n|
            live = _unrot_live_lines(Lj)
            cube = Lj * 2 * Lj * Nc * B
            w2 = Lj * Nm * Lj * B
            grid = Nm * Lj * Nm * GB
            fft = 5.0 * Nm * math.log2(Nm)
            if Lj >= BETA_FFT_MIN_L:
                add("contract_inv", Lj, nnz * B, 4.0 * terms)
                add("beta_gemm_inv", Lj, nnz * B + 2 * live * Lj * B, live * fft)
            else:
                add("contract_inv", Lj, cube, 4.0 * terms)
                add("beta_gemm_inv", Lj, 2 * cube, 2.0 * Lj * Lj * 2 * 2 * Lj * Nc)
            add("alpha_dft_inv", Lj, Lj * cols * B + w2, Lj * Lj * fft)
            add("gamma_dft_inv", Lj, w2 + grid, Nm * Lj * fft)
            add("gamma_dft_fwd", Lj, grid + w2, Nm * Lj * fft)
            add("alpha_dft_fwd", Lj, w2 + Lj * cols * B, Lj * Lj * fft)
            add("beta_gemm_fwd", Lj, Lj * cols * B + nnz * B, 2.0 * 2 * Lj * nnz)
            add("contract_fwd", Lj, terms * B, 4.0 * terms)
            continue
        terms = sum((l + 1) * (l + 1) * (l // 2 + 1) for l in range(g["llo"], g["lhi"] + 1))
        cube = Lj * Lj * Ne * B
        w2 = Lj * Nm * (h + 1) * B
        grid = Nm * Lj * Nm * GB
        v1 = Lj * Nm * Ne * B
        fft = 5.0 * Nm * math.log2(Nm)
        add("contract_inv", Lj, cube, 4.0 * terms)
        if Lj >= BETA_FFT_MIN_L:  # one DFT line per even/odd m' line pair
            add("beta_gemm_inv", Lj, 2 * cube, ((Lj + 1) // 2) * Ne * fft)
        else:
            add("beta_gemm_inv", Lj, 2 * cube, 2.0 * Lj * Lj * 2 * Lj * Ne)
        add("alpha_dft_inv", Lj, cube + w2, Lj * (h + 1) * fft)
        add("gamma_dft_inv", Lj, w2 + grid, Nm * Lj * fft)
        add("gamma_dft_fwd", Lj, grid + v1, Nm * Lj * fft)
        add("alpha_dft_fwd", Lj, v1 + cube, Lj * Ne * fft)
        add("beta_gemm_fwd", Lj, 2 * cube, 2.0 * Lj * Lj * 2 * Lj * Ne)
        add("contract_fwd", Lj, cube, 4.0 * terms)
    return m


def whole_roofline(L, lam, J0, prec, NB, GB, ms, unrot=False):
    """Roofline of the whole round trip: t_roof = max(bytes / HBM peak,
    contraction flops / matrix peak + DFT flops / vector peak) with bytes the
    grids written once and read once plus the maps, contraction flops 4 per
    (l, m >= 0, m' >= 0, even n) term with l >= max(m, m', |n|) (x3 for split
    BF16), DFT flops 5 n log2 n per complex line of length n = 2L_j - 1 over
    the beta, alpha and gamma lines of a (2L_j - 1) x L_j x (2L_j - 1) grid in
    both directions, halved for the real signal.  Unrotated curvelets: one
    contraction term per (l, m >= 0, m' <= l, n = +-l)."""
    gb = 2 * grid_bytes(L, lam, J0, GB)
    Lp = min(int(math.ceil(lam ** J0)), L)
    maps = 2 * L * (2 * L - 1) * 8 + 2 * Lp * (2 * Lp - 1) * 8
    nbytes = NB * (gb + maps)
    con = dft = 0.0
    for g in scale_geoms(L, lam, J0):
        Lj, Nm = g["L"], g["Nm"]
        if unrot:
            terms = sum((l + 1) * (l + 1) * (2 if l else 1)
                        for l in range(g["llo"], g["lhi"] + 1))
        else:
            terms = sum((l + 1) * (l + 1) * (2 * (l // 2) + 1)
                        for l in range(g["llo"], g["lhi"] + 1))
        con += 2 * 4.0 * terms
        fft = 5.0 * Nm * math.log2(Nm)
        # per direction: beta lines (m, n), alpha lines (b, n), gamma lines (a, b)
        dft += 2 * 0.5 * fft * (Nm * Nm + Lj * Nm + Nm * Lj)
    con *= NB * (3 if prec == "bf16x3" else 1)
    dft *= NB
    peak_c = {"fp64": FP64_PEAK_TFLOPS, "fp32": FP32_PEAK_TFLOPS,
              "bf16x3": BF16_MFMA_PEAK_TFLOPS}[prec]
    peak_v = FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS
    t_mem = nbytes / (HBM_PEAK_GBS * 1e9) * 1e3
    t_cmp = (con / (peak_c * 1e12) + dft / (peak_v * 1e12)) * 1e3
    t_roof = max(t_mem, t_cmp)
    return {"t_roof_ms": t_roof, "bound": "hbm" if t_mem >= t_cmp else "compute",
            "frac": t_roof / ms, "bytes": nbytes, "contraction_flops": con,
            "dft_flops": dft}


def rule_roofline(stage, Lj, GB, flops_per_launch, t_launch, peak_tf):
    """Roofline of one launch by the measurement rule: the algorithmic bytes
    are the grid elements a launch writes (analysis) or reads (synthesis) once
    -- only the gamma DFT stages touch the grids, one scale's grid per launch,
    (2L_j-1) x L_j x (2L_j-1) elements of GB bytes -- and the algorithmic flops
    those the method needs (``stage_models``).  A stage without grid IO is
    priced by its flops against the matrix cores (contractions, beta GEMMs) or
    the vector units (the other DFT stages)."""
    if stage.startswith("gamma"):
        nbytes = (2 * Lj - 1) * Lj * (2 * Lj - 1) * GB
        r = {"bound": "hbm", "achieved": nbytes / t_launch / 1e9, "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "bytes_per_launch": nbytes}
    else:
        r = {"bound": "mfma" if stage.startswith(("contract", "beta_gemm")) else "alu",
             "achieved": flops_per_launch / t_launch / 1e12, "peak": peak_tf, "unit": "TFLOP/s"}
    r["frac"] = r["achieved"] / r["peak"]
    return r


def copy_ceiling(stage_gbs, nbytes=512 << 20, reps=5):
    """The HBM rate a plain device copy reaches on this GPU (bytes read plus
    bytes written per second, 512 MiB: twice the 256 MB last-level cache),
    timed with HIP events, and the dominant launch's stage IO rate as a
    fraction of it -- the practical ceiling beside the nominal 8 TB/s."""
    import torch

    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    return {"GBs": gbs, "bytes": 2 * nbytes, "stage_io_frac": stage_gbs / gbs}


def bluestein_size(Lj):
    n = 2 * (2 * Lj - 1) - 1
    P = 8
    while P < n:
        P *= 2
    return P


def kernel_symbol(stage, Lj, prec, real_grids=False, unrot=False):
    """HIP kernel (template instance) that runs a stage at band-limit L_j."""
    c = "cd" if prec == "fp64" else "cf"
    P = bluestein_size(Lj)
    u = "Unrot" if unrot else ""
    # the packed gamma stages at even L_j run one FFT at half length at
    # 1024 <= P <= 4096
    even = Lj % 2 == 0 and not unrot
    odd = "Odd" if (even and 1024 <= P <= 4096) else ""
    io = {"alpha_dft_inv": u + "InvAlphaIO", "alpha_dft_fwd": u + "FwdAlphaIO",
          "gamma_dft_inv": u + ("InvGammaPack%sIO" % odd if P >= 256 else "InvGammaIO"),
          "gamma_dft_fwd": u + ("FwdGammaPack%sIO" % odd if P >= 256 else "FwdGammaIO")}
    if stage in io:
        targs = c
        if stage.startswith("gamma"):  # grid element type
            targs += ", " + (("double" if prec == "fp64" else "float") if real_grids else c)
        eng = "k_blue_r16<%d, %s<%s> >" % (P, io[stage], targs) if P >= 256 else \
              "k_bluestein<%d, ..., %s<%s> >" % (P, io[stage], targs)
        return eng
    mode = {"fp64": "", "fp32": "<1>", "bf16x3": "<2>"}[prec]
    if stage == "beta_gemm_inv" and Lj >= BETA_FFT_MIN_L:
        # complex64 at FFT size 4096: written line-major, then transposed
        io = "BetaInvLineIO" if (prec != "fp64" and P == 4096 and not unrot) else "BetaInvPairIO"
        return "k_blue_r16<%d, %s%s<%s> >" % (P, "Unrot" if unrot else "", io, c)
    if stage.startswith("beta"):
        if prec == "fp64":
            return "k_beta_mfma"
        # template instance: precision mode, K = L_j a multiple of 4
        return "k_beta_mfma_mx%s" % (mode[:-1] + (", true>" if Lj % 4 == 0 else ", false>"))
    if unrot and stage in ("contract_inv", "contract_fwd"):
        return "k_unrot_%s<%s>" % (stage, c)
    if stage == "contract_inv":
        return "k_contract_inv_mfma" if prec == "fp64" else "k_contract_inv_mx" + mode
    if stage == "contract_fwd":
        return "k_contract_fwd_m1" if prec == "fp64" else "k_contract_fwd_mx1" + mode
    if stage == "reduce_fwd":
        return "k_reduce_groups<%s>" % c
    return stage


def source_fingerprint():
    """sha1 of the library sources: counter figures taken from another build
    do not describe this one."""
    import hashlib
    hsh = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_1511_05578_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            hsh.update(name.encode() + f.read())
    return hsh.hexdigest()[:16]


def recorded_traffic(workload_key, kernel, finest=False):
    """HBM bytes per launch of `kernel` from a committed counter summary of
    this workload and this source fingerprint, else None.  finest: the launch
    of interest is one of the finest scales', and a kernel that every scale
    shares has its largest launches recorded separately ("top")."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    fp = source_fingerprint()
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                if not line.startswith("TRAFFIC_JSON "):
                    continue
                try:
                    rec = json.loads(line[len("TRAFFIC_JSON "):])
                except ValueError:
                    continue
                if rec.get("workload") != workload_key or rec.get("source") != fp:
                    continue
                k = rec.get("kernels", {}).get(kernel)
                if k:
                    if finest and "top" in k:
                        k = k["top"]
                    return k["fetch_bytes"] + k["write_bytes"]
    return None


def grid_bytes(L, lam=2.0, J0=2, B=16.0):
    """Bytes of one map's grids, B bytes per element."""
    return sum(g["Nm"] * g["L"] * g["Nm"] * B for g in scale_geoms(L, lam, J0))


def point_source_flm(L, theta, phi, amp):
    """Harmonic coefficients sum_k amp_k conj(Y_lm(theta_k, phi_k)) of
    band-limited point sources (flat, length L^2), for building the large
    workload's input.  Y_lm from the fully normalised associated Legendre
    functions (Condon-Shortley phase), by the standard recurrences:
    P_00 = 1/sqrt(4 pi), P_mm = -sqrt((2m+1)/(2m)) sin(t) P_{m-1,m-1},
    P_{m+1,m} = sqrt(2m+3) cos(t) P_mm and, for l >= m+2,
    P_lm = a (cos(t) P_{l-1,m} - b P_{l-2,m}) with a = sqrt((4l^2-1)/(l^2-m^2)),
    b = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)); vectorised over m and the sources."""
    import numpy as np
    x = np.cos(np.asarray(theta, dtype=np.float64))[None, :]
    sx = np.sin(np.asarray(theta, dtype=np.float64))[None, :]
    K = x.shape[1]
    m = np.arange(L, dtype=np.float64)[:, None]
    fac = np.ones((L, 1))
    fac[1:, 0] = -np.sqrt((2 * m[1:, 0] + 1) / (2 * m[1:, 0]))
    steps = fac * sx * np.ones((L, K))
    steps[0] = 1.0
    diag = np.cumprod(steps, axis=0) / math.sqrt(4 * math.pi)  # P_mm
    ph = np.exp(-1j * np.outer(np.arange(L), np.asarray(phi, dtype=np.float64)))  # [m, k]
    w = ph * np.asarray(amp, dtype=np.float64)[None, :]
    out = np.zeros(L * L, dtype=np.complex128)
    p2 = np.zeros((L, K))
    p1 = np.zeros((L, K))
    for l in range(L):
        p0 = np.zeros((L, K))
        if l >= 2:
            mm = m[:l - 1]
            a = np.sqrt((4.0 * l * l - 1) / (l * l - mm * mm))
            b = np.sqrt(((l - 1.0) ** 2 - mm * mm) / (4.0 * (l - 1) ** 2 - 1))
            p0[:l - 1] = a * (x * p1[:l - 1] - b * p2[:l - 1])
        if l >= 1:
            p0[l - 1] = math.sqrt(2 * l + 1) * x[0] * diag[l - 1]
        p0[l] = diag[l]
        vals = np.sum(p0[:l + 1] * w[:l + 1], axis=1)  # m = 0..l
        base = l * l + l
        out[base:base + l + 1] = vals
        ms = np.arange(1, l + 1)
        out[base - ms] = ((-1.0) ** ms) * np.conj(vals[1:])
        p2, p1 = p1, p0
    return out


def large_leg(steps=3, L=1024, n_sources=64):
    """The large workload: one real map at L = 1024 (Gaussian field, seed 0,
    plus 64 band-limited point sources, seed 1, peaks 1..10 x the field's rms)
    through the streaming interface (one complex64 grid resident at a time),
    FP32 MFMA contractions, FP64 Delta and final accumulation.  One warm-up
    round trip, then `steps` timed ones."""
    import torch
    from paper_1511_05578_amd import api, inputs
    lam, J0 = 2.0, 2
    t_setup = time.perf_counter()
    ctx = api.Context(L, 0)
    try:
        ctx.prepare(L, lam, J0)
        f = inputs.gaussian_real_flm(L, seed=0)
        th, ph, a = inputs.point_sources(n_sources, seed=1)
        f = f + point_source_flm(L, th, ph, inputs.source_amplitudes(a, f, L))
        fmap = ctx.sht_inverse(torch.from_numpy(f).cuda(), L)
        rec, _ = ctx.round_trip_streamed(fmap, lam, J0, precision="fp32")
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t_setup
        t0 = time.perf_counter()
        for _ in range(steps):
            rec, _ = ctx.round_trip_streamed(fmap, lam, J0, precision="fp32")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        err = (torch.linalg.norm(rec - fmap) / torch.linalg.norm(fmap)).item()
        del rec, fmap
    finally:
        torch.cuda.synchronize()
        ctx.close()
        torch.cuda.empty_cache()
    return {"workload": "1 real spin-0 map with %d point sources, L=%d, lambda=2, J0=2, J=%d, "
                        "complex64 grids streamed one scale at a time, FP32 MFMA contractions, "
                        "FP64 Delta and final accumulation" % (n_sources, L, api.num_scales(L)),
            "value": 1e3 / ms, "unit": "transforms/s", "ms_per_step": ms, "steps": steps,
            "warmup": 1, "round_trip_rel_l2": err, "setup_s": setup_s}


def precision_leg(prec, steps=2, L=512, batch=16):
    """The precision workload: a batch of 16 real maps at L = 512 (Gaussian
    fields, seeds 0..15) through one batched analysis and synthesis with the
    l-contraction and beta GEMMs in FP32 or split BF16 on the matrix cores
    (complex64 grids; Delta and the final accumulation in FP64).  One warm-up
    round trip, then `steps` timed ones; the error of map 0's grids against
    the FP64 path, relative L2 and max-abs relative."""
    import torch
    from paper_1511_05578_amd import api, inputs
    lam, J0 = 2.0, 2
    ctx = api.Context(L, 0)
    try:
        ctx.prepare(L, lam, J0)
        maps = torch.stack([ctx.sht_inverse(torch.from_numpy(inputs.gaussian_real_flm(L, seed=s))
                                            .cuda(), L) for s in range(batch)]).contiguous()
        scal, grids = ctx.alloc_outputs(L, lam, J0, batch, precision=prec)
        rec = torch.empty_like(maps)

        def step():
            ctx.curvelet_analysis(maps, lam, J0, out=(scal, grids), precision=prec)
            ctx.curvelet_synthesis(scal, grids, L, lam, J0, out=rec, precision=prec)

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        err = (torch.linalg.norm(rec - maps) / torch.linalg.norm(maps)).item()
        _, g64 = ctx.curvelet_analysis(maps[:1], lam, J0, precision="fp64")
        num = den = mx = mref = 0.0
        for a, b in zip(grids[0], g64[0]):
            for i0 in range(0, a.shape[0], 64):  # in slabs: bounded temporaries
                d = a[i0:i0 + 64].to(b.dtype) - b[i0:i0 + 64]
                num += torch.linalg.norm(d).item() ** 2
                den += torch.linalg.norm(b[i0:i0 + 64]).item() ** 2
                mx = max(mx, d.abs().max().item())
                mref = max(mref, b[i0:i0 + 64].abs().max().item())
                del d
            del a, b
        del g64, grids, scal, rec, maps, step
    finally:
        torch.cuda.synchronize()
        ctx.close()
        torch.cuda.empty_cache()
    return {"workload": "batch of %d real spin-0 maps, L=%d, lambda=2, J0=2, J=%d, complex64 grids, "
                        "%s MFMA contractions and beta GEMMs, FP64 Delta and final accumulation"
                        % (batch, L, api.num_scales(L), {"fp32": "FP32", "bf16x3": "split-BF16"}[prec]),
            "value": batch * 1e3 / ms, "unit": "maps/s", "ms_per_batch": ms, "steps": steps,
            "warmup": 1, "round_trip_rel_l2": err,
            "vs_fp64_path": {"grids_rel_l2": math.sqrt(num / den), "grids_max_abs_rel": mx / mref}}


def serving_leg(n=128, rho=0.7, bandlimits=(64, 128, 256, 512), slots=4):
    """The serving workload on a short trace: closed-loop capacity of the
    continuous-batching server (4 stream slots, same-L batching, HBM admission)
    and of the plain path (one request at a time, one slot, no batching), then
    `n` requests with Poisson arrivals (seed 1) at `rho` x the server's
    capacity and band-limits uniform over `bandlimits` (seed 2), served by both:
    throughput and p50 / p99 latency."""
    import torch
    from paper_1511_05578_amd import inputs, serving
    out = {"requests": n, "load": rho, "bandlimits": list(bandlimits)}
    _, Ls_cap = inputs.serving_trace(64, tuple(bandlimits), 1.0, seed_arrivals=1, seed_sizes=2)
    res = {}
    for name, nslots, mb in (("served", slots, 4), ("plain", 1, 1)):
        srv = serving.CurveletServer(L_max=max(bandlimits), slots=nslots, max_batch=mb)
        try:
            srv.prepare(bandlimits)
            cap = serving.measure_capacity(srv, Ls_cap, n=64)  # the same 64 requests for both
            res[name] = {"capacity_req_per_s": cap, "slots": nslots, "max_batch": mb}
            if name == "served":
                rate = rho * cap
            arr, Ls = inputs.serving_trace(n, tuple(bandlimits), rate, seed_arrivals=1,
                                           seed_sizes=2)
            reqs = serving.make_requests(srv, n, Ls, arr)
            t0 = time.perf_counter()
            done = srv.run(reqs)
            wall = time.perf_counter() - t0
            st = serving.latency_stats(done)
            st["served_req_per_s"] = len(done) / wall
            res[name].update(st)
            del reqs, done
        finally:
            srv.close()
            torch.cuda.empty_cache()
    out["offered_req_per_s"] = rate
    out.update(res)
    return out


def cpu_model():
    """Model name of the host CPU (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(L, lam=2.0, J0=2, unrot=False):
    """Oracle round-trip time at this workload, from a bounded sample: one beta
    row per scale of the analysis and one Gauss-Legendre node per scale of the
    synthesis (plus that scale's full alpha/gamma Fourier step), scaled by the
    rows / nodes each scale has.  Also returns the sampled oracle rows
    {scale index: (row b, grid[:, b, :])} of the seed-0 map."""
    import numpy as np
    from oracle import curvelet as ocurv
    from oracle import sht as osht
    from paper_1511_05578_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    try:  # the BLAS pool the oracle's matrix products actually use
        import threadpoolctl
        np.ones((64, 64)) @ np.ones((64, 64))
        pools = [p["num_threads"] for p in threadpoolctl.threadpool_info()
                 if p.get("user_api") == "blas"]
        if pools:
            threads = max(pools)
    except ImportError:
        pass
    plan = ocurv.Plan(L, lam, J0, rotated=not unrot)
    f = inputs.gaussian_real_flm(L, seed=0)
    t_an = 0.0
    t_sy = 0.0
    t0 = time.perf_counter()
    rows = {}
    for s, j in enumerate(plan.scales):
        Lj = plan.Lj[j]
        a = time.perf_counter()
        row = ocurv.analysis_scale(plan, f, j, rows=[Lj // 2])
        rows[s] = (Lj // 2, row)
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
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": "L=%d: 1 beta row per scale of the analysis and 1 Gauss-Legendre node per "
                      "scale of the synthesis (with its full alpha/gamma step), extrapolated by "
                      "rows/nodes per scale, plus one SHT pair; %.1f s sampled, estimated %.1f s "
                      "per round trip" % (L, wall, t_total)}, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--point-sources", type=int, default=0,
                    help="add this many point sources to each map (projected onto band-limit L)")
    ap.add_argument("--stream", action="store_true",
                    help="one scale at a time through the streaming interface (batch 1)")
    ap.add_argument("--real-grids", action="store_true",
                    help="real (float64 / float32) grids instead of complex ones")
    ap.add_argument("--unrotated", action="store_true",
                    help="coefficients of the unrotated curvelets (|n| = l Wigner path)")
    ap.add_argument("--graph", action="store_true",
                    help="also capture one step in a HIP graph and report its replay time "
                         "(graph_replay_ms_per_step; not the headline value)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the secondary workloads (L=1024 streamed FP32, L=512 batch 16 FP32 and "
                         "BF16x3, serving trace)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="after timing, copy BYTES of device memory once (a plain copy kernel "
                         "of known size, for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1511_05578_amd import api, inputs

    L, lam, J0, NB, prec = args.L, 2.0, 2, args.batch, args.precision
    EB = 16.0 if prec == "fp64" else 8.0  # complex element of the intermediates
    RG = args.real_grids
    UR = args.unrotated
    GB = EB / 2 if RG else EB  # grid element
    ctx = api.Context(L, 0)
    ctx.prepare(L, lam, J0)
    if args.stream and NB != 1:
        print("--stream runs one map per step (--batch 1)", file=sys.stderr)
        sys.exit(2)

    def make_map(s):
        f = inputs.gaussian_real_flm(L, seed=s)
        if args.point_sources:
            th, ph, a = inputs.point_sources(args.point_sources, seed=100 + s)
            f = f + point_source_flm(L, th, ph, inputs.source_amplitudes(a, f, L))
        return ctx.sht_inverse(torch.from_numpy(f).cuda(), L)

    maps = torch.stack([make_map(s) for s in range(NB)]).contiguous()
    rec = torch.empty((NB, L, 2 * L - 1), dtype=torch.float64, device="cuda")
    if args.stream:
        grids = None

        def step():
            r, _ = ctx.round_trip_streamed(maps[0], lam, J0, precision=prec, real_grids=RG,
                                           unrotated=UR)
            rec[0].copy_(r)
    else:
        scal, grids = ctx.alloc_outputs(L, lam, J0, NB, precision=prec, real_grids=RG)

        def step():
            ctx.curvelet_analysis(maps, lam, J0, out=(scal, grids), precision=prec, real_grids=RG,
                                  unrotated=UR)
            ctx.curvelet_synthesis(scal, grids, L, lam, J0, out=rec, precision=prec,
                                   real_grids=RG, unrotated=UR)

    models = stage_models(L, lam, J0, EB, GB, UR)
    # Warm-up: every launch timed (per-stage breakdown, dominant kernel);
    # the first step, which may still build plans, is left out.
    if args.warmup > 0:
        step()
    ctx.profile_enable(True)
    for _ in range(args.warmup - 1):
        step()
    torch.cuda.synchronize()
    nprof = max(args.warmup - 1, 0)
    prof = ctx.profile_read()
    detail = ctx.profile_read_detail()
    err = (torch.linalg.norm(rec - maps) / torch.linalg.norm(maps)).item()
    print("warm-up done, round trip rel L2 %.3e" % err, file=sys.stderr, flush=True)
    top = None
    if nprof:
        # dominant kernel: the (stage, L_j) pair with the most device time
        top = max((k for k in detail if k in models), key=lambda k: detail[k][1])

    # Timed region: only the dominant kernel's launches carry timing events
    # (with none known, every launch does).
    ctx.profile_enable(True)
    if top is not None:
        ctx.profile_filter(top[0], top[1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tdetail = ctx.profile_read_detail()
    ctx.profile_filter(None)
    ctx.profile_enable(False)
    if top is None:
        prof, nprof = ctx.profile_read(), args.steps
        detail = tdetail
        top = max((k for k in detail if k in models), key=lambda k: detail[k][1])
    print("timed %d steps" % args.steps, file=sys.stderr, flush=True)

    graph_ms = None
    if args.graph and not args.stream:
        # one step captured (timing events off) and replayed K times
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            step()
        gr.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            gr.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        del gr

    vs64 = None
    if prec != "fp64" and grids is not None:
        # the first map's grids against the FP64 path's
        s64, g64 = ctx.curvelet_analysis(maps[:1], lam, J0, precision="fp64", real_grids=RG,
                                         unrotated=UR)
        num = den = 0.0
        mx = mref = 0.0
        for a, b in zip(grids[0], g64[0]):
            for i0 in range(0, a.shape[0], 64):  # in slabs: bounded temporaries
                d = a[i0:i0 + 64].to(b.dtype) - b[i0:i0 + 64]
                num += torch.linalg.norm(d).item() ** 2
                den += torch.linalg.norm(b[i0:i0 + 64]).item() ** 2
                mx = max(mx, d.abs().max().item())
                mref = max(mref, b[i0:i0 + 64].abs().max().item())
                del d
        vs64 = {"grids_rel_l2": math.sqrt(num / den), "grids_max_abs_rel": mx / mref}
        del s64, g64

    ms = dt * 1e3 / args.steps
    stages = {k: {"launches": v[0] / nprof, "ms_per_step": v[1] / nprof}
              for k, v in prof.items() if v[0]}
    n_launch, t_ms = tdetail[top]
    t_top = t_ms * 1e-3 / n_launch  # s per launch
    nb, nf, nscales = models[top]
    bytes_per_launch = nb / nscales  # one launch per scale per map
    flops_per_launch = nf / nscales
    peak_tf = stage_peak(top[0], prec)
    roof = rule_roofline(top[0], top[1], GB, flops_per_launch, t_top, peak_tf)
    # the same launch priced by its whole stage IO (input plane read once and
    # output written once), which the measurement rule does not count
    roof["stage_io"] = {"bytes": bytes_per_launch,
                        "achieved_GBs": bytes_per_launch / t_top / 1e9,
                        "frac_hbm": bytes_per_launch / t_top / 1e9 / HBM_PEAK_GBS}
    wkey = "L%d_b%d_%s%s%s%s%s" % (L, NB, prec, "_stream" if args.stream else "",
                                   "_ps%d" % args.point_sources if args.point_sources else "",
                                   "_rg" if RG else "", "_unrot" if UR else "")
    sym = kernel_symbol(top[0], top[1], prec, RG, UR)
    roof["traffic"] = recorded_traffic(wkey, sym, finest=top[1] == L)
    roof["kernel"] = sym
    roof["stage"] = top[0]
    roof["L_j"] = top[1]
    roof["launch_ms"] = t_top * 1e3
    roof["algorithmic_per_launch"] = {"bytes": bytes_per_launch, "flops": flops_per_launch}
    roof["copy_ceiling"] = copy_ceiling(bytes_per_launch / t_top / 1e9)
    if args.copy_calibration:
        x = torch.ones(args.copy_calibration // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    gname = ("float64" if prec == "fp64" else "float32") if RG else \
        ("complex128" if prec == "fp64" else "complex64")
    work = ("%d real spin-0 map%s%s, L=%d, lambda=2, J0=2, J=%d, N_j=L_j, %s%s grids%s, %s, "
            "analysis+synthesis round trip" % (
                NB, "" if NB == 1 else "s",
                " with %d point sources" % args.point_sources if args.point_sources else "",
                L, api.num_scales(L), "unrotated-curvelet " if UR else "", gname,
                " streamed one scale at a time" if args.stream else "",
                {"fp64": "FP64 throughout",
                 "fp32": "FP32 MFMA contractions, FP32 FFT/beta",
                 "bf16x3": "split-BF16 MFMA contractions, FP32 FFT/beta"}[prec]))
    out = {
        "metric": METRIC,
        "value": NB * 1e3 / ms,
        "unit": "transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[prec],
        "data": "synthetic: f_lm ~ N(0,(l+1)^-2) real-map coefficients, seeds 0..%d" % (NB - 1),
        "config": {"workload": work, "L": L, "lambda": lam, "J0": J0, "batch": NB,
                   "precision": prec, "stream": bool(args.stream), "unrotated": bool(UR),
                   "point_sources": args.point_sources, "grid_bytes": NB * grid_bytes(L, lam, J0, GB)},
        "round_trip_rel_l2": err,
        "source": source_fingerprint(),
        "hbm_roofline_ms": 2 * NB * grid_bytes(L, lam, J0, GB) / (HBM_PEAK_GBS * 1e9) * 1e3,
        "whole_roofline": whole_roofline(L, lam, J0, prec, NB, GB, ms, UR),
        "roofline": roof,
        "stages": stages,
        "stages_by_bandlimit": {"%s@%d" % k: round(v[1] / nprof, 4) for k, v in sorted(detail.items())},
    }
    if vs64 is not None:
        out["vs_fp64_path"] = vs64
    if graph_ms is not None:
        out["graph_replay_ms_per_step"] = graph_ms
    if not args.no_cpu:
        out["cpu_baseline"], orows = cpu_baseline(L, lam, J0, UR)
        if grids is not None and not args.point_sources:
            # the first map (seed 0) against the oracle's sampled beta rows
            import numpy as np
            num = den = mx = mref = 0.0
            for s_, (b, row) in orows.items():
                g = grids[0][s_][:, b:b + 1, :].cpu().numpy().astype(np.complex128)
                d = g - row
                num += float(np.sum(np.abs(d) ** 2))
                den += float(np.sum(np.abs(row) ** 2))
                mx = max(mx, float(np.abs(d).max()))
                mref = max(mref, float(np.abs(row).max()))
            out["vs_oracle_sampled"] = {"grids_rel_l2": math.sqrt(num / den),
                                        "grids_max_abs_rel": mx / mref,
                                        "rows": "beta row L_j/2 of every scale, map 0"}
    ctx.close()
    del grids
    torch.cuda.empty_cache()
    if not args.no_legs and args.L == 256 and NB == 1 and prec == "fp64" and not UR \
            and not args.stream:
        # the other configurations of the metric, measured in the same run
        print("large workload (L=1024 streamed FP32)", file=sys.stderr, flush=True)
        out["large"] = large_leg()
        print("serving trace", file=sys.stderr, flush=True)
        out["serving"] = serving_leg()
        print("precision workloads (L=512, 16 maps)", file=sys.stderr, flush=True)
        out["precision"] = {p: precision_leg(p) for p in ("fp32", "bf16x3")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
