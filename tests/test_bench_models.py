"""Host logic of the benchmark: work models of the unrotated path and kernel
names, against brute-force enumeration of the unrotated cube."""
import math

import numpy as np
import pytest

import bench


def _cube_entries(Lj):
    """(m', m, n) of the unrotated cube that can be non-zero: m, m' >= 0,
    |n| < L_j, max(m, m') <= l = |n| (the kernel is non-zero only at |n| = l)."""
    return [(mp, m, n) for n in range(-(Lj - 1), Lj) for m in range(Lj) for mp in range(Lj)
            if max(m, mp) <= abs(n)]


def _live_lines_brute(Lj):
    # line pair (m, column c): rows (m, s = 0, 1); row (m, s) holds the n of
    # parity (m + s) mod 2 in increasing order, so column c holds the c-th such n
    count = 0
    for m in range(Lj):
        cols = {}
        for s in (0, 1):
            ns = [n for n in range(-(Lj - 1), Lj) if (n - m - s) % 2 == 0]
            for c, n in enumerate(ns):
                cols.setdefault(c, []).append(n)
        count += sum(1 for ns in cols.values() if any(m <= abs(n) for n in ns))
    return count


@pytest.mark.parametrize("Lj", [2, 3, 8, 9, 16, 33])
def test_unrot_live_lines_match_brute_force(Lj):
    assert bench._unrot_live_lines(Lj) == _live_lines_brute(Lj)


def test_unrot_models_count_the_needed_work():
    L = 16
    B = 16.0
    m = bench.stage_models(L, 2.0, 2, B, unrot=True)
    terms = {}  # scales of equal L_j share a model entry (summed)
    for g in bench.scale_geoms(L, 2.0, 2):
        ent = _cube_entries(g["L"])
        terms[g["L"]] = terms.get(g["L"], 0) + len(
            [e for e in ent if g["llo"] <= abs(e[2]) <= g["lhi"]])
    for Lj, t in terms.items():
        ent = _cube_entries(Lj)
        nnz = len(ent)
        cols = len({(mm, n) for _, mm, n in ent})  # columns with m <= |n|
        nb, nf, n_launch = m[("contract_fwd", Lj)]
        assert nf == pytest.approx(4.0 * t)
        nb, nf, _ = m[("beta_gemm_fwd", Lj)]
        per = nb / n_launch
        assert per == pytest.approx(Lj * cols * B + nnz * B)
        assert nf / n_launch == pytest.approx(4.0 * Lj * nnz)


def test_whole_roofline_bytes_do_not_depend_on_rotation():
    a = bench.whole_roofline(64, 2.0, 2, "fp64", 1, 16.0, 1.0)
    b = bench.whole_roofline(64, 2.0, 2, "fp64", 1, 16.0, 1.0, True)
    assert a["bytes"] == b["bytes"] and a["dft_flops"] == b["dft_flops"]
    assert b["contraction_flops"] < a["contraction_flops"]


def test_kernel_symbols():
    assert bench.kernel_symbol("contract_inv", 256, "fp64", unrot=True) == "k_unrot_contract_inv<cd>"
    assert bench.kernel_symbol("contract_fwd", 512, "fp32", unrot=True) == "k_unrot_contract_fwd<cf>"
    assert bench.kernel_symbol("contract_inv", 256, "fp64") == "k_contract_inv_mfma"
    assert bench.kernel_symbol("alpha_dft_inv", 256, "fp64", unrot=True) == \
        "k_blue_r16<1024, UnrotInvAlphaIO<cd> >"
    assert bench.kernel_symbol("gamma_dft_fwd", 256, "fp64", True, True) == \
        "k_blue_r16<1024, UnrotFwdGammaPackIO<cd, double> >"
    assert bench.kernel_symbol("beta_gemm_fwd", 256, "fp32") == "k_beta_mfma_mx<1, true>"
    assert bench.kernel_symbol("beta_gemm_inv", 13, "bf16x3") == "k_beta_mfma_mx<2, false>"
    assert bench.kernel_symbol("gamma_dft_fwd", 512, "fp32") == \
        "k_blue_r16<2048, FwdGammaPackOddIO<cf, cf> >"
    assert bench.kernel_symbol("gamma_dft_fwd", 512, "fp64") == \
        "k_blue_r16<2048, FwdGammaPackOddIO<cd, cd> >"
    assert bench.kernel_symbol("gamma_dft_fwd", 515, "fp64") == \
        "k_blue_r16<4096, FwdGammaPackIO<cd, cd> >"
    assert bench.bluestein_size(256) == 1024 and bench.bluestein_size(1024) == 4096
    assert math.isclose(bench.stage_peak("contract_inv", "bf16x3"), bench.BF16_MFMA_PEAK_TFLOPS)


def test_bench_point_sources_match_library_ylm():
    # the benchmark's own Legendre recurrence for its large workload's input
    import scipy.special as sps
    L = 20
    th = np.array([0.05, 1.3, 3.1])
    ph = np.array([0.2, 3.3, 6.0])
    amp = np.array([2.0, 1.0, 0.5])
    f = bench.point_source_flm(L, th, ph, amp)
    for l in range(L):
        for m in range(-l, l + 1):
            ref = np.sum(amp * np.conj(sps.sph_harm_y(l, m, th, ph)))
            assert abs(f[l * l + l + m] - ref) < 1e-13
