// Odd-length McEwen-Wiaux DFTs (lengths 2L-1) as Bluestein chirp-z transforms
// over power-of-two Stockham FFTs held in LDS.
//
// Every MW DFT is out[k] = scale * sum_j in[j] exp(sigma 2 pi i j k / Nd) for a
// window of inputs j in [j0, j0+Kin) and outputs k in [k0, k0+Kout).  With
// jk = (j^2 + k^2 - (k-j)^2)/2 this is a chirp pre-multiply, a linear
// convolution with a chirp (a circular one of power-of-two length P >=
// Kin+Kout-1, its spectrum precomputed on the host with the 1/P and `scale`
// folded in), and a chirp post-multiply.  The inverse FFT is the forward one
// between two conjugations.
//
// A work-group of 256 threads transforms LINES lines; each line lives in its
// own P-element LDS slice and is worked on by 256/LINES threads.  The stage
// IO policies below gather / scatter each stage's lines with the symmetries
// the stage uses (reality of the map, evenness of n, parity in beta).
#include "cvl_device.h"

namespace cvl {

// In-place Stockham FFT of one LDS line (forward, tw[x] = e^{-2 pi i x / P}).
// Radix-4 stages first, then one radix-2 stage when log2 P is odd.  Every
// thread of the work-group must call it (it synchronises the work-group).
template <int P, int TPL>
__device__ __forceinline__ void fft_lds(cd *buf, const cd *__restrict__ tw, int lane) {
    constexpr int Q = P / 4;
    constexpr int B4 = (Q + TPL - 1) / TPL;
    int Ns = 1;
    for (; Ns * 4 <= P; Ns *= 4) {
        cd v[B4][4];
        const int step = P / (4 * Ns);
#pragma unroll
        for (int i = 0; i < B4; ++i) {
            const int j = lane + i * TPL;
            if (j < Q) {
                const int k = j & (Ns - 1);
                v[i][0] = buf[j];
                v[i][1] = cmul(buf[j + Q], tw[k * step]);
                v[i][2] = cmul(buf[j + 2 * Q], tw[2 * k * step]);
                v[i][3] = cmul(buf[j + 3 * Q], tw[3 * k * step]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < B4; ++i) {
            const int j = lane + i * TPL;
            if (j < Q) {
                const int k = j & (Ns - 1);
                const cd a0 = cadd(v[i][0], v[i][2]), a1 = csub(v[i][0], v[i][2]);
                const cd b0 = cadd(v[i][1], v[i][3]), b1 = csub(v[i][1], v[i][3]);
                const cd mib1 = cd{b1.y, -b1.x};  // -i * b1
                const int d = (j / Ns) * Ns * 4 + k;
                buf[d] = cadd(a0, b0);
                buf[d + Ns] = cadd(a1, mib1);
                buf[d + 2 * Ns] = csub(a0, b0);
                buf[d + 3 * Ns] = csub(a1, mib1);
            }
        }
        __syncthreads();
    }
    if (Ns < P) {  // radix-2, Ns = P/2
        constexpr int H = P / 2;
        constexpr int B2 = (H + TPL - 1) / TPL;
        cd v[B2][2];
#pragma unroll
        for (int i = 0; i < B2; ++i) {
            const int j = lane + i * TPL;
            if (j < H) {
                v[i][0] = buf[j];
                v[i][1] = cmul(buf[j + H], tw[j]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < B2; ++i) {
            const int j = lane + i * TPL;
            if (j < H) {
                buf[j] = cadd(v[i][0], v[i][1]);
                buf[j + H] = csub(v[i][0], v[i][1]);
            }
        }
        __syncthreads();
    }
}

template <int P>
struct LinesFor {
    static constexpr int v = (4096 / P) > 64 ? 64 : (4096 / P) < 1 ? 1 : (4096 / P);
};

template <int P, int LINES, bool IN_IL, bool OUT_IL, class IO>
__global__ __launch_bounds__(256) void k_bluestein(IO io, int nlines, BluesteinDev B) {
    extern __shared__ cd smem[];
    constexpr int TPL = 256 / LINES;
    const int tid = threadIdx.x;
    const int li = tid / TPL, lane = tid % TPL;
    const int line0 = blockIdx.x * LINES;
    for (int idx = tid; idx < LINES * P; idx += 256) {
        int l, t;
        if (IN_IL) {
            l = idx % LINES;
            t = idx / LINES;
        } else {
            l = idx / P;
            t = idx % P;
        }
        const int line = line0 + l;
        cd v = cd{0.0, 0.0};
        if (t < B.Kin && line < nlines) v = cmul(io.load(line, B.j0 + t), B.pre[t]);
        smem[l * P + t] = v;
    }
    __syncthreads();
    cd *buf = smem + li * P;
    fft_lds<P, TPL>(buf, B.tw, lane);
    for (int t = lane; t < P; t += TPL) buf[t] = cconj(cmul(buf[t], B.vhat[t]));
    __syncthreads();
    fft_lds<P, TPL>(buf, B.tw, lane);
    for (int idx = tid; idx < LINES * B.Kout; idx += 256) {
        int l, t;
        if (OUT_IL) {
            l = idx % LINES;
            t = idx / LINES;
        } else {
            l = idx / B.Kout;
            t = idx % B.Kout;
        }
        const int line = line0 + l;
        if (line < nlines) {
            const cd c = cconj(smem[l * P + t + B.Kin - 1]);
            io.store(line, B.k0 + t, cmul(c, B.post[t]));
        }
    }
}

template <bool IN_IL, bool OUT_IL, class IO>
static hipError_t run_bluestein(const IO &io, int nlines, const BluesteinDev &B,
                                hipStream_t st) {
    if (nlines <= 0) return hipSuccess;
#define CVL_BLUE_CASE(PP)                                                              \
    case PP: {                                                                          \
        constexpr int LN = LinesFor<PP>::v;                                             \
        const int grid = (nlines + LN - 1) / LN;                                        \
        hipLaunchKernelGGL((k_bluestein<PP, LN, IN_IL, OUT_IL, IO>), dim3(grid),        \
                           dim3(256), LN * PP * sizeof(cd), st, io, nlines, B);         \
        return hipGetLastError();                                                       \
    }
    switch (B.P) {
        CVL_BLUE_CASE(8)
        CVL_BLUE_CASE(16)
        CVL_BLUE_CASE(32)
        CVL_BLUE_CASE(64)
        CVL_BLUE_CASE(128)
        CVL_BLUE_CASE(256)
        CVL_BLUE_CASE(512)
        CVL_BLUE_CASE(1024)
        CVL_BLUE_CASE(2048)
        CVL_BLUE_CASE(4096)
        default:
            return hipErrorInvalidValue;
    }
#undef CVL_BLUE_CASE
}

// ---------------------------------------------------------------------------
// Curvelet (real map, even n) stage IO.
// Cube / plane layouts: X, W1, V2, Z: [r][m][nn] with m in [0, L), nn = n/2 + h,
// row length Nep.  W2: [b][a][k], k = n/2 in [0, h].  V1: [b][a][nn].
// ---------------------------------------------------------------------------

// alpha DFT of the analysis: line (b, k >= 0); input over m in (-L, L) with the
// reality condition W1(b, -m, -n) = conj W1(b, m, n); output a in [0, 2L-1).
struct InvAlphaIO {
    const cd *W1;
    cd *W2;
    int L, h, Nep, Nm;
    __device__ cd load(int line, int m) const {
        const int b = line / (h + 1), k = line % (h + 1);
        if (m >= 0) return W1[((size_t)b * L + m) * Nep + h + k];
        return cconj(W1[((size_t)b * L - m) * Nep + h - k]);
    }
    __device__ void store(int line, int a, cd v) const {
        const int b = line / (h + 1), k = line % (h + 1);
        W2[((size_t)b * Nm + a) * (h + 1) + k] = v;
    }
};

// gamma DFT of the analysis: line (a, b); input over n in (-L, L): even n from
// W2 (n < 0 by conjugation), odd n zero; output g, written as (re, 0).
struct InvGammaIO {
    const cd *W2;
    cd *grid;
    int L, h, Nm;
    __device__ cd load(int line, int n) const {
        if (n & 1) return cd{0.0, 0.0};
        const int a = line / L, b = line % L;
        const int k = n >= 0 ? n / 2 : -n / 2;
        const cd v = W2[((size_t)b * Nm + a) * (h + 1) + k];
        return n >= 0 ? v : cconj(v);
    }
    __device__ void store(int line, int g, cd v) const {
        grid[(size_t)line * Nm + g] = cd{v.x, 0.0};
    }
};

// gamma DFT of the synthesis: line (a, b) of the complex grid; even n kept.
struct FwdGammaIO {
    const cd *grid;
    cd *V1;
    int L, h, Nm, Nep;
    __device__ cd load(int line, int g) const { return grid[(size_t)line * Nm + g]; }
    __device__ void store(int line, int n, cd v) const {
        if (n & 1) return;
        const int a = line / L, b = line % L;
        V1[((size_t)b * Nm + a) * Nep + (n / 2 + h)] = v;
    }
};

// alpha DFT of the synthesis: line (b, nn); outputs m in [0, L).
struct FwdAlphaIO {
    const cd *V1;
    cd *V2;
    int L, Ne, Nm, Nep;
    __device__ cd load(int line, int a) const {
        const int b = line / Ne, nn = line % Ne;
        return V1[((size_t)b * Nm + a) * Nep + nn];
    }
    __device__ void store(int line, int m, cd v) const {
        const int b = line / Ne, nn = line % Ne;
        V2[((size_t)b * L + m) * Nep + nn] = v;
    }
};

struct ShtInvPhiIO {
    const cd *G;
    double *map;
    int L, Nm;
    __device__ cd load(int t, int m) const {
        return m >= 0 ? G[(size_t)t * L + m] : cconj(G[(size_t)t * L - m]);
    }
    __device__ void store(int t, int p, cd v) const { map[(size_t)t * Nm + p] = v.x; }
};

struct ShtFwdPhiIO {
    const double *map;
    cd *F1;
    int L, Nm;
    __device__ cd load(int t, int p) const { return cd{map[(size_t)t * Nm + p], 0.0}; }
    __device__ void store(int t, int m, cd v) const { F1[(size_t)t * L + m] = v; }
};

hipError_t launch_inv_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *W1,
                            cd *W2, hipStream_t st) {
    InvAlphaIO io{W1, W2, g.L, g.h, g.Nep, g.Nm};
    return run_bluestein<true, true>(io, g.L * (g.h + 1), B, st);
}
hipError_t launch_inv_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *W2,
                            cd *grid, hipStream_t st) {
    InvGammaIO io{W2, grid, g.L, g.h, g.Nm};
    return run_bluestein<false, false>(io, g.Nm * g.L, B, st);
}
hipError_t launch_fwd_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *grid,
                            cd *V1, hipStream_t st) {
    FwdGammaIO io{grid, V1, g.L, g.h, g.Nm, g.Nep};
    return run_bluestein<false, false>(io, g.Nm * g.L, B, st);
}
hipError_t launch_fwd_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *V1,
                            cd *V2, hipStream_t st) {
    FwdAlphaIO io{V1, V2, g.L, g.Ne, g.Nm, g.Nep};
    return run_bluestein<true, true>(io, g.L * g.Ne, B, st);
}
hipError_t launch_sht_inv_phi(int L, const BluesteinDev &B, const cd *G, double *map,
                              hipStream_t st) {
    ShtInvPhiIO io{G, map, L, 2 * L - 1};
    return run_bluestein<false, false>(io, L, B, st);
}
hipError_t launch_sht_fwd_phi(int L, const BluesteinDev &B, const double *map, cd *F1,
                              hipStream_t st) {
    ShtFwdPhiIO io{map, F1, L, 2 * L - 1};
    return run_bluestein<false, false>(io, L, B, st);
}

// ---------------------------------------------------------------------------
// General complex Wigner transforms: all m in (-L, L), all n in (-N, N).
// Cube / plane layouts: [r][m + L - 1][n + N - 1] with row length Nnp.
// ---------------------------------------------------------------------------
static inline int nnp_of(int N) { return ((2 * N - 1) + 31) / 32 * 32; }

struct GenInvAlphaIO {  // line (b, n); in m; out a
    const cd *W1;
    cd *W2;
    int L, Nn, Nnp, Nm;
    __device__ cd load(int line, int m) const {
        const int b = line / Nn, n = line % Nn;
        return W1[((size_t)b * Nm + (m + L - 1)) * Nnp + n];
    }
    __device__ void store(int line, int a, cd v) const {
        const int b = line / Nn, n = line % Nn;
        W2[((size_t)b * Nm + a) * Nnp + n] = v;
    }
};
struct GenInvGammaIO {  // line (a, b); in n; out g
    const cd *W2;
    cd *grid;
    int L, N, Nnp, Nm, Ng;
    __device__ cd load(int line, int n) const {
        const int a = line / L, b = line % L;
        return W2[((size_t)b * Nm + a) * Nnp + (n + N - 1)];
    }
    __device__ void store(int line, int g, cd v) const { grid[(size_t)line * Ng + g] = v; }
};
struct GenFwdGammaIO {  // line (a, b); in g; out n
    const cd *grid;
    cd *V1;
    int L, N, Nnp, Nm, Ng;
    __device__ cd load(int line, int g) const { return grid[(size_t)line * Ng + g]; }
    __device__ void store(int line, int n, cd v) const {
        const int a = line / L, b = line % L;
        V1[((size_t)b * Nm + a) * Nnp + (n + N - 1)] = v;
    }
};
struct GenFwdAlphaIO {  // line (b, n); in a; out m
    const cd *V1;
    cd *V2;
    int L, Nn, Nnp, Nm;
    __device__ cd load(int line, int a) const {
        const int b = line / Nn, n = line % Nn;
        return V1[((size_t)b * Nm + a) * Nnp + n];
    }
    __device__ void store(int line, int m, cd v) const {
        const int b = line / Nn, n = line % Nn;
        V2[((size_t)b * Nm + (m + L - 1)) * Nnp + n] = v;
    }
};

hipError_t launch_gen_inv_alpha(int L, int N, const BluesteinDev &B, const cd *W1,
                                cd *W2, hipStream_t st) {
    GenInvAlphaIO io{W1, W2, L, 2 * N - 1, nnp_of(N), 2 * L - 1};
    return run_bluestein<true, true>(io, L * (2 * N - 1), B, st);
}
hipError_t launch_gen_inv_gamma(int L, int N, const BluesteinDev &B, const cd *W2,
                                cd *grid, hipStream_t st) {
    GenInvGammaIO io{W2, grid, L, N, nnp_of(N), 2 * L - 1, 2 * N - 1};
    return run_bluestein<false, false>(io, (2 * L - 1) * L, B, st);
}
hipError_t launch_gen_fwd_gamma(int L, int N, const BluesteinDev &B, const cd *grid,
                                cd *V1, hipStream_t st) {
    GenFwdGammaIO io{grid, V1, L, N, nnp_of(N), 2 * L - 1, 2 * N - 1};
    return run_bluestein<false, false>(io, (2 * L - 1) * L, B, st);
}
hipError_t launch_gen_fwd_alpha(int L, int N, const BluesteinDev &B, const cd *V1,
                                cd *V2, hipStream_t st) {
    GenFwdAlphaIO io{V1, V2, L, 2 * N - 1, nnp_of(N), 2 * L - 1};
    return run_bluestein<true, true>(io, L * (2 * N - 1), B, st);
}

}  // namespace cvl
