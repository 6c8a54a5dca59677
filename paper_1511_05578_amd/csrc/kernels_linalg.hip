// Dense kernels of the curvelet transform on gfx950, all FP64:
//  * Delta = d(pi/2) quarter table by the Trapani-Navaza recursion;
//  * the parity-folded beta stage as a real-matrix x complex-data GEMM;
//  * the l-contraction of the analysis (harmonic product f_lm Psi_ln folded
//    into the Fourier-cube sum over l) and the Delta-projection + Psi
//    contraction of the synthesis;
//  * dense Wigner contractions for general F^l_mn;
//  * small SHT helpers.
#include "cvl_device.h"

namespace cvl {

// ---------------------------------------------------------------------------
// Delta table: tab[off(l) + r*(l+1) + c] = Delta^l_{r,c}, 0 <= r, c <= l.
// Top rows (r = l) from the previous l:
//   Delta^l_{l,0} = -sqrt((2l-1)/(2l)) Delta^{l-1}_{l-1,0}
//   Delta^l_{l,c} = sqrt(l(2l-1)/(2(l+c)(l+c-1))) Delta^{l-1}_{l-1,c-1}
// then every column downwards (r = l-1 .. 0):
//   Delta^l_{r,c} = 2c/sqrt((l-r)(l+r+1)) Delta^l_{r+1,c}
//                   - sqrt((l-r-1)(l+r+2)/((l-r)(l+r+1))) Delta^l_{r+2,c}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_delta_toprows(double *tab, int Lmax) {
    const int tid = threadIdx.x;
    if (tid == 0) tab[0] = 1.0;
    __syncthreads();
    for (int l = 1; l < Lmax; ++l) {
        const double *prev = tab + delta_off(l - 1) + (int64_t)(l - 1) * l;
        double *row = tab + delta_off(l) + (int64_t)l * (l + 1);
        for (int c = tid; c <= l; c += blockDim.x) {
            double v;
            if (c == 0)
                v = -sqrt((2.0 * l - 1.0) / (2.0 * l)) * prev[0];
            else
                v = sqrt((double)l * (2.0 * l - 1.0) /
                         (2.0 * (double)(l + c) * (double)(l + c - 1))) * prev[c - 1];
            row[c] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_delta_fill(double *tab, int Lmax) {
    const int l = blockIdx.x;
    if (l == 0) return;
    double *blk = tab + delta_off(l);
    const int w = l + 1;
    for (int c = threadIdx.x; c <= l; c += blockDim.x) {
        double d2 = 0.0;                      // Delta_{r+2, c}
        double d1 = blk[(int64_t)l * w + c];  // Delta_{r+1, c}
        for (int r = l - 1; r >= 0; --r) {
            const double den = (double)(l - r) * (double)(l + r + 1);
            const double a = 2.0 * c / sqrt(den);
            const double b = sqrt((double)(l - r - 1) * (double)(l + r + 2) / den);
            const double d0 = a * d1 - b * d2;
            blk[(int64_t)r * w + c] = d0;
            d2 = d1;
            d1 = d0;
        }
    }
}

hipError_t launch_delta_toprows(double *tab, int Lmax, hipStream_t st) {
    hipLaunchKernelGGL(k_delta_toprows, dim3(1), dim3(1024), 0, st, tab, Lmax);
    return hipGetLastError();
}
hipError_t launch_delta_fill(double *tab, int Lmax, hipStream_t st) {
    hipLaunchKernelGGL(k_delta_fill, dim3(Lmax), dim3(256), 0, st, tab, Lmax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Parity-folded beta stage: out[r][c] = (i^par) * sum_k A^{par(c)}[r][k] in[k][c].
// Real GEMM over interleaved (re, im) columns for layouts whose column parity
// varies inside a tile (general Wigner transforms): both matrices are applied
// and each column keeps its parity's result.  Tile 64 rows x 32 complex
// columns x 16 k; each thread owns 4 rows x 2 complex columns.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_beta_gemm(int M, int K, int ncols, int Nep, int mode,
                                                   int par0, const double *__restrict__ Ae,
                                                   const double *__restrict__ Ao,
                                                   const double *__restrict__ in,
                                                   double *__restrict__ out) {
    __shared__ double As[2][16][64];
    __shared__ double Bs[16][64];
    const int tid = threadIdx.x;
    const int tr = tid / 16, tc = tid % 16;
    const int r0 = blockIdx.y * 64;
    const int c0 = blockIdx.x * 32;  // complex column base
    const size_t ld = 2 * (size_t)ncols;
    auto parity = [&](int c) -> int {
        if (mode == 0) return (c / Nep) & 1;
        return ((c / Nep) + (c % Nep) + par0) & 1;
    };
    double acc[4][4], acc2[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[i][e] = acc2[i][e] = 0.0;
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int i = tid; i < 1024; i += 256) {
            const int rr = i / 16, kk = i % 16;
            const int r = r0 + rr, k = k0 + kk;
            const bool ok = (r < M && k < K);
            As[0][kk][rr] = ok ? Ae[(size_t)r * K + k] : 0.0;
            As[1][kk][rr] = ok ? Ao[(size_t)r * K + k] : 0.0;
        }
        for (int i = tid; i < 1024; i += 256) {
            const int kk = i / 64, cc = i % 64;
            const int k = k0 + kk;
            const size_t col = 2 * (size_t)c0 + cc;
            Bs[kk][cc] = (k < K && col < ld) ? in[(size_t)k * ld + col] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double b[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) b[e] = Bs[kk][tc * 4 + e];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double a = As[0][kk][tr + 16 * i];
                const double ao = As[1][kk][tr + 16 * i];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    acc[i][e] += a * b[e];
                    acc2[i][e] += ao * b[e];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + tr + 16 * i;
        if (r >= M) continue;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = c0 + tc * 2 + q;
            if (c >= ncols) continue;
            const int par = parity(c);
            const double re = par ? acc2[i][2 * q] : acc[i][2 * q];
            const double im = par ? acc2[i][2 * q + 1] : acc[i][2 * q + 1];
            double *o = out + (size_t)r * ld + 2 * (size_t)c;
            if (par) {
                o[0] = -im;
                o[1] = re;
            } else {
                o[0] = re;
                o[1] = im;
            }
        }
    }
}

// MFMA version for the curvelet layout (every 32-complex-column tile inside one
// m, so one parity per tile).  Tile 128 rows x 64 real columns x 16 k; wave w
// owns rows [32w, 32w+32) as 2 x 4 blocks of v_mfma_f64_16x16x4f64, whose lane
// layout is A[l%16][l/16], B[l/16][l%16], D[4r + l/16][l%16].  The factor i of
// odd parity is applied to the result: (re, im) -> (-im, re).  The next K
// tile is loaded into registers while the current one is multiplied.
// uL > 0: the synthesis cube of the unrotated curvelets at band-limit uL,
// whose outputs are read only at m' <= l and m <= l (l = |n|); a tile with
// none of those is skipped (its outputs are left unwritten).
typedef double cvl_d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256, 4) void k_beta_mfma(int M, int K, int ncols, int Nep,
                                                   const double *__restrict__ Ae,
                                                   const double *__restrict__ Ao,
                                                   const double *__restrict__ in,
                                                   double *__restrict__ out, int uL) {
    __shared__ double As[128][17];
    __shared__ double Bs[16][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // logical tile (row tile fastest: the row tiles of one column tile share
    // its B operand, so they run together on one XCD)
    const int nrt = (M + 127) / 128;
    const int lg = xcd_group(blockIdx.x, gridDim.x);
    const int r0 = (lg % nrt) * 128;
    const int c0 = (lg / nrt) * 32;  // complex column base
    if (uL > 0) {  // uniform over the work-group
        const int rho = c0 / Nep, m = rho >> 1, pn = ((rho & 1) + m) & 1;
        const int h = (uL - 1) >> 1, ho = uL >> 1;
        const int cb = c0 % Nep, clast = pn ? 2 * ho - 1 : 2 * h;  // last column in use
        int lmax = -1;  // n is monotone in the column, so max |n| is at an end
        if (cb <= clast) {
            const int ce = cb + 31 < clast ? cb + 31 : clast;
            const int n0 = pn ? 2 * (cb - ho) + 1 : 2 * (cb - h);
            const int n1 = pn ? 2 * (ce - ho) + 1 : 2 * (ce - h);
            lmax = max(n0 < 0 ? -n0 : n0, n1 < 0 ? -n1 : n1);
        }
        if (m > lmax || r0 > lmax) return;
    }
    const size_t ld = 2 * (size_t)ncols;
    const int par = (c0 / Nep) & 1;
    const double *A = par ? Ao : Ae;
    cvl_d4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = cvl_d4{0.0, 0.0, 0.0, 0.0};
    const int lr = lane & 15, lk = lane >> 4;
    // Next K tile held in registers while the current one is multiplied.
    // A whole tile (the usual case) loads without guards, so no load result
    // is consumed (and waited for) before the next iteration stores it.
    double ra[8];
    double2 rb[2];
    const int kkb = tid >> 4, ccb = (tid & 15) * 4;  // 4 doubles = 2 complex
    const double *Arow = A + (size_t)r0 * K;
    const size_t col = 2 * (size_t)c0 + ccb;
    auto fetch = [&](int k0) {
        const int k = k0 + kkb;
        if (r0 + 128 <= M && k0 + 16 <= K && 2 * (size_t)c0 + 64 <= ld) {  // uniform
            // element q: row (tid >> 4) + 16 q, column k0 + (tid & 15)
            const double *pa = Arow + (uint32_t)((tid >> 4) * K + (tid & 15) + k0);
            const uint32_t step = 16u * (uint32_t)K;
#pragma unroll
            for (int q = 0; q < 8; ++q) ra[q] = pa[q * step];
            const double2 *src = reinterpret_cast<const double2 *>(in + (size_t)k * ld + col);
            rb[0] = src[0];
            rb[1] = src[1];
            return;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + 256 * q;
            const int r = idx >> 4, kq = k0 + (idx & 15);
            ra[q] = (r0 + r < M && kq < K) ? Arow[(uint32_t)(r * K + kq)] : 0.0;
        }
        rb[0] = make_double2(0.0, 0.0);
        rb[1] = make_double2(0.0, 0.0);
        if (k < K && col + 3 < ld) {
            const double2 *src = reinterpret_cast<const double2 *>(in + (size_t)k * ld + col);
            rb[0] = src[0];
            rb[1] = src[1];
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + 256 * q;
            As[idx >> 4][idx & 15] = ra[q];
        }
        *reinterpret_cast<double2 *>(&Bs[kkb][ccb]) = rb[0];
        *reinterpret_cast<double2 *>(&Bs[kkb][ccb + 2]) = rb[1];
        __syncthreads();
        if (k0 + 16 < K) fetch(k0 + 16);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int k = 4 * ks + lk;
            const double a0 = As[32 * w + lr][k];
            const double a1 = As[32 * w + 16 + lr][k];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double b = Bs[k][16 * j + lr];
                acc[0][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc[0][j], 0, 0, 0);
                acc[1][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc[1][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // Odd parity: the factor i on the input columns, (re, im) -> (-im, re),
    // applied to the result instead (the GEMM is linear in its columns).
    // Column 16 j + lr: re at even lr, im at odd lr; the partner is lane ^ 1.
    if (par) {
        const double sg = (lr & 1) ? 1.0 : -1.0;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[i][j][r] = sg * __shfl_xor(acc[i][j][r], 1);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + 32 * w + 16 * i + 4 * r + lk;
                const size_t col = 2 * (size_t)c0 + 16 * j + lr;
                if (row < M && col < ld) out[(size_t)row * ld + col] = acc[i][j][r];
            }
}

hipError_t launch_beta_gemm_unrot_fwd(const ScaleGeom &g, const double *Aeven,
                                     const double *Aodd, const cd *in, cd *out, hipStream_t st) {
    const int ncols = 2 * g.L * g.Nep;
    if (g.Nep % 32 != 0) return hipErrorInvalidValue;
    dim3 grid(((ncols + 31) / 32) * ((g.L + 127) / 128));
    hipLaunchKernelGGL(k_beta_mfma, grid, dim3(256), 0, st, g.L, g.L, ncols, g.Nep, Aeven, Aodd,
                       (const double *)in, (double *)out, g.L);
    return hipGetLastError();
}

hipError_t launch_beta_gemm(int M, int K, int ncols, int Nep, int mode, int par0,
                            const double *Aeven, const double *Aodd, const cd *in, cd *out,
                            hipStream_t st) {
    if (mode == 0 && Nep % 32 == 0) {
        dim3 g(((ncols + 31) / 32) * ((M + 127) / 128));
        hipLaunchKernelGGL(k_beta_mfma, g, dim3(256), 0, st, M, K, ncols, Nep, Aeven, Aodd,
                           (const double *)in, (double *)out, 0);
        return hipGetLastError();
    }
    dim3 grid((ncols + 31) / 32, (M + 63) / 64);
    hipLaunchKernelGGL(k_beta_gemm, grid, dim3(256), 0, st, M, K, ncols, Nep, mode, par0, Aeven,
                       Aodd, (const double *)in, (double *)out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Analysis contraction of one curvelet scale (Fourier cube, parity-folded):
//   P_e/o[m][k] = sum_{l even/odd} (Delta^l_{m'm} f_lm) (Delta^l_{m',2k} Psi_{l,2k})
//   X[m'][m][h+k] = (-1)^k i^{-m} (P_e + P_o)
//   X[m'][m][h-k] = (-1)^k i^{-m} (-1)^{m'} (P_e - P_o)
// over l in [max(llo, m', m, 2k), lhi], on FP64 MFMA.  Work-group: one m',
// 64 m x 32 k.  The GEMM rows are (component c, m):
// A[(c, m)][l] = c-part of Delta^l_{m'm} f_lm, B[l][k] = Delta^l_{m',2k} Psi_{l,2k}.
// A chunk covers 32 consecutive l (16 of each parity = four K = 4 steps), the
// next chunk's raw operands prefetched into registers.  Wave w: parity
// p = w & 1, component c = w >> 1; 64 m x 32 k as 4 x 2 blocks of 16 x 16
// (operand layouts: A[row = lane%16][K = lane/16], B[K = lane/16]
// [col = lane%16], result row 4r + lane/16, column lane%16).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void k_contract_inv_mfma(ScaleGeom g, int Lf,
                                                              const double *__restrict__ delta,
                                                              const cd *__restrict__ fpad,
                                                              const double *__restrict__ psi,
                                                              cd *__restrict__ X) {
    // As[p][c][i][mm] (l = lb + p + 2i), Bs[p][i][kk]; then R[p][mm][kk] for
    // one component at a time in the epilogue.  Pads 66 / 34 spread the four
    // 16-lane groups of an operand read over the LDS banks.
    __shared__ double smem[2 * 2 * 16 * 66 + 2 * 16 * 34];
    double(*As)[2][16][66] = reinterpret_cast<double(*)[2][16][66]>(smem);
    double(*Bs)[16][34] = reinterpret_cast<double(*)[16][34]>(smem + 2 * 2 * 16 * 66);
    const int L = g.L, h = g.h;
    // logical tile: k tile fastest, then m tile, then m' (tiles of one m'
    // share its Delta rows; the tiles of one m' run on one XCD)
    const int nkt = (h + 1 + 31) / 32, nmt = (L + 63) / 64;
    const int lg = xcd_group_runs(blockIdx.x, gridDim.x, nkt * nmt);
    const int mp = lg / (nkt * nmt);
    const int m0 = ((lg / nkt) % nmt) * 64, k0 = (lg % nkt) * 32;
    // w is the same across a wave: readfirstlane lets the compiler keep it,
    // the l of each staged row and that row's offsets in scalar registers.
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int p = w & 1, c = w >> 1;
    const int li = lane & 15, lq = lane >> 4;
    cvl_d4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = cvl_d4{0.0, 0.0, 0.0, 0.0};
    int lstart = g.llo;
    if (mp > lstart) lstart = mp;
    if (m0 > lstart) lstart = m0;
    if (2 * k0 > lstart) lstart = 2 * k0;
    const int lend = g.lhi;
    // The next chunk's raw operands, prefetched while the current one is
    // multiplied.  A element q of a thread: parity pp = q >> 2, i = w + 4 (q & 3),
    // mm = lane, so l = lb + pp + 2 i is uniform over the wave.  B element q:
    // parity = lane >> 5, i = w + 4 q, kk = lane & 31 (two l per wave, both
    // offsets scalar).  Loads out of range read element 0; their bit in `okm`
    // is clear and the value is replaced by 0 only when the next iteration
    // stores it, so that no load is waited for before the multiply.
    double ra[8], rb2[4], rp[4];
    cd rf[8];
    uint32_t okm = 0;
    auto fetch = [&](int lb) {
        const int m = m0 + lane;
        okm = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int l = lb + (q >> 2) + 2 * (w + 4 * (q & 3));
            const bool lok = l >= lstart && l <= lend;
            const bool ok = lok && m <= l && m < L;
            const uint32_t dro = lok ? delta_off32(l) + (uint32_t)(mp * (l + 1)) : 0u;
            const uint32_t fro = lok ? (uint32_t)(l * Lf) : 0u;
            const uint32_t mi = ok ? (uint32_t)m : 0u;
            ra[q] = delta[(size_t)(dro + mi)];
            rf[q] = fpad[(size_t)(fro + mi)];
            okm |= ok ? 1u << q : 0u;
        }
        const int hi = lane >> 5, k = k0 + (lane & 31);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int la = lb + 2 * (w + 4 * q);
            const bool ok0 = la >= lstart && la <= lend, ok1 = la + 1 >= lstart && la + 1 <= lend;
            const uint32_t d0 = ok0 ? delta_off32(la) + (uint32_t)(mp * (la + 1)) : 0u;
            const uint32_t d1 = ok1 ? delta_off32(la + 1) + (uint32_t)(mp * (la + 2)) : 0u;
            const uint32_t p0 = ok0 ? (uint32_t)(la * (h + 1)) : 0u;
            const uint32_t p1 = ok1 ? (uint32_t)((la + 1) * (h + 1)) : 0u;
            const int l = la + hi;
            const bool ok = (hi ? ok1 : ok0) && k <= h && 2 * k <= l;
            const uint32_t ki = ok ? (uint32_t)k : 0u;
            rb2[q] = delta[(size_t)((hi ? d1 : d0) + 2u * ki)];
            rp[q] = psi[(size_t)((hi ? p1 : p0) + ki)];
            okm |= ok ? 1u << (8 + q) : 0u;
        }
    };
    const int lb0 = lstart & ~1;
    if (lb0 <= lend) fetch(lb0);
    for (int lb = lb0; lb <= lend; lb += 32) {
        // A: 2 parities x 16 l x 64 m complex; B: 2 parities x 16 l x 32 k
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = w + 4 * (q & 3), pp = q >> 2;
            const bool ok = (okm >> q) & 1u;
            As[pp][0][i][lane] = ok ? ra[q] * rf[q].x : 0.0;
            As[pp][1][i][lane] = ok ? ra[q] * rf[q].y : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            Bs[lane >> 5][w + 4 * q][lane & 31] = ((okm >> (8 + q)) & 1u) ? rb2[q] * rp[q] : 0.0;
        __syncthreads();
        if (lb + 32 <= lend) fetch(lb + 32);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int i = 4 * ks + lq;
            double b[2];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) b[cb] = Bs[p][i][16 * cb + li];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const double a = As[p][c][i][16 * rb + li];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[cb], acc[rb][cb], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // Epilogue, one component at a time through LDS: s = P_e + P_o, d = P_e - P_o.
    double(*R)[64][33] = reinterpret_cast<double(*)[64][33]>(smem);
    double sv[2][8], dv[2][8];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
        if (c == cc) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        R[p][16 * rb + 4 * r + lq][16 * cb + li] = acc[rb][cb][r];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx & 31, mm = idx >> 5;
            sv[cc][q] = R[0][mm][kk] + R[1][mm][kk];
            dv[cc][q] = R[0][mm][kk] - R[1][mm][kk];
        }
        __syncthreads();
    }
    const int Nep = g.Nep;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int idx = tid + 256 * q;
        const int kk = idx & 31, mm = idx >> 5;
        const int m = m0 + mm, k = k0 + kk;
        if (m >= L || k > h) continue;
        const double sk = (k & 1) ? -1.0 : 1.0;
        cd *row = X + ((size_t)mp * L + m) * Nep;
        row[h + k] = ipow(cscale(cd{sv[0][q], sv[1][q]}, sk), -m);
        if (k > 0) {
            const double sm = (mp & 1) ? -sk : sk;
            row[h - k] = ipow(cscale(cd{dv[0][q], dv[1][q]}, sm), -m);
        }
    }
}

hipError_t launch_contract_inv(const ScaleGeom &g, int Lf, const double *delta, const cd *fpad,
                               const double *psi, cd *X, hipStream_t st) {
    const int nkt = (g.h + 1 + 31) / 32;
    dim3 grid(((g.L + 63) / 64) * nkt * g.L);
    hipLaunchKernelGGL(k_contract_inv_mfma, grid, dim3(256), 0, st, g, Lf, delta, fpad, psi, X);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Synthesis contraction of one curvelet scale:
//   f_lm = i^m sum_{m'} Delta^l_{m'm} sum_k Z^{par(l)}[m'][m][k] B'[k][l],
//   B'[k][l] = (-1)^k Delta^l_{m',2k} Psi_{l,2k},
//   Z^{+/-}[m'][m][k] = Z[m'][m][h+k] +/- (-1)^{m'} Z[m'][m][h-k]  (k > 0),
//   Z^{+/-}[m'][m][0] = Z[m'][m][h].
// One m' per work-group column: the partials part[m'][l][m] =
// Delta^l_{m'm} T_{m'}[l][m] are summed over m' in a fixed order afterwards.
// ---------------------------------------------------------------------------
// Sum of the group partials into the FP64 accumulator,
//   facc[l][m] += i^m sum_grp part[grp][l][m],
// over the groups that can hold an m' <= l (m' of group grp: [grp*gsz,
// (grp+1)*gsz)).  Work-group: one l, 64 m x 4 slices of the groups; slice s
// sums groups s, s+4, ... in FP64, the slices are then added in a fixed order.
template <class P>
__global__ __launch_bounds__(256) void k_reduce_groups(ScaleGeom g, int Lf,
                                                       const P *__restrict__ part, int ngroups,
                                                       cd *__restrict__ facc) {
    __shared__ cd red[4][64];
    const int L = g.L;
    const int l = g.llo + blockIdx.y;
    const int mm = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int m = blockIdx.x * 64 + mm;
    const int gsz = (L + ngroups - 1) / ngroups;
    int gmax = l / gsz;
    if (gmax > ngroups - 1) gmax = ngroups - 1;
    double sx = 0.0, sy = 0.0;
    if (m <= l && m < L) {
        const P *src = part + (size_t)l * L + m;
        const size_t gs = (size_t)L * L;
        int grp = sl;
        // four independent loads in flight per step
        for (; grp + 12 <= gmax; grp += 16) {
            const P a = src[grp * gs], b = src[(grp + 4) * gs], c = src[(grp + 8) * gs],
                    d = src[(grp + 12) * gs];
            sx += (double)a.x;
            sy += (double)a.y;
            sx += (double)b.x;
            sy += (double)b.y;
            sx += (double)c.x;
            sy += (double)c.y;
            sx += (double)d.x;
            sy += (double)d.y;
        }
        for (; grp <= gmax; grp += 4) {
            const P a = src[grp * gs];
            sx += (double)a.x;
            sy += (double)a.y;
        }
    }
    red[sl][mm] = cd{sx, sy};
    __syncthreads();
    if (sl == 0 && m <= l && m < L) {
        const cd t = cadd(cadd(red[0][mm], red[1][mm]), cadd(red[2][mm], red[3][mm]));
        cd *o = facc + (size_t)l * Lf + m;
        *o = cadd(*o, ipow(t, m));
    }
}

template <class P>
static hipError_t launch_reduce_groups(const ScaleGeom &g, int Lf, const P *part, int ngroups,
                                       cd *facc, hipStream_t st) {
    const int nl = g.lhi - g.llo + 1;
    if (nl <= 0) return hipSuccess;
    dim3 grid((g.L + 63) / 64, nl);
    hipLaunchKernelGGL(k_reduce_groups<P>, grid, dim3(256), 0, st, g, Lf, part, ngroups, facc);
    return hipGetLastError();
}

// The contraction on FP64 MFMA.  Work-group tile: 64 l (32 of each parity,
// l = l0 + par + 2i) x 64 m for one m':
//   T[l][m] = sum_k B'[k][l] Z^{par(l)}[m'][m][k]   (A = B'^T real, B = Z^T complex)
//   part[m'][l][m] = Delta^l_{m'm} T[l][m]   (applied in the MFMA output layout;
//   the Delta row of each l is contiguous in m, so those loads coalesce).
// Wave (wp, wm): parity wp, 32 l x 32 m, [2 l blocks][2 m blocks][re/im].
// With no running sum over m' held, the next K chunk's operands (raw Delta,
// Psi and the two Z half rows) are prefetched into registers while the
// current chunk is multiplied.
__global__ __launch_bounds__(256, 2) void k_contract_fwd_m1(ScaleGeom g,
                                                         const double *__restrict__ delta,
                                                         const cd *__restrict__ Z,
                                                         const double *__restrict__ psi,
                                                         cd *__restrict__ part) {
    __shared__ double Bt[2][16][33];
    __shared__ double Zr[2][16][65], Zi[2][16][65];
    const int L = g.L, h = g.h, Nep = g.Nep;
    const int lbase = g.llo & ~1;
    const int nl = g.lhi - lbase + 1;
    const int nlt = (nl + 63) / 64, nmt = (L + 63) / 64;
    // logical tile: l tile fastest, then m tile, then m'; all tiles of one m'
    // run on one XCD (those of one (m', m tile) read the same cube rows, those
    // of one (m', l tile) the same Delta rows)
    const int lg = xcd_group_runs(blockIdx.x, gridDim.x, nlt * nmt);
    const int m0 = ((lg / nlt) % nmt) * 64;
    const int l0 = lbase + (lg % nlt) * 64;
    const int mp = lg / (nlt * nmt);
    int ltop = l0 + 63;
    if (ltop > g.lhi) ltop = g.lhi;
    // entries the reduction never reads (m > l or m' > l for the whole tile)
    if (m0 > ltop || mp > ltop) return;
    int kmax = ltop / 2;
    if (kmax > h) kmax = h;
    const double smp = (mp & 1) ? -1.0 : 1.0;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wp = w & 1, wm = w >> 1;
    const int li = lane & 15, lq = lane >> 4;
    // staging assignment: element q of this thread
    //   B'^T: kk = idx & 15, i = (idx >> 4) & 31, par = idx >> 9 (l = l0 + par + 2 i)
    //   Z:    kk = idx & 15, mm = idx >> 4
    double rd[4], rp[4];
    cd rzp[4], rzn[4];
    const cd *zt = Z + ((size_t)mp * L + m0) * Nep;  // cube row (m', m0)
    auto fetch = [&](int kb) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx & 15, i = (idx >> 4) & 31, par = idx >> 9;
            const int l = l0 + par + 2 * i, k = kb + kk;
            const bool ok = k <= kmax && l <= g.lhi && 2 * k <= l && mp <= l;
            rd[q] = ok ? delta[(size_t)(delta_row32(l, mp) + (uint32_t)(2 * k))] : 0.0;
            rp[q] = ok ? psi[(size_t)(uint32_t)(l * (h + 1) + k)] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx & 15, mm = idx >> 4;
            const int k = kb + kk, m = m0 + mm;
            const bool ok = k <= kmax && m < L;
            // 32-bit offsets inside the tile's rows (64 rows of Nep <= 1024)
            const cd *row = zt + (uint32_t)((ok ? mm : 0) * Nep);
            rzp[q] = ok ? row[h + k] : cd{0.0, 0.0};
            rzn[q] = (ok && k > 0) ? row[h - k] : cd{0.0, 0.0};
        }
    };
    cvl_d4 t[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) t[a][b][c] = cvl_d4{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int kb = 0; kb <= kmax; kb += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx & 15, i = (idx >> 4) & 31, par = idx >> 9;
            const double v = rd[q] * rp[q];
            Bt[par][kk][i] = (kk & 1) ? -v : v;  // (-1)^k, k = kb + kk with kb even
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx & 15, mm = idx >> 4;
            // k = 0: Z^+ = Z^- = Z[h] (rzn is zero there)
            const cd zn = cscale(rzn[q], smp);
            const cd vp = cadd(rzp[q], zn), vm = csub(rzp[q], zn);
            Zr[0][kk][mm] = vp.x;
            Zi[0][kk][mm] = vp.y;
            Zr[1][kk][mm] = vm.x;
            Zi[1][kk][mm] = vm.y;
        }
        __syncthreads();
        if (kb + 16 <= kmax) fetch(kb + 16);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = 4 * ks + lq;
            double a[2], zr[2], zi[2];
#pragma unroll
            for (int lf = 0; lf < 2; ++lf) a[lf] = Bt[wp][kk][16 * lf + li];
#pragma unroll
            for (int mj = 0; mj < 2; ++mj) {
                zr[mj] = Zr[wp][kk][32 * wm + 16 * mj + li];
                zi[mj] = Zi[wp][kk][32 * wm + 16 * mj + li];
            }
#pragma unroll
            for (int lf = 0; lf < 2; ++lf)
#pragma unroll
                for (int mj = 0; mj < 2; ++mj) {
                    t[lf][mj][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[lf], zr[mj],
                                                                        t[lf][mj][0], 0, 0, 0);
                    t[lf][mj][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[lf], zi[mj],
                                                                        t[lf][mj][1], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // part[m'][l][m] = Delta^l_{m'm} T[l][m]  (output layout: row 4r + lq of block lf).
    // The 16 Delta values of a thread are loaded together (out-of-range ones
    // read element 0 and are replaced by 0 when used), then the products stored.
    double dd[2][4][2];
#pragma unroll
    for (int lf = 0; lf < 2; ++lf)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int l = l0 + wp + 2 * (16 * lf + 4 * r + lq);
            const uint32_t dro = (l <= g.lhi && mp <= l) ? delta_row32(l, mp) : 0u;
#pragma unroll
            for (int mj = 0; mj < 2; ++mj) {
                const int m = m0 + 32 * wm + 16 * mj + li;
                const bool ok = l <= g.lhi && m < L && mp <= l && m <= l;
                dd[lf][r][mj] = delta[(size_t)(dro + (ok ? (uint32_t)m : 0u))];
            }
        }
    cd *pbase = part + (size_t)mp * L * L;
#pragma unroll
    for (int lf = 0; lf < 2; ++lf)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int l = l0 + wp + 2 * (16 * lf + 4 * r + lq);
            if (l > g.lhi) continue;
#pragma unroll
            for (int mj = 0; mj < 2; ++mj) {
                const int m = m0 + 32 * wm + 16 * mj + li;
                if (m >= L) continue;
                const double d = (mp <= l && m <= l) ? dd[lf][r][mj] : 0.0;
                pbase[(uint32_t)(l * L + m)] = cd{d * t[lf][mj][0][r], d * t[lf][mj][1][r]};
            }
        }
}

hipError_t launch_contract_fwd(const ScaleGeom &g, const double *delta, const cd *Z,
                               const double *psi, cd *part, hipStream_t st) {
    if (g.lhi < g.llo) return hipSuccess;
    const int nl = g.lhi - (g.llo & ~1) + 1;
    dim3 grid(((g.L + 63) / 64) * ((nl + 63) / 64) * g.L);
    hipLaunchKernelGGL(k_contract_fwd_m1, grid, dim3(256), 0, st, g, delta, Z, psi, part);
    return hipGetLastError();
}

hipError_t launch_reduce_fwd(const ScaleGeom &g, int Lf, const cd *part, int ngroups, cd *facc,
                             hipStream_t st) {
    return launch_reduce_groups(g, Lf, part, ngroups, facc, st);
}
hipError_t launch_reduce_fwd_mx(const ScaleGeom &g, int Lf, const cf *part, int ngroups,
                                cd *facc, hipStream_t st) {
    return launch_reduce_groups(g, Lf, part, ngroups, facc, st);
}

// ---------------------------------------------------------------------------
// Unrotated curvelets (Sec. III-A-1): the kernel Psi~_ln is zero unless
// |n| = l, so each Fourier-cube entry takes one l and the contractions are
// O(L^3) per scale.  pd[m'][l] = Delta^l_{m'l} Psi~_{l,l} (zero for m' > l and
// outside the kernel support; row length L_j); Psi~_{l,-l} = (-1)^l Psi~_{l,l}
// and Delta^l_{m',-l} = (-1)^(l+m') Delta^l_{m',l}.
//
// Analysis: X[m'][m][n] = i^(n-m) s Delta^l_{m'm} pd[m'][l] f_lm, l = |n|,
// s = (-1)^m' for n < 0 (the two signs above), zero unless m <= l and m' <= l.
// dense: every cube entry is written (zeros included, unused columns too), as
// the beta GEMM reads them all; otherwise only the entries with m <= l and
// m' <= l (the ones the beta FFT reads).  Work-group: one m'
// and two m (four cube rows, all columns).  The per-l factors of those rows
// (Delta^l_{m'm}, pd[m'][l], f_lm) are staged in LDS first, one read per l,
// so each cube entry costs LDS reads and one coalesced store.  xcd_group keeps
// a plane's Delta rows in one L2.
// ---------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(256) void k_unrot_contract_inv(ScaleGeom g, int Lf,
                                                            const double *__restrict__ delta,
                                                            const cd *__restrict__ fpad,
                                                            const double *__restrict__ pd,
                                                            C *__restrict__ X, int nmb,
                                                            int dense) {
    extern __shared__ __align__(16) char smem_raw[];
    const int L = g.L, Nep = g.Nep;
    cd *fv = reinterpret_cast<cd *>(smem_raw);                   // [2][L]: f_{l, m0 + i}
    double *dmm = reinterpret_cast<double *>(smem_raw) + 4 * L;  // [2][L]: Delta^l_{m', m0 + i}
    double *dml = dmm + 2 * L;                                   // [L]: pd[m'][l]
    const int lg = xcd_group(blockIdx.x, gridDim.x);
    const int mp = lg / nmb, m0 = 2 * (lg % nmb);
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        const double p = pd[(size_t)mp * L + l];
        const bool on = p != 0.0;  // implies m' <= l
        double d0 = 0.0, d1 = 0.0;
        cd f0 = cd{0.0, 0.0}, f1 = cd{0.0, 0.0};
        if (on && m0 <= l) {
            const double *row = delta + delta_row32(l, mp);
            d0 = row[m0];
            f0 = fpad[(size_t)l * Lf + m0];
            if (m0 + 1 <= l) {
                d1 = row[m0 + 1];
                f1 = fpad[(size_t)l * Lf + m0 + 1];
            }
        }
        dmm[l] = d0;
        dmm[L + l] = d1;
        fv[l] = f0;
        fv[L + l] = f1;
        dml[l] = p;
    }
    __syncthreads();
    const int ho = L >> 1;
    const int nrow = m0 + 1 < L ? 4 : 2;
    for (int e = threadIdx.x; e < nrow * Nep; e += blockDim.x) {
        const int r = e / Nep, c = e % Nep;
        const int mi = r >> 1, m = m0 + mi;
        const int pn = ((r & 1) + m) & 1;  // parity of n
        cd out = cd{0.0, 0.0};
        bool keep = dense != 0;
        if (pn ? c < 2 * ho : c <= 2 * g.h) {
            const int n = pn ? 2 * (c - ho) + 1 : 2 * (c - g.h);
            const int l = n < 0 ? -n : n;
            double w = dmm[mi * L + l] * dml[l];
            if (n < 0 && (mp & 1)) w = -w;
            const cd f = fv[mi * L + l];
            out = ipow(cd{w * f.x, w * f.y}, n - m);
            keep = keep || (m <= l && mp <= l);
        }
        if (keep) X[((size_t)mp * 2 * L + 2 * m0 + r) * Nep + c] = cmk<C>(out.x, out.y);
    }
}

template <class C>
static hipError_t unrot_contract_inv_t(const ScaleGeom &g, int Lf, const double *delta,
                                       const cd *fpad, const double *pd, C *X, bool dense,
                                       hipStream_t st) {
    const int nmb = (g.L + 1) / 2;
    const size_t lds = (size_t)7 * g.L * sizeof(double);  // <= 56 KiB for L_j <= 1024
    if (lds > 65536) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_unrot_contract_inv<C>, dim3(nmb * g.L), dim3(256), lds, st, g, Lf, delta,
                       fpad, pd, X, nmb, dense ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_unrot_contract_inv(const ScaleGeom &g, int Lf, const double *delta,
                                     const cd *fpad, const double *pd, cd *X, bool dense,
                                     hipStream_t st) {
    return unrot_contract_inv_t(g, Lf, delta, fpad, pd, X, dense, st);
}
hipError_t launch_unrot_contract_inv(const ScaleGeom &g, int Lf, const double *delta,
                                     const cd *fpad, const double *pd, cf *X, bool dense,
                                     hipStream_t st) {
    return unrot_contract_inv_t(g, Lf, delta, fpad, pd, X, dense, st);
}

// Synthesis: with Y the beta-projected cube (m' >= 0, the -m' half folded in),
//   F~^l_{m,+-l} = i^(m-+l) sum_{m'<=l} Delta^l_{m'm} Delta^l_{m',+-l} Y[m'][m][+-l]
// and f_lm = Psi~_{l,l} F~^l_{m,l} + Psi~_{l,-l} F~^l_{m,-l}, i.e.
//   facc[l][m] += i^(m-l) sum_{m'<=l} Delta^l_{m'm} pd[m'][l]
//                 (Y[m'][m][l] + (-1)^(l+m') Y[m'][m][-l])      (n = 0 once).
// Work-group: one m, 64 consecutive l (lanes), the m' sum split over the four
// waves (m' = w mod 4), four m' per wave in flight, the wave sums added in
// LDS in wave order, all in FP64.  Y[.][m][+-l] and pd[m'][.] of neighbouring
// l are neighbours in memory (Y: two cube rows, one per parity of l).
template <class C>
__global__ __launch_bounds__(256) void k_unrot_contract_fwd(ScaleGeom g, int Lf,
                                                            const double *__restrict__ delta,
                                                            const C *__restrict__ Y,
                                                            const double *__restrict__ pd,
                                                            cd *__restrict__ facc) {
    __shared__ double red[4][64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = blockIdx.y;
    const int l = blockIdx.x * 64 + lane;
    const int L = g.L;
    const bool live = l < L && l >= m && l >= g.llo && l <= g.lhi;
    double sx = 0.0, sy = 0.0;
    if (live) {
        const size_t plane = (size_t)2 * L * g.Nep;
        const C *yp = Y + unrot_off(g, m, l);
        const C *ym = Y + unrot_off(g, m, -l);
        const double *dm = delta + (size_t)(delta_off32(l) + (uint32_t)m);  // Delta^l_{m'm} at dm[m' (l + 1)]
        const double *pl = pd + l;                    // pd[m'][l] at pl[m' L]
        const double both = l > 0 ? 1.0 : 0.0;
        int mp = w;
        for (; mp + 12 <= l; mp += 16) {
            double dd[4];
            C a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = mp + 4 * u;
                dd[u] = dm[(int64_t)q * (l + 1)] * pl[(size_t)q * L];
                a[u] = yp[q * plane];
                b[u] = ym[q * plane];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double sb = ((l + mp + 4 * u) & 1) ? -both : both;
                sx += dd[u] * ((double)a[u].x + sb * (double)b[u].x);
                sy += dd[u] * ((double)a[u].y + sb * (double)b[u].y);
            }
        }
        for (; mp <= l; mp += 4) {
            const double d = dm[(int64_t)mp * (l + 1)] * pl[(size_t)mp * L];
            const C a = yp[mp * plane], b = ym[mp * plane];
            const double sb = ((l + mp) & 1) ? -both : both;
            sx += d * ((double)a.x + sb * (double)b.x);
            sy += d * ((double)a.y + sb * (double)b.y);
        }
    }
    red[w][lane][0] = sx;
    red[w][lane][1] = sy;
    __syncthreads();
    if (w == 0 && live) {
        double tx = red[0][lane][0], ty = red[0][lane][1];
        for (int q = 1; q < 4; ++q) {
            tx += red[q][lane][0];
            ty += red[q][lane][1];
        }
        cd *o = facc + (size_t)l * Lf + m;
        *o = cadd(*o, ipow(cd{tx, ty}, m - l));
    }
}

template <class C>
static hipError_t unrot_contract_fwd_t(const ScaleGeom &g, int Lf, const double *delta,
                                       const C *Y, const double *pd, cd *facc, hipStream_t st) {
    hipLaunchKernelGGL(k_unrot_contract_fwd<C>, dim3((g.L + 63) / 64, g.L), dim3(256), 0, st, g,
                       Lf, delta, Y, pd, facc);
    return hipGetLastError();
}
hipError_t launch_unrot_contract_fwd(const ScaleGeom &g, int Lf, const double *delta,
                                     const cd *Y, const double *pd, cd *facc, hipStream_t st) {
    return unrot_contract_fwd_t(g, Lf, delta, Y, pd, facc, st);
}
hipError_t launch_unrot_contract_fwd(const ScaleGeom &g, int Lf, const double *delta,
                                     const cf *Y, const double *pd, cd *facc, hipStream_t st) {
    return unrot_contract_fwd_t(g, Lf, delta, Y, pd, facc, st);
}

// ---------------------------------------------------------------------------
// General Wigner contractions (dense F^l_mn, any m, n).  Delta^l_{m',-k} =
// (-1)^(l+m') Delta^l_{m',k}.  Layouts: F[l][m+L-1][n+N-1] (row 2N-1),
// X / Z[m'][m+L-1][n+N-1] (row Nnp).
// ---------------------------------------------------------------------------
__global__ void k_gen_contract_inv(int L, int N, int Nnp, const double *__restrict__ delta,
                                   const cd *__restrict__ F, cd *__restrict__ X) {
    const int Nm = 2 * L - 1, Nn = 2 * N - 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int mp = blockIdx.y;
    if (idx >= Nm * Nnp) return;
    const int mi = idx / Nnp, ni = idx % Nnp;
    cd *o = X + ((size_t)mp * Nm + mi) * Nnp + ni;
    if (ni >= Nn) {
        *o = cd{0.0, 0.0};
        return;
    }
    const int m = mi - (L - 1), n = ni - (N - 1);
    const int am = m < 0 ? -m : m, an = n < 0 ? -n : n;
    int l0 = am > an ? am : an;
    if (mp > l0) l0 = mp;
    cd s = cd{0.0, 0.0};
    for (int l = l0; l < L; ++l) {
        const double *row = delta + delta_row32(l, mp);
        double w = row[am] * row[an] * (2.0 * l + 1.0) * (1.0 / (8.0 * M_PI * M_PI));
        const int flip = ((m < 0) + (n < 0)) * ((l + mp) & 1);
        if (flip & 1) w = -w;
        const cd f = F[((size_t)l * Nm + mi) * Nn + ni];
        s.x += w * f.x;
        s.y += w * f.y;
    }
    *o = ipow(s, n - m);
}

__global__ void k_gen_contract_fwd(int L, int N, int Nnp, const double *__restrict__ delta,
                                   const cd *__restrict__ Z, cd *__restrict__ F) {
    const int Nm = 2 * L - 1, Nn = 2 * N - 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (idx >= Nm * Nn) return;
    const int mi = idx / Nn, ni = idx % Nn;
    const int m = mi - (L - 1), n = ni - (N - 1);
    const int am = m < 0 ? -m : m, an = n < 0 ? -n : n;
    cd *o = F + ((size_t)l * Nm + mi) * Nn + ni;
    if (am > l || an > l) {
        *o = cd{0.0, 0.0};
        return;
    }
    cd s = cd{0.0, 0.0};
    for (int mp = 0; mp <= l; ++mp) {
        const double *row = delta + delta_row32(l, mp);
        double w = row[am] * row[an];
        const int flip = ((m < 0) + (n < 0)) * ((l + mp) & 1);
        if (flip & 1) w = -w;
        const cd z = Z[((size_t)mp * Nm + mi) * Nnp + ni];
        s.x += w * z.x;
        s.y += w * z.y;
    }
    *o = ipow(s, m - n);
}

// Spin-s curvelets rotated to the North pole (Sec. II-B; rho* = (0, theta_j, 0)
// with theta_j = arccos(-s / lambda^j)): the kernel coefficients Psi_ln are
// real but non-zero at every n, and the signal has no reality condition, so
// each scale runs on the general Wigner layouts with the harmonic product
// folded into the contraction:
//   X[m'][m][n] = i^{n-m} sum_l Delta^l_{m'm} Delta^l_{m'n} f_lm Psi_ln,
// l over the kernel support [llo, lhi] and l >= max(|m|, |n|, m'); f flat
// (band-limit Lf), psi [l][n + L - 1] (rows of 2L - 1).  The synthesis
// contracts the forward Wigner coefficients with Psi:
//   acc[l^2 + l + m] += sum_n F^l_mn Psi_ln.
__global__ void k_spin_contract_inv(int L, int Nnp, int llo, int lhi,
                                    const double *__restrict__ delta, const cd *__restrict__ flm,
                                    const double *__restrict__ psi, cd *__restrict__ X) {
    const int Nm = 2 * L - 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int mp = blockIdx.y;
    if (idx >= Nm * Nnp) return;
    const int mi = idx / Nnp, ni = idx % Nnp;
    cd *o = X + ((size_t)mp * Nm + mi) * Nnp + ni;
    if (ni >= Nm) {
        *o = cd{0.0, 0.0};
        return;
    }
    const int m = mi - (L - 1), n = ni - (L - 1);
    const int am = m < 0 ? -m : m, an = n < 0 ? -n : n;
    int l0 = am > an ? am : an;
    if (mp > l0) l0 = mp;
    if (llo > l0) l0 = llo;
    const int l1 = lhi < L - 1 ? lhi : L - 1;
    cd s = cd{0.0, 0.0};
    for (int l = l0; l <= l1; ++l) {
        const double *row = delta + delta_row32(l, mp);
        double w = row[am] * row[an] * psi[(size_t)l * Nm + ni];
        const int flip = ((m < 0) + (n < 0)) * ((l + mp) & 1);
        if (flip & 1) w = -w;
        const cd f = flm[(size_t)l * l + l + m];
        s.x += w * f.x;
        s.y += w * f.y;
    }
    *o = ipow(s, n - m);
}

// One thread per (l, m) of l < L: a fixed-order sum over n.
__global__ void k_spin_reduce_fwd(int L, const cd *__restrict__ F, const double *__restrict__ psi,
                                  cd *__restrict__ acc) {
    const int Nm = 2 * L - 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L * L) return;
    int l = (int)sqrt((double)idx);
    while (l * l > idx) --l;
    while ((l + 1) * (l + 1) <= idx) ++l;
    const int m = idx - l * l - l;
    const cd *row = F + ((size_t)l * Nm + m + L - 1) * Nm;
    const double *ps = psi + (size_t)l * Nm;
    cd s = cd{0.0, 0.0};
    for (int ni = L - 1 - l; ni <= L - 1 + l; ++ni) {
        const double w = ps[ni];
        s.x += w * row[ni].x;
        s.y += w * row[ni].y;
    }
    acc[idx] = cadd(acc[idx], s);
}

hipError_t launch_spin_contract_inv(int L, int llo, int lhi, const double *delta, const cd *flm,
                                    const double *psi, cd *X, hipStream_t st) {
    const int Nnp = ((2 * L - 1) + 31) / 32 * 32;
    const int n = (2 * L - 1) * Nnp;
    hipLaunchKernelGGL(k_spin_contract_inv, dim3((n + 255) / 256, L), dim3(256), 0, st, L, Nnp,
                       llo, lhi, delta, flm, psi, X);
    return hipGetLastError();
}
hipError_t launch_spin_reduce_fwd(int L, const cd *F, const double *psi, cd *acc, hipStream_t st) {
    hipLaunchKernelGGL(k_spin_reduce_fwd, dim3((L * L + 255) / 256), dim3(256), 0, st, L, F, psi,
                       acc);
    return hipGetLastError();
}

hipError_t launch_gen_contract_inv(int L, int N, const double *delta, const cd *F, cd *X,
                                   hipStream_t st) {
    const int Nnp = ((2 * N - 1) + 31) / 32 * 32;
    const int n = (2 * L - 1) * Nnp;
    hipLaunchKernelGGL(k_gen_contract_inv, dim3((n + 255) / 256, L), dim3(256), 0, st, L, N,
                       Nnp, delta, F, X);
    return hipGetLastError();
}
hipError_t launch_gen_contract_fwd(int L, int N, const double *delta, const cd *Z, cd *F,
                                   hipStream_t st) {
    const int Nnp = ((2 * N - 1) + 31) / 32 * 32;
    const int n = (2 * L - 1) * (2 * N - 1);
    hipLaunchKernelGGL(k_gen_contract_fwd, dim3((n + 255) / 256, L), dim3(256), 0, st, L, N,
                       Nnp, delta, Z, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// SHT (spin 0) helpers.  c_l = sqrt((2l+1)/(4 pi)).
//   inverse: F[m'][m] = i^{-m} sum_{l>=max(m,m')} c_l Delta^l_{m'm} Delta^l_{m'0} f_lm
//   forward: f_lm = i^m c_l sum_{m'<=l} Delta^l_{m'm} Delta^l_{m'0} Z[m'][m]
// (Delta^l_{m'0} = 0 when l + m' is odd.)
// ---------------------------------------------------------------------------
// Work-group: 64 consecutive m (lanes) of one m' (inverse) or one l
// (forward), the sum split over the four waves (every fourth term) and the
// wave sums added in LDS in wave order: four times the work-groups of one
// thread per output, which at L = 256 would leave one work-group per CU.
__global__ __launch_bounds__(256) void k_sht_inv_delta(int L, int Lf,
                                                       const double *__restrict__ delta,
                                                       const cd *__restrict__ fpad,
                                                       cd *__restrict__ F) {
    __shared__ double red[4][64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int mp = blockIdx.y, m = blockIdx.x * 64 + lane;
    double sx = 0.0, sy = 0.0;
    if (m < L) {
        int l0 = m > mp ? m : mp;
        if ((l0 + mp) & 1) ++l0;
        for (int l = l0 + 2 * w; l < L; l += 8) {
            const double *row = delta + delta_row32(l, mp);
            const double c = sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) * row[m] * row[0];
            const cd f = fpad[(size_t)l * Lf + m];
            sx += c * f.x;
            sy += c * f.y;
        }
    }
    red[w][lane][0] = sx;
    red[w][lane][1] = sy;
    __syncthreads();
    if (w == 0 && m < L) {
        double tx = red[0][lane][0], ty = red[0][lane][1];
        for (int q = 1; q < 4; ++q) {
            tx += red[q][lane][0];
            ty += red[q][lane][1];
        }
        F[(size_t)mp * L + m] = ipow(cd{tx, ty}, -m);
    }
}

__global__ __launch_bounds__(256) void k_sht_fwd_delta(int L, int Lf,
                                                       const double *__restrict__ delta,
                                                       const cd *__restrict__ Z,
                                                       cd *__restrict__ fpad) {
    __shared__ double red[4][64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int l = blockIdx.y, m = blockIdx.x * 64 + lane;
    double sx = 0.0, sy = 0.0;
    if (m <= l) {
        for (int mp = (l & 1) + 2 * w; mp <= l; mp += 8) {
            const double *row = delta + delta_row32(l, mp);
            const double c = row[m] * row[0];
            const cd z = Z[(size_t)mp * L + m];
            sx += c * z.x;
            sy += c * z.y;
        }
    }
    red[w][lane][0] = sx;
    red[w][lane][1] = sy;
    __syncthreads();
    if (w == 0 && m < L) {
        cd *o = fpad + (size_t)l * Lf + m;
        if (m > l) {
            *o = cd{0.0, 0.0};
        } else {
            double tx = red[0][lane][0], ty = red[0][lane][1];
            for (int q = 1; q < 4; ++q) {
                tx += red[q][lane][0];
                ty += red[q][lane][1];
            }
            *o = ipow(cscale(cd{tx, ty}, sqrt((2.0 * l + 1.0) / (4.0 * M_PI))), m);
        }
    }
}

hipError_t launch_sht_inv_delta(int L, int Lf, const double *delta, const cd *fpad, cd *F,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_sht_inv_delta, dim3((L + 63) / 64, L), dim3(256), 0, st, L, Lf, delta,
                       fpad, F);
    return hipGetLastError();
}
hipError_t launch_sht_fwd_delta(int L, int Lf, const double *delta, const cd *Z, cd *fpad,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_sht_fwd_delta, dim3((L + 63) / 64, L), dim3(256), 0, st, L, Lf, delta,
                       Z, fpad);
    return hipGetLastError();
}
// ---------------------------------------------------------------------------
// Spin-s SHT of complex maps (Sec. II-A: sY_lm = (-1)^s c_l d^l_{m,-s}(theta)
// e^{i m phi}, c_l = sqrt((2l+1)/(4 pi))), every m in (-L, L), column
// c = m + L - 1.  Through the Fourier factorisation of d with Delta = d(pi/2):
//   inverse: F[m'][c] = (-1)^s i^{-(m+s)} sum_{l >= max(|m|,|s|,m')}
//                         c_l Delta^l_{m'm} Delta^l_{m',-s} f_lm,   m' >= 0
//   forward: f_lm = (-1)^s i^{m+s} c_l sum_{m'<=l} Delta^l_{m'm} Delta^l_{m',-s} Z[m'][c]
// (the theta stage folds -m' onto m' with the parity (-1)^{m+s} of the
// product in m').  Quarter-table entries for negative indices:
// Delta^l_{m',-k} = (-1)^{l+m'} Delta^l_{m'k}.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double spin_sign(int l, int mp, int m, int s) {
    // sign of Delta^l_{m'm} Delta^l_{m',-s} relative to row[|m|] row[|s|]
    int q = 0;
    if (m < 0) q += l + mp;
    if (s > 0) q += l + mp;
    return (q & 1) ? -1.0 : 1.0;
}

__global__ __launch_bounds__(256) void k_sht_inv_delta_spin(int L, int s,
                                                            const double *__restrict__ delta,
                                                            const cd *__restrict__ flm,
                                                            cd *__restrict__ F) {
    __shared__ double red[4][64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int Nm = 2 * L - 1;
    const int mp = blockIdx.y, c = blockIdx.x * 64 + lane, m = c - (L - 1);
    const int am = m < 0 ? -m : m, as = s < 0 ? -s : s;
    double sx = 0.0, sy = 0.0;
    if (c < Nm) {
        int l0 = am > mp ? am : mp;
        if (as > l0) l0 = as;
        for (int l = l0 + w; l < L; l += 4) {
            const double *row = delta + delta_row32(l, mp);
            const double v = sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) * row[am] * row[as] *
                             spin_sign(l, mp, m, s);
            const cd f = flm[(size_t)l * l + l + m];
            sx += v * f.x;
            sy += v * f.y;
        }
    }
    red[w][lane][0] = sx;
    red[w][lane][1] = sy;
    __syncthreads();
    if (w == 0 && c < Nm) {
        double tx = red[0][lane][0], ty = red[0][lane][1];
        for (int q = 1; q < 4; ++q) {
            tx += red[q][lane][0];
            ty += red[q][lane][1];
        }
        cd v = ipow(cd{tx, ty}, -(m + s));
        if (s & 1) v = cd{-v.x, -v.y};
        F[(size_t)mp * Nm + c] = v;
    }
}

__global__ __launch_bounds__(256) void k_sht_fwd_delta_spin(int L, int s,
                                                            const double *__restrict__ delta,
                                                            const cd *__restrict__ Z,
                                                            cd *__restrict__ flm) {
    __shared__ double red[4][64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int Nm = 2 * L - 1;
    const int l = blockIdx.y, k = blockIdx.x * 64 + lane, m = k - l;  // m in [-l, l]
    const int am = m < 0 ? -m : m, as = s < 0 ? -s : s;
    const bool live = k <= 2 * l && as <= l;
    double sx = 0.0, sy = 0.0;
    if (live) {
        for (int mp = w; mp <= l; mp += 4) {
            const double *row = delta + delta_row32(l, mp);
            const double v = row[am] * row[as] * spin_sign(l, mp, m, s);
            const cd z = Z[(size_t)mp * Nm + m + L - 1];
            sx += v * z.x;
            sy += v * z.y;
        }
    }
    red[w][lane][0] = sx;
    red[w][lane][1] = sy;
    __syncthreads();
    if (w == 0 && k <= 2 * l) {
        cd v{0.0, 0.0};
        if (live) {
            double tx = red[0][lane][0], ty = red[0][lane][1];
            for (int q = 1; q < 4; ++q) {
                tx += red[q][lane][0];
                ty += red[q][lane][1];
            }
            v = ipow(cscale(cd{tx, ty}, sqrt((2.0 * l + 1.0) / (4.0 * M_PI))), m + s);
            if (s & 1) v = cd{-v.x, -v.y};
        }
        flm[(size_t)l * l + k] = v;
    }
}

hipError_t launch_sht_inv_delta_spin(int L, int s, const double *delta, const cd *flm, cd *F,
                                     hipStream_t st) {
    hipLaunchKernelGGL(k_sht_inv_delta_spin, dim3((2 * L - 1 + 63) / 64, L), dim3(256), 0, st,
                       L, s, delta, flm, F);
    return hipGetLastError();
}
hipError_t launch_sht_fwd_delta_spin(int L, int s, const double *delta, const cd *Z, cd *flm,
                                     hipStream_t st) {
    hipLaunchKernelGGL(k_sht_fwd_delta_spin, dim3((2 * L - 1 + 63) / 64, L), dim3(256), 0, st,
                       L, s, delta, Z, flm);
    return hipGetLastError();
}

// theta stage of the SHT: out[r][m] = (i^(p)) sum_k A^{p}[r][k] in[k][m],
// p = (m + par0) & 1, r < Mrows, k < Kdim, m < ncols (columns: m >= 0 of a
// real spin-0 map with par0 = 0; or every m of a spin-s map, column
// m + L - 1, with par0 the parity offset that makes p the parity of m + s).
// Work-group: an 8 x 8 output tile, K in chunks
// of 32 through LDS, each chunk's 32 terms split over the four waves (8 each)
// and the wave sums added in LDS in wave order; small tiles so that there are
// enough work-groups to fill the device at the band-limits of the SHT.
__global__ __launch_bounds__(256) void k_sht_theta(int L, int par0, int Mrows, int Kdim,
                                                   const double *__restrict__ Ae,
                                                   const double *__restrict__ Ao,
                                                   const cd *__restrict__ in,
                                                   cd *__restrict__ out) {
    __shared__ double As[2][8][33];
    __shared__ cd Bs[32][9];
    __shared__ double red[4][64][2];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tx = lane & 7, ty = lane >> 3;
    const int m = blockIdx.x * 8 + tx, r = blockIdx.y * 8 + ty;
    const int par = (m + par0) & 1;
    double re = 0.0, im = 0.0;
    for (int k0 = 0; k0 < Kdim; k0 += 32) {
        {
            const int i = threadIdx.x;  // 256 = 8 rows x 32 k
            const int rr = i >> 5, kk = i & 31;
            const int rg = blockIdx.y * 8 + rr, k = k0 + kk;
            const bool ok = rg < Mrows && k < Kdim;
            As[0][rr][kk] = ok ? Ae[(size_t)rg * Kdim + k] : 0.0;
            As[1][rr][kk] = ok ? Ao[(size_t)rg * Kdim + k] : 0.0;
            const int kb = i >> 3, mm = i & 7;  // 256 = 32 k x 8 m
            const int kg = k0 + kb, mg = blockIdx.x * 8 + mm;
            Bs[kb][mm] = (kg < Kdim && mg < L) ? in[(size_t)kg * L + mg] : cd{0.0, 0.0};
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kk = 8 * w + q;
            const double a = As[par][ty][kk];
            const cd b = Bs[kk][tx];
            re += a * b.x;
            im += a * b.y;
        }
        __syncthreads();
    }
    red[w][lane][0] = re;
    red[w][lane][1] = im;
    __syncthreads();
    if (w == 0 && r < Mrows && m < L) {
        double sr = red[0][lane][0], si = red[0][lane][1];
        for (int q = 1; q < 4; ++q) {
            sr += red[q][lane][0];
            si += red[q][lane][1];
        }
        out[(size_t)r * L + m] = par ? cd{-si, sr} : cd{sr, si};
    }
}

hipError_t launch_sht_theta(int L, int Mrows, int Kdim, int, const double *Aeven,
                            const double *Aodd, const cd *in, cd *out, hipStream_t st) {
    dim3 grid((L + 7) / 8, (Mrows + 7) / 8);
    hipLaunchKernelGGL(k_sht_theta, grid, dim3(256), 0, st, L, 0, Mrows, Kdim, Aeven, Aodd, in,
                       out);
    return hipGetLastError();
}
hipError_t launch_sht_theta_cols(int ncols, int par0, int Mrows, int Kdim, const double *Aeven,
                                 const double *Aodd, const cd *in, cd *out, hipStream_t st) {
    dim3 grid((ncols + 7) / 8, (Mrows + 7) / 8);
    hipLaunchKernelGGL(k_sht_theta, grid, dim3(256), 0, st, ncols, par0 & 1, Mrows, Kdim, Aeven,
                       Aodd, in, out);
    return hipGetLastError();
}

// f (flat l^2+l+m) <-> fpad [l][m], m >= 0.
// flm[l^2 + l + m] (=|+=) fpad[l][|m|] (negative m by the reality condition).
__global__ void k_flm_unpack(int L, const cd *__restrict__ fpad, cd *__restrict__ flm,
                             int accumulate) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L * L) return;
    int l = (int)sqrt((double)idx);
    while (l * l > idx) --l;
    while ((l + 1) * (l + 1) <= idx) ++l;
    const int m = idx - l * l - l;
    cd v = fpad[(size_t)l * L + (m < 0 ? -m : m)];
    if (m < 0) v = cscale(cconj(v), (m & 1) ? -1.0 : 1.0);
    flm[idx] = accumulate ? cadd(flm[idx], v) : v;
}
__global__ void k_flm_pack(int L, const cd *__restrict__ flm, cd *__restrict__ fpad) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L * L) return;
    const int l = idx / L, m = idx % L;
    fpad[idx] = (m <= l) ? flm[(size_t)l * l + l + m] : cd{0.0, 0.0};
}
hipError_t launch_flm_unpack(int L, const cd *fpad, cd *flm, int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_flm_unpack, dim3((L * L + 255) / 256), dim3(256), 0, st, L, fpad, flm,
                       accumulate);
    return hipGetLastError();
}
hipError_t launch_flm_pack(int L, const cd *flm, cd *fpad, hipStream_t st) {
    hipLaunchKernelGGL(k_flm_pack, dim3((L * L + 255) / 256), dim3(256), 0, st, L, flm, fpad);
    return hipGetLastError();
}

// Complex signals as two real parts: every f_lm (flat) <-> the coefficients
// a, b (padded [l][m], m >= 0) of the real and imaginary parts of the signal,
// each obeying the reality condition (x_{l,-m} = (-1)^m conj x_lm):
//   a_lm = (f_lm + (-1)^m conj f_{l,-m}) / 2,  b_lm = (f_lm - (-1)^m conj f_{l,-m}) / (2i),
//   f_lm = a_lm + i b_lm (every m, negative m of a and b by their reality).
__global__ void k_flm_split(int L, const cd *__restrict__ flm, cd *__restrict__ fa,
                            cd *__restrict__ fb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L * L) return;
    const int l = idx / L, m = idx % L;
    cd a{0.0, 0.0}, b{0.0, 0.0};
    if (m <= l) {
        const cd p = flm[(size_t)l * l + l + m];
        cd q = cconj(flm[(size_t)l * l + l - m]);
        if (m & 1) q = cd{-q.x, -q.y};
        a = cd{0.5 * (p.x + q.x), 0.5 * (p.y + q.y)};
        // (p - q) / (2i) = -i (p - q) / 2
        b = cd{0.5 * (p.y - q.y), -0.5 * (p.x - q.x)};
    }
    fa[idx] = a;
    fb[idx] = b;
}
__global__ void k_flm_combine(int L, const cd *__restrict__ fa, const cd *__restrict__ fb,
                              cd *__restrict__ flm, int accumulate) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L * L) return;
    int l = (int)sqrt((double)idx);
    while (l * l > idx) --l;
    while ((l + 1) * (l + 1) <= idx) ++l;
    const int m = idx - l * l - l, am = m < 0 ? -m : m;
    cd a = fa[(size_t)l * L + am], b = fb[(size_t)l * L + am];
    if (m < 0) {
        const double sg = (am & 1) ? -1.0 : 1.0;
        a = cd{sg * a.x, -sg * a.y};
        b = cd{sg * b.x, -sg * b.y};
    }
    const cd v{a.x - b.y, a.y + b.x};
    flm[idx] = accumulate ? cadd(flm[idx], v) : v;
}
hipError_t launch_flm_split(int L, const cd *flm, cd *fa, cd *fb, hipStream_t st) {
    hipLaunchKernelGGL(k_flm_split, dim3((L * L + 255) / 256), dim3(256), 0, st, L, flm, fa, fb);
    return hipGetLastError();
}
hipError_t launch_flm_combine(int L, const cd *fa, const cd *fb, cd *flm, int accumulate,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_flm_combine, dim3((L * L + 255) / 256), dim3(256), 0, st, L, fa, fb,
                       flm, accumulate);
    return hipGetLastError();
}

// Flat coefficients (index l^2 + l + m, the same for every band-limit):
// dst (=|+=) fac[l] src for l < Lphi, every m.
__global__ void k_scale_flat(int Lphi, const double *__restrict__ fac, const cd *__restrict__ src,
                             cd *__restrict__ dst, int accumulate) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Lphi * Lphi) return;
    int l = (int)sqrt((double)idx);
    while (l * l > idx) --l;
    while ((l + 1) * (l + 1) <= idx) ++l;
    const cd v = cscale(src[idx], fac[l]);
    dst[idx] = accumulate ? cadd(dst[idx], v) : v;
}
hipError_t launch_scale_flat(int Lphi, const double *fac, const cd *src, cd *dst, int accumulate,
                             hipStream_t st) {
    const int n = Lphi * Lphi;
    hipLaunchKernelGGL(k_scale_flat, dim3((n + 255) / 256), dim3(256), 0, st, Lphi, fac, src, dst,
                       accumulate);
    return hipGetLastError();
}

// dst[l][m] (=|+=) fac[l] * src[l][m] for l < Lphi, m <= l.
__global__ void k_scale_flm(int Lphi, int Lsrc, int Ldst, const double *__restrict__ fac,
                            const cd *__restrict__ src, cd *__restrict__ dst, int accumulate) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Lphi * Lphi) return;
    const int l = idx / Lphi, m = idx % Lphi;
    cd v = (m <= l) ? cscale(src[(size_t)l * Lsrc + m], fac[l]) : cd{0.0, 0.0};
    cd *o = dst + (size_t)l * Ldst + m;
    if (accumulate) {
        if (m <= l) *o = cadd(*o, v);
    } else {
        *o = v;
    }
}
hipError_t launch_scale_flm(int Lphi, int Lsrc, int Ldst, const double *fac, const cd *src,
                            cd *dst, int accumulate, hipStream_t st) {
    const int n = Lphi * Lphi;
    hipLaunchKernelGGL(k_scale_flm, dim3((n + 255) / 256), dim3(256), 0, st, Lphi, Lsrc, Ldst,
                       fac, src, dst, accumulate);
    return hipGetLastError();
}

__global__ void k_zero(cd *p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = cd{0.0, 0.0};
}
hipError_t launch_zero(cd *p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

__global__ void k_add(cd *dst, const cd *src, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = cadd(dst[i], src[i]);
}
hipError_t launch_add(cd *dst, const cd *src, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}

}  // namespace cvl
