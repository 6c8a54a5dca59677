// Reduced-precision dense kernels of the curvelet transform on gfx950.
//
// The l-contractions of the analysis and of the synthesis run on the matrix
// cores with FP32 accumulation, in one of two operand precisions:
//   * FP32: v_mfma_f32_16x16x4_f32;
//   * BF16x3: each FP32 operand split as x = hi + lo (two bfloat16, hi the
//     nearest bfloat16 to x, lo the nearest to x - hi) and a*b taken as
//     hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 (the lo*lo term,
//     relative size 2^-16, is dropped).
// Delta stays FP64 in HBM; each element is multiplied by its FP64 partner
// (f_lm, or Psi) before rounding to FP32, so the operands carry one rounding.
// The beta stage is a GEMM on the matrix cores in the same operand precision
// (FP32, or split BF16); the FFT stages run in FP32 elsewhere.
//
// Lane layouts (16 x 16 output block, 64 lanes, lane = 16 q + i, i < 16):
//   f32 16x16x4:   A[i][q], B[q][i];           D[4q + r][i] in result reg r
//   bf16 16x16x32: A[i][8q + e], B[8q + e][i]; D[4q + r][i]
// For K = 32 both modes give lane (q, i) the operand elements k = 8q + e,
// e < 8 (the FP32 mode issues one K = 4 product per e; the order of the
// terms of a sum over k does not change the sum's definition).
#include "cvl_device.h"

namespace cvl {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// One lane's eight K-elements of an MFMA operand, in the working format.
template <int MODE>
struct Op;
template <>
struct Op<PREC_FP32> {
    float v[8];
    __device__ __forceinline__ void set(const float x[8]) {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = x[e];
    }
};
template <>
struct Op<PREC_BF16X3> {
    bf8v hi, lo;
    __device__ __forceinline__ void set(const float x[8]) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const __bf16 h = (__bf16)x[e];
            hi[e] = h;
            lo[e] = (__bf16)(x[e] - (float)h);
        }
    }
};

// acc += A B over the 32 K-elements of a chunk.
__device__ __forceinline__ f4v mma32(const Op<PREC_FP32> &a, const Op<PREC_FP32> &b, f4v acc) {
#pragma unroll
    for (int e = 0; e < 8; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[e], b.v[e], acc, 0, 0, 0);
    return acc;
}
__device__ __forceinline__ f4v mma32(const Op<PREC_BF16X3> &a, const Op<PREC_BF16X3> &b,
                                     f4v acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, acc, 0, 0, 0);
    return acc;
}

// Operand loads of one K tile of the FP32 beta GEMMs (128 rows x 32 k of A,
// 32 k x 64 real columns of the input) into registers: A as four 16-byte
// pieces along k (eight threads per 128-byte row segment; single values when
// K is not a multiple of 4), the input as eight single values down k (a wave
// reads one 256-byte row segment per load), so that both land in LDS
// k-contiguous per row and column.  Indices are clamped into the operands, so
// every load is in bounds and none is guarded: no load result is consumed,
// and so waited for, before the next iteration stores the registers to LDS.
// Rows past M only feed outputs that are not stored; k past K is zeroed in A
// when the tile is staged (the clamped input rows it meets are finite).
// Columns are always whole (ncols is a multiple of 32).
template <bool KV4>
__device__ __forceinline__ void beta_fetch_f32(const float *__restrict__ A,
                                               const float *__restrict__ in, int M, int K,
                                               size_t ld, int r0, int c0, int k0, int tid,
                                               float4 (&ra)[4], float (&rb)[8]) {
    const int ar = tid >> 3, ak = 4 * (tid & 7);   // A: rows ar + 32 q, k0 + ak .. + 3
    const int bc = tid & 63, bk = 4 * (tid >> 6);  // input: column bc, k0 + bk + 16 g + e
    const float *Arow = A + (size_t)r0 * K;
    const int rmax = M - 1 - r0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t rofs = (uint32_t)min(ar + 32 * q, rmax) * (uint32_t)K;
        if constexpr (KV4) {
            ra[q] = *reinterpret_cast<const float4 *>(Arow + rofs + min(k0 + ak, K - 4));
        } else {
            float x[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = Arow[rofs + min(k0 + ak + e, K - 1)];
            ra[q] = make_float4(x[0], x[1], x[2], x[3]);
        }
    }
    const float *pb = in + (size_t)k0 * ld + 2 * (size_t)c0 + bc;
    const int kmax = K - 1 - k0;
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            rb[4 * g + e] = pb[(uint32_t)min(bk + 16 * g + e, kmax) * (uint32_t)ld];
}

// One K tile in LDS, k-contiguous: As[row][k], Bt[column][k]; rows of 36
// floats keep the 16-byte writes and reads free of bank conflicts.
struct BetaTileF32 {
    float As[128][36];
    float Bt[64][36];
};

__device__ __forceinline__ void beta_stage_f32(BetaTileF32 &t, float4 (&ra)[4],
                                               const float (&rb)[8], int tid, int k0, int K) {
    const int ar = tid >> 3, ak = 4 * (tid & 7);
    const int bc = tid & 63, bk = 4 * (tid >> 6);
    if (k0 + 32 > K) {  // last, partial K tile (uniform): zero A past K
        const int kk = k0 + ak;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ra[q].x = kk < K ? ra[q].x : 0.f;
            ra[q].y = kk + 1 < K ? ra[q].y : 0.f;
            ra[q].z = kk + 2 < K ? ra[q].z : 0.f;
            ra[q].w = kk + 3 < K ? ra[q].w : 0.f;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<float4 *>(&t.As[ar + 32 * q][ak]) = ra[q];
#pragma unroll
    for (int g = 0; g < 2; ++g)
        *reinterpret_cast<float4 *>(&t.Bt[bc][bk + 16 * g]) =
            make_float4(rb[4 * g], rb[4 * g + 1], rb[4 * g + 2], rb[4 * g + 3]);
}

__device__ __forceinline__ float f4get(const float4 &v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}

// A lane's eight k of one 16-row (or 16-column) block: k = 8 lq + e.  The
// MFMA of step e sums its four k-lanes lq, so a K tile's 32 k are covered
// once, in an order that lets each lane read its eight k as two 16-byte words.
__device__ __forceinline__ void beta_operand(const float (&row)[36], int lq, float (&x)[8]) {
    const float4 *src = reinterpret_cast<const float4 *>(&row[8 * lq]);
    const float4 x0 = src[0], x1 = src[1];
    x[0] = x0.x; x[1] = x0.y; x[2] = x0.z; x[3] = x0.w;
    x[4] = x1.x; x[5] = x1.y; x[6] = x1.z; x[7] = x1.w;
}

// The factor i of the odd beta parity, (re, im) -> (-im, re), applied to the
// result of the GEMM on the raw columns (it is linear in them): in the 16 x 16
// MFMA output layout column li holds re at even li, im at odd li, and the
// partner column sits in lane ^ 1.
__device__ __forceinline__ void beta_odd_parity(f4v (&acc)[2][4], int li) {
    const float sg = (li & 1) ? 1.f : -1.f;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = sg * __shfl_xor(acc[i][j][r], 1);
}

__device__ __forceinline__ void beta_store_f32(const f4v (&acc)[2][4], float *__restrict__ out,
                                               int M, size_t ld, int r0, int c0, int w, int li,
                                               int lq) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + 32 * w + 16 * i + 4 * lq + r;
                const size_t col = 2 * (size_t)c0 + 16 * j + li;
                if (row < M && col < ld) out[(size_t)row * ld + col] = acc[i][j][r];
            }
}

// ---------------------------------------------------------------------------
// Parity-folded beta stage in FP32 (curvelet layout, Nep % 32 == 0):
//   out[r][c] = (i^par(c)) sum_k A^{par(c)}[r][k] in[k][c].
// Tile 128 rows x 64 real columns x 32 k; wave w owns rows [32w, 32w+32) as
// 2 x 4 blocks of v_mfma_f32_16x16x4_f32 (MODE PREC_FP32) or of split-BF16
// v_mfma_f32_16x16x32_bf16 triples (PREC_BF16X3, operands split in
// registers).  The next K tile is loaded into registers while the current one
// is multiplied; the odd parity's factor i is applied to the result.
// ---------------------------------------------------------------------------
template <int MODE, bool KV4>
__global__ __launch_bounds__(256, MODE == PREC_FP32 ? 4 : 3) void k_beta_mfma_mx(int M, int K, int ncols, int Nep,
                                                      const float *__restrict__ Ae,
                                                      const float *__restrict__ Ao,
                                                      const float *__restrict__ in,
                                                      float *__restrict__ out) {
    __shared__ __align__(16) BetaTileF32 t;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // logical tile (row tile fastest: the row tiles of one column tile share
    // its B operand, so they run together on one XCD)
    const int nrt = (M + 127) / 128;
    const int lg = xcd_group(blockIdx.x, gridDim.x);
    const int r0 = (lg % nrt) * 128;
    const int c0 = (lg / nrt) * 32;  // complex column base
    const size_t ld = 2 * (size_t)ncols;
    const int par = (c0 / Nep) & 1;
    const float *A = par ? Ao : Ae;
    f4v acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    const int li = lane & 15, lq = lane >> 4;
    float4 ra[4];
    float rb[8];
    beta_fetch_f32<KV4>(A, in, M, K, ld, r0, c0, 0, tid, ra, rb);
    for (int k0 = 0; k0 < K; k0 += 32) {
        beta_stage_f32(t, ra, rb, tid, k0, K);
        __syncthreads();
        if (k0 + 32 < K) beta_fetch_f32<KV4>(A, in, M, K, ld, r0, c0, k0 + 32, tid, ra, rb);
        if constexpr (MODE == PREC_FP32) {
            // two halves of four k (one 16-byte read per operand), step e
            // outermost: eight independent accumulators between two products
            // into the same one
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float4 a4[2], b4[4];
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    a4[i] = *reinterpret_cast<const float4 *>(&t.As[32 * w + 16 * i + li][8 * lq + 4 * h]);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    b4[j] = *reinterpret_cast<const float4 *>(&t.Bt[16 * j + li][8 * lq + 4 * h]);
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int i = 0; i < 2; ++i)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                f4get(a4[i], e), f4get(b4[j], e), acc[i][j], 0, 0, 0);
            }
        } else {
            Op<MODE> aop[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                float x[8];
                beta_operand(t.As[32 * w + 16 * i + li], lq, x);
                aop[i].set(x);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float x[8];
                beta_operand(t.Bt[16 * j + li], lq, x);
                Op<MODE> bop;
                bop.set(x);
#pragma unroll
                for (int i = 0; i < 2; ++i) acc[i][j] = mma32(aop[i], bop, acc[i][j]);
            }
        }
        __syncthreads();
    }
    if (par) beta_odd_parity(acc, li);
    beta_store_f32(acc, out, M, ld, r0, c0, w, li, lq);
}

hipError_t launch_beta_gemm_f32(int mode, int M, int K, int ncols, int Nep, const float *Aeven,
                                const float *Aodd, const cf *in, cf *out, hipStream_t st) {
    // whole 32-column tiles; 32 input rows of 2 ncols floats within 32-bit offsets
    if (Nep % 32 != 0 || ncols % 32 != 0 || M < 1 || K < 1 ||
        (uint64_t)32 * 2 * (uint64_t)ncols >= ((uint64_t)1 << 32))
        return hipErrorInvalidValue;
    dim3 g((ncols / 32) * ((M + 127) / 128));
    const bool v4 = K % 4 == 0;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, g, dim3(256), 0, st, M, K, ncols, Nep, Aeven, Aodd,
                           (const float *)in, (float *)out);
    };
    if (mode == PREC_BF16X3)
        v4 ? go(k_beta_mfma_mx<PREC_BF16X3, true>) : go(k_beta_mfma_mx<PREC_BF16X3, false>);
    else
        v4 ? go(k_beta_mfma_mx<PREC_FP32, true>) : go(k_beta_mfma_mx<PREC_FP32, false>);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Analysis contraction of one scale, reduced precision (cube X in complex64):
//   P_e/o[m][k] = sum_{l even/odd} (Delta^l_{m'm} f_lm) (Delta^l_{m',2k} Psi_{l,2k})
//   X[m'][m][h+k] = (-1)^k i^{-m} (P_e + P_o)
//   X[m'][m][h-k] = (-1)^k i^{-m} (-1)^{m'} (P_e - P_o)
// for l in [max(llo, m', m, 2k), lhi].  Work-group: one m', 64 m x 32 k.  The
// GEMM rows are (component c, m): A[(c, m)][l] = c-part of Delta f, B[l][k].
// A chunk covers 64 consecutive l (32 of each parity = one K = 32 step).
// Wave w: parity p = w & 1, component c = w >> 1; 64 rows x 32 columns as
// 4 x 2 blocks.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_contract_inv_mx(ScaleGeom g, int Lf,
                                                         const double *__restrict__ delta,
                                                         const cd *__restrict__ fpad,
                                                         const double *__restrict__ psi,
                                                         cf *__restrict__ X) {
    // As[p][c][i][mm] (l = lb + p + 2i), Bs[p][i][kk]; reused for the results
    // R[p][c][mm][kk] after the l loop.
    // Row pads (66, 34) put the four 16-lane groups of an operand read on
    // disjoint LDS banks.
    __shared__ float smem[2 * 2 * 32 * 66 + 2 * 32 * 34];
    float(*As)[2][32][66] = reinterpret_cast<float(*)[2][32][66]>(smem);
    float(*Bs)[32][34] = reinterpret_cast<float(*)[32][34]>(smem + 2 * 2 * 32 * 66);
    const int L = g.L, h = g.h;
    // logical tile: k tile fastest, then m tile, then m' (see k_contract_inv_mfma)
    const int nkt = (h + 1 + 31) / 32, nmt = (L + 63) / 64;
    const int lg = xcd_group_runs(blockIdx.x, gridDim.x, nkt * nmt);
    const int mp = lg / (nkt * nmt);
    const int m0 = ((lg / nkt) % nmt) * 64, k0 = (lg % nkt) * 32;
    // w is the same across a wave: readfirstlane lets the compiler keep it,
    // the l of each staged row and that row's offsets in scalar registers.
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int p = w & 1, c = w >> 1;
    const int li = lane & 15, lq = lane >> 4;
    f4v acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
    int lstart = g.llo;
    if (mp > lstart) lstart = mp;
    if (m0 > lstart) lstart = m0;
    if (2 * k0 > lstart) lstart = 2 * k0;
    const int lend = g.lhi;
    // l chunks from the top down, at boundaries common to the whole launch:
    // the tiles of one m tile (and of one k tile) then read the same Delta
    // rows at about the same time, while the L2 still holds them (tiles
    // differ only in where they stop, at their lstart).
    const int ltop = (lend + 2) & ~1;  // even, past lend
    const int m = m0 + lane, hi = lane >> 5, k = k0 + (lane & 31);
    for (int lb = ltop - 64; lb + 63 >= lstart; lb -= 64) {
        // A: 2 parities x 32 l x 64 m complex, 16 per thread in two batches
        // of 8 loads in flight.  Element q: parity q >> 3, i = w + 4 (q & 7),
        // mm = lane (l uniform over the wave).  Loads out of range read
        // element 0 and are replaced by 0.
#pragma unroll
        for (int hb = 0; hb < 16; hb += 8) {
            double dv[8];
            cd fv[8];
            uint32_t okb = 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int q = hb + e, l = lb + (q >> 3) + 2 * (w + 4 * (q & 7));
                const bool lok = l >= lstart && l <= lend;
                const bool ok = lok && m <= l && m < L;
                const uint32_t dro = lok ? delta_row32(l, mp) : 0u;
                const uint32_t fro = lok ? (uint32_t)(l * Lf) : 0u;
                const uint32_t mi = ok ? (uint32_t)m : 0u;
                dv[e] = delta[(size_t)(dro + mi)];
                fv[e] = fpad[(size_t)(fro + mi)];
                okb |= ok ? 1u << e : 0u;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int q = hb + e, pp = q >> 3, i = w + 4 * (q & 7);
                const bool ok = (okb >> e) & 1u;
                As[pp][0][i][lane] = ok ? (float)(dv[e] * fv[e].x) : 0.f;
                As[pp][1][i][lane] = ok ? (float)(dv[e] * fv[e].y) : 0.f;
            }
        }
        // B: 2 parities x 32 l x 32 k, 8 per thread, all in flight together.
        // Element e: parity e >> 2, i = 2 w + (lane >> 5) + 8 (e & 3), kk =
        // lane & 31: two l per wave, both row offsets scalar.
        {
            double dv[8], pv[8];
            uint32_t okb = 0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int la = lb + (e >> 2) + 2 * (2 * w + 8 * (e & 3));  // l at hi = 0
                const bool ok0 = la >= lstart && la <= lend;
                const bool ok1 = la + 2 >= lstart && la + 2 <= lend;
                const uint32_t d0 = ok0 ? delta_row32(la, mp) : 0u;
                const uint32_t d1 = ok1 ? delta_row32(la + 2, mp) : 0u;
                const uint32_t p0 = ok0 ? (uint32_t)(la * (h + 1)) : 0u;
                const uint32_t p1 = ok1 ? (uint32_t)((la + 2) * (h + 1)) : 0u;
                const int l = la + 2 * hi;
                const bool ok = (hi ? ok1 : ok0) && k <= h && 2 * k <= l;
                const uint32_t ki = ok ? (uint32_t)k : 0u;
                dv[e] = delta[(size_t)((hi ? d1 : d0) + 2u * ki)];
                pv[e] = psi[(size_t)((hi ? p1 : p0) + ki)];
                okb |= ok ? 1u << e : 0u;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int pp = e >> 2, i = 2 * w + hi + 8 * (e & 3);
                Bs[pp][i][lane & 31] = ((okb >> e) & 1u) ? (float)(dv[e] * pv[e]) : 0.f;
            }
        }
        __syncthreads();
        Op<MODE> bop[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = Bs[p][8 * lq + e][16 * cb + li];
            bop[cb].set(x);
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = As[p][c][8 * lq + e][16 * rb + li];
            Op<MODE> aop;
            aop.set(x);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = mma32(aop, bop[cb], acc[rb][cb]);
        }
        __syncthreads();
    }
    // results to LDS: R[p][c][mm][kk]
    float(*R)[2][64][33] = reinterpret_cast<float(*)[2][64][33]>(smem);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) R[p][c][16 * rb + 4 * lq + r][16 * cb + li] = acc[rb][cb][r];
    __syncthreads();
    const int Nep = g.Nep;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int idx = tid + 256 * q;
        const int kk = idx & 31, mm = idx >> 5;
        const int m = m0 + mm, k = k0 + kk;
        if (m >= L || k > h) continue;
        const cf pe = cf{R[0][0][mm][kk], R[0][1][mm][kk]};
        const cf po = cf{R[1][0][mm][kk], R[1][1][mm][kk]};
        const float sk = (k & 1) ? -1.f : 1.f;
        cf *row = X + ((size_t)mp * L + m) * Nep;
        row[h + k] = ipow(cscale(cadd(pe, po), sk), -m);
        if (k > 0) {
            const float sm = (mp & 1) ? -sk : sk;
            row[h - k] = ipow(cscale(csub(pe, po), sm), -m);
        }
    }
}

hipError_t launch_contract_inv_mx(int mode, const ScaleGeom &g, int Lf, const double *delta,
                                  const cd *fpad, const double *psi, cf *X, hipStream_t st) {
    const int nkt = (g.h + 1 + 31) / 32;
    dim3 grid(((g.L + 63) / 64) * nkt * g.L);
    if (mode == PREC_FP32)
        hipLaunchKernelGGL(k_contract_inv_mx<PREC_FP32>, grid, dim3(256), 0, st, g, Lf, delta,
                           fpad, psi, X);
    else
        hipLaunchKernelGGL(k_contract_inv_mx<PREC_BF16X3>, grid, dim3(256), 0, st, g, Lf, delta,
                           fpad, psi, X);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Synthesis contraction of one scale, reduced precision (cube Z in complex64):
//   f_lm = i^m sum_{m'} Delta^l_{m'm} sum_k Z^{par(l)}[m'][m][k] B'[k][l],
//   B'[k][l] = (-1)^k Delta^l_{m',2k} Psi_{l,2k},
//   Z^{+/-}[m'][m][k] = Z[m'][m][h+k] +/- (-1)^{m'} Z[m'][m][h-k]  (k > 0),
//   Z^{+/-}[m'][m][0] = Z[m'][m][h].
// Work-group tile: 64 l (32 of each parity, l = l0 + par + 2i) x 64 m for one
// m': T[l][m] = sum_k B'[k][l] Z^par[m][k] on the matrix cores (K chunks of
// 32), then part[m'][l][m] = Delta^l_{m'm} T[l][m] (complex64) in the output
// layout.  Wave (wp, wm): parity wp, 32 l x 32 m, [2 l blocks][2 m blocks]
// [re/im].  The partials are summed over m' in FP64 afterwards.  With no
// running sum over m' held, the next K chunk's operands (raw Delta, Psi and
// the two Z half rows) are prefetched into registers while the current chunk
// is multiplied.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256, 2) void k_contract_fwd_mx1(ScaleGeom g,
                                                           const double *__restrict__ delta,
                                                           const cf *__restrict__ Z,
                                                           const double *__restrict__ psi,
                                                           cf *__restrict__ part) {
    __shared__ float Bt[2][32][34];       // [par][k][i]
    __shared__ float Zs[2][2][32][66];    // [par][re/im][k][mm]
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
    const float smp = (mp & 1) ? -1.f : 1.f;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wp = w & 1, wm = w >> 1;
    const int li = lane & 15, lq = lane >> 4;
    // staging assignment: element q of this thread
    //   B'^T: kk = idx & 31, i = (idx >> 5) & 31, par = idx >> 10 (l = l0 + par + 2 i)
    //   Z:    kk = idx & 31, mm = idx >> 5
    double rd[8], rp[8];
    cf rzp[8], rzn[8];
    const cf *zt = Z + ((size_t)mp * L + m0) * Nep;  // cube row (m', m0)
    auto fetch = [&](int kb) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx & 31, i = (idx >> 5) & 31, par = idx >> 10;
            const int l = l0 + par + 2 * i, k = kb + kk;
            const bool ok = k <= kmax && l <= g.lhi && 2 * k <= l && mp <= l;
            rd[q] = ok ? delta[(size_t)(delta_row32(l, mp) + (uint32_t)(2 * k))] : 0.0;
            rp[q] = ok ? psi[(size_t)(uint32_t)(l * (h + 1) + k)] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx & 31, mm = idx >> 5;
            const int k = kb + kk, m = m0 + mm;
            const bool ok = k <= kmax && m < L;
            // 32-bit offsets inside the tile's rows (64 rows of Nep <= 1024)
            const cf *row = zt + (uint32_t)((ok ? mm : 0) * Nep);
            rzp[q] = ok ? row[h + k] : cf{0.f, 0.f};
            rzn[q] = (ok && k > 0) ? row[h - k] : cf{0.f, 0.f};
        }
    };
    f4v t[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) t[a][b][cc] = f4v{0.f, 0.f, 0.f, 0.f};
    fetch(0);
    for (int kb = 0; kb <= kmax; kb += 32) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx & 31, i = (idx >> 5) & 31, par = idx >> 10;
            const double dv = rd[q] * rp[q];  // formed in FP64, rounded once
            Bt[par][kk][i] = (float)((kk & 1) ? -dv : dv);  // (-1)^k, kb even
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx & 31, mm = idx >> 5;
            // k = 0: Z^+ = Z^- = Z[h] (rzn is zero there)
            const cf zn = cscale(rzn[q], smp);
            const cf vp = cadd(rzp[q], zn), vm = csub(rzp[q], zn);
            Zs[0][0][kk][mm] = vp.x;
            Zs[0][1][kk][mm] = vp.y;
            Zs[1][0][kk][mm] = vm.x;
            Zs[1][1][kk][mm] = vm.y;
        }
        __syncthreads();
        if (kb + 32 <= kmax) fetch(kb + 32);
        Op<MODE> aop[2];
#pragma unroll
        for (int lf = 0; lf < 2; ++lf) {
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = Bt[wp][8 * lq + e][16 * lf + li];
            aop[lf].set(x);
        }
#pragma unroll
        for (int mj = 0; mj < 2; ++mj)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                float x[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = Zs[wp][cc][8 * lq + e][32 * wm + 16 * mj + li];
                Op<MODE> bop;
                bop.set(x);
#pragma unroll
                for (int lf = 0; lf < 2; ++lf) t[lf][mj][cc] = mma32(aop[lf], bop, t[lf][mj][cc]);
            }
        __syncthreads();
    }
    // part[m'][l][m] = Delta^l_{m'm} T: output row 4 lq + r of block lf, column li.
    // The 8 Delta values of a block are loaded together (out-of-range ones
    // read element 0 and are replaced by 0 when used), then the products stored.
    cf *pbase = part + (size_t)mp * L * L;
#pragma unroll
    for (int lf = 0; lf < 2; ++lf) {
        double dd[4][2];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int l = l0 + wp + 2 * (16 * lf + 4 * lq + r);
            const uint32_t dro = (l <= g.lhi && mp <= l) ? delta_row32(l, mp) : 0u;
#pragma unroll
            for (int mj = 0; mj < 2; ++mj) {
                const int m = m0 + 32 * wm + 16 * mj + li;
                const bool ok = l <= g.lhi && m < L && mp <= l && m <= l;
                dd[r][mj] = delta[(size_t)(dro + (ok ? (uint32_t)m : 0u))];
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int l = l0 + wp + 2 * (16 * lf + 4 * lq + r);
            if (l > g.lhi) continue;
#pragma unroll
            for (int mj = 0; mj < 2; ++mj) {
                const int m = m0 + 32 * wm + 16 * mj + li;
                if (m >= L) continue;
                const float d = (mp <= l && m <= l) ? (float)dd[r][mj] : 0.f;
                pbase[(uint32_t)(l * L + m)] = cf{d * t[lf][mj][0][r], d * t[lf][mj][1][r]};
            }
        }
    }
}

hipError_t launch_contract_fwd_mx(int mode, const ScaleGeom &g, const double *delta,
                                  const cf *Z, const double *psi, cf *part, hipStream_t st) {
    if (g.lhi < g.llo) return hipSuccess;
    const int nl = g.lhi - (g.llo & ~1) + 1;
    dim3 grid(((g.L + 63) / 64) * ((nl + 63) / 64) * g.L);
    if (mode == PREC_FP32)
        hipLaunchKernelGGL(k_contract_fwd_mx1<PREC_FP32>, grid, dim3(256), 0, st, g, delta, Z,
                           psi, part);
    else
        hipLaunchKernelGGL(k_contract_fwd_mx1<PREC_BF16X3>, grid, dim3(256), 0, st, g, delta, Z,
                           psi, part);
    return hipGetLastError();
}

}  // namespace cvl
