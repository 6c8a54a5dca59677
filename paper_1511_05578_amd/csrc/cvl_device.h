// Device-side types and launch wrappers shared by the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace cvl {

struct __align__(16) cd {
    double x, y;
};

__host__ __device__ __forceinline__ cd mk(double x, double y) { return cd{x, y}; }
__host__ __device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__host__ __device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__host__ __device__ __forceinline__ cd cmul(cd a, cd b) {
    return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ __forceinline__ cd cconj(cd a) { return cd{a.x, -a.y}; }
__host__ __device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.x * s, a.y * s}; }
// Single-precision complex (the reduced-precision path: complex64 grids and
// cubes).  The same operations as cd, so templated code works on both.
struct __align__(8) cf {
    float x, y;
};
__host__ __device__ __forceinline__ cf cadd(cf a, cf b) { return cf{a.x + b.x, a.y + b.y}; }
__host__ __device__ __forceinline__ cf csub(cf a, cf b) { return cf{a.x - b.x, a.y - b.y}; }
__host__ __device__ __forceinline__ cf cmul(cf a, cf b) {
    return cf{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ __forceinline__ cf cconj(cf a) { return cf{a.x, -a.y}; }
__host__ __device__ __forceinline__ cf cscale(cf a, float s) { return cf{a.x * s, a.y * s}; }

// multiply by i^q (q taken mod 4, may be negative)
template <class C>
__host__ __device__ __forceinline__ C ipow(C a, int q) {
    switch (q & 3) {
        case 0: return a;
        case 1: return C{-a.y, a.x};
        case 2: return C{-a.x, -a.y};
        default: return C{a.y, -a.x};
    }
}

// Real component type of a complex type.
template <class C> struct RealOf;
template <> struct RealOf<cd> { using T = double; };
template <> struct RealOf<cf> { using T = float; };
template <class C> using real_t = typename RealOf<C>::T;

// Complex constant of type C from double components.
template <class C>
__host__ __device__ __forceinline__ C cmk(double x, double y) {
    return C{(real_t<C>)x, (real_t<C>)y};
}

// Precision of a curvelet call (values of cvl_params.precision).
enum Precision { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16X3 = 2 };

// Work-groups are dealt to the 8 XCDs (each with its own L2) round-robin by
// index.  Kernels whose neighbouring logical work-groups share data (cache
// lines of interleaved lines, Delta rows, cube rows, GEMM operand tiles)
// remap the hardware index so that each XCD gets a contiguous range of
// logical groups: hardware index b runs on XCD b % 8 and processes group
// start(b % 8) + b / 8.  A bijection of [0, n) for any n.
__device__ __forceinline__ int xcd_group(int b, int n) {
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// The same in chunks: logical groups come in runs of G that share data (all
// tiles of one m', say) while runs differ in cost; each XCD gets whole runs,
// dealt round-robin (run r to XCD r % 8), which keeps the sharing inside one
// L2 and the load balanced across XCDs.  Groups past the last full round of
// 8 runs keep their index.  A bijection of [0, n).
__device__ __forceinline__ int xcd_group_runs(int b, int n, int G) {
    const int full = (n / (8 * G)) * 8 * G;
    if (b >= full) return b;
    const int x = b & 7, i = b >> 3;
    return ((i / G) * 8 + x) * G + (i % G);
}

// Offset of block l in the quarter Delta table: sum_{k<l} (k+1)^2.
__host__ __device__ __forceinline__ int64_t delta_off(int l) {
    return (int64_t)l * (l + 1) * (2 * l + 1) / 6;
}
// The same offset in 32-bit arithmetic, exact for l <= 2048 (the table of
// L = 2048 has 2.86e9 < 2^32 entries): l (l + 1) / 2 is exact, its product with
// 2l + 1 is a multiple of 3, and a multiple of 3 below 2^32 divided by 3 is its
// product with the inverse of 3 modulo 2^32.  Row m' of block l starts at
// delta_off32(l) + m' (l + 1), also below 2^32.
__host__ __device__ __forceinline__ uint32_t delta_off32(int l) {
    const uint32_t t = (uint32_t)l * (uint32_t)(l + 1) / 2u;
    return t * (uint32_t)(2 * l + 1) * 0xAAAAAAABu;
}
__host__ __device__ __forceinline__ uint32_t delta_row32(int l, int mp) {
    return delta_off32(l) + (uint32_t)mp * (uint32_t)(l + 1);
}

// Device tables of one Bluestein DFT configuration (see host::Bluestein), in
// the working precision of the transform.
template <class C>
struct BlueT {
    int Nd, P, Kin, j0, Kout, k0;
    const C *pre, *post, *vhat, *tw;
};
using BluesteinDev = BlueT<cd>;
using BluesteinF = BlueT<cf>;

// Geometry of one curvelet scale (or one SHT / Wigner band-limit).
struct ScaleGeom {
    int L;     // band-limit L_j (alpha band-limit M = L_j too)
    int Nm;    // 2L - 1
    int h;     // (L-1)/2: even n = 2k with |k| <= h
    int Ne;    // 2h + 1 even-n values
    int Nep;   // Ne padded to a multiple of 32 (cube row length)
    int llo, lhi;  // l range where the curvelet kernel is non-zero (inclusive)
};

// Cube of the unrotated curvelets (Sec. III-A-1: kernel coefficients only at
// |n| = l, so every n in (-L, L) occurs): m >= 0 only (the reality condition
// gives m < 0), element (m, n) in row 2m + ((m + n) & 1), so that each row
// has one parity of m + n (the parity of the beta extension), at the column
// of n within its parity class: h + n/2 for even n, L/2 + (n - 1)/2 (floor)
// for odd n.  Row length Nep (>= both class sizes), 2L rows per plane.
__host__ __device__ __forceinline__ int unrot_col(const ScaleGeom &g, int n) {
    return (n & 1) ? (g.L >> 1) + ((n - 1) >> 1) : g.h + (n >> 1);
}
__host__ __device__ __forceinline__ size_t unrot_off(const ScaleGeom &g, int m, int n) {
    return (size_t)(2 * m + ((m + n) & 1)) * g.Nep + unrot_col(g, n);
}
// Columns in use in an unrotated-cube row: max(2h + 1, 2 (L/2)).
__host__ __device__ __forceinline__ int unrot_cols(const ScaleGeom &g) {
    const int e = 2 * g.h + 1, o = 2 * (g.L >> 1);
    return e > o ? e : o;
}

// ---- launch wrappers (defined in the .hip files) ----
hipError_t launch_delta_toprows(double *tab, int Lmax, hipStream_t st);
hipError_t launch_delta_fill(double *tab, int Lmax, hipStream_t st);

// Bluestein stages.  Each returns hipSuccess or the launch error.
hipError_t launch_inv_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *W1,
                            cd *W2, hipStream_t st);
// gamma stages: complex grids (zero imaginary parts) or real grids
hipError_t launch_inv_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *W2,
                            cd *grid, hipStream_t st);
hipError_t launch_inv_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *W2,
                            double *grid, hipStream_t st);
hipError_t launch_fwd_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *grid,
                            cd *V1, hipStream_t st);
hipError_t launch_fwd_gamma(const ScaleGeom &g, const BluesteinDev &B, const double *grid,
                            cd *V1, hipStream_t st);
hipError_t launch_fwd_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *V1,
                            cd *V2, hipStream_t st);
// beta DFT of the analysis as an FFT (line pairs of opposite m-parity):
// X [m'][m][nn] (m' >= 0) -> W1 [b][m][nn], b < L; B: length 2L-1, inputs
// j in (-L, L), outputs k' in (-L, L).
hipError_t launch_inv_beta_dft(const ScaleGeom &g, const BluesteinDev &B, const cd *X, cd *W1,
                               hipStream_t st);
hipError_t launch_inv_beta_dft(const ScaleGeom &g, const BluesteinF &B, const cf *X, cf *W1,
                               hipStream_t st);
// The same, each line's outputs contiguous in b: T[(m Nep + nn) L + b]; then
// launch_beta_lines_to_planes moves T into the W1 layout [b][m][nn].  Used
// in complex64 where one line fills a work-group (FFT size 4096).
hipError_t launch_inv_beta_dft_lines(const ScaleGeom &g, const BluesteinDev &B, const cd *X,
                                     cd *T, hipStream_t st);
hipError_t launch_inv_beta_dft_lines(const ScaleGeom &g, const BluesteinF &B, const cf *X,
                                     cf *T, hipStream_t st);
hipError_t launch_beta_lines_to_planes(const ScaleGeom &g, const cd *T, cd *W1, hipStream_t st);
hipError_t launch_beta_lines_to_planes(const ScaleGeom &g, const cf *T, cf *W1, hipStream_t st);

// The same four stages in single precision (complex64 cubes and grids).
hipError_t launch_inv_alpha(const ScaleGeom &g, const BluesteinF &B, const cf *W1, cf *W2,
                            hipStream_t st);
hipError_t launch_inv_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *W2, cf *grid,
                            hipStream_t st);
hipError_t launch_inv_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *W2,
                            float *grid, hipStream_t st);
hipError_t launch_fwd_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *grid, cf *V1,
                            hipStream_t st);
hipError_t launch_fwd_gamma(const ScaleGeom &g, const BluesteinF &B, const float *grid,
                            cf *V1, hipStream_t st);
hipError_t launch_fwd_alpha(const ScaleGeom &g, const BluesteinF &B, const cf *V1, cf *V2,
                            hipStream_t st);
hipError_t launch_sht_inv_phi(int L, const BluesteinDev &B, const cd *G, double *map,
                              hipStream_t st);
hipError_t launch_sht_fwd_phi(int L, const BluesteinDev &B, const double *map, cd *F1,
                              hipStream_t st);
// general complex Wigner transforms (all m, all n)
hipError_t launch_gen_inv_alpha(int L, int N, const BluesteinDev &B, const cd *W1,
                                cd *W2, hipStream_t st);
hipError_t launch_gen_inv_gamma(int L, int N, const BluesteinDev &B, const cd *W2,
                                cd *grid, hipStream_t st);
hipError_t launch_gen_fwd_gamma(int L, int N, const BluesteinDev &B, const cd *grid,
                                cd *V1, hipStream_t st);
hipError_t launch_gen_fwd_alpha(int L, int N, const BluesteinDev &B, const cd *V1,
                                cd *V2, hipStream_t st);

// Parity-folded beta stage as a real-matrix x complex-data GEMM:
// out[r][c] = sum_k A^{par(c)}[r][k] in[k][c] (times i for odd parity), rows
// r < M, k < K, complex columns c < ncols.  Column parity: (c / Nep) & 1 when
// mode == 0 (curvelet layout, parity of m), ((c / Nep) + (c % Nep) + par0) & 1
// when mode == 1 (general layout [m][n], parity of m + n).
hipError_t launch_beta_gemm(int M, int K, int ncols, int Nep, int mode, int par0,
                            const double *Aeven, const double *Aodd, const cd *in,
                            cd *out, hipStream_t st);

// The same GEMM (FP64) for the synthesis cube of the unrotated curvelets
// (2 L_j rows of Nep columns per plane): only the outputs at m' <= l, m <= l
// (l = |n|) are computed, the others are left unwritten.
hipError_t launch_beta_gemm_unrot_fwd(const ScaleGeom &g, const double *Aeven,
                                     const double *Aodd, const cd *in, cd *out, hipStream_t st);

// Reduced-precision dense stages (FP32 data; see kernels_mixed.hip).
hipError_t launch_beta_gemm_f32(int mode, int M, int K, int ncols, int Nep, const float *Aeven,
                                const float *Aodd, const cf *in, cf *out, hipStream_t st);
hipError_t launch_contract_inv_mx(int mode, const ScaleGeom &g, int Lf, const double *delta,
                                  const cd *fpad, const double *psi, cf *X, hipStream_t st);
hipError_t launch_contract_fwd_mx(int mode, const ScaleGeom &g, const double *delta,
                                  const cf *Z, const double *psi, cf *part, hipStream_t st);
hipError_t launch_reduce_fwd_mx(const ScaleGeom &g, int Lf, const cf *part, int ngroups,
                                cd *facc, hipStream_t st);

// Curvelet contractions.
hipError_t launch_contract_inv(const ScaleGeom &g, int Lf, const double *delta,
                               const cd *fpad, const double *psi, cd *X, hipStream_t st);
// part[m'][l][m] (one m' per group; the reductions take ngroups = L_j)
hipError_t launch_contract_fwd(const ScaleGeom &g, const double *delta, const cd *Z,
                               const double *psi, cd *part, hipStream_t st);
hipError_t launch_reduce_fwd(const ScaleGeom &g, int Lf, const cd *part, int ngroups,
                             cd *facc, hipStream_t st);

// Unrotated curvelets: the stages on the unrotated cube layout (unrot_off).
// W2 / V1 planes: [b][a][n], n in [0, L) (n < 0 by the reality condition).
// pd[m'][l] = Delta^l_{m'l} Psi~_{l,l}, L_j x L_j (Psi~_{l,-l} = (-1)^l Psi~_{l,l},
// zero for other n).
// dense: write every cube entry (the beta GEMM reads them all); otherwise only
// those with m <= l and m' <= l, the ones the beta FFT reads
hipError_t launch_unrot_contract_inv(const ScaleGeom &g, int Lf, const double *delta,
                                     const cd *fpad, const double *pd, cd *X, bool dense,
                                     hipStream_t st);
hipError_t launch_unrot_contract_inv(const ScaleGeom &g, int Lf, const double *delta,
                                     const cd *fpad, const double *pd, cf *X, bool dense,
                                     hipStream_t st);
hipError_t launch_unrot_contract_fwd(const ScaleGeom &g, int Lf, const double *delta,
                                     const cd *Y, const double *pd, cd *facc, hipStream_t st);
hipError_t launch_unrot_contract_fwd(const ScaleGeom &g, int Lf, const double *delta,
                                     const cf *Y, const double *pd, cd *facc, hipStream_t st);
hipError_t launch_unrot_inv_beta_dft(const ScaleGeom &g, const BluesteinDev &B, const cd *X,
                                     cd *W1, hipStream_t st);
hipError_t launch_unrot_inv_beta_dft(const ScaleGeom &g, const BluesteinF &B, const cf *X,
                                     cf *W1, hipStream_t st);
hipError_t launch_unrot_inv_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *W1,
                                  cd *W2, hipStream_t st);
hipError_t launch_unrot_inv_alpha(const ScaleGeom &g, const BluesteinF &B, const cf *W1,
                                  cf *W2, hipStream_t st);
hipError_t launch_unrot_inv_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *W2,
                                  cd *grid, hipStream_t st);
hipError_t launch_unrot_inv_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *W2,
                                  double *grid, hipStream_t st);
hipError_t launch_unrot_inv_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *W2,
                                  cf *grid, hipStream_t st);
hipError_t launch_unrot_inv_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *W2,
                                  float *grid, hipStream_t st);
hipError_t launch_unrot_fwd_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *grid,
                                  cd *V1, hipStream_t st);
hipError_t launch_unrot_fwd_gamma(const ScaleGeom &g, const BluesteinDev &B,
                                  const double *grid, cd *V1, hipStream_t st);
hipError_t launch_unrot_fwd_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *grid,
                                  cf *V1, hipStream_t st);
hipError_t launch_unrot_fwd_gamma(const ScaleGeom &g, const BluesteinF &B, const float *grid,
                                  cf *V1, hipStream_t st);
hipError_t launch_unrot_fwd_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *V1,
                                  cd *V2, hipStream_t st);
hipError_t launch_unrot_fwd_alpha(const ScaleGeom &g, const BluesteinF &B, const cf *V1,
                                  cf *V2, hipStream_t st);

// General Wigner contractions (dense F^l_mn).
hipError_t launch_gen_contract_inv(int L, int N, const double *delta, const cd *F,
                                   cd *X, hipStream_t st);
hipError_t launch_gen_contract_fwd(int L, int N, const double *delta, const cd *Z,
                                   cd *F, hipStream_t st);

// Rotated spin-s curvelets on the general layouts (see kernels_linalg.hip).
hipError_t launch_spin_contract_inv(int L, int llo, int lhi, const double *delta, const cd *flm,
                                    const double *psi, cd *X, hipStream_t st);
hipError_t launch_spin_reduce_fwd(int L, const cd *F, const double *psi, cd *acc, hipStream_t st);

// SHT helpers.
hipError_t launch_sht_inv_delta(int L, int Lf, const double *delta, const cd *fpad,
                                cd *F, hipStream_t st);
hipError_t launch_sht_theta(int L, int Mrows, int Kdim, int mode_fwd, const double *Aeven,
                            const double *Aodd, const cd *in, cd *out, hipStream_t st);
hipError_t launch_sht_fwd_delta(int L, int Lf, const double *delta, const cd *Z, cd *fpad,
                                hipStream_t st);
hipError_t launch_flm_unpack(int L, const cd *fpad, cd *flm, int accumulate, hipStream_t st);
hipError_t launch_flm_pack(int L, const cd *flm, cd *fpad, hipStream_t st);
hipError_t launch_scale_flm(int Lphi, int Lsrc, int Ldst, const double *fac, const cd *src,
                            cd *dst, int accumulate, hipStream_t st);
// Spin-s SHT of complex maps (every m, columns m + L - 1 of rows of 2L - 1).
hipError_t launch_sht_inv_delta_spin(int L, int s, const double *delta, const cd *flm, cd *F,
                                     hipStream_t st);
hipError_t launch_sht_fwd_delta_spin(int L, int s, const double *delta, const cd *Z, cd *flm,
                                     hipStream_t st);
hipError_t launch_sht_theta_cols(int ncols, int par0, int Mrows, int Kdim, const double *Aeven,
                                 const double *Aodd, const cd *in, cd *out, hipStream_t st);
hipError_t launch_sht_inv_phi_cplx(int L, const BluesteinDev &B, const cd *G, cd *map,
                                   hipStream_t st);
hipError_t launch_sht_fwd_phi_cplx(int L, const BluesteinDev &B, const cd *map, cd *F1,
                                   hipStream_t st);
// Complex signals as two real parts (coefficient sets a, b with the reality
// condition, padded [l][m >= 0]); flat coefficients of every m.
hipError_t launch_flm_split(int L, const cd *flm, cd *fa, cd *fb, hipStream_t st);
hipError_t launch_flm_combine(int L, const cd *fa, const cd *fb, cd *flm, int accumulate,
                              hipStream_t st);
hipError_t launch_scale_flat(int Lphi, const double *fac, const cd *src, cd *dst, int accumulate,
                             hipStream_t st);
// gamma stages of complex grids: W2a / V1a carry the real part's
// coefficients, W2b / V1b the imaginary part's.
hipError_t launch_inv_gamma_cplx(const ScaleGeom &g, const BluesteinDev &B, const cd *W2a,
                                 const cd *W2b, cd *grid, hipStream_t st);
hipError_t launch_inv_gamma_cplx(const ScaleGeom &g, const BluesteinF &B, const cf *W2a,
                                 const cf *W2b, cf *grid, hipStream_t st);
hipError_t launch_fwd_gamma_cplx(const ScaleGeom &g, const BluesteinDev &B, const cd *grid,
                                 cd *V1a, cd *V1b, hipStream_t st);
hipError_t launch_fwd_gamma_cplx(const ScaleGeom &g, const BluesteinF &B, const cf *grid,
                                 cf *V1a, cf *V1b, hipStream_t st);
hipError_t launch_unrot_inv_gamma_cplx(const ScaleGeom &g, const BluesteinDev &B,
                                       const cd *W2a, const cd *W2b, cd *grid, hipStream_t st);
hipError_t launch_unrot_inv_gamma_cplx(const ScaleGeom &g, const BluesteinF &B,
                                       const cf *W2a, const cf *W2b, cf *grid, hipStream_t st);
hipError_t launch_unrot_fwd_gamma_cplx(const ScaleGeom &g, const BluesteinDev &B,
                                       const cd *grid, cd *V1a, cd *V1b, hipStream_t st);
hipError_t launch_unrot_fwd_gamma_cplx(const ScaleGeom &g, const BluesteinF &B,
                                       const cf *grid, cf *V1a, cf *V1b, hipStream_t st);
hipError_t launch_zero(cd *p, size_t n, hipStream_t st);
hipError_t launch_add(cd *dst, const cd *src, size_t n, hipStream_t st);  // dst += src

}  // namespace cvl
