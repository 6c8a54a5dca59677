/*
 * curvelet.h - C ABI of the MI355X (gfx950) spherical curvelet transform.
 *
 * Transform: second-generation scale-discretised curvelets on the sphere
 * (Chan, Leistedt, Kitching, McEwen, IEEE TSP 65(1), 2017).  Every numerical
 * step runs in hand-written HIP kernels; the host only validates, builds
 * tables and launches.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Sampling (Sec. III-A-2): McEwen-Wiaux.  A sphere map of band-limit L is a
 *   row-major array [t][p] of L x (2L-1) samples at theta_t = pi(2t+1)/(2L-1),
 *   phi_p = 2 pi p/(2L-1).  An SO(3) grid of band-limits (L, N) is a row-major
 *   array [a][b][g] of (2L-1) x L x (2N-1) samples at alpha_a = 2 pi a/(2L-1),
 *   beta_b = pi(2b+1)/(2L-1), gamma_g = 2 pi g/(2N-1).
 * - Harmonic coefficients f_lm (Sec. II-A) are complex128, flat, index
 *   l*l + l + m, 0 <= l < L, |m| <= l.  Wigner coefficients F^l_mn are a dense
 *   complex128 array [l][m + L - 1][n + N - 1] (entries with |m| > l or
 *   |n| > l are ignored on input and written as zero on output).
 * - Conventions of Sec. II-A: zyz Euler angles, D^l_mn = e^{-ima} d^l_mn(b)
 *   e^{-ing}, Condon-Shortley phase, Y_lm = sqrt((2l+1)/4pi) d^l_{m0} e^{imphi}.
 * - All data pointers are DEVICE pointers owned by the caller.  The library
 *   never allocates or frees them.  Scratch memory is the caller's workspace
 *   `ws` of `ws_bytes` bytes (size from cvl_workspace_bytes, or for the
 *   per-scale streaming calls cvl_scale_workspace_bytes); the library
 *   itself allocates only inside cvl_context_create (the resident Delta table)
 *   and on the first use of a new (L, lambda, J0) (its kernel and DFT tables,
 *   kept until cvl_context_destroy; cvl_prepare builds them ahead of time).
 * - `stream` is a hipStream_t (NULL = legacy default stream).  Every call only
 *   enqueues work on that stream and returns; results are ready when the
 *   stream is.  Calls that share a workspace must be ordered on one stream.
 *   The batched curvelet calls run the scales below the top band-limit on a
 *   side stream of the caller's stream (created by the context on first use,
 *   default priority), forked and joined with events inside the call, so the
 *   caller still sees plain stream order.
 * - Graph capture: once the tables of (L, lambda, J0) exist (cvl_prepare or a
 *   first call) the curvelet calls allocate nothing and enqueue only kernels
 *   and event records, so with per-stage timing off they can be captured into
 *   a HIP graph on the caller's stream and replayed.
 * - Return value: CVL_OK, or a negative CVL_E* code.  Arguments are validated
 *   before anything is enqueued; on error nothing is written to any output and
 *   cvl_last_error() (thread-local) describes the failure.  NaN/Inf inputs are
 *   not checked: they propagate to the outputs.
 * - Precision: by default every step is IEEE FP64 (round to nearest, FMA
 *   contraction).  The curvelet calls also offer a reduced-precision path
 *   (cvl_params.precision): complex64 (or float32) coefficient grids, the two
 *   l-contractions on the matrix cores in FP32 or in split bfloat16 ("BF16x3",
 *   a*b = hi*hi + hi*lo + lo*hi) with FP32 accumulation, the beta stage and the
 *   FFTs in FP32, while the Delta table, the SHTs, the scaling part and the
 *   final accumulation of the synthesis over scales stay FP64.
 *   Results are bitwise run-to-run deterministic (no atomics, fixed orders).
 */
#ifndef CURVELET_H
#define CURVELET_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CVL_OK = 0,
    CVL_EINVAL = -1,       /* invalid argument */
    CVL_ENOMEM = -2,       /* workspace too small or device allocation failed */
    CVL_EDEVICE = -3,      /* HIP runtime error */
    CVL_EUNSUPPORTED = -4  /* valid request outside what this build implements */
};

/* Flags of cvl_params. */
#define CVL_REAL 1u        /* real map (f_{l,-m} = (-1)^m conj f_lm); unset: complex map */
#define CVL_REAL_GRIDS 2u  /* curvelet grids of real elements (see cvl_curvelet_analysis) */
#define CVL_UNROTATED 4u   /* coefficients of the unrotated curvelets (see cvl_curvelet_analysis) */

/* Precision of the curvelet calls (cvl_params.precision). */
#define CVL_FP64 0         /* everything FP64, complex128 (or double) grids */
#define CVL_FP32 1         /* FP32 MFMA contractions, FP32 FFT/beta, complex64 (or float) grids */
#define CVL_BF16X3 2       /* split-bfloat16 MFMA contractions, otherwise as CVL_FP32 */

typedef struct { double re, im; } cvl_c128;   /* layout of torch.complex128 */
typedef struct { float re, im; } cvl_c64;     /* layout of torch.complex64 */

typedef struct cvl_ctx cvl_ctx;

/* Curvelet parameters (Sec. II-B).  L: band-limit of the map (>= 2).
 * N: azimuthal band-limit of the curvelets; curvelets have none, so N must be
 * 0 or L (each scale then uses N_j = L_j).  lambda > 1: dilation.  J0 >= 1:
 * lowest curvelet scale, J0 <= J where J = ceil(log_lambda L).  spin: the
 * spin s of the signal and of the curvelets (Sec. II-A, II-B), |s| < L; a
 * real map (CVL_REAL) has spin 0.  precision: CVL_FP64, CVL_FP32 or
 * CVL_BF16X3 (curvelet calls only; it selects the grid element type).
 * flags: CVL_REAL for a real map [t][p] of doubles (unset: a complex map of
 * cvl_c128, with complex grids), optionally CVL_REAL_GRIDS (real maps only)
 * and CVL_UNROTATED; other bits are rejected.  Spin s != 0 needs
 * CVL_UNROTATED (CVL_EUNSUPPORTED otherwise).  The workspace size depends on
 * CVL_UNROTATED and CVL_REAL (cvl_workspace_bytes).  The odd-length DFTs run
 * on power-of-two FFTs of at most 4096 points, which bounds L (and N) at 1024
 * for the curvelet, Wigner and complex-map SHT calls (the real-map SHTs reach
 * a little higher); a larger L returns CVL_EUNSUPPORTED before any launch. */
typedef struct {
    int L;
    int N;
    double lambda;
    int J0;
    int spin;
    int precision;
    unsigned flags;
} cvl_params;

/* Create a context on HIP device `device` holding the quarter table
 * Delta^l_{m'm} = d^l_{m'm}(pi/2), 0 <= m', m <= l < L_max (Sec. III-A-2,
 * the Delta projection; built on the device by the Trapani-Navaza recursion),
 * 8 * L_max(L_max+1)(2L_max+1)/6 bytes.  Synchronous.  2 <= L_max <= 2048. */
int cvl_context_create(cvl_ctx **ctx, int L_max, int device);

/* Release the context and every table it owns (synchronises the device). */
void cvl_context_destroy(cvl_ctx *ctx);

/* J = ceil(log_lambda L), the top scale needed for admissibility (Sec. II-D). */
int cvl_num_scales(const cvl_params *p, int *J);

/* Per-scale band-limits L_j = min(ceil(lambda^(j+1)), L) and N_j = L_j
 * (Sec. III-A-3, multiresolution).  Grid of scale j: (2L_j-1) x L_j x (2N_j-1). */
int cvl_scale_shape(const cvl_params *p, int j, int *Lj, int *Nj);

/* Band-limit of the scaling-coefficient map, L_Phi = min(ceil(lambda^J0), L). */
int cvl_scaling_bandlimit(const cvl_params *p, int *Lphi);

/* Workspace bytes needed by cvl_curvelet_analysis / cvl_curvelet_synthesis
 * for `batch` maps (the workspace is reused map after map).  It includes the
 * buffers of the scales those calls run concurrently on side streams. */
int cvl_workspace_bytes(const cvl_params *p, int batch, size_t *bytes);

/* Workspace bytes needed by the per-scale calls of the streaming interface
 * (cvl_curvelet_analysis_scale, cvl_curvelet_synthesis_scale,
 * cvl_curvelet_scaling_analysis, cvl_curvelet_scaling_synthesis): they run
 * on the caller's stream alone, so they need no side-stream buffers and this
 * is at most cvl_workspace_bytes(p, 1, ...).  Errors: CVL_EINVAL for invalid
 * parameters or a NULL `bytes`. */
int cvl_scale_workspace_bytes(const cvl_params *p, size_t *bytes);

/* Workspace bytes needed by the SHT (L; real and complex maps) and Wigner
 * (L, N) entry points. */
int cvl_sht_workspace_bytes(int L, size_t *bytes);
int cvl_wigner_workspace_bytes(int L, int N, size_t *bytes);

/* Build (synchronously) the tables of parameters `p` so that later calls with
 * the same (L, lambda, J0) allocate nothing. */
int cvl_prepare(cvl_ctx *ctx, const cvl_params *p);

/* Forward SHT of a real spin-0 map (L x (2L-1) doubles) to f_lm (L^2 complex,
 * negative m filled by f_{l,-m} = (-1)^m conj f_lm).  MW sampling theorem
 * (Sec. III-A-2 applied with n = 0).  spin must be 0.  2 <= L <= L_max. */
int cvl_sht_forward(cvl_ctx *ctx, int L, int spin, const double *map,
                    cvl_c128 *flm, void *ws, size_t ws_bytes, void *stream);

/* Inverse SHT to a real map: uses f_lm for m >= 0 and assumes the reality
 * condition for m < 0 (the m < 0 entries are not read). */
int cvl_sht_inverse(cvl_ctx *ctx, int L, int spin, const cvl_c128 *flm,
                    double *map, void *ws, size_t ws_bytes, void *stream);

/* Forward spin-s SHT of a complex map (L x (2L-1) cvl_c128, MW sampling) to
 * the f_lm of every m (flat, L^2 entries; zero for l < |s|):
 * f_lm = <f, sY_lm> with sY_lm = (-1)^s sqrt((2l+1)/4pi) d^l_{m,-s}(theta)
 * e^{i m phi} (Sec. II-A), exact for band-limited maps (the MW sampling
 * theorem; Sec. III-A-2's steps with n = -s).  -L < spin < L. */
int cvl_sht_forward_complex(cvl_ctx *ctx, int L, int spin, const cvl_c128 *map,
                            cvl_c128 *flm, void *ws, size_t ws_bytes, void *stream);

/* Inverse spin-s SHT: the complex map sum_lm f_lm sY_lm (every m read;
 * entries with l < |s| ignored). */
int cvl_sht_inverse_complex(cvl_ctx *ctx, int L, int spin, const cvl_c128 *flm,
                            cvl_c128 *map, void *ws, size_t ws_bytes, void *stream);

/* Inverse Wigner transform (Sec. II-A, Sec. III-A-2): complex grid
 * W(rho) = sum_lmn (2l+1)/(8pi^2) F^l_mn D^{l*}_mn(rho), general complex F,
 * 1 <= N <= L <= L_max. */
int cvl_wigner_inverse(cvl_ctx *ctx, int L, int N, const cvl_c128 *flmn,
                       cvl_c128 *grid, void *ws, size_t ws_bytes, void *stream);

/* Forward Wigner transform (exact for band-limited grids):
 * F^l_mn = <W, D^{l*}_mn>, via the alpha/gamma DFT, the beta extension, the
 * beta DFT, the sin(beta) weight correlation and the Delta projection
 * (Sec. III-A-2). */
int cvl_wigner_forward(cvl_ctx *ctx, int L, int N, const cvl_c128 *grid,
                       cvl_c128 *flmn, void *ws, size_t ws_bytes, void *stream);

/* Curvelet analysis (Sec. II-D-1) of `batch` maps (contiguous, batch x L x
 * (2L-1) doubles with CVL_REAL, else cvl_c128 of spin p->spin).  Outputs per
 * map i:
 *   scal_maps + i * L_Phi * (2L_Phi-1): the scaling coefficients as a spin-0
 *     MW map of band-limit L_Phi (doubles for a real map, else cvl_c128);
 *   grids[i * nJ + (j - J0)], nJ = J - J0 + 1: SO(3) grid W^(j)[a][b][g] of
 *     scale j, (2L_j-1) x L_j x (2L_j-1), of cvl_c128 (CVL_FP64) or cvl_c64
 *     (CVL_FP32, CVL_BF16X3) elements.  For a real map the curvelet
 *     coefficients are real: the imaginary parts are written as 0.  For a
 *     complex map f = f_a + i f_b they are W_a + i W_b (the curvelets'
 *     coefficients obey the reality condition): the two parts' coefficients
 *     run through the real-signal stages and meet in one complex gamma DFT
 *     per grid line, so a complex map costs two real maps.  With
 *     CVL_REAL_GRIDS the elements are double (CVL_FP64) or float instead,
 *     holding the same real parts: the conjugate symmetry of real signals
 *     halves the grids' memory and traffic (Sec. III-A-3).
 *   By default the curvelets are the ones rotated to the North pole (Sec.
 *     II-B), W^(j)(rho) = <f, R_rho psi^(j)>.  With CVL_UNROTATED the grids
 *     hold the coefficients of the unrotated curvelets psi~^(j) (directional
 *     component zeta~, harmonic coefficients only at |n| = l) instead,
 *     W~^(j)(rho) = <f, R_rho psi~^(j)> = W^(j)(rho rho*^-1) with
 *     rho* = (0, pi/2, 0) (Sec. III-A-1); their Wigner transforms need one l
 *     per (m, n) rather than a sum over l, O(L_j^3) per scale.  Same shapes,
 *     element types and synthesis (exact reconstruction) with the same flag.
 * `grids` is a HOST array of batch * nJ device pointers. */
int cvl_curvelet_analysis(cvl_ctx *ctx, const cvl_params *p, int batch,
                          const void *maps, void *scal_maps,
                          void *const *grids, void *ws, size_t ws_bytes,
                          void *stream);

/* Bytes of the static device scratch of cvl_curvelet_analysis_noalloc. */
#define CVL_NOALLOC_SCRATCH_BYTES (80u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * analysis as cvl_curvelet_analysis, with the same arguments and results,
 * but with no workspace argument and no allocation of any kind.  Its scratch
 * is a static device array of CVL_NOALLOC_SCRATCH_BYTES (80 MiB) per GPU,
 * held by the library until the process ends, so a call must fit it: it
 * needs cvl_scale_workspace_bytes(p) bytes (FP64 real maps up to L = 128,
 * for example); larger ones return CVL_ENOMEM.  Every stage runs on the
 * caller's stream (no side stream).  Requirements, checked before anything
 * is enqueued: the tables of (L, lambda, J0) exist (cvl_prepare, else
 * CVL_EINVAL) and per-stage timing is off (CVL_EINVAL).  Every call on one
 * GPU shares that GPU's scratch, which keeps the last call's contents:
 * calls that overlap on one GPU (on different streams, or from different
 * contexts or threads) race; order them on one stream. */
int cvl_curvelet_analysis_noalloc(cvl_ctx *ctx, const cvl_params *p, int batch,
                                  const void *maps, void *scal_maps,
                                  void *const *grids, void *stream);

/* Curvelet synthesis (Sec. II-D-2, exact reconstruction): the inverse of
 * cvl_curvelet_analysis on its range.  With CVL_REAL: synthesis is linear,
 * and a grid's imaginary part only feeds the imaginary part of the
 * synthesised map, so the real map returned is the synthesis of the grids'
 * real parts (the imaginary parts are not used).  Without CVL_REAL the
 * complex grids and scaling maps give complex maps of spin p->spin.  Writes
 * `batch` maps.  Same layouts (and CVL_REAL_GRIDS element types) as
 * cvl_curvelet_analysis. */
int cvl_curvelet_synthesis(cvl_ctx *ctx, const cvl_params *p, int batch,
                           const void *scal_maps, const void *const *grids,
                           void *maps, void *ws, size_t ws_bytes, void *stream);

/* Streaming interface: the same transform one scale at a time, so that only
 * one scale's grid need be resident (Sec. II-D; the synthesis is a sum over
 * scales in harmonic space, Sec. II-D-2).  flm / flm_acc are L^2 complex128
 * harmonic coefficients in the layout of cvl_sht_forward (with CVL_REAL:
 * negative m by the reality condition; else every m, as from
 * cvl_sht_forward_complex, and the scaling maps are cvl_c128).  Workspace:
 * cvl_scale_workspace_bytes(p).  A round trip is
 *   cvl_sht_forward(map) -> flm;  cvl_curvelet_scaling_analysis(flm) -> scal;
 *   per scale j: cvl_curvelet_analysis_scale(flm, j) -> grid,
 *                cvl_curvelet_synthesis_scale(grid, j) adds into flm_acc;
 *   cvl_curvelet_scaling_synthesis(scal) adds into flm_acc;
 *   cvl_sht_inverse(flm_acc) -> map
 * with flm_acc zeroed by the caller first.  The sum is the one
 * cvl_curvelet_synthesis forms (in another order: equal up to rounding). */

/* Grid of scale j (same layout and element type as cvl_curvelet_analysis). */
int cvl_curvelet_analysis_scale(cvl_ctx *ctx, const cvl_params *p, int j,
                                const cvl_c128 *flm, void *grid, void *ws,
                                size_t ws_bytes, void *stream);

/* flm_acc += f^(j)_lm, the synthesis of scale j's grid (with CVL_REAL: of
 * its real part). */
int cvl_curvelet_synthesis_scale(cvl_ctx *ctx, const cvl_params *p, int j,
                                 const void *grid, cvl_c128 *flm_acc, void *ws,
                                 size_t ws_bytes, void *stream);

/* Scaling coefficients: spin-0 MW map of band-limit L_Phi (Sec. II-D-1). */
int cvl_curvelet_scaling_analysis(cvl_ctx *ctx, const cvl_params *p,
                                  const cvl_c128 *flm, void *scal_map,
                                  void *ws, size_t ws_bytes, void *stream);

/* flm_acc += the scaling part of the synthesis (Sec. II-D-2). */
int cvl_curvelet_scaling_synthesis(cvl_ctx *ctx, const cvl_params *p,
                                   const void *scal_map, cvl_c128 *flm_acc,
                                   void *ws, size_t ws_bytes, void *stream);

/* Host copy of the kernel tables of `p` (no device work; usable without a
 * GPU): kappa[(j - J0) * L + l] = kappa^(j)(l) for J0 <= j <= J, and
 * phi[l] = Phi_l0 (Sec. II-B).  kappa needs (J - J0 + 1) * L doubles, phi L. */
int cvl_kernel_tables(const cvl_params *p, double *kappa, double *phi);

/* Per-stage device time accounting for benchmarks.  When enabled, every
 * kernel launch of the calls that follow is bracketed by HIP events on the
 * call's stream; cvl_profile_read synchronises those events and returns, for
 * stage index i < *n, its name, launch count and total milliseconds. */
int cvl_profile_enable(cvl_ctx *ctx, int on);
int cvl_profile_read(cvl_ctx *ctx, int max, int *n, const char **names,
                     int *launches, double *ms);

/* Restrict the per-launch timing to the launches of stage index `stage`
 * (names as in cvl_profile_read) at band-limit `bandlimit`; stage -1 times
 * every launch again.  Timing few launches keeps the events' own cost out of
 * the work being measured.  Errors: CVL_EINVAL for a stage index outside
 * [-1, number of stages). */
int cvl_profile_filter(cvl_ctx *ctx, int stage, int bandlimit);

/* The same times split by (stage, band-limit): row i < min(*n, max) is stage
 * index stage[i] (names as in cvl_profile_read) at band-limit bandlimit[i]
 * (the scale's L_j, or the SHT's L), with its launch count and milliseconds. */
int cvl_profile_read_detail(cvl_ctx *ctx, int max, int *n, int *stage,
                            int *bandlimit, int *launches, double *ms);

/* Copy block l of the resident Delta table to host memory (synchronous):
 * out[m' * (l+1) + m] = Delta^l_{m'm} = d^l_{m'm}(pi/2), 0 <= m', m <= l < L_max. */
int cvl_delta_block(cvl_ctx *ctx, int l, double *out);

/* Thread-local description of the last error (empty string if none). */
const char *cvl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CURVELET_H */
