// C ABI of the curvelet transform: validation, resident tables, workspace
// carving and the launch sequences of every entry point.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/curvelet.h"
#include "cvl_device.h"
#include "host_tables.h"

using namespace cvl;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e__ = (expr);                                                           \
        if (e__ != hipSuccess)                                                             \
            return fail(CVL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e__));      \
    } while (0)

constexpr size_t kAlign = 256;
// Scales with L_j at least this run the analysis beta stage as an FFT
// (O(L^3 log L)) instead of the dense parity-folded GEMM (O(L^4)).
constexpr int kBetaFftMinL = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum Stage {
    ST_SHT_PHI,
    ST_SHT_THETA,
    ST_SHT_DELTA,
    ST_CONTRACT_INV,
    ST_BETA_INV,
    ST_ALPHA_INV,
    ST_GAMMA_INV,
    ST_GAMMA_FWD,
    ST_ALPHA_FWD,
    ST_BETA_FWD,
    ST_CONTRACT_FWD,
    ST_REDUCE_FWD,
    ST_MISC,
    ST_COUNT
};
const char *kStageNames[ST_COUNT] = {"sht_phi_dft",     "sht_theta",       "sht_delta",
                                     "contract_inv",    "beta_gemm_inv",   "alpha_dft_inv",
                                     "gamma_dft_inv",   "gamma_dft_fwd",   "alpha_dft_fwd",
                                     "beta_gemm_fwd",   "contract_fwd",    "reduce_fwd",
                                     "misc"};

struct DeviceArena {
    std::vector<void *> ptrs;
    ~DeviceArena() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    int upload(const std::vector<T> &v, T **out) {
        void *p = nullptr;
        size_t bytes = v.size() * sizeof(T);
        if (bytes == 0) bytes = sizeof(T);
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) return fail(CVL_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        ptrs.push_back(p);
        if (!v.empty()) {
            e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(CVL_EDEVICE, "hipMemcpy failed: %s", hipGetErrorString(e));
        }
        *out = (T *)p;
        return CVL_OK;
    }
};

struct BetaTabs {  // parity-folded beta matrices of one band-limit
    double *Cinv = nullptr, *Sinv = nullptr, *Qp = nullptr, *Qs = nullptr;
};
struct BetaTabsF {  // the same, rounded to FP32 (reduced-precision path)
    float *Cinv = nullptr, *Sinv = nullptr, *Qp = nullptr, *Qs = nullptr;
};

struct ScaleRt {
    int j;
    ScaleGeom g;
    double *psi;  // [l][k]: Psi^(j)_{l,2k}
    double *pd;   // [m'][l]: Delta^l_{m'l} Psi~^(j)_{l,l} (unrotated curvelets)
    BetaTabs beta;
    BluesteinDev inv_full, fwd_full;
    BetaTabsF betaf;
    BluesteinF inv_full_f, fwd_full_f;
    int ngroups;  // m' groups of the synthesis contraction
    bool beta_fft;  // analysis beta stage as an FFT (large L_j) instead of a GEMM
    // ... written line-major and transposed into W1 (FFT size 4096: one line
    // per work-group), in complex64; W1 then lives in the first cube buffer,
    // W2 in the second.  (In complex128 the wider stores merge well enough
    // that the transpose costs more than it saves: L = 1024, 37.2 ms per
    // launch direct against 39.5 ms line-major and transposed.)
    bool beta_lines;
    BluesteinDev beta_inv;
    BluesteinF beta_inv_f;
};

struct Plan {
    int L, J0, J, Lphi;
    double lambda;
    std::vector<ScaleRt> scales;
    double *phifac;  // [Lphi]: sqrt(4pi/(2l+1)) Phi_l0
};

struct ShtRt {
    int L;
    BetaTabs beta;  // factor 2 pi
    BluesteinDev inv, fwd;
    BluesteinDev fwd_c;  // phi DFT of a complex map: every m
};

struct GenRt {
    int L, N;
    BetaTabs beta;  // factor (2 pi)^2
    BluesteinDev a_inv, a_fwd, g_inv, g_fwd;
};

}  // namespace

// Scratch of cvl_curvelet_analysis_noalloc: a file-scope device array of
// CVL_NOALLOC_SCRATCH_BYTES, one copy per GPU, held while the library is
// loaded.  In host code the name `scratch` is a host-side stand-in, not a
// device address: its address on each device comes from hipGetSymbolAddress
// (cvl_context_create, with the context's device current) and is the only
// handle host code passes on.
static __device__ __align__(256) unsigned char scratch[CVL_NOALLOC_SCRATCH_BYTES];

struct cvl_ctx {
    int device = 0;
    int Lmax = 0;
    double *delta = nullptr;
    void *scratch_dev = nullptr;  // this device's copy of `scratch`
    std::mutex mu;
    DeviceArena arena;
    std::map<int, cd *> tw;
    std::map<int, cf *> tw_f;
    std::map<std::tuple<int, int, int, int, int, int, int>, BluesteinDev> blue;
    std::map<std::tuple<int, int, int, int, int, int, int>, BluesteinF> blue_f;
    std::map<std::pair<int, int>, BetaTabs> beta;  // (L, factor id)
    std::map<std::pair<int, int>, BetaTabsF> beta_f;
    std::map<std::tuple<int, double, int>, std::unique_ptr<Plan>> plans;
    std::map<int, std::unique_ptr<ShtRt>> sht;
    std::map<std::pair<int, int>, std::unique_ptr<GenRt>> gen;
    // Psi of the rotated spin-s curvelets per scale, [l][n + L_j - 1], keyed
    // (L, lambda, J0, spin)
    std::map<std::tuple<int, double, int, int>, std::vector<double *>> spin_psi;
    // side stream (and its fork / join events) per caller stream
    struct Side {
        hipStream_t s = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
    };
    std::map<hipStream_t, Side> side;
    // profiling
    bool prof = false;
    int pf_stage = -1, pf_tag = 0;  // only this (stage, band-limit) when pf_stage >= 0
    std::vector<hipEvent_t> pool;
    std::vector<std::tuple<int, int, hipEvent_t, hipEvent_t>> rec;  // stage, tag, events
    double stage_ms[ST_COUNT] = {0};
    int stage_n[ST_COUNT] = {0};
    std::map<std::pair<int, int>, std::pair<int, double>> detail;  // (stage, tag) -> (n, ms)
};

namespace {

int get_twiddles(cvl_ctx *c, int P, const cd **out) {
    auto it = c->tw.find(P);
    if (it != c->tw.end()) {
        *out = it->second;
        return CVL_OK;
    }
    auto t = host::twiddles(P);
    std::vector<cd> v(P);
    for (int i = 0; i < P; ++i) v[i] = cd{t[i].real(), t[i].imag()};
    cd *d;
    int rc = c->arena.upload(v, &d);
    if (rc) return rc;
    c->tw[P] = d;
    *out = d;
    return CVL_OK;
}

int get_bluestein(cvl_ctx *c, int Nd, int Kin, int j0, int Kout, int k0, int sigma,
                  BluesteinDev *out) {
    auto key = std::make_tuple(Nd, Kin, j0, Kout, k0, sigma, 0);
    auto it = c->blue.find(key);
    if (it != c->blue.end()) {
        *out = it->second;
        return CVL_OK;
    }
    const double scale = sigma < 0 ? 1.0 / Nd : 1.0;
    host::Bluestein B = host::make_bluestein(Nd, Kin, j0, Kout, k0, sigma, scale);
    if (B.P > 4096) return fail(CVL_EUNSUPPORTED, "DFT length %d needs FFT size %d > 4096", Nd, B.P);
    if (B.P >= 256 && 2 * std::max(Kin, Kout) > B.P + B.P / 16)
        return fail(CVL_EUNSUPPORTED, "DFT window (%d in, %d out) too wide for FFT size %d", Kin,
                    Kout, B.P);
    auto cv = [](const std::vector<std::complex<double>> &s) {
        std::vector<cd> v(s.size());
        for (size_t i = 0; i < s.size(); ++i) v[i] = cd{s[i].real(), s[i].imag()};
        return v;
    };
    BluesteinDev D{};
    D.Nd = Nd;
    D.P = B.P;
    D.Kin = Kin;
    D.j0 = j0;
    D.Kout = Kout;
    D.k0 = k0;
    cd *pre, *post, *vhat;
    int rc;
    if ((rc = c->arena.upload(cv(B.pre), &pre))) return rc;
    if ((rc = c->arena.upload(cv(B.post), &post))) return rc;
    if ((rc = c->arena.upload(cv(B.vhat), &vhat))) return rc;
    const cd *tw;
    if ((rc = get_twiddles(c, B.P, &tw))) return rc;
    D.pre = pre;
    D.post = post;
    D.vhat = vhat;
    D.tw = tw;
    c->blue[key] = D;
    *out = D;
    return CVL_OK;
}

// factor id 0: (2 pi)^2 (Wigner), 1: 2 pi (SHT)
int get_beta(cvl_ctx *c, int L, int fid, BetaTabs *out) {
    auto key = std::make_pair(L, fid);
    auto it = c->beta.find(key);
    if (it != c->beta.end()) {
        *out = it->second;
        return CVL_OK;
    }
    std::vector<double> C, S, Qp, Qs;
    host::beta_inverse_mats(L, C, S);
    host::beta_forward_mats(L, fid == 0 ? 4.0 * M_PI * M_PI : 2.0 * M_PI, Qp, Qs);
    BetaTabs T;
    int rc;
    if ((rc = c->arena.upload(C, &T.Cinv))) return rc;
    if ((rc = c->arena.upload(S, &T.Sinv))) return rc;
    if ((rc = c->arena.upload(Qp, &T.Qp))) return rc;
    if ((rc = c->arena.upload(Qs, &T.Qs))) return rc;
    c->beta[key] = T;
    *out = T;
    return CVL_OK;
}

// FP32 copies of the DFT tables (computed in extended precision, rounded once).
int get_bluestein_f(cvl_ctx *c, int Nd, int Kin, int j0, int Kout, int k0, int sigma,
                    BluesteinF *out) {
    auto key = std::make_tuple(Nd, Kin, j0, Kout, k0, sigma, 0);
    auto it = c->blue_f.find(key);
    if (it != c->blue_f.end()) {
        *out = it->second;
        return CVL_OK;
    }
    const double scale = sigma < 0 ? 1.0 / Nd : 1.0;
    host::Bluestein B = host::make_bluestein(Nd, Kin, j0, Kout, k0, sigma, scale);
    if (B.P > 4096) return fail(CVL_EUNSUPPORTED, "DFT length %d needs FFT size %d > 4096", Nd, B.P);
    if (B.P >= 256 && 2 * std::max(Kin, Kout) > B.P + B.P / 16)
        return fail(CVL_EUNSUPPORTED, "DFT window (%d in, %d out) too wide for FFT size %d", Kin,
                    Kout, B.P);
    auto cv = [](const std::vector<std::complex<double>> &v) {
        std::vector<cf> o(v.size());
        for (size_t i = 0; i < v.size(); ++i) o[i] = cf{(float)v[i].real(), (float)v[i].imag()};
        return o;
    };
    BluesteinF D{};
    D.Nd = Nd;
    D.P = B.P;
    D.Kin = Kin;
    D.j0 = j0;
    D.Kout = Kout;
    D.k0 = k0;
    cf *pre, *post, *vhat;
    int rc;
    if ((rc = c->arena.upload(cv(B.pre), &pre))) return rc;
    if ((rc = c->arena.upload(cv(B.post), &post))) return rc;
    if ((rc = c->arena.upload(cv(B.vhat), &vhat))) return rc;
    auto tw = c->tw_f.find(B.P);
    if (tw == c->tw_f.end()) {
        cf *d;
        if ((rc = c->arena.upload(cv(host::twiddles(B.P)), &d))) return rc;
        tw = c->tw_f.emplace(B.P, d).first;
    }
    D.pre = pre;
    D.post = post;
    D.vhat = vhat;
    D.tw = tw->second;
    c->blue_f[key] = D;
    *out = D;
    return CVL_OK;
}

int get_beta_f(cvl_ctx *c, int L, int fid, BetaTabsF *out) {
    auto key = std::make_pair(L, fid);
    auto it = c->beta_f.find(key);
    if (it != c->beta_f.end()) {
        *out = it->second;
        return CVL_OK;
    }
    std::vector<double> C, S, Qp, Qs;
    host::beta_inverse_mats(L, C, S);
    host::beta_forward_mats(L, fid == 0 ? 4.0 * M_PI * M_PI : 2.0 * M_PI, Qp, Qs);
    auto cv = [](const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); };
    BetaTabsF T;
    int rc;
    if ((rc = c->arena.upload(cv(C), &T.Cinv))) return rc;
    if ((rc = c->arena.upload(cv(S), &T.Sinv))) return rc;
    if ((rc = c->arena.upload(cv(Qp), &T.Qp))) return rc;
    if ((rc = c->arena.upload(cv(Qs), &T.Qs))) return rc;
    c->beta_f[key] = T;
    *out = T;
    return CVL_OK;
}

int num_scales(int L, double lam) {
    int J = 0;
    double p = 1.0;
    while (p < L) {
        p *= lam;
        ++J;
    }
    return J;
}
int scale_bandlimit(int j, int L, double lam) {
    double v = std::ceil(std::pow(lam, j + 1) - 1e-9);
    return v >= L ? L : (int)v;
}
int scaling_bandlimit(int L, double lam, int J0) {
    double v = std::ceil(std::pow(lam, J0) - 1e-9);
    return v >= L ? L : (int)v;
}

int check_params(const cvl_params *p, int *J) {
    if (!p) return fail(CVL_EINVAL, "params is NULL");
    if (p->L < 2 || p->L > 2048) return fail(CVL_EINVAL, "L=%d outside [2, 2048]", p->L);
    if (p->N != 0 && p->N != p->L)
        return fail(CVL_EINVAL, "N=%d: curvelets have no azimuthal band-limit, N must be 0 or L",
                    p->N);
    if (!(p->lambda > 1.0) || !std::isfinite(p->lambda))
        return fail(CVL_EINVAL, "lambda=%g must be a finite number > 1", p->lambda);
    int JJ = num_scales(p->L, p->lambda);
    if (p->J0 < 1 || p->J0 > JJ)
        return fail(CVL_EINVAL, "J0=%d outside [1, J=%d]", p->J0, JJ);
    if (p->precision != CVL_FP64 && p->precision != CVL_FP32 && p->precision != CVL_BF16X3)
        return fail(CVL_EINVAL, "precision=%d is not CVL_FP64, CVL_FP32 or CVL_BF16X3",
                    p->precision);
    if (p->flags & ~(CVL_REAL | CVL_REAL_GRIDS | CVL_UNROTATED))
        return fail(CVL_EINVAL, "flags=0x%x: unknown bits", p->flags);
    if (p->flags & CVL_REAL) {
        if (p->spin != 0)
            return fail(CVL_EINVAL, "spin=%d: a spin signal is complex (clear CVL_REAL)", p->spin);
    } else {
        if (p->flags & CVL_REAL_GRIDS)
            return fail(CVL_EINVAL, "CVL_REAL_GRIDS needs a real map (CVL_REAL): the "
                                    "coefficients of a complex map are complex");
        if (p->spin <= -p->L || p->spin >= p->L)
            return fail(CVL_EINVAL, "spin=%d outside (-L, L)", p->spin);
        if (p->spin != 0 && !(p->flags & CVL_UNROTATED) && p->precision != CVL_FP64)
            return fail(CVL_EUNSUPPORTED, "spin=%d: the rotated spin curvelets run in FP64 only",
                        p->spin);
    }
    if (J) *J = JJ;
    return CVL_OK;
}

// The analysis beta DFT of band-limit L_j is written line-major and then
// transposed when its Bluestein size (>= 4 L_j - 3) is 4096, i.e. from
// L_j = 513 on (see launch_inv_beta_dft_lines).
bool beta_lines_of(int Lj) { return Lj >= kBetaFftMinL && 4 * Lj - 3 > 2048; }

ScaleGeom geom_of(int Lj) {
    ScaleGeom g{};
    g.L = Lj;
    g.Nm = 2 * Lj - 1;
    g.h = (Lj - 1) / 2;
    g.Ne = 2 * g.h + 1;
    g.Nep = (g.Ne + 31) / 32 * 32;
    g.llo = 0;
    g.lhi = Lj - 1;
    return g;
}

// Element counts of the two cube-sized workspace buffers of a curvelet call.
// m' groups of the synthesis contraction of a scale: one m' per group (the
// contraction then keeps no running sum over m', and the group reduction
// sums only the groups that can hold an m' <= l).
int fwd_groups(const ScaleGeom &g) { return g.L; }

// Elements of the two cube buffers of the scales at the top band-limit
// (b0, b1) and of the side scales below it (sb0, sb1), which run
// concurrently on a side stream with buffers of their own.
void curvelet_buf_elems(int L, double lam, int J0, int J, bool unrot, size_t *b0, size_t *b1,
                        size_t *sb0, size_t *sb1) {
    *b0 = *b1 = *sb0 = *sb1 = 0;
    const int top = scale_bandlimit(J, L, lam);
    for (int j = J0; j <= J; ++j) {
        ScaleGeom g = geom_of(scale_bandlimit(j, L, lam));
        // unrotated: 2 L_j cube rows per plane, W2 / V1 rows of L_j entries,
        // no partial sums
        size_t cube = (size_t)g.L * (unrot ? 2 * g.L : g.L) * g.Nep;
        size_t w2 = (size_t)g.L * g.Nm * (unrot ? g.L : g.h + 1);
        size_t part = unrot ? 0 : (size_t)g.L * g.L * g.L;  // at most L_j groups
        // line-major beta: W2 in the second buffer
        const size_t w2b = (!unrot && beta_lines_of(g.L)) ? w2 : 0;
        size_t *x0 = g.L < top ? sb0 : b0, *x1 = g.L < top ? sb1 : b1;
        *x0 = std::max({*x0, cube, w2});
        *x1 = std::max({*x1, cube, part, w2b});
    }
}

// Workspace bytes of a curvelet call: two cube buffers for the top scales and
// four L x L (plus the scaling band-limit's) complex128 planes; the batched
// calls add two cube buffers and a plane for the side scales (cube elements
// complex128, or complex64 in reduced precision).  The per-scale calls
// (scale_call) need only the first part: they run on one stream.
// Elements of the W2 / V1 plane buffer of a complex signal's second part:
// the largest plane of the top scales (*top) and of the side scales (*side).
void curvelet_plane_elems(int L, double lam, int J0, int J, bool unrot, size_t *top,
                          size_t *side) {
    *top = *side = 0;
    const int T = scale_bandlimit(J, L, lam);
    for (int j = J0; j <= J; ++j) {
        ScaleGeom g = geom_of(scale_bandlimit(j, L, lam));
        const size_t w2 = (size_t)g.L * g.Nm * (unrot ? g.L : g.h + 1);
        size_t *x = g.L < T ? side : top;
        *x = std::max(*x, w2);
    }
}

size_t curvelet_ws_bytes(int L, double lam, int J0, int J, int precision, bool unrot,
                         bool scale_call, bool cplx = false) {
    size_t b0, b1, sb0, sb1, p2, sp2;
    curvelet_buf_elems(L, lam, J0, J, unrot, &b0, &b1, &sb0, &sb1);
    curvelet_plane_elems(L, lam, J0, J, unrot, &p2, &sp2);
    const size_t esz = precision == CVL_FP64 ? 16 : 8;
    const int Lphi = scaling_bandlimit(L, lam, J0);
    size_t small = 4 * (size_t)L * L + 2 * (size_t)Lphi * Lphi;
    size_t base = align_up(b0 * esz) + align_up(b1 * esz) + align_up(small * 16) + 8 * kAlign;
    // complex signals: the second part's plane, its padded coefficients and
    // accumulator, the flat coefficients and the complex SHT's scratch at L
    // and at L_Phi
    const size_t L2 = align_up((size_t)L * L * 16);
    const size_t sht = align_up((size_t)L * (2 * L - 1) * 16);
    const size_t shtp = align_up((size_t)Lphi * (2 * Lphi - 1) * 16);
    if (cplx) base += align_up(p2 * esz) + 3 * L2 + 2 * sht + 2 * shtp + 8 * kAlign;
    if (scale_call) return base;
    const size_t plane = align_up((size_t)L * L * 16);
    size_t side = align_up(sb0 * esz) + align_up(sb1 * esz) + plane + 3 * kAlign;
    if (cplx) side += align_up(sp2 * esz) + plane + 2 * kAlign;
    return base + side;
}

// Rotated spin-s curvelets (kernel coefficients at every n, no reality
// condition) run on the general Wigner layouts, every scale on the caller's
// stream: two general cube buffers and the dense Wigner coefficients of the
// top scale, the flat coefficients and accumulator, the complex SHT scratch.
bool spin_rotated(const cvl_params *p) {
    return !(p->flags & CVL_REAL) && !(p->flags & CVL_UNROTATED) && p->spin != 0;
}
size_t spin_ws_bytes(int L, double lam, int J0, int J) {
    const int T = scale_bandlimit(J, L, lam), Lphi = scaling_bandlimit(L, lam, J0);
    const size_t Nm = 2 * T - 1, Nnp = (Nm + 31) / 32 * 32;
    const size_t gen = align_up((size_t)T * Nm * Nnp * 16), F = align_up((size_t)T * Nm * Nm * 16);
    const size_t L2 = align_up((size_t)L * L * 16), sht = align_up((size_t)L * (2 * L - 1) * 16);
    const size_t shtp = align_up((size_t)Lphi * (2 * Lphi - 1) * 16);
    return 2 * gen + F + 2 * L2 + 2 * sht + 2 * shtp + align_up((size_t)Lphi * Lphi * 16) +
           10 * kAlign;
}
size_t ws_bytes_of(const cvl_params *p, int J, bool scale_call) {
    if (spin_rotated(p)) return spin_ws_bytes(p->L, p->lambda, p->J0, J);
    return curvelet_ws_bytes(p->L, p->lambda, p->J0, J, p->precision,
                             (p->flags & CVL_UNROTATED) != 0, scale_call, !(p->flags & CVL_REAL));
}

int get_plan(cvl_ctx *c, const cvl_params *p, Plan **out) {
    int J;
    int rc = check_params(p, &J);
    if (rc) return rc;
    if (p->L > c->Lmax) return fail(CVL_EINVAL, "L=%d exceeds the context's L_max=%d", p->L, c->Lmax);
    auto key = std::make_tuple(p->L, p->lambda, p->J0);
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->plans.find(key);
    if (it != c->plans.end()) {
        *out = it->second.get();
        return CVL_OK;
    }
    std::unique_ptr<Plan> P(new Plan);
    P->L = p->L;
    P->J0 = p->J0;
    P->J = J;
    P->lambda = p->lambda;
    P->Lphi = scaling_bandlimit(p->L, p->lambda, p->J0);
    const int L = p->L;
    std::vector<double> kap = host::kappa_table(L, p->lambda, p->J0, J);
    std::vector<double> phi = host::phi_table(L, p->lambda, p->J0);
    std::vector<double> acol = host::delta_col_l(L);
    for (int j = p->J0; j <= J; ++j) {
        ScaleRt S{};
        S.j = j;
        const int Lj = scale_bandlimit(j, L, p->lambda);
        S.g = geom_of(Lj);
        const double *kj = &kap[(size_t)(j - p->J0) * L];
        int llo = Lj, lhi = Lj - 1;
        for (int l = 0; l < Lj; ++l)
            if (kj[l] > 0.0) {
                if (l < llo) llo = l;
                lhi = l;
            }
        S.g.llo = llo;
        S.g.lhi = lhi;
        S.ngroups = fwd_groups(S.g);
        const int h = S.g.h;
        std::vector<double> psi((size_t)Lj * (h + 1), 0.0);
        for (int l = 0; l < Lj; ++l)
            for (int k = 0; 2 * k <= l && k <= h; ++k)
                psi[(size_t)l * (h + 1) + k] = std::sqrt((2.0 * l + 1.0) / (8.0 * M_PI * M_PI)) *
                                               kj[l] * std::sqrt(2.0) * acol[(size_t)l * L + 2 * k];
        if ((rc = c->arena.upload(psi, &S.psi))) return rc;
        // unrotated: Psi~_{l,l} = sqrt((2l+1)/(8 pi^2)) kappa_j(l) zeta~_{l,l},
        // zeta~_{l,l} = 1/sqrt 2, times Delta^l_{m'l} (zero for m' > l)
        std::vector<double> pd((size_t)Lj * Lj, 0.0);
        for (int l = 0; l < Lj; ++l) {
            const double ps = std::sqrt((2.0 * l + 1.0) / (8.0 * M_PI * M_PI)) * kj[l] /
                              std::sqrt(2.0);
            for (int mp = 0; mp <= l; ++mp)
                pd[(size_t)mp * Lj + l] = acol[(size_t)l * L + mp] * ps;
        }
        if ((rc = c->arena.upload(pd, &S.pd))) return rc;
        if ((rc = get_beta(c, Lj, 0, &S.beta))) return rc;
        const int Nm = 2 * Lj - 1;
        if ((rc = get_bluestein(c, Nm, Nm, -(Lj - 1), Nm, 0, +1, &S.inv_full))) return rc;
        if ((rc = get_bluestein(c, Nm, Nm, 0, Nm, -(Lj - 1), -1, &S.fwd_full))) return rc;
        if ((rc = get_beta_f(c, Lj, 0, &S.betaf))) return rc;
        if ((rc = get_bluestein_f(c, Nm, Nm, -(Lj - 1), Nm, 0, +1, &S.inv_full_f))) return rc;
        if ((rc = get_bluestein_f(c, Nm, Nm, 0, Nm, -(Lj - 1), -1, &S.fwd_full_f))) return rc;
        S.beta_fft = Lj >= kBetaFftMinL;
        S.beta_lines = false;
        if (S.beta_fft) {
            if ((rc = get_bluestein(c, Nm, Nm, -(Lj - 1), Nm, -(Lj - 1), +1, &S.beta_inv))) return rc;
            if ((rc = get_bluestein_f(c, Nm, Nm, -(Lj - 1), Nm, -(Lj - 1), +1, &S.beta_inv_f)))
                return rc;
            S.beta_lines = beta_lines_of(Lj);
        }
        P->scales.push_back(S);
    }
    std::vector<double> pf(P->Lphi);
    for (int l = 0; l < P->Lphi; ++l) pf[l] = std::sqrt(4.0 * M_PI / (2.0 * l + 1.0)) * phi[l];
    if ((rc = c->arena.upload(pf, &P->phifac))) return rc;
    *out = P.get();
    c->plans[key] = std::move(P);
    return CVL_OK;
}

int get_sht(cvl_ctx *c, int L, ShtRt **out) {
    // caller holds c->mu
    auto it = c->sht.find(L);
    if (it != c->sht.end()) {
        *out = it->second.get();
        return CVL_OK;
    }
    std::unique_ptr<ShtRt> S(new ShtRt);
    S->L = L;
    int rc;
    if ((rc = get_beta(c, L, 1, &S->beta))) return rc;
    const int Nm = 2 * L - 1;
    if ((rc = get_bluestein(c, Nm, Nm, -(L - 1), Nm, 0, +1, &S->inv))) return rc;
    if ((rc = get_bluestein(c, Nm, Nm, 0, L, 0, -1, &S->fwd))) return rc;
    if ((rc = get_bluestein(c, Nm, Nm, 0, Nm, -(L - 1), -1, &S->fwd_c))) return rc;
    *out = S.get();
    c->sht[L] = std::move(S);
    return CVL_OK;
}

// ---- profiling ----
// Band-limit of the scale (or SHT) whose kernels are being enqueued on this
// thread; recorded with each timed launch.
thread_local int g_tag = 0;
struct TagScope {
    int prev;
    explicit TagScope(int t) : prev(g_tag) { g_tag = t; }
    ~TagScope() { g_tag = prev; }
};

struct Prof {
    cvl_ctx *c;
    hipStream_t st;
    int stage, tag;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Prof(cvl_ctx *c_, hipStream_t s, int stg) : c(c_), st(s), stage(stg), tag(g_tag) {
        if (!c->prof || (c->pf_stage >= 0 && (stage != c->pf_stage || tag != c->pf_tag))) return;
        e0 = take();
        e1 = take();
        if (e0) (void)hipEventRecord(e0, st);
    }
    hipEvent_t take() {
        std::lock_guard<std::mutex> lk(c->mu);
        if (!c->pool.empty()) {
            hipEvent_t e = c->pool.back();
            c->pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~Prof() {
        if (!c->prof || !e0 || !e1) return;
        (void)hipEventRecord(e1, st);
        std::lock_guard<std::mutex> lk(c->mu);
        c->rec.emplace_back(stage, tag, e0, e1);
    }
};

#define LAUNCH(stage, call)                                                                \
    do {                                                                                   \
        Prof pr__(ctx, st, stage);                                                         \
        hipError_t e__ = (call);                                                           \
        if (e__ != hipSuccess)                                                             \
            return fail(CVL_EDEVICE, "launch of %s failed: %s", kStageNames[stage],        \
                        hipGetErrorString(e__));                                           \
    } while (0)

struct Carver {
    char *p;
    size_t left;
    template <class T>
    T *take(size_t n) {
        size_t b = align_up(n * sizeof(T));
        if (b > left) return nullptr;
        T *r = (T *)p;
        p += b;
        left -= b;
        return r;
    }
};

// ---- SHT launch sequences (device scratch passed in) ----
int sht_forward_run(cvl_ctx *ctx, ShtRt *S, const double *map, cd *fpad, int Lf, cd *F1,
                    cd *Zs, hipStream_t st) {
    const int L = S->L;
    TagScope tag(L);
    LAUNCH(ST_SHT_PHI, launch_sht_fwd_phi(L, S->fwd, map, F1, st));
    LAUNCH(ST_SHT_THETA, launch_sht_theta(L, L, L, 1, S->beta.Qp, S->beta.Qs, F1, Zs, st));
    LAUNCH(ST_SHT_DELTA, launch_sht_fwd_delta(L, Lf, ctx->delta, Zs, fpad, st));
    return CVL_OK;
}

int sht_inverse_run(cvl_ctx *ctx, ShtRt *S, const cd *fpad, int Lf, double *map, cd *F,
                    cd *G, hipStream_t st) {
    const int L = S->L;
    TagScope tag(L);
    LAUNCH(ST_SHT_DELTA, launch_sht_inv_delta(L, Lf, ctx->delta, fpad, F, st));
    LAUNCH(ST_SHT_THETA, launch_sht_theta(L, L, L, 0, S->beta.Cinv, S->beta.Sinv, F, G, st));
    LAUNCH(ST_SHT_PHI, launch_sht_inv_phi(L, S->inv, G, map, st));
    return CVL_OK;
}

// Spin-s SHT of a complex map [t][p] (L x (2L-1) complex128) to the flat
// f_lm of every m, and back (scratch: two L x (2L-1) complex buffers).
int sht_forward_cplx_run(cvl_ctx *ctx, ShtRt *S, int spin, const cd *map, cd *flm, cd *F1,
                         cd *Zs, hipStream_t st) {
    const int L = S->L, Nm = 2 * L - 1;
    TagScope tag(L);
    LAUNCH(ST_SHT_PHI, launch_sht_fwd_phi_cplx(L, S->fwd_c, map, F1, st));
    LAUNCH(ST_SHT_THETA, launch_sht_theta_cols(Nm, spin - L + 1, L, L, S->beta.Qp, S->beta.Qs,
                                               F1, Zs, st));
    LAUNCH(ST_SHT_DELTA, launch_sht_fwd_delta_spin(L, spin, ctx->delta, Zs, flm, st));
    return CVL_OK;
}

int sht_inverse_cplx_run(cvl_ctx *ctx, ShtRt *S, int spin, const cd *flm, cd *map, cd *F,
                         cd *G, hipStream_t st) {
    const int L = S->L, Nm = 2 * L - 1;
    TagScope tag(L);
    LAUNCH(ST_SHT_DELTA, launch_sht_inv_delta_spin(L, spin, ctx->delta, flm, F, st));
    LAUNCH(ST_SHT_THETA, launch_sht_theta_cols(Nm, spin - L + 1, L, L, S->beta.Cinv,
                                               S->beta.Sinv, F, G, st));
    LAUNCH(ST_SHT_PHI, launch_sht_inv_phi_cplx(L, S->inv, G, map, st));
    return CVL_OK;
}

int check_ctx(cvl_ctx *ctx) {
    if (!ctx) return fail(CVL_EINVAL, "context is NULL");
    return CVL_OK;
}

int set_device(cvl_ctx *ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(CVL_EDEVICE, "hipSetDevice(%d): %s", ctx->device, hipGetErrorString(e));
    return CVL_OK;
}

}  // namespace

extern "C" {

static int get_spin_psi(cvl_ctx *ctx, const Plan *P, int spin, const std::vector<double *> **out);
static int get_gen(cvl_ctx *ctx, int L, int N, GenRt **out);

const char *cvl_last_error(void) { return g_err.c_str(); }

int cvl_context_create(cvl_ctx **out, int L_max, int device) {
    g_err.clear();
    if (!out) return fail(CVL_EINVAL, "ctx out-pointer is NULL");
    *out = nullptr;
    if (L_max < 2 || L_max > 2048) return fail(CVL_EINVAL, "L_max=%d outside [2, 2048]", L_max);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(CVL_EDEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(CVL_EINVAL, "device=%d outside [0, %d)", device, ndev);
    std::unique_ptr<cvl_ctx> c(new cvl_ctx);
    c->device = device;
    c->Lmax = L_max;
    HIP_TRY(hipSetDevice(device));
    // device address of the static scratch on this device (set-up of the
    // allocation-free entry point; allocates nothing)
    {
        void *sp = nullptr;
        e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !sp)
            return fail(CVL_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        c->scratch_dev = sp;
    }
    size_t n = (size_t)delta_off(L_max);
    void *p = nullptr;
    e = hipMalloc(&p, n * sizeof(double));
    if (e != hipSuccess) return fail(CVL_ENOMEM, "Delta table of %zu bytes: %s", n * sizeof(double), hipGetErrorString(e));
    c->arena.ptrs.push_back(p);
    c->delta = (double *)p;
    HIP_TRY(launch_delta_toprows(c->delta, L_max, nullptr));
    HIP_TRY(launch_delta_fill(c->delta, L_max, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    *out = c.release();
    return CVL_OK;
}

void cvl_context_destroy(cvl_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &r : ctx->rec) {
        (void)hipEventDestroy(std::get<2>(r));
        (void)hipEventDestroy(std::get<3>(r));
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    for (auto &kv : ctx->side) {
        (void)hipEventDestroy(kv.second.fork);
        (void)hipEventDestroy(kv.second.join);
        (void)hipStreamDestroy(kv.second.s);
    }
    delete ctx;
}

int cvl_num_scales(const cvl_params *p, int *J) {
    g_err.clear();
    if (!J) return fail(CVL_EINVAL, "J out-pointer is NULL");
    return check_params(p, J);
}

int cvl_scale_shape(const cvl_params *p, int j, int *Lj, int *Nj) {
    g_err.clear();
    int J, rc = check_params(p, &J);
    if (rc) return rc;
    if (j < p->J0 || j > J) return fail(CVL_EINVAL, "scale j=%d outside [%d, %d]", j, p->J0, J);
    if (!Lj || !Nj) return fail(CVL_EINVAL, "output pointer is NULL");
    *Lj = scale_bandlimit(j, p->L, p->lambda);
    *Nj = *Lj;
    return CVL_OK;
}

int cvl_scaling_bandlimit(const cvl_params *p, int *Lphi) {
    g_err.clear();
    int rc = check_params(p, nullptr);
    if (rc) return rc;
    if (!Lphi) return fail(CVL_EINVAL, "output pointer is NULL");
    *Lphi = scaling_bandlimit(p->L, p->lambda, p->J0);
    return CVL_OK;
}

int cvl_workspace_bytes(const cvl_params *p, int batch, size_t *bytes) {
    g_err.clear();
    int J, rc = check_params(p, &J);
    if (rc) return rc;
    if (batch < 1) return fail(CVL_EINVAL, "batch=%d < 1", batch);
    if (!bytes) return fail(CVL_EINVAL, "bytes out-pointer is NULL");
    *bytes = ws_bytes_of(p, J, false);
    return CVL_OK;
}

int cvl_scale_workspace_bytes(const cvl_params *p, size_t *bytes) {
    g_err.clear();
    int J, rc = check_params(p, &J);
    if (rc) return rc;
    if (!bytes) return fail(CVL_EINVAL, "bytes out-pointer is NULL");
    *bytes = ws_bytes_of(p, J, true);
    return CVL_OK;
}

int cvl_sht_workspace_bytes(int L, size_t *bytes) {
    g_err.clear();
    if (L < 2 || L > 2048) return fail(CVL_EINVAL, "L=%d outside [2, 2048]", L);
    if (!bytes) return fail(CVL_EINVAL, "bytes out-pointer is NULL");
    // real maps: three L x L complex buffers; complex maps: two L x (2L-1)
    *bytes = std::max(3 * align_up((size_t)L * L * 16),
                      2 * align_up((size_t)L * (2 * L - 1) * 16)) + kAlign;
    return CVL_OK;
}

int cvl_wigner_workspace_bytes(int L, int N, size_t *bytes) {
    g_err.clear();
    if (L < 1 || L > 2048 || N < 1 || N > L) return fail(CVL_EINVAL, "need 1 <= N <= L <= 2048 (L=%d, N=%d)", L, N);
    if (!bytes) return fail(CVL_EINVAL, "bytes out-pointer is NULL");
    const size_t Nnp = ((2 * N - 1) + 31) / 32 * 32;
    const size_t one = (size_t)L * (2 * L - 1) * Nnp * 16;
    *bytes = 2 * align_up(one) + kAlign;
    return CVL_OK;
}

int cvl_prepare(cvl_ctx *ctx, const cvl_params *p) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    Plan *P;
    if ((rc = get_plan(ctx, p, &P))) return rc;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ShtRt *S;
        if ((rc = get_sht(ctx, P->L, &S))) return rc;
        if ((rc = get_sht(ctx, P->Lphi, &S))) return rc;
    }
    if (spin_rotated(p)) {  // the kernel coefficients and general Wigner tables
        const std::vector<double *> *psi;
        if ((rc = get_spin_psi(ctx, P, p->spin, &psi))) return rc;
        for (const ScaleRt &S : P->scales) {
            GenRt *G;
            if ((rc = get_gen(ctx, S.g.L, S.g.L, &G))) return rc;
        }
    }
    return CVL_OK;
}

int cvl_kernel_tables(const cvl_params *p, double *kappa, double *phi) {
    g_err.clear();
    int J, rc = check_params(p, &J);
    if (rc) return rc;
    if (!kappa || !phi) return fail(CVL_EINVAL, "output pointer is NULL");
    auto k = host::kappa_table(p->L, p->lambda, p->J0, J);
    auto f = host::phi_table(p->L, p->lambda, p->J0);
    std::memcpy(kappa, k.data(), k.size() * sizeof(double));
    std::memcpy(phi, f.data(), f.size() * sizeof(double));
    return CVL_OK;
}

int cvl_sht_forward(cvl_ctx *ctx, int L, int spin, const double *map, cvl_c128 *flm, void *ws,
                    size_t ws_bytes, void *stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (L < 2 || L > ctx->Lmax) return fail(CVL_EINVAL, "L=%d outside [2, L_max=%d]", L, ctx->Lmax);
    if (spin != 0) return fail(CVL_EUNSUPPORTED, "spin=%d: only spin 0 is implemented", spin);
    if (!map || !flm || !ws) return fail(CVL_EINVAL, "NULL device pointer");
    size_t need;
    cvl_sht_workspace_bytes(L, &need);
    if (ws_bytes < need) return fail(CVL_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    if ((rc = set_device(ctx))) return rc;
    ShtRt *S;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if ((rc = get_sht(ctx, L, &S))) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    Carver cv{(char *)ws, ws_bytes};
    cd *fpad = cv.take<cd>((size_t)L * L);
    cd *F1 = cv.take<cd>((size_t)L * L);
    cd *Zs = cv.take<cd>((size_t)L * L);
    if ((rc = sht_forward_run(ctx, S, map, fpad, L, F1, Zs, st))) return rc;
    LAUNCH(ST_MISC, launch_flm_unpack(L, fpad, (cd *)flm, 0, st));
    return CVL_OK;
}

int cvl_sht_inverse(cvl_ctx *ctx, int L, int spin, const cvl_c128 *flm, double *map, void *ws,
                    size_t ws_bytes, void *stream) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (L < 2 || L > ctx->Lmax) return fail(CVL_EINVAL, "L=%d outside [2, L_max=%d]", L, ctx->Lmax);
    if (spin != 0) return fail(CVL_EUNSUPPORTED, "spin=%d: only spin 0 is implemented", spin);
    if (!map || !flm || !ws) return fail(CVL_EINVAL, "NULL device pointer");
    size_t need;
    cvl_sht_workspace_bytes(L, &need);
    if (ws_bytes < need) return fail(CVL_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    if ((rc = set_device(ctx))) return rc;
    ShtRt *S;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if ((rc = get_sht(ctx, L, &S))) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    Carver cv{(char *)ws, ws_bytes};
    cd *fpad = cv.take<cd>((size_t)L * L);
    cd *F = cv.take<cd>((size_t)L * L);
    cd *G = cv.take<cd>((size_t)L * L);
    LAUNCH(ST_MISC, launch_flm_pack(L, (const cd *)flm, fpad, st));
    return sht_inverse_run(ctx, S, fpad, L, map, F, G, st);
}

static int check_sht_call(cvl_ctx *ctx, int L, int spin, const void *a, const void *b, void *ws,
                          size_t ws_bytes, ShtRt **S) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (L < 2 || L > ctx->Lmax) return fail(CVL_EINVAL, "L=%d outside [2, L_max=%d]", L, ctx->Lmax);
    if (spin <= -L || spin >= L) return fail(CVL_EINVAL, "spin=%d outside (-L, L)", spin);
    if (!a || !b || !ws) return fail(CVL_EINVAL, "NULL device pointer");
    size_t need;
    cvl_sht_workspace_bytes(L, &need);
    if (ws_bytes < need) return fail(CVL_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    if ((rc = set_device(ctx))) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return get_sht(ctx, L, S);
}

int cvl_sht_forward_complex(cvl_ctx *ctx, int L, int spin, const cvl_c128 *map, cvl_c128 *flm,
                            void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    ShtRt *S;
    int rc = check_sht_call(ctx, L, spin, map, flm, ws, ws_bytes, &S);
    if (rc) return rc;
    Carver cv{(char *)ws, ws_bytes};
    cd *F1 = cv.take<cd>((size_t)L * (2 * L - 1));
    cd *Zs = cv.take<cd>((size_t)L * (2 * L - 1));
    return sht_forward_cplx_run(ctx, S, spin, (const cd *)map, (cd *)flm, F1, Zs,
                                (hipStream_t)stream);
}

int cvl_sht_inverse_complex(cvl_ctx *ctx, int L, int spin, const cvl_c128 *flm, cvl_c128 *map,
                            void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    ShtRt *S;
    int rc = check_sht_call(ctx, L, spin, flm, map, ws, ws_bytes, &S);
    if (rc) return rc;
    Carver cv{(char *)ws, ws_bytes};
    cd *F = cv.take<cd>((size_t)L * (2 * L - 1));
    cd *G = cv.take<cd>((size_t)L * (2 * L - 1));
    return sht_inverse_cplx_run(ctx, S, spin, (const cd *)flm, (cd *)map, F, G,
                                (hipStream_t)stream);
}

static int get_gen(cvl_ctx *ctx, int L, int N, GenRt **out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto key = std::make_pair(L, N);
    auto it = ctx->gen.find(key);
    if (it != ctx->gen.end()) {
        *out = it->second.get();
        return CVL_OK;
    }
    std::unique_ptr<GenRt> G(new GenRt);
    G->L = L;
    G->N = N;
    int rc;
    if ((rc = get_beta(ctx, L, 0, &G->beta))) return rc;
    const int Nm = 2 * L - 1, Ng = 2 * N - 1;
    if ((rc = get_bluestein(ctx, Nm, Nm, -(L - 1), Nm, 0, +1, &G->a_inv))) return rc;
    if ((rc = get_bluestein(ctx, Nm, Nm, 0, Nm, -(L - 1), -1, &G->a_fwd))) return rc;
    if ((rc = get_bluestein(ctx, Ng, Ng, -(N - 1), Ng, 0, +1, &G->g_inv))) return rc;
    if ((rc = get_bluestein(ctx, Ng, Ng, 0, Ng, -(N - 1), -1, &G->g_fwd))) return rc;
    *out = G.get();
    ctx->gen[key] = std::move(G);
    return CVL_OK;
}

static int check_wigner(cvl_ctx *ctx, int L, int N, const void *a, const void *b, void *ws,
                        size_t ws_bytes) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (L < 1 || L > ctx->Lmax || N < 1 || N > L)
        return fail(CVL_EINVAL, "need 1 <= N <= L <= L_max=%d (L=%d, N=%d)", ctx->Lmax, L, N);
    if (!a || !b || !ws) return fail(CVL_EINVAL, "NULL device pointer");
    size_t need;
    cvl_wigner_workspace_bytes(L, N, &need);
    if (ws_bytes < need) return fail(CVL_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    return CVL_OK;
}

int cvl_wigner_inverse(cvl_ctx *ctx, int L, int N, const cvl_c128 *flmn, cvl_c128 *grid, void *ws,
                       size_t ws_bytes, void *stream) {
    g_err.clear();
    int rc = check_wigner(ctx, L, N, flmn, grid, ws, ws_bytes);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    GenRt *G;
    if ((rc = get_gen(ctx, L, N, &G))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t Nnp = ((2 * N - 1) + 31) / 32 * 32;
    const size_t one = (size_t)L * (2 * L - 1) * Nnp;
    Carver cv{(char *)ws, ws_bytes};
    cd *b0 = cv.take<cd>(one);
    cd *b1 = cv.take<cd>(one);
    const int ncols = (2 * L - 1) * (int)Nnp;
    LAUNCH(ST_CONTRACT_INV, launch_gen_contract_inv(L, N, ctx->delta, (const cd *)flmn, b0, st));
    LAUNCH(ST_BETA_INV, launch_beta_gemm(L, L, ncols, (int)Nnp, 1, (L + N) & 1, G->beta.Cinv,
                                         G->beta.Sinv, b0, b1, st));
    LAUNCH(ST_ALPHA_INV, launch_gen_inv_alpha(L, N, G->a_inv, b1, b0, st));
    LAUNCH(ST_GAMMA_INV, launch_gen_inv_gamma(L, N, G->g_inv, b0, (cd *)grid, st));
    return CVL_OK;
}

int cvl_wigner_forward(cvl_ctx *ctx, int L, int N, const cvl_c128 *grid, cvl_c128 *flmn, void *ws,
                       size_t ws_bytes, void *stream) {
    g_err.clear();
    int rc = check_wigner(ctx, L, N, grid, flmn, ws, ws_bytes);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    GenRt *G;
    if ((rc = get_gen(ctx, L, N, &G))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t Nnp = ((2 * N - 1) + 31) / 32 * 32;
    const size_t one = (size_t)L * (2 * L - 1) * Nnp;
    Carver cv{(char *)ws, ws_bytes};
    cd *b0 = cv.take<cd>(one);
    cd *b1 = cv.take<cd>(one);
    const int ncols = (2 * L - 1) * (int)Nnp;
    LAUNCH(ST_GAMMA_FWD, launch_gen_fwd_gamma(L, N, G->g_fwd, (const cd *)grid, b0, st));
    LAUNCH(ST_ALPHA_FWD, launch_gen_fwd_alpha(L, N, G->a_fwd, b0, b1, st));
    LAUNCH(ST_BETA_FWD, launch_beta_gemm(L, L, ncols, (int)Nnp, 1, (L + N) & 1, G->beta.Qp,
                                         G->beta.Qs, b1, b0, st));
    LAUNCH(ST_CONTRACT_FWD, launch_gen_contract_fwd(L, N, ctx->delta, b0, (cd *)flmn, st));
    return CVL_OK;
}

static int check_curvelet_call(cvl_ctx *ctx, const cvl_params *p, int batch, const void *a,
                               const void *b, const void *grids, void *ws, size_t ws_bytes,
                               Plan **P, bool scale_call = false) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (batch < 1) return fail(CVL_EINVAL, "batch=%d < 1", batch);
    if (!a || !b || !grids || !ws) return fail(CVL_EINVAL, "NULL pointer argument");
    if ((rc = set_device(ctx))) return rc;
    if ((rc = get_plan(ctx, p, P))) return rc;
    const size_t need = ws_bytes_of(p, (*P)->J, scale_call);
    if (ws_bytes < need)
        return fail(CVL_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ShtRt *S;
    if ((rc = get_sht(ctx, (*P)->L, &S))) return rc;
    if ((rc = get_sht(ctx, (*P)->Lphi, &S))) return rc;
    return CVL_OK;
}

struct CurveletBufs {
    void *b0, *b1;
    cd *fpad, *facc, *s0, *s1, *fphi;
    // complex signals: the second (imaginary) part's W2 / V1 plane, padded
    // coefficients and accumulator; the flat coefficients of every m; the
    // complex SHT's scratch at L (c0, c1) and at L_Phi (cp0, cp1)
    void *b2;
    cd *fpadb, *faccb, *flat, *c0, *c1, *cp0, *cp1;
    void *sb0, *sb1;  // cube buffers of the side scales
    cd *sfacc;        // harmonic accumulator of the side scales' synthesis
    void *sb2;        // complex signals: the side scales' second plane and
    cd *sfaccb;       // second accumulator
};

static CurveletBufs carve_curvelet(const Plan *P, int precision, bool unrot, bool cplx,
                                   void *ws, size_t ws_bytes) {
    size_t b0, b1, sb0, sb1, p2, sp2;
    curvelet_buf_elems(P->L, P->lambda, P->J0, P->J, unrot, &b0, &b1, &sb0, &sb1);
    curvelet_plane_elems(P->L, P->lambda, P->J0, P->J, unrot, &p2, &sp2);
    const size_t esz = precision == CVL_FP64 ? 16 : 8;
    // the per-scale calls may pass the first part only: the side-stream
    // buffers then come out null, and those calls do not use them
    Carver cv{(char *)ws, ws_bytes};
    CurveletBufs B{};
    B.b0 = cv.take<char>(b0 * esz);
    B.b1 = cv.take<char>(b1 * esz);
    const size_t L2 = (size_t)P->L * P->L;
    B.fpad = cv.take<cd>(L2);
    B.facc = cv.take<cd>(L2);
    B.s0 = cv.take<cd>(L2);
    B.s1 = cv.take<cd>(L2);
    B.fphi = cv.take<cd>((size_t)P->Lphi * P->Lphi);
    if (cplx) {
        B.b2 = cv.take<char>(p2 * esz);
        B.fpadb = cv.take<cd>(L2);
        B.faccb = cv.take<cd>(L2);
        B.flat = cv.take<cd>(L2);
        B.c0 = cv.take<cd>((size_t)P->L * (2 * P->L - 1));
        B.c1 = cv.take<cd>((size_t)P->L * (2 * P->L - 1));
        B.cp0 = cv.take<cd>((size_t)P->Lphi * (2 * P->Lphi - 1));
        B.cp1 = cv.take<cd>((size_t)P->Lphi * (2 * P->Lphi - 1));
    }
    B.sb0 = cv.take<char>(sb0 * esz);
    B.sb1 = cv.take<char>(sb1 * esz);
    B.sfacc = cv.take<cd>(L2);
    if (cplx) {
        B.sb2 = cv.take<char>(sp2 * esz);
        B.sfaccb = cv.take<cd>(L2);
    }
    return B;
}

// The buffers a side-scale run uses: its own cubes and accumulators, the
// shared (read-only) padded harmonic coefficients.
static CurveletBufs side_bufs(const CurveletBufs &B) {
    CurveletBufs S = B;
    S.b0 = B.sb0;
    S.b1 = B.sb1;
    S.facc = B.sfacc;
    S.b2 = B.sb2;
    S.faccb = B.sfaccb;
    return S;
}

static bool real_grids(const cvl_params *p) { return (p->flags & CVL_REAL_GRIDS) != 0; }
static bool complex_map(const cvl_params *p) { return (p->flags & CVL_REAL) == 0; }
static bool unrotated(const cvl_params *p) { return (p->flags & CVL_UNROTATED) != 0; }

// Analysis of one scale of the unrotated curvelets (same buffers and stages
// as the rotated one, on the unrotated cube layout).
extern "C++" {
template <class C, class G, class BT>
static int unrot_analysis_t(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                            const BT &full, const BT &beta_inv, const CurveletBufs &B, G *grid,
                            hipStream_t st) {
    const ScaleGeom &g = S.g;
    C *b0 = (C *)B.b0, *b1 = (C *)B.b1;
    LAUNCH(ST_CONTRACT_INV,
           launch_unrot_contract_inv(g, P->L, ctx->delta, B.fpad, S.pd, b0, !S.beta_fft, st));
    const int ncols = 2 * g.L * g.Nep;
    if (S.beta_fft)
        LAUNCH(ST_BETA_INV, launch_unrot_inv_beta_dft(g, beta_inv, b0, b1, st));
    else if (precision == CVL_FP64)
        LAUNCH(ST_BETA_INV, launch_beta_gemm(g.L, g.L, ncols, g.Nep, 0, 0, S.beta.Cinv,
                                             S.beta.Sinv, (const cd *)b0, (cd *)b1, st));
    else
        LAUNCH(ST_BETA_INV, launch_beta_gemm_f32(precision, g.L, g.L, ncols, g.Nep, S.betaf.Cinv,
                                                 S.betaf.Sinv, (const cf *)b0, (cf *)b1, st));
    LAUNCH(ST_ALPHA_INV, launch_unrot_inv_alpha(g, full, b1, b0, st));
    LAUNCH(ST_GAMMA_INV, launch_unrot_inv_gamma(g, full, b0, grid, st));
    return CVL_OK;
}

template <class C, class G, class BT>
static int unrot_synthesis_t(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                             const BT &full, const CurveletBufs &B, const G *grid,
                             hipStream_t st) {
    const ScaleGeom &g = S.g;
    C *b0 = (C *)B.b0, *b1 = (C *)B.b1;
    LAUNCH(ST_GAMMA_FWD, launch_unrot_fwd_gamma(g, full, grid, b0, st));
    LAUNCH(ST_ALPHA_FWD, launch_unrot_fwd_alpha(g, full, b0, b1, st));
    const int ncols = 2 * g.L * g.Nep;
    if (precision == CVL_FP64)
        LAUNCH(ST_BETA_FWD, launch_beta_gemm_unrot_fwd(g, S.beta.Qp, S.beta.Qs, (const cd *)b1,
                                                       (cd *)b0, st));
    else
        LAUNCH(ST_BETA_FWD, launch_beta_gemm_f32(precision, g.L, g.L, ncols, g.Nep, S.betaf.Qp,
                                                 S.betaf.Qs, (const cf *)b1, (cf *)b0, st));
    LAUNCH(ST_CONTRACT_FWD,
           launch_unrot_contract_fwd(g, P->L, ctx->delta, (const C *)b0, S.pd, B.facc, st));
    return CVL_OK;
}
}  // extern "C++"

// Analysis of one scale from the padded harmonic coefficients B.fpad into a
// complex (zero imaginary parts) or, with real_grid, a real grid.
static int analysis_scale_run(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                              bool real_grid, bool unrot, const CurveletBufs &B, void *grid_out,
                              hipStream_t st) {
    const ScaleGeom &g = S.g;
    const int L = P->L;
    TagScope tag(g.L);
    if (unrot) {
        if (precision == CVL_FP64)
            return real_grid ? unrot_analysis_t<cd>(ctx, P, S, precision, S.inv_full, S.beta_inv, B,
                                                    (double *)grid_out, st)
                             : unrot_analysis_t<cd>(ctx, P, S, precision, S.inv_full, S.beta_inv, B,
                                                    (cd *)grid_out, st);
        return real_grid ? unrot_analysis_t<cf>(ctx, P, S, precision, S.inv_full_f, S.beta_inv_f, B,
                                                (float *)grid_out, st)
                         : unrot_analysis_t<cf>(ctx, P, S, precision, S.inv_full_f, S.beta_inv_f, B,
                                                (cf *)grid_out, st);
    }
    // X in b0; W1 in b1 (in b0 after a line-major beta DFT); W2 in the other one
    // (complex128: W1 in b1, W2 in b0)
    if (precision != CVL_FP64) {
        cf *b0 = (cf *)B.b0, *b1 = (cf *)B.b1, *w1 = b1;
        LAUNCH(ST_CONTRACT_INV,
               launch_contract_inv_mx(precision, g, L, ctx->delta, B.fpad, S.psi, b0, st));
        if (S.beta_lines) {
            LAUNCH(ST_BETA_INV, launch_inv_beta_dft_lines(g, S.beta_inv_f, b0, b1, st));
            LAUNCH(ST_BETA_INV, launch_beta_lines_to_planes(g, b1, b0, st));
            w1 = b0;
        } else if (S.beta_fft) {
            LAUNCH(ST_BETA_INV, launch_inv_beta_dft(g, S.beta_inv_f, b0, b1, st));
        } else {
            LAUNCH(ST_BETA_INV, launch_beta_gemm_f32(precision, g.L, g.L, g.L * g.Nep, g.Nep,
                                                     S.betaf.Cinv, S.betaf.Sinv, b0, b1, st));
        }
        cf *w2 = w1 == b0 ? b1 : b0;
        LAUNCH(ST_ALPHA_INV, launch_inv_alpha(g, S.inv_full_f, w1, w2, st));
        if (real_grid)
            LAUNCH(ST_GAMMA_INV, launch_inv_gamma(g, S.inv_full_f, w2, (float *)grid_out, st));
        else
            LAUNCH(ST_GAMMA_INV, launch_inv_gamma(g, S.inv_full_f, w2, (cf *)grid_out, st));
        return CVL_OK;
    }
    cd *b0 = (cd *)B.b0, *b1 = (cd *)B.b1;
    LAUNCH(ST_CONTRACT_INV, launch_contract_inv(g, L, ctx->delta, B.fpad, S.psi, b0, st));
    if (S.beta_fft)
        LAUNCH(ST_BETA_INV, launch_inv_beta_dft(g, S.beta_inv, b0, b1, st));
    else
        LAUNCH(ST_BETA_INV, launch_beta_gemm(g.L, g.L, g.L * g.Nep, g.Nep, 0, 0, S.beta.Cinv,
                                             S.beta.Sinv, b0, b1, st));
    LAUNCH(ST_ALPHA_INV, launch_inv_alpha(g, S.inv_full, b1, b0, st));
    if (real_grid)
        LAUNCH(ST_GAMMA_INV, launch_inv_gamma(g, S.inv_full, b0, (double *)grid_out, st));
    else
        LAUNCH(ST_GAMMA_INV, launch_inv_gamma(g, S.inv_full, b0, (cd *)grid_out, st));
    return CVL_OK;
}

// Synthesis of one scale (real parts of a complex grid, or a real grid): adds
// f^(j)_lm into the padded accumulator B.facc.
static int synthesis_scale_run(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                               bool real_grid, bool unrot, const CurveletBufs &B,
                               const void *grid_in, hipStream_t st) {
    const ScaleGeom &g = S.g;
    const int L = P->L;
    TagScope tag(g.L);
    if (unrot) {
        if (precision == CVL_FP64)
            return real_grid ? unrot_synthesis_t<cd>(ctx, P, S, precision, S.fwd_full, B,
                                                     (const double *)grid_in, st)
                             : unrot_synthesis_t<cd>(ctx, P, S, precision, S.fwd_full, B,
                                                     (const cd *)grid_in, st);
        return real_grid ? unrot_synthesis_t<cf>(ctx, P, S, precision, S.fwd_full_f, B,
                                                 (const float *)grid_in, st)
                         : unrot_synthesis_t<cf>(ctx, P, S, precision, S.fwd_full_f, B,
                                                 (const cf *)grid_in, st);
    }
    if (precision != CVL_FP64) {
        cf *b0 = (cf *)B.b0, *b1 = (cf *)B.b1;
        const BluesteinF &F = S.fwd_full_f;
        if (real_grid)
            LAUNCH(ST_GAMMA_FWD, launch_fwd_gamma(g, F, (const float *)grid_in, b0, st));
        else
            LAUNCH(ST_GAMMA_FWD, launch_fwd_gamma(g, F, (const cf *)grid_in, b0, st));
        LAUNCH(ST_ALPHA_FWD, launch_fwd_alpha(g, S.fwd_full_f, b0, b1, st));
        LAUNCH(ST_BETA_FWD, launch_beta_gemm_f32(precision, g.L, g.L, g.L * g.Nep, g.Nep, S.betaf.Qp,
                                                 S.betaf.Qs, b1, b0, st));
        LAUNCH(ST_CONTRACT_FWD,
               launch_contract_fwd_mx(precision, g, ctx->delta, b0, S.psi, b1, st));
        LAUNCH(ST_REDUCE_FWD, launch_reduce_fwd_mx(g, L, b1, S.ngroups, B.facc, st));
        return CVL_OK;
    }
    cd *b0 = (cd *)B.b0, *b1 = (cd *)B.b1;
    if (real_grid)
        LAUNCH(ST_GAMMA_FWD, launch_fwd_gamma(g, S.fwd_full, (const double *)grid_in, b0, st));
    else
        LAUNCH(ST_GAMMA_FWD, launch_fwd_gamma(g, S.fwd_full, (const cd *)grid_in, b0, st));
    LAUNCH(ST_ALPHA_FWD, launch_fwd_alpha(g, S.fwd_full, b0, b1, st));
    LAUNCH(ST_BETA_FWD, launch_beta_gemm(g.L, g.L, g.L * g.Nep, g.Nep, 0, 0, S.beta.Qp,
                                         S.beta.Qs, b1, b0, st));
    LAUNCH(ST_CONTRACT_FWD, launch_contract_fwd(g, ctx->delta, b0, S.psi, b1, st));
    LAUNCH(ST_REDUCE_FWD, launch_reduce_fwd(g, L, b1, S.ngroups, B.facc, st));
    return CVL_OK;
}

// ---- complex signals: each scale runs the real-signal stages twice, on the
// coefficients of the signal's real part (B.fpad) and imaginary part
// (B.fpadb), up to their W2 planes, and one complex gamma DFT combines the
// two into the complex grid W = W_a + i W_b (the curvelets' harmonic
// coefficients obey the reality condition, so each part's coefficients are
// real and the analysis is linear).  The synthesis splits each complex grid
// line into its two real parts' coefficients and accumulates them into
// B.facc and B.faccb. ----
extern "C++" {
template <class C> struct FullTabs;
template <> struct FullTabs<cd> {
    static const BluesteinDev &inv(const ScaleRt &S) { return S.inv_full; }
    static const BluesteinDev &fwd(const ScaleRt &S) { return S.fwd_full; }
    static const BluesteinDev &beta(const ScaleRt &S) { return S.beta_inv; }
};
template <> struct FullTabs<cf> {
    static const BluesteinF &inv(const ScaleRt &S) { return S.inv_full_f; }
    static const BluesteinF &fwd(const ScaleRt &S) { return S.fwd_full_f; }
    static const BluesteinF &beta(const ScaleRt &S) { return S.beta_inv_f; }
};

static hipError_t beta_gemm_any(int precision, int M, int K, int ncols, int Nep,
                                const BetaTabs &T64, const BetaTabsF &T32, bool inverse,
                                const void *in, void *out, hipStream_t st) {
    if (precision == CVL_FP64)
        return launch_beta_gemm(M, K, ncols, Nep, 0, 0, inverse ? T64.Cinv : T64.Qp,
                                inverse ? T64.Sinv : T64.Qs, (const cd *)in, (cd *)out, st);
    return launch_beta_gemm_f32(precision, M, K, ncols, Nep, inverse ? T32.Cinv : T32.Qp,
                                inverse ? T32.Sinv : T32.Qs, (const cf *)in, (cf *)out, st);
}

// Analysis stages of one part (padded coefficients fp) up to its W2 plane
// (cube scratch b0, b1): into w2, or, with w2 null, into whichever cube
// buffer the stages leave free (b0, or b1 after a line-major beta DFT);
// *w2_out receives the plane.
template <class C>
static int analysis_to_w2(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                          bool unrot, const cd *fp, C *b0, C *b1, C *w2, C **w2_out,
                          hipStream_t st) {
    const ScaleGeom &g = S.g;
    const int L = P->L;
    if (unrot) {
        LAUNCH(ST_CONTRACT_INV,
               launch_unrot_contract_inv(g, L, ctx->delta, fp, S.pd, b0, !S.beta_fft, st));
        if (S.beta_fft)
            LAUNCH(ST_BETA_INV, launch_unrot_inv_beta_dft(g, FullTabs<C>::beta(S), b0, b1, st));
        else
            LAUNCH(ST_BETA_INV, beta_gemm_any(precision, g.L, g.L, 2 * g.L * g.Nep, g.Nep,
                                              S.beta, S.betaf, true, b0, b1, st));
        C *dst = w2 ? w2 : b0;
        LAUNCH(ST_ALPHA_INV, launch_unrot_inv_alpha(g, FullTabs<C>::inv(S), b1, dst, st));
        *w2_out = dst;
        return CVL_OK;
    }
    if constexpr (std::is_same<C, cd>::value)
        LAUNCH(ST_CONTRACT_INV, launch_contract_inv(g, L, ctx->delta, fp, S.psi, b0, st));
    else
        LAUNCH(ST_CONTRACT_INV,
               launch_contract_inv_mx(precision, g, L, ctx->delta, fp, S.psi, b0, st));
    C *w1 = b1;
    if (S.beta_lines && std::is_same<C, cf>::value) {
        LAUNCH(ST_BETA_INV, launch_inv_beta_dft_lines(g, FullTabs<C>::beta(S), b0, b1, st));
        LAUNCH(ST_BETA_INV, launch_beta_lines_to_planes(g, b1, b0, st));
        w1 = b0;
    } else if (S.beta_fft) {
        LAUNCH(ST_BETA_INV, launch_inv_beta_dft(g, FullTabs<C>::beta(S), b0, b1, st));
    } else {
        LAUNCH(ST_BETA_INV, beta_gemm_any(precision, g.L, g.L, g.L * g.Nep, g.Nep, S.beta,
                                          S.betaf, true, b0, b1, st));
    }
    C *dst = w2 ? w2 : (w1 == b0 ? b1 : b0);
    LAUNCH(ST_ALPHA_INV, launch_inv_alpha(g, FullTabs<C>::inv(S), w1, dst, st));
    *w2_out = dst;
    return CVL_OK;
}

// Synthesis stages of one part from its V1 plane v1 (which may be b0) into
// the padded accumulator acc (cube scratch b0, b1).
template <class C>
static int synthesis_from_v1(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                             bool unrot, C *v1, C *b0, C *b1, cd *acc, hipStream_t st) {
    const ScaleGeom &g = S.g;
    const int L = P->L;
    if (unrot) {
        LAUNCH(ST_ALPHA_FWD, launch_unrot_fwd_alpha(g, FullTabs<C>::fwd(S), v1, b1, st));
        if (precision == CVL_FP64)
            LAUNCH(ST_BETA_FWD, launch_beta_gemm_unrot_fwd(g, S.beta.Qp, S.beta.Qs,
                                                           (const cd *)b1, (cd *)b0, st));
        else
            LAUNCH(ST_BETA_FWD, beta_gemm_any(precision, g.L, g.L, 2 * g.L * g.Nep, g.Nep,
                                              S.beta, S.betaf, false, b1, b0, st));
        LAUNCH(ST_CONTRACT_FWD,
               launch_unrot_contract_fwd(g, L, ctx->delta, (const C *)b0, S.pd, acc, st));
        return CVL_OK;
    }
    LAUNCH(ST_ALPHA_FWD, launch_fwd_alpha(g, FullTabs<C>::fwd(S), v1, b1, st));
    LAUNCH(ST_BETA_FWD, beta_gemm_any(precision, g.L, g.L, g.L * g.Nep, g.Nep, S.beta, S.betaf,
                                      false, b1, b0, st));
    if constexpr (std::is_same<C, cd>::value) {
        LAUNCH(ST_CONTRACT_FWD, launch_contract_fwd(g, ctx->delta, b0, S.psi, b1, st));
        LAUNCH(ST_REDUCE_FWD, launch_reduce_fwd(g, L, b1, S.ngroups, acc, st));
    } else {
        LAUNCH(ST_CONTRACT_FWD,
               launch_contract_fwd_mx(precision, g, ctx->delta, b0, S.psi, b1, st));
        LAUNCH(ST_REDUCE_FWD, launch_reduce_fwd_mx(g, L, b1, S.ngroups, acc, st));
    }
    return CVL_OK;
}

template <class C>
static int analysis_scale_cplx_t(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                                 bool unrot, const CurveletBufs &B, C *grid, hipStream_t st) {
    C *b0 = (C *)B.b0, *b1 = (C *)B.b1, *b2 = (C *)B.b2, *wa = nullptr, *wb = nullptr;
    int rc = analysis_to_w2<C>(ctx, P, S, precision, unrot, B.fpad, b0, b1, b2, &wa, st);
    if (!rc) rc = analysis_to_w2<C>(ctx, P, S, precision, unrot, B.fpadb, b0, b1, nullptr, &wb, st);
    if (rc) return rc;
    if (unrot)
        LAUNCH(ST_GAMMA_INV, launch_unrot_inv_gamma_cplx(S.g, FullTabs<C>::inv(S), wa, wb, grid, st));
    else
        LAUNCH(ST_GAMMA_INV, launch_inv_gamma_cplx(S.g, FullTabs<C>::inv(S), wa, wb, grid, st));
    return CVL_OK;
}

template <class C>
static int synthesis_scale_cplx_t(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                                  bool unrot, const CurveletBufs &B, const C *grid,
                                  hipStream_t st) {
    C *b0 = (C *)B.b0, *b1 = (C *)B.b1, *b2 = (C *)B.b2;
    if (unrot)
        LAUNCH(ST_GAMMA_FWD, launch_unrot_fwd_gamma_cplx(S.g, FullTabs<C>::fwd(S), grid, b2, b0, st));
    else
        LAUNCH(ST_GAMMA_FWD, launch_fwd_gamma_cplx(S.g, FullTabs<C>::fwd(S), grid, b2, b0, st));
    // the imaginary part first: its V1 plane sits in b0, which the stages reuse
    int rc = synthesis_from_v1<C>(ctx, P, S, precision, unrot, b0, b0, b1, B.faccb, st);
    if (!rc) rc = synthesis_from_v1<C>(ctx, P, S, precision, unrot, b2, b0, b1, B.facc, st);
    return rc;
}

static int analysis_scale_cplx(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                               bool unrot, const CurveletBufs &B, void *grid, hipStream_t st) {
    TagScope tag(S.g.L);
    if (precision == CVL_FP64)
        return analysis_scale_cplx_t<cd>(ctx, P, S, precision, unrot, B, (cd *)grid, st);
    return analysis_scale_cplx_t<cf>(ctx, P, S, precision, unrot, B, (cf *)grid, st);
}

static int synthesis_scale_cplx(cvl_ctx *ctx, const Plan *P, const ScaleRt &S, int precision,
                                bool unrot, const CurveletBufs &B, const void *grid,
                                hipStream_t st) {
    TagScope tag(S.g.L);
    if (precision == CVL_FP64)
        return synthesis_scale_cplx_t<cd>(ctx, P, S, precision, unrot, B, (const cd *)grid, st);
    return synthesis_scale_cplx_t<cf>(ctx, P, S, precision, unrot, B, (const cf *)grid, st);
}

}  // extern "C++"

// ---- side stream: the scales below the top band-limit run concurrently with
// the top ones (they only meet in the sum over scales); every call forks and
// joins it with events, so callers see plain stream order. ----
static int get_side(cvl_ctx *ctx, hipStream_t st, cvl_ctx::Side **out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->side.find(st);
    if (it == ctx->side.end()) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(ctx->device);
        cvl_ctx::Side sd;
        hipError_t e = hipStreamCreateWithFlags(&sd.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sd.join, hipEventDisableTiming);
        (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            if (sd.join) (void)hipEventDestroy(sd.join);
            if (sd.fork) (void)hipEventDestroy(sd.fork);
            if (sd.s) (void)hipStreamDestroy(sd.s);
            return fail(CVL_EDEVICE, "side stream creation failed: %s", hipGetErrorString(e));
        }
        it = ctx->side.emplace(st, sd).first;
    }
    *out = &it->second;
    return CVL_OK;
}

static int side_fork(cvl_ctx::Side *sd, hipStream_t st) {
    hipError_t e = hipEventRecord(sd->fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(sd->s, sd->fork, 0);
    return e == hipSuccess ? CVL_OK : fail(CVL_EDEVICE, "side fork: %s", hipGetErrorString(e));
}

static int side_join(cvl_ctx::Side *sd, hipStream_t st) {
    hipError_t e = hipEventRecord(sd->join, sd->s);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, sd->join, 0);
    return e == hipSuccess ? CVL_OK : fail(CVL_EDEVICE, "side join: %s", hipGetErrorString(e));
}

// Leading scales (ordered by band-limit) below the top band-limit.
static int side_count(const Plan *P) {
    const int top = P->scales.back().g.L;
    int n = 0;
    while (n < (int)P->scales.size() && P->scales[n].g.L < top) ++n;
    return n;
}

static int analysis_scales(cvl_ctx *ctx, const Plan *P, const cvl_params *p,
                           const CurveletBufs &B, void *const *grids, int s0, int s1,
                           hipStream_t st) {
    for (int s = s0; s < s1; ++s) {
        int rc = analysis_scale_run(ctx, P, P->scales[s], p->precision, real_grids(p),
                                    unrotated(p), B,
                                    grids[s], st);
        if (rc) return rc;
    }
    return CVL_OK;
}

// Scaling part of the analysis: (W^Phi)_lm = phifac_l f_lm, then the inverse
// SHT at L_Phi into the scaling map (scratch X.s0, X.s1).
static int scaling_analysis_run(cvl_ctx *ctx, const Plan *P, ShtRt *SP, const CurveletBufs &X,
                                double *smap, hipStream_t st) {
    LAUNCH(ST_MISC, launch_scale_flm(P->Lphi, P->L, P->Lphi, P->phifac, X.fpad, X.fphi, 0, st));
    return sht_inverse_run(ctx, SP, X.fphi, P->Lphi, smap, X.s0, X.s1, st);
}

// Scaling part of the synthesis: forward SHT of the scaling map at L_Phi, then
// X.facc[l][m] += phifac_l (W^Phi)_lm.
static int scaling_synthesis_run(cvl_ctx *ctx, const Plan *P, ShtRt *SP, const CurveletBufs &X,
                                 const double *smap, hipStream_t st) {
    int rc = sht_forward_run(ctx, SP, smap, X.fphi, P->Lphi, X.s0, X.s1, st);
    if (rc) return rc;
    LAUNCH(ST_MISC, launch_scale_flm(P->Lphi, P->Lphi, P->L, P->phifac, X.fphi, X.facc, 1, st));
    return CVL_OK;
}

// Scaling part of the analysis of a complex signal: (W^Phi)_lm = phifac_l
// f_lm on the flat coefficients of every m (X.flat), then the complex spin-0
// inverse SHT at L_Phi (the scaling coefficients are a spin-0 map).
static int scaling_analysis_cplx_run(cvl_ctx *ctx, const Plan *P, ShtRt *SP,
                                     const CurveletBufs &X, cd *smap, hipStream_t st) {
    LAUNCH(ST_MISC, launch_scale_flat(P->Lphi, P->phifac, X.flat, X.fphi, 0, st));
    return sht_inverse_cplx_run(ctx, SP, 0, X.fphi, smap, X.cp0, X.cp1, st);
}

// Forward complex spin-0 SHT of the scaling map into X.fphi (flat); the
// caller adds phifac_l times it into the synthesised coefficients.
static int scaling_synthesis_cplx_run(cvl_ctx *ctx, ShtRt *SP, const CurveletBufs &X,
                                      const cd *smap, hipStream_t st) {
    return sht_forward_cplx_run(ctx, SP, 0, smap, X.fphi, X.cp0, X.cp1, st);
}

static int analysis_scales_cplx(cvl_ctx *ctx, const Plan *P, const cvl_params *p,
                                const CurveletBufs &B, void *const *grids, int s0, int s1,
                                hipStream_t st) {
    for (int s = s0; s < s1; ++s) {
        int rc = analysis_scale_cplx(ctx, P, P->scales[s], p->precision, unrotated(p), B,
                                     grids[s], st);
        if (rc) return rc;
    }
    return CVL_OK;
}

// Zeroes B.facc and B.faccb, then adds the synthesis of scales [s0, s1).
static int synthesis_scales_cplx(cvl_ctx *ctx, const Plan *P, const cvl_params *p,
                                 const CurveletBufs &B, const void *const *grids, int s0,
                                 int s1, hipStream_t st) {
    LAUNCH(ST_MISC, launch_zero(B.facc, (size_t)P->L * P->L, st));
    LAUNCH(ST_MISC, launch_zero(B.faccb, (size_t)P->L * P->L, st));
    for (int s = s0; s < s1; ++s) {
        int rc = synthesis_scale_cplx(ctx, P, P->scales[s], p->precision, unrotated(p), B,
                                      grids[s], st);
        if (rc) return rc;
    }
    return CVL_OK;
}

// Zeroes B.facc, then adds the synthesis of scales [s0, s1) into it.
static int synthesis_scales(cvl_ctx *ctx, const Plan *P, const cvl_params *p,
                            const CurveletBufs &B, const void *const *grids, int s0, int s1,
                            hipStream_t st) {
    LAUNCH(ST_MISC, launch_zero(B.facc, (size_t)P->L * P->L, st));
    for (int s = s0; s < s1; ++s) {
        int rc = synthesis_scale_run(ctx, P, P->scales[s], p->precision, real_grids(p),
                                     unrotated(p), B,
                                     grids[s], st);
        if (rc) return rc;
    }
    return CVL_OK;
}

static int curvelet_analysis_cplx(cvl_ctx *ctx, const cvl_params *p, const Plan *P, int batch,
                                  const cd *maps, cd *scal_maps, void *const *grids,
                                  const CurveletBufs &B, hipStream_t st, bool side_ok) {
    const CurveletBufs BS = side_bufs(B);
    const int L = P->L, Lp = P->Lphi, nJ = P->J - P->J0 + 1;
    const int nside = side_ok ? side_count(P) : 0;
    ShtRt *SL = ctx->sht[L].get(), *SP = ctx->sht[Lp].get();
    cvl_ctx::Side *sd = nullptr;
    int rc;
    if (nside > 0 && (rc = get_side(ctx, st, &sd))) return rc;
    for (int bi = 0; bi < batch; ++bi) {
        const cd *map = maps + (size_t)bi * L * (2 * L - 1);
        cd *smap = scal_maps + (size_t)bi * Lp * (2 * Lp - 1);
        void *const *g = grids + (size_t)bi * nJ;
        if ((rc = sht_forward_cplx_run(ctx, SL, p->spin, map, B.flat, B.c0, B.c1, st))) return rc;
        LAUNCH(ST_MISC, launch_flm_split(L, B.flat, B.fpad, B.fpadb, st));
        if (!sd && (rc = scaling_analysis_cplx_run(ctx, P, SP, B, smap, st))) return rc;
        if (sd && (rc = side_fork(sd, st))) return rc;
        rc = analysis_scales_cplx(ctx, P, p, B, g, nside, nJ, st);
        if (!rc && sd) rc = scaling_analysis_cplx_run(ctx, P, SP, BS, smap, sd->s);
        if (!rc && sd) rc = analysis_scales_cplx(ctx, P, p, BS, g, 0, nside, sd->s);
        const int rj = sd ? side_join(sd, st) : CVL_OK;
        if (rc || (rc = rj)) return rc;
    }
    return CVL_OK;
}

static int curvelet_synthesis_cplx(cvl_ctx *ctx, const cvl_params *p, const Plan *P, int batch,
                                   const cd *scal_maps, const void *const *grids, cd *maps,
                                   const CurveletBufs &B, hipStream_t st) {
    const CurveletBufs BS = side_bufs(B);
    const int L = P->L, Lp = P->Lphi, nside = side_count(P), nJ = P->J - P->J0 + 1;
    ShtRt *SL = ctx->sht[L].get(), *SP = ctx->sht[Lp].get();
    cvl_ctx::Side *sd = nullptr;
    int rc;
    if (nside > 0 && (rc = get_side(ctx, st, &sd))) return rc;
    for (int bi = 0; bi < batch; ++bi) {
        const cd *smap = scal_maps + (size_t)bi * Lp * (2 * Lp - 1);
        cd *map = maps + (size_t)bi * L * (2 * L - 1);
        const void *const *g = grids + (size_t)bi * nJ;
        if (sd && (rc = side_fork(sd, st))) return rc;
        rc = synthesis_scales_cplx(ctx, P, p, B, g, nside, nJ, st);
        if (!rc && sd) rc = synthesis_scales_cplx(ctx, P, p, BS, g, 0, nside, sd->s);
        if (!rc && sd) rc = scaling_synthesis_cplx_run(ctx, SP, BS, smap, sd->s);
        const int rj = sd ? side_join(sd, st) : CVL_OK;
        if (rc || (rc = rj)) return rc;
        if (sd) {
            LAUNCH(ST_MISC, launch_add(B.facc, BS.facc, (size_t)L * L, st));
            LAUNCH(ST_MISC, launch_add(B.faccb, BS.faccb, (size_t)L * L, st));
        } else if ((rc = scaling_synthesis_cplx_run(ctx, SP, B, smap, st))) {
            return rc;
        }
        LAUNCH(ST_MISC, launch_flm_combine(L, B.facc, B.faccb, B.flat, 0, st));
        LAUNCH(ST_MISC, launch_scale_flat(Lp, P->phifac, B.fphi, B.flat, 1, st));
        if ((rc = sht_inverse_cplx_run(ctx, SL, p->spin, B.flat, map, B.c0, B.c1, st))) return rc;
    }
    return CVL_OK;
}

// ---- rotated spin-s curvelets (general Wigner layouts, caller's stream) ----
static int get_spin_psi(cvl_ctx *ctx, const Plan *P, int spin, const std::vector<double *> **out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto key = std::make_tuple(P->L, P->lambda, P->J0, spin);
    auto it = ctx->spin_psi.find(key);
    if (it == ctx->spin_psi.end()) {
        const int L = P->L;
        std::vector<double> kap = host::kappa_table(L, P->lambda, P->J0, P->J);
        std::vector<double *> tabs;
        for (const ScaleRt &S : P->scales) {
            const int Lj = S.g.L, Nm = 2 * Lj - 1;
            // theta_j = arccos(-s / lambda^j), clamped to [0, pi] where lambda^j < |s|
            const double c = std::max(-1.0, std::min(1.0, -spin / std::pow(P->lambda, S.j)));
            std::vector<double> z = host::zeta_rotated(Lj, std::acos(c));
            const double *kj = &kap[(size_t)(S.j - P->J0) * L];
            for (int l = 0; l < Lj; ++l) {
                const double f = std::sqrt((2.0 * l + 1.0) / (8.0 * M_PI * M_PI)) * kj[l];
                for (int n = 0; n < Nm; ++n) z[(size_t)l * Nm + n] *= f;
            }
            double *d;
            int rc = ctx->arena.upload(z, &d);
            if (rc) return rc;
            tabs.push_back(d);
        }
        it = ctx->spin_psi.emplace(key, std::move(tabs)).first;
    }
    *out = &it->second;
    return CVL_OK;
}

struct SpinBufs {
    cd *g0, *g1, *F, *flat, *acc, *c0, *c1, *cp0, *cp1, *fphi;
};

static SpinBufs carve_spin(const Plan *P, void *ws, size_t ws_bytes) {
    const int T = P->scales.back().g.L, L = P->L, Lp = P->Lphi;
    const size_t Nm = 2 * T - 1, Nnp = (Nm + 31) / 32 * 32;
    Carver cv{(char *)ws, ws_bytes};
    SpinBufs B{};
    B.g0 = cv.take<cd>((size_t)T * Nm * Nnp);
    B.g1 = cv.take<cd>((size_t)T * Nm * Nnp);
    B.F = cv.take<cd>((size_t)T * Nm * Nm);
    B.flat = cv.take<cd>((size_t)L * L);
    B.acc = cv.take<cd>((size_t)L * L);
    B.c0 = cv.take<cd>((size_t)L * (2 * L - 1));
    B.c1 = cv.take<cd>((size_t)L * (2 * L - 1));
    B.cp0 = cv.take<cd>((size_t)Lp * (2 * Lp - 1));
    B.cp1 = cv.take<cd>((size_t)Lp * (2 * Lp - 1));
    B.fphi = cv.take<cd>((size_t)Lp * Lp);
    return B;
}

// Grid of scale s from the flat coefficients B.flat.
static int spin_analysis_scale(cvl_ctx *ctx, const Plan *P, int s, const double *psi,
                               const SpinBufs &B, cd *grid, hipStream_t st) {
    const ScaleGeom &g = P->scales[s].g;
    const int Lj = g.L;
    TagScope tag(Lj);
    GenRt *G;
    int rc = get_gen(ctx, Lj, Lj, &G);
    if (rc) return rc;
    const int Nnp = ((2 * Lj - 1) + 31) / 32 * 32, ncols = (2 * Lj - 1) * Nnp;
    LAUNCH(ST_CONTRACT_INV,
           launch_spin_contract_inv(Lj, g.llo, g.lhi, ctx->delta, B.flat, psi, B.g0, st));
    LAUNCH(ST_BETA_INV, launch_beta_gemm(Lj, Lj, ncols, Nnp, 1, 0, G->beta.Cinv, G->beta.Sinv,
                                         B.g0, B.g1, st));
    LAUNCH(ST_ALPHA_INV, launch_gen_inv_alpha(Lj, Lj, G->a_inv, B.g1, B.g0, st));
    LAUNCH(ST_GAMMA_INV, launch_gen_inv_gamma(Lj, Lj, G->g_inv, B.g0, grid, st));
    return CVL_OK;
}

// acc (flat) += the synthesis of scale s's grid.
static int spin_synthesis_scale(cvl_ctx *ctx, const Plan *P, int s, const double *psi,
                                const SpinBufs &B, const cd *grid, cd *acc, hipStream_t st) {
    const int Lj = P->scales[s].g.L;
    TagScope tag(Lj);
    GenRt *G;
    int rc = get_gen(ctx, Lj, Lj, &G);
    if (rc) return rc;
    const int Nnp = ((2 * Lj - 1) + 31) / 32 * 32, ncols = (2 * Lj - 1) * Nnp;
    LAUNCH(ST_GAMMA_FWD, launch_gen_fwd_gamma(Lj, Lj, G->g_fwd, grid, B.g0, st));
    LAUNCH(ST_ALPHA_FWD, launch_gen_fwd_alpha(Lj, Lj, G->a_fwd, B.g0, B.g1, st));
    LAUNCH(ST_BETA_FWD, launch_beta_gemm(Lj, Lj, ncols, Nnp, 1, 0, G->beta.Qp, G->beta.Qs, B.g1,
                                         B.g0, st));
    LAUNCH(ST_CONTRACT_FWD, launch_gen_contract_fwd(Lj, Lj, ctx->delta, B.g0, B.F, st));
    LAUNCH(ST_REDUCE_FWD, launch_spin_reduce_fwd(Lj, B.F, psi, acc, st));
    return CVL_OK;
}

static int spin_analysis_run(cvl_ctx *ctx, const cvl_params *p, const Plan *P, int batch,
                             const cd *maps, cd *scal_maps, void *const *grids, void *ws,
                             size_t ws_bytes, hipStream_t st) {
    const std::vector<double *> *psi;
    int rc = get_spin_psi(ctx, P, p->spin, &psi);
    if (rc) return rc;
    const SpinBufs B = carve_spin(P, ws, ws_bytes);
    const int L = P->L, Lp = P->Lphi, nJ = P->J - P->J0 + 1;
    ShtRt *SL = ctx->sht[L].get(), *SP = ctx->sht[Lp].get();
    for (int bi = 0; bi < batch; ++bi) {
        const cd *map = maps + (size_t)bi * L * (2 * L - 1);
        cd *smap = scal_maps + (size_t)bi * Lp * (2 * Lp - 1);
        if ((rc = sht_forward_cplx_run(ctx, SL, p->spin, map, B.flat, B.c0, B.c1, st))) return rc;
        LAUNCH(ST_MISC, launch_scale_flat(Lp, P->phifac, B.flat, B.fphi, 0, st));
        if ((rc = sht_inverse_cplx_run(ctx, SP, 0, B.fphi, smap, B.cp0, B.cp1, st))) return rc;
        for (int s = 0; s < nJ; ++s)
            if ((rc = spin_analysis_scale(ctx, P, s, (*psi)[s], B,
                                          (cd *)grids[(size_t)bi * nJ + s], st)))
                return rc;
    }
    return CVL_OK;
}

static int spin_synthesis_run(cvl_ctx *ctx, const cvl_params *p, const Plan *P, int batch,
                              const cd *scal_maps, const void *const *grids, cd *maps, void *ws,
                              size_t ws_bytes, hipStream_t st) {
    const std::vector<double *> *psi;
    int rc = get_spin_psi(ctx, P, p->spin, &psi);
    if (rc) return rc;
    const SpinBufs B = carve_spin(P, ws, ws_bytes);
    const int L = P->L, Lp = P->Lphi, nJ = P->J - P->J0 + 1;
    ShtRt *SL = ctx->sht[L].get(), *SP = ctx->sht[Lp].get();
    for (int bi = 0; bi < batch; ++bi) {
        const cd *smap = scal_maps + (size_t)bi * Lp * (2 * Lp - 1);
        cd *map = maps + (size_t)bi * L * (2 * L - 1);
        LAUNCH(ST_MISC, launch_zero(B.acc, (size_t)L * L, st));
        for (int s = 0; s < nJ; ++s)
            if ((rc = spin_synthesis_scale(ctx, P, s, (*psi)[s], B,
                                           (const cd *)grids[(size_t)bi * nJ + s], B.acc, st)))
                return rc;
        if ((rc = sht_forward_cplx_run(ctx, SP, 0, smap, B.fphi, B.cp0, B.cp1, st))) return rc;
        LAUNCH(ST_MISC, launch_scale_flat(Lp, P->phifac, B.fphi, B.acc, 1, st));
        if ((rc = sht_inverse_cplx_run(ctx, SL, p->spin, B.acc, map, B.c0, B.c1, st))) return rc;
    }
    return CVL_OK;
}

// The analysis launches of a validated call.  side_ok: the scales below the
// top band-limit may run on the caller stream's side stream (the workspace
// then holds their buffers too); otherwise every stage runs on the caller's
// stream, in the first part of the workspace.
static int curvelet_analysis_run(cvl_ctx *ctx, const cvl_params *p, const Plan *P, int batch,
                                 const void *maps_v, void *scal_maps_v, void *const *grids,
                                 void *ws, size_t ws_bytes, hipStream_t st, bool side_ok) {
    int rc;
    const int nJ = P->J - P->J0 + 1;
    ShtRt *SL = ctx->sht[P->L].get(), *SP = ctx->sht[P->Lphi].get();
    if (spin_rotated(p))
        return spin_analysis_run(ctx, p, P, batch, (const cd *)maps_v, (cd *)scal_maps_v, grids,
                                 ws, ws_bytes, st);
    CurveletBufs B = carve_curvelet(P, p->precision, unrotated(p), complex_map(p), ws, ws_bytes);
    if (complex_map(p))
        return curvelet_analysis_cplx(ctx, p, P, batch, (const cd *)maps_v, (cd *)scal_maps_v,
                                      grids, B, st, side_ok);
    const double *maps = (const double *)maps_v;
    double *scal_maps = (double *)scal_maps_v;
    const CurveletBufs BS = side_bufs(B);
    const int L = P->L, Lp = P->Lphi, nside = side_ok ? side_count(P) : 0;
    cvl_ctx::Side *sd = nullptr;
    if (nside > 0 && (rc = get_side(ctx, st, &sd))) return rc;
    for (int bi = 0; bi < batch; ++bi) {
        const double *map = maps + (size_t)bi * L * (2 * L - 1);
        double *smap = scal_maps + (size_t)bi * Lp * (2 * Lp - 1);
        void *const *g = grids + (size_t)bi * nJ;
        if ((rc = sht_forward_run(ctx, SL, map, B.fpad, L, B.s0, B.s1, st))) return rc;
        // the scaling part goes with the side scales when there is a side stream
        // (it only reads the padded coefficients), else on the caller's stream
        if (!sd && (rc = scaling_analysis_run(ctx, P, SP, B, smap, st))) return rc;
        if (sd && (rc = side_fork(sd, st))) return rc;
        // top scales enqueued first, so that the caller's stream starts on them
        // while the side scales' launches are still being enqueued
        rc = analysis_scales(ctx, P, p, B, g, nside, nJ, st);
        if (!rc && sd) rc = scaling_analysis_run(ctx, P, SP, BS, smap, sd->s);
        if (!rc && sd) rc = analysis_scales(ctx, P, p, BS, g, 0, nside, sd->s);
        // joined even after an error: the next map (or call) reuses the buffers
        const int rj = sd ? side_join(sd, st) : CVL_OK;
        if (rc || (rc = rj)) return rc;
    }
    return CVL_OK;
}

int cvl_curvelet_analysis(cvl_ctx *ctx, const cvl_params *p, int batch, const void *maps_v,
                          void *scal_maps_v, void *const *grids, void *ws, size_t ws_bytes,
                          void *stream) {
    g_err.clear();
    Plan *P;
    int rc = check_curvelet_call(ctx, p, batch, maps_v, scal_maps_v, grids, ws, ws_bytes, &P);
    if (rc) return rc;
    const int nJ = P->J - P->J0 + 1;
    for (int i = 0; i < batch * nJ; ++i)
        if (!grids[i]) return fail(CVL_EINVAL, "grids[%d] is NULL", i);
    return curvelet_analysis_run(ctx, p, P, batch, maps_v, scal_maps_v, grids, ws, ws_bytes,
                                 (hipStream_t)stream, true);
}

int cvl_curvelet_analysis_noalloc(cvl_ctx *ctx, const cvl_params *p, int batch,
                                  const void *maps, void *scal_maps, void *const *grids,
                                  void *stream) {
    g_err.clear();
    int J, rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_params(p, &J))) return rc;
    if (batch < 1) return fail(CVL_EINVAL, "batch=%d < 1", batch);
    if (!maps || !scal_maps || !grids) return fail(CVL_EINVAL, "NULL pointer argument");
    if (p->L > ctx->Lmax) return fail(CVL_EINVAL, "L=%d exceeds the context's L_max=%d", p->L, ctx->Lmax);
    if (!ctx->scratch_dev) return fail(CVL_EDEVICE, "no device address for the static scratch");
    const Plan *P = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->prof)
            return fail(CVL_EINVAL, "per-stage timing is on: its events would be created here");
        auto it = ctx->plans.find(std::make_tuple(p->L, p->lambda, p->J0));
        if (it == ctx->plans.end() || !ctx->sht.count(p->L) ||
            !ctx->sht.count(it->second->Lphi))
            return fail(CVL_EINVAL, "the tables of (L=%d, lambda=%g, J0=%d) are not built: call "
                                    "cvl_prepare first", p->L, p->lambda, p->J0);
        P = it->second.get();
    }
    const size_t need = ws_bytes_of(p, P->J, true);
    if (need > (size_t)CVL_NOALLOC_SCRATCH_BYTES)
        return fail(CVL_ENOMEM, "this call needs %zu bytes of scratch, above the static %zu",
                    need, (size_t)CVL_NOALLOC_SCRATCH_BYTES);
    const int nJ = P->J - P->J0 + 1;
    for (int i = 0; i < batch * nJ; ++i)
        if (!grids[i]) return fail(CVL_EINVAL, "grids[%d] is NULL", i);
    if ((rc = set_device(ctx))) return rc;
    return curvelet_analysis_run(ctx, p, P, batch, maps, scal_maps, grids, ctx->scratch_dev, need,
                                 (hipStream_t)stream, false);
}

int cvl_curvelet_synthesis(cvl_ctx *ctx, const cvl_params *p, int batch, const void *scal_maps_v,
                           const void *const *grids, void *maps_v, void *ws, size_t ws_bytes,
                           void *stream) {
    g_err.clear();
    Plan *P;
    int rc = check_curvelet_call(ctx, p, batch, scal_maps_v, maps_v, grids, ws, ws_bytes, &P);
    if (rc) return rc;
    const int nJ = P->J - P->J0 + 1;
    for (int i = 0; i < batch * nJ; ++i)
        if (!grids[i]) return fail(CVL_EINVAL, "grids[%d] is NULL", i);
    ShtRt *SL = ctx->sht[P->L].get(), *SP = ctx->sht[P->Lphi].get();
    hipStream_t st = (hipStream_t)stream;
    if (spin_rotated(p))
        return spin_synthesis_run(ctx, p, P, batch, (const cd *)scal_maps_v, grids, (cd *)maps_v,
                                  ws, ws_bytes, st);
    CurveletBufs B = carve_curvelet(P, p->precision, unrotated(p), complex_map(p), ws, ws_bytes);
    if (complex_map(p))
        return curvelet_synthesis_cplx(ctx, p, P, batch, (const cd *)scal_maps_v, grids,
                                       (cd *)maps_v, B, st);
    const double *scal_maps = (const double *)scal_maps_v;
    double *maps = (double *)maps_v;
    const CurveletBufs BS = side_bufs(B);
    const int L = P->L, Lp = P->Lphi, nside = side_count(P);
    cvl_ctx::Side *sd = nullptr;
    if (nside > 0 && (rc = get_side(ctx, st, &sd))) return rc;
    for (int bi = 0; bi < batch; ++bi) {
        const double *smap = scal_maps + (size_t)bi * Lp * (2 * Lp - 1);
        double *map = maps + (size_t)bi * L * (2 * L - 1);
        const void *const *g = grids + (size_t)bi * nJ;
        // top scales into B.facc; the side scales and then the scaling part
        // into the side accumulator, added in afterwards (a fixed order:
        // results are deterministic)
        if (sd && (rc = side_fork(sd, st))) return rc;
        rc = synthesis_scales(ctx, P, p, B, g, nside, nJ, st);
        if (!rc && sd) rc = synthesis_scales(ctx, P, p, BS, g, 0, nside, sd->s);
        if (!rc && sd) rc = scaling_synthesis_run(ctx, P, SP, BS, smap, sd->s);
        const int rj = sd ? side_join(sd, st) : CVL_OK;
        if (rc || (rc = rj)) return rc;
        if (sd) LAUNCH(ST_MISC, launch_add(B.facc, BS.facc, (size_t)L * L, st));
        if (!sd && (rc = scaling_synthesis_run(ctx, P, SP, B, smap, st))) return rc;
        if ((rc = sht_inverse_run(ctx, SL, B.facc, L, map, B.s0, B.s1, st))) return rc;
    }
    return CVL_OK;
}

// ---- streaming interface: one scale at a time, harmonic-space accumulator ----
static int check_scale_call(cvl_ctx *ctx, const cvl_params *p, int j, const void *a,
                            const void *b, void *ws, size_t ws_bytes, Plan **P, int *s) {
    int rc = check_curvelet_call(ctx, p, 1, a, b, a, ws, ws_bytes, P, true);
    if (rc) return rc;
    if (j < (*P)->J0 || j > (*P)->J)
        return fail(CVL_EINVAL, "scale j=%d outside [J0=%d, J=%d]", j, (*P)->J0, (*P)->J);
    if (s) *s = j - (*P)->J0;
    return CVL_OK;
}

int cvl_curvelet_analysis_scale(cvl_ctx *ctx, const cvl_params *p, int j, const cvl_c128 *flm,
                                void *grid, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    Plan *P;
    int s, rc = check_scale_call(ctx, p, j, flm, grid, ws, ws_bytes, &P, &s);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (spin_rotated(p)) {
        const std::vector<double *> *psi;
        if ((rc = get_spin_psi(ctx, P, p->spin, &psi))) return rc;
        SpinBufs SB = carve_spin(P, ws, ws_bytes);
        SB.flat = (cd *)flm;  // read only
        return spin_analysis_scale(ctx, P, s, (*psi)[s], SB, (cd *)grid, st);
    }
    CurveletBufs B = carve_curvelet(P, p->precision, unrotated(p), complex_map(p), ws, ws_bytes);
    if (complex_map(p)) {
        LAUNCH(ST_MISC, launch_flm_split(P->L, (const cd *)flm, B.fpad, B.fpadb, st));
        return analysis_scale_cplx(ctx, P, P->scales[s], p->precision, unrotated(p), B, grid, st);
    }
    LAUNCH(ST_MISC, launch_flm_pack(P->L, (const cd *)flm, B.fpad, st));
    return analysis_scale_run(ctx, P, P->scales[s], p->precision, real_grids(p), unrotated(p), B,
                              grid, st);
}

int cvl_curvelet_synthesis_scale(cvl_ctx *ctx, const cvl_params *p, int j, const void *grid,
                                 cvl_c128 *flm_acc, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    Plan *P;
    int s, rc = check_scale_call(ctx, p, j, grid, flm_acc, ws, ws_bytes, &P, &s);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (spin_rotated(p)) {
        const std::vector<double *> *psi;
        if ((rc = get_spin_psi(ctx, P, p->spin, &psi))) return rc;
        const SpinBufs SB = carve_spin(P, ws, ws_bytes);
        return spin_synthesis_scale(ctx, P, s, (*psi)[s], SB, (const cd *)grid, (cd *)flm_acc, st);
    }
    CurveletBufs B = carve_curvelet(P, p->precision, unrotated(p), complex_map(p), ws, ws_bytes);
    const int L = P->L;
    if (complex_map(p)) {
        LAUNCH(ST_MISC, launch_zero(B.facc, (size_t)L * L, st));
        LAUNCH(ST_MISC, launch_zero(B.faccb, (size_t)L * L, st));
        if ((rc = synthesis_scale_cplx(ctx, P, P->scales[s], p->precision, unrotated(p), B, grid,
                                       st)))
            return rc;
        LAUNCH(ST_MISC, launch_flm_combine(L, B.facc, B.faccb, (cd *)flm_acc, 1, st));
        return CVL_OK;
    }
    LAUNCH(ST_MISC, launch_zero(B.facc, (size_t)L * L, st));
    if ((rc = synthesis_scale_run(ctx, P, P->scales[s], p->precision, real_grids(p), unrotated(p),
                                  B, grid, st)))
        return rc;
    LAUNCH(ST_MISC, launch_flm_unpack(L, B.facc, (cd *)flm_acc, 1, st));
    return CVL_OK;
}

int cvl_curvelet_scaling_analysis(cvl_ctx *ctx, const cvl_params *p, const cvl_c128 *flm,
                                  void *scal_map_v, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    Plan *P;
    int rc = check_curvelet_call(ctx, p, 1, flm, scal_map_v, flm, ws, ws_bytes, &P, true);
    if (rc) return rc;
    ShtRt *SP = ctx->sht[P->Lphi].get();
    hipStream_t st = (hipStream_t)stream;
    CurveletBufs B = carve_curvelet(P, p->precision, unrotated(p), complex_map(p), ws, ws_bytes);
    const int L = P->L, Lp = P->Lphi;
    if (spin_rotated(p)) {  // the same steps in the buffers of that layout
        const SpinBufs SB = carve_spin(P, ws, ws_bytes);
        LAUNCH(ST_MISC, launch_scale_flat(Lp, P->phifac, (const cd *)flm, SB.fphi, 0, st));
        return sht_inverse_cplx_run(ctx, SP, 0, SB.fphi, (cd *)scal_map_v, SB.cp0, SB.cp1, st);
    }
    if (complex_map(p)) {
        LAUNCH(ST_MISC, launch_scale_flat(Lp, P->phifac, (const cd *)flm, B.fphi, 0, st));
        return sht_inverse_cplx_run(ctx, SP, 0, B.fphi, (cd *)scal_map_v, B.cp0, B.cp1, st);
    }
    double *scal_map = (double *)scal_map_v;
    LAUNCH(ST_MISC, launch_flm_pack(L, (const cd *)flm, B.fpad, st));
    LAUNCH(ST_MISC, launch_scale_flm(Lp, L, Lp, P->phifac, B.fpad, B.fphi, 0, st));
    return sht_inverse_run(ctx, SP, B.fphi, Lp, scal_map, B.s0, B.s1, st);
}

int cvl_curvelet_scaling_synthesis(cvl_ctx *ctx, const cvl_params *p, const void *scal_map_v,
                                   cvl_c128 *flm_acc, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    Plan *P;
    int rc = check_curvelet_call(ctx, p, 1, scal_map_v, flm_acc, scal_map_v, ws, ws_bytes, &P, true);
    if (rc) return rc;
    ShtRt *SP = ctx->sht[P->Lphi].get();
    hipStream_t st = (hipStream_t)stream;
    CurveletBufs B = carve_curvelet(P, p->precision, unrotated(p), complex_map(p), ws, ws_bytes);
    const int L = P->L, Lp = P->Lphi;
    if (complex_map(p)) {
        CurveletBufs X = B;
        if (spin_rotated(p)) {  // the same steps in the buffers of that layout
            const SpinBufs SB = carve_spin(P, ws, ws_bytes);
            X.fphi = SB.fphi;
            X.cp0 = SB.cp0;
            X.cp1 = SB.cp1;
        }
        if ((rc = sht_forward_cplx_run(ctx, SP, 0, (const cd *)scal_map_v, X.fphi, X.cp0, X.cp1,
                                       st)))
            return rc;
        LAUNCH(ST_MISC, launch_scale_flat(Lp, P->phifac, X.fphi, (cd *)flm_acc, 1, st));
        return CVL_OK;
    }
    const double *scal_map = (const double *)scal_map_v;
    if ((rc = sht_forward_run(ctx, SP, scal_map, B.fphi, Lp, B.s0, B.s1, st))) return rc;
    LAUNCH(ST_MISC, launch_zero(B.facc, (size_t)L * L, st));
    LAUNCH(ST_MISC, launch_scale_flm(Lp, Lp, L, P->phifac, B.fphi, B.facc, 1, st));
    LAUNCH(ST_MISC, launch_flm_unpack(L, B.facc, (cd *)flm_acc, 1, st));
    return CVL_OK;
}

int cvl_delta_block(cvl_ctx *ctx, int l, double *out) {
    g_err.clear();
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (l < 0 || l >= ctx->Lmax) return fail(CVL_EINVAL, "l=%d outside [0, L_max=%d)", l, ctx->Lmax);
    if (!out) return fail(CVL_EINVAL, "out is NULL");
    if ((rc = set_device(ctx))) return rc;
    HIP_TRY(hipMemcpy(out, ctx->delta + delta_off(l), sizeof(double) * (size_t)(l + 1) * (l + 1),
                      hipMemcpyDeviceToHost));
    return CVL_OK;
}

int cvl_profile_enable(cvl_ctx *ctx, int on) {
    g_err.clear();
    if (!ctx) return fail(CVL_EINVAL, "context is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->prof = on != 0;
    for (int i = 0; i < ST_COUNT; ++i) {
        ctx->stage_ms[i] = 0;
        ctx->stage_n[i] = 0;
    }
    ctx->detail.clear();
    return CVL_OK;
}

int cvl_profile_filter(cvl_ctx *ctx, int stage, int bandlimit) {
    g_err.clear();
    if (!ctx) return fail(CVL_EINVAL, "context is NULL");
    if (stage < -1 || stage >= ST_COUNT)
        return fail(CVL_EINVAL, "stage index %d outside [-1, %d)", stage, (int)ST_COUNT);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->pf_stage = stage;
    ctx->pf_tag = bandlimit;
    return CVL_OK;
}

// Waits for the recorded launches and adds their times to the totals.
static int profile_drain(cvl_ctx *ctx) {
    std::vector<std::tuple<int, int, hipEvent_t, hipEvent_t>> rec;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        rec.swap(ctx->rec);
    }
    for (auto &r : rec) {
        hipEvent_t e0 = std::get<2>(r), e1 = std::get<3>(r);
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        const int stg = std::get<0>(r);
        ctx->stage_ms[stg] += t;
        ctx->stage_n[stg] += 1;
        auto &d = ctx->detail[std::make_pair(stg, std::get<1>(r))];
        d.first += 1;
        d.second += t;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &r : rec) {
        ctx->pool.push_back(std::get<2>(r));
        ctx->pool.push_back(std::get<3>(r));
    }
    return CVL_OK;
}

int cvl_profile_read(cvl_ctx *ctx, int max, int *n, const char **names, int *launches,
                     double *ms) {
    g_err.clear();
    if (!ctx || !n) return fail(CVL_EINVAL, "NULL argument");
    int rc = profile_drain(ctx);
    if (rc) return rc;
    *n = ST_COUNT;
    for (int i = 0; i < ST_COUNT && i < max; ++i) {
        if (names) names[i] = kStageNames[i];
        if (launches) launches[i] = ctx->stage_n[i];
        if (ms) ms[i] = ctx->stage_ms[i];
    }
    return CVL_OK;
}

int cvl_profile_read_detail(cvl_ctx *ctx, int max, int *n, int *stage, int *bandlimit,
                            int *launches, double *ms) {
    g_err.clear();
    if (!ctx || !n) return fail(CVL_EINVAL, "NULL argument");
    int rc = profile_drain(ctx);
    if (rc) return rc;
    *n = (int)ctx->detail.size();
    int i = 0;
    for (auto &kv : ctx->detail) {
        if (i >= max) break;
        if (stage) stage[i] = kv.first.first;
        if (bandlimit) bandlimit[i] = kv.first.second;
        if (launches) launches[i] = kv.second.first;
        if (ms) ms[i] = kv.second.second;
        ++i;
    }
    return CVL_OK;
}

}  // extern "C"
