// Odd-length McEwen-Wiaux DFTs (lengths 2L-1) as Bluestein chirp-z transforms
// over power-of-two Stockham FFTs.
//
// Every MW DFT is out[k] = scale * sum_j in[j] exp(sigma 2 pi i j k / Nd) for a
// window of inputs j in [j0, j0+Kin) and outputs k in [k0, k0+Kout).  With
// jk = (j^2 + k^2 - (k-j)^2)/2 this is a chirp pre-multiply, a linear
// convolution with a chirp (a circular one of power-of-two length P >=
// Kin+Kout-1, its spectrum precomputed on the host with the 1/P and `scale`
// folded in), and a chirp post-multiply.  The inverse FFT is the forward one
// between two conjugations.
//
// Two engines: for P <= 128 a work-group of 256 threads transforms LINES
// lines with radix-4 stages in LDS; for P >= 256 a register-resident radix-16
// engine.  The stage IO policies gather / scatter each stage's lines with the
// symmetries the stage uses (reality of the map, evenness of n) and say whether
// a line is contiguous in memory (DIRECT) or interleaved with its neighbours
// (STAGED through LDS so that global accesses stay coalesced).  Each policy
// resolves a line to a context (base pointers) once; element accesses are then
// plain offsets.
#include <type_traits>
#include <utility>

#include "cvl_device.h"

namespace cvl {

// An IO policy may declare `bool live(int line)`: a line for which it returns
// false is all zero on input and its output is never read, so a work-group of
// the register engine whose lines are all dead returns at once.
template <class T, class = void>
struct HasLive : std::false_type {};
template <class T>
struct HasLive<T, std::void_t<decltype(std::declval<const T &>().live(0))>> : std::true_type {};

// An IO policy may declare `static constexpr bool kOddIn`: its inputs are
// non-zero only at odd window positions t (and t < P/2), so the register
// engine's first FFT is a half-length FFT of the odd samples; or
// `kOddOut`: only odd output positions are read, so its second FFT is a
// half-length FFT of the folded sequence.  (Both for P = 1024, T = 64.)
template <class T, class = void>
struct OddIn : std::false_type {};
template <class T>
struct OddIn<T, std::void_t<decltype(T::kOddIn)>> : std::integral_constant<bool, T::kOddIn> {};
template <class T, class = void>
struct OddOut : std::false_type {};
template <class T>
struct OddOut<T, std::void_t<decltype(T::kOddOut)>> : std::integral_constant<bool, T::kOddOut> {};

// Output modes: IO_PAIR hands the policy output pairs (k, -k) of a symmetric
// window, line by line; IO_STAGED_PAIR does the same with the work-group's
// lines interleaved (neighbouring lines neighbouring in memory).
enum { IO_DIRECT = 0, IO_STAGED = 1, IO_PAIR = 2, IO_STAGED_PAIR = 3 };



// In-place Stockham FFT of one LDS line (forward, tw[x] = e^{-2 pi i x / P}).
// Radix-4 stages first, then one radix-2 stage when log2 P is odd.  Every
// thread of the work-group must call it (it synchronises the work-group).
template <int P, int TPL, class C>
__device__ __forceinline__ void fft_lds(C *buf, const C *__restrict__ tw, int lane) {
    constexpr int Q = P / 4;
    constexpr int B4 = (Q + TPL - 1) / TPL;
    int Ns = 1;
    for (; Ns * 4 <= P; Ns *= 4) {
        C v[B4][4];
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
                const C a0 = cadd(v[i][0], v[i][2]), a1 = csub(v[i][0], v[i][2]);
                const C b0 = cadd(v[i][1], v[i][3]), b1 = csub(v[i][1], v[i][3]);
                const C mib1 = C{b1.y, -b1.x};  // -i * b1
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
        C v[B2][2];
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

// Lines per 256-thread work-group of the small engine: P/4 threads per line
// (one radix-4 butterfly each per stage), at most 64 lines.  Few lines per
// group keep enough work-groups to spread small stages over the device.
template <int P>
struct LinesFor {
    static constexpr int v = (1024 / P) > 64 ? 64 : (1024 / P) < 1 ? 1 : (1024 / P);
};

template <int P, int LINES, class IO>
__global__ __launch_bounds__(256) void k_bluestein(IO io, int nlines, BlueT<typename IO::C> B) {
    using C = typename IO::C;
    constexpr bool IN_IL = IO::kLoad == IO_STAGED, OUT_IL = IO::kStore == IO_STAGED;
    extern __shared__ __align__(16) char smem_raw[];
    C *smem = reinterpret_cast<C *>(smem_raw);
    constexpr int TPL = 256 / LINES;
    const int tid = threadIdx.x;
    const int li = tid / TPL, lane = tid % TPL;
    const int line0 = xcd_group(blockIdx.x, gridDim.x) * LINES;
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
        C v = C{0, 0};
        if (t < B.Kin && line < nlines) v = cmul(io.load(io.at(line), B.j0 + t), B.pre[t]);
        smem[l * P + t] = v;
    }
    __syncthreads();
    C *buf = smem + li * P;
    fft_lds<P, TPL>(buf, B.tw, lane);
    for (int t = lane; t < P; t += TPL) buf[t] = cconj(cmul(buf[t], B.vhat[t]));
    __syncthreads();
    fft_lds<P, TPL>(buf, B.tw, lane);
    for (int t = lane; t < B.Kout; t += TPL) buf[t] = cmul(cconj(buf[t]), B.post[t]);
    __syncthreads();
    if constexpr (IO::kStore == IO_PAIR || IO::kStore == IO_STAGED_PAIR) {
        const int line = line0 + li;
        if (line < nlines) {
            const auto c = io.at(line);
            const int K = -B.k0;
            for (int k = lane; k <= K; k += TPL)
                io.store_pair(c, k, buf[k + K], buf[K - k]);
        }
    } else {
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
            if (line < nlines) io.store(io.at(line), B.k0 + t, smem[l * P + t]);
        }
    }
}

// ---------------------------------------------------------------------------
// Register-resident Bluestein engine for P >= 256.
//
// A line of P points is held by T = P/16 threads, 16 complex values each;
// after every FFT thread t holds elements t + T*s (s = 0..15).  The FFT is a
// Stockham transform with two radix-16 passes (Ns = 1, 16) and, for P > 256,
// a last radix-(P/256) pass (Ns = 256).  Passes exchange data through a
// padded LDS line (index e + e/16).  Because the forward FFT ends with the
// layout the next FFT's first pass reads, the chirp-spectrum multiply and the
// second FFT need no exchange in between.
// ---------------------------------------------------------------------------
template <class C>
__device__ __forceinline__ C mul_mi(C a) { return C{a.y, -a.x}; }  // -i * a

template <class C>
__device__ __forceinline__ void bfly4(C &x0, C &x1, C &x2, C &x3) {
    const C a0 = cadd(x0, x2), a1 = csub(x0, x2);
    const C b0 = cadd(x1, x3), b1 = mul_mi(csub(x1, x3));
    x0 = cadd(a0, b0);
    x2 = csub(a0, b0);
    x1 = cadd(a1, b1);
    x3 = csub(a1, b1);
}
template <class C>
__device__ __forceinline__ void bfly2(C &x0, C &x1) {
    const C a = cadd(x0, x1);
    x1 = csub(x0, x1);
    x0 = a;
}

// e^{-2 pi i e / 16} for the exponents a 4x4 split of the 16-point DFT needs.
#define CVL_C1 0.92387953251128675613
#define CVL_S1 0.38268343236508977173
#define CVL_R2 0.70710678118654752440

// 16-point forward DFT, natural order in and out (4 x 4 split).
template <class C>
__device__ __forceinline__ void dft16(C v[16]) {
#pragma unroll
    for (int r0 = 0; r0 < 4; ++r0) bfly4(v[r0], v[r0 + 4], v[r0 + 8], v[r0 + 12]);
    v[5] = cmul(v[5], cmk<C>(CVL_C1, -CVL_S1));
    v[9] = cmul(v[9], cmk<C>(CVL_R2, -CVL_R2));
    v[13] = cmul(v[13], cmk<C>(CVL_S1, -CVL_C1));
    v[6] = cmul(v[6], cmk<C>(CVL_R2, -CVL_R2));
    v[10] = mul_mi(v[10]);
    v[14] = cmul(v[14], cmk<C>(-CVL_R2, -CVL_R2));
    v[7] = cmul(v[7], cmk<C>(CVL_S1, -CVL_C1));
    v[11] = cmul(v[11], cmk<C>(-CVL_R2, -CVL_R2));
    v[15] = cmul(v[15], cmk<C>(-CVL_C1, CVL_S1));
#pragma unroll
    for (int k0 = 0; k0 < 4; ++k0) bfly4(v[4 * k0], v[4 * k0 + 1], v[4 * k0 + 2], v[4 * k0 + 3]);
    C t[16];
#pragma unroll
    for (int k0 = 0; k0 < 4; ++k0)
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) t[k0 + 4 * k1] = v[4 * k0 + k1];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = t[k];
}

// 8-point forward DFT (4 x 2 split), natural order.
template <class C>
__device__ __forceinline__ void dft8(C *v) {
    bfly4(v[0], v[2], v[4], v[6]);
    bfly4(v[1], v[3], v[5], v[7]);
    v[3] = cmul(v[3], cmk<C>(CVL_R2, -CVL_R2));
    v[5] = mul_mi(v[5]);
    v[7] = cmul(v[7], cmk<C>(-CVL_R2, -CVL_R2));
#pragma unroll
    for (int k0 = 0; k0 < 4; ++k0) bfly2(v[2 * k0], v[2 * k0 + 1]);
    C t[8];
#pragma unroll
    for (int k0 = 0; k0 < 4; ++k0) {
        t[k0] = v[2 * k0];
        t[k0 + 4] = v[2 * k0 + 1];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = t[k];
}

template <int R, class C>
__device__ __forceinline__ void dft_small(C *v) {
    if constexpr (R == 2) {
        bfly2(v[0], v[1]);
    } else if constexpr (R == 4) {
        bfly4(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        dft8(v);
    } else {
        dft16(v);
    }
}

__device__ __forceinline__ int lpad(int e) { return e + (e >> 4); }
// Padded offset of an offset o that is a multiple of 16:
// lpad(e + o) = lpad(e) + lpo(o) for every e.
__host__ __device__ constexpr int lpo(int o) { return o + (o >> 4); }

// Keeps loaded values in registers at this point: an empty asm statement that
// takes them as inputs, so that the compiler issues (and waits for) a whole
// batch of loads here instead of sinking each load into the conditional block
// that uses it, one wait per element.
template <class C>
__device__ __forceinline__ void materialize(const C &v) {
    asm volatile("" ::"v"(v.x), "v"(v.y));
}

// Orders one line's LDS exchange.  When a line lives in a single wavefront
// (P <= 1024) the exchange is wave-local: a wavefront-scope fence keeps the
// compiler from moving LDS accesses across it, and a wave's LDS instructions
// complete in order, so no work-group barrier is needed.  Larger lines span
// several wavefronts and synchronise the work-group.
template <int P>
__device__ __forceinline__ void line_sync() {
    if constexpr (P / 16 <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int P>
struct R16 {
    static constexpr int T = P / 16;                 // threads per line
    static constexpr int WG = T < 256 ? 256 : T;     // threads per work-group (>= 4 waves)
    static constexpr int LINES = WG / T;             // lines per work-group
    static constexpr int RC = P / 256;               // radix of the last pass (1: none)
    static constexpr int LW = P + P / 16 + 4;        // reals per LDS line (padded)
};

// Moves one line between passes through LDS, one real component at a time
// (the LDS line holds P reals): v[k] leaves to padded index wb + wo(k), v[r]
// arrives from padded index rb + ro(r).  The bases are per thread, the
// offsets compile-time constants, so every access is one base register plus
// an immediate offset.
template <int P, class C, class WO, class RO>
__device__ __forceinline__ void exchange(C v[16], real_t<C> *lds, int wb, WO wo, int rb, RO ro) {
    real_t<C> nx[16];
    real_t<C> *w = lds + wb;
    const real_t<C> *r = lds + rb;
#pragma unroll
    for (int k = 0; k < 16; ++k) w[wo(k)] = v[k].x;
    line_sync<P>();
#pragma unroll
    for (int i = 0; i < 16; ++i) nx[i] = r[ro(i)];
    line_sync<P>();
#pragma unroll
    for (int k = 0; k < 16; ++k) w[wo(k)] = v[k].y;
    line_sync<P>();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = C{nx[i], r[ro(i)]};
    line_sync<P>();
}

// v[r] *= w^r for r = 1..15 (w^r from w by a product tree, used as produced).
template <class C>
__device__ __forceinline__ void twiddle16(C v[16], C w1) {
    const C w2 = cmul(w1, w1), w4 = cmul(w2, w2), w8 = cmul(w4, w4);
    const C w3 = cmul(w2, w1);
    v[1] = cmul(v[1], w1);
    v[2] = cmul(v[2], w2);
    v[3] = cmul(v[3], w3);
    v[4] = cmul(v[4], w4);
    v[5] = cmul(v[5], cmul(w4, w1));
    v[6] = cmul(v[6], cmul(w4, w2));
    v[7] = cmul(v[7], cmul(w4, w3));
    v[8] = cmul(v[8], w8);
    v[9] = cmul(v[9], cmul(w8, w1));
    v[10] = cmul(v[10], cmul(w8, w2));
    v[11] = cmul(v[11], cmul(w8, w3));
    const C w12 = cmul(w8, w4);
    v[12] = cmul(v[12], w12);
    v[13] = cmul(v[13], cmul(w12, w1));
    v[14] = cmul(v[14], cmul(w12, w2));
    v[15] = cmul(v[15], cmul(w12, w3));
}

// v[r] *= w^r for r = 1..7 (w^r from w by a product tree, used as produced).
template <class C>
__device__ __forceinline__ void twiddle8(C v[8], C w1) {
    const C w2 = cmul(w1, w1), w4 = cmul(w2, w2), w3 = cmul(w2, w1);
    v[1] = cmul(v[1], w1);
    v[2] = cmul(v[2], w2);
    v[3] = cmul(v[3], w3);
    v[4] = cmul(v[4], w4);
    v[5] = cmul(v[5], cmul(w4, w1));
    v[6] = cmul(v[6], cmul(w4, w2));
    v[7] = cmul(v[7], cmul(w4, w3));
}

// u[e] *= W^{j + (P/16) e}, e = 0..7, W = e^{-2 pi i / P}: W^j from the table
// times powers of the constant W^{P/16} = e^{-i pi / 8} (the same for every P).
template <class C>
__device__ __forceinline__ void twiddle_stride16th(C u[8], C wj) {
    const C c1 = cmk<C>(CVL_C1, -CVL_S1);  // e^{-i pi / 8}
    C w = wj;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        u[e] = cmul(u[e], w);
        if (e < 7) w = cmul(w, c1);
    }
}

// Forward FFT of one line; v[s] = element tid + T*s on entry and on exit.
template <int P, class C>
__device__ __forceinline__ void fft_r16(C v[16], real_t<C> *lds, const C *__restrict__ tw,
                                        int tid) {
    constexpr int T = R16<P>::T, RC = R16<P>::RC;
    dft16(v);  // pass Ns = 1: butterfly tid, no twiddles
    // element 16 tid + k leaves v[k] (lpad = 17 tid + k), element tid + T r
    // arrives in v[r] (T is a multiple of 16)
    const int rb = lpad(tid);
    exchange<P>(
        v, lds, 17 * tid, [](int k) { return k; }, rb, [](int r) { return lpo(T * r); });
    twiddle16(v, tw[(tid & 15) * (P / 256)]);
    dft16(v);  // pass Ns = 16
    if constexpr (RC > 1) {
        constexpr int NB = 16 / RC;  // butterflies per thread
        // element (tid >> 4) 256 + (tid & 15) + 16 k leaves v[k], element
        // tid + T (idx / RC) + 256 (idx % RC) arrives in v[idx]
        exchange<P>(
            v, lds, lpad((tid >> 4) * 256 + (tid & 15)), [](int k) { return lpo(16 * k); }, rb,
            [](int idx) { return lpo(T * (idx / RC) + 256 * (idx % RC)); });
        // v[q*RC + r] = element j + 256 r, j = tid + T q
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int j = tid + T * q;
            C *u = &v[q * RC];
            const C w1 = tw[j];
            if constexpr (RC == 2) {
                u[1] = cmul(u[1], w1);
            } else if constexpr (RC == 4) {
                const C w2 = cmul(w1, w1);
                u[1] = cmul(u[1], w1);
                u[2] = cmul(u[2], w2);
                u[3] = cmul(u[3], cmul(w2, w1));
            } else if constexpr (RC == 8) {
                twiddle8(u, w1);
            } else {
                twiddle16(u, w1);
            }
            dft_small<RC>(u);
        }
        // element j + 256 r = tid + T (q + r NB): reorder to v[q + r NB]
        C t[16];
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int r = 0; r < RC; ++r) t[q + r * NB] = v[q * RC + r];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = t[k];
    }
}

// Moves 8 values per thread through the LDS line (one real component at a
// time), as `exchange` does for 16.
template <int P, class C, class WO, class RO>
__device__ __forceinline__ void exchange8(C v[8], real_t<C> *lds, int wb, WO wo, int rb, RO ro) {
    real_t<C> nx[8];
    real_t<C> *w = lds + wb;
    const real_t<C> *r = lds + rb;
#pragma unroll
    for (int k = 0; k < 8; ++k) w[wo(k)] = v[k].x;
    line_sync<P>();
#pragma unroll
    for (int i = 0; i < 8; ++i) nx[i] = r[ro(i)];
    line_sync<P>();
#pragma unroll
    for (int k = 0; k < 8; ++k) w[wo(k)] = v[k].y;
    line_sync<P>();
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = C{nx[i], r[ro(i)]};
    line_sync<P>();
}

// Forward FFT of N = P/2 points held by the T = P/16 threads of a P-point
// line, 8 each: v[s] = element tid + T s on entry and on exit.  Stockham,
// radix-8 passes (Ns = 1, 8, 64) and, for N > 512, a last radix-(N/512) pass
// (Ns = 512) of 8/R butterflies per thread; twiddles e^{-2 pi i x / N} =
// tw[2x] of the P-point table.
template <int P, class C>
__device__ __forceinline__ void fft_r8_half(C v[8], real_t<C> *lds, const C *__restrict__ tw,
                                            int tid) {
    constexpr int N = P / 2, T = P / 16, R = N / 512;
    static_assert(N >= 512 && N <= 2048, "half-length FFT of a 1024- to 4096-point line");
    dft8(v);  // pass Ns = 1: outputs 8 tid + k
    const int rb = lpad(tid);
    exchange8<P>(
        v, lds, lpad(8 * tid), [](int k) { return k; }, rb, [](int r) { return lpo(T * r); });
    {  // pass Ns = 8: twiddle w^{r k}, w = e^{-2 pi i / 64}, k = tid mod 8
        twiddle8(v, tw[(P / 64) * (tid & 7)]);
        dft8(v);  // outputs (tid / 8) 64 + (tid mod 8) + 8 k'
    }
    exchange8<P>(
        v, lds, lpad((tid >> 3) * 64 + (tid & 7)), [](int k) { return lpo(8 * k); }, rb,
        [](int r) { return lpo(T * r); });
    // pass Ns = 64: twiddle w^{r k}, w = e^{-2 pi i / 512}, k = tid mod 64;
    // outputs (tid / 64) 512 + (tid mod 64) + 64 k'
    twiddle8(v, tw[(P / 512) * (tid & 63)]);
    dft8(v);
    if constexpr (R > 1) {
        constexpr int NB = 8 / R;  // butterflies per thread
        // element j + 512 r (j = tid + T q) arrives in v[q R + r]
        exchange8<P>(
            v, lds, lpad((tid >> 6) * 512 + (tid & 63)), [](int k) { return lpo(64 * k); }, rb,
            [](int idx) { return lpo(T * (idx / R) + 512 * (idx % R)); });
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            C *u = &v[q * R];
            const C w1 = tw[2 * (tid + T * q)];  // w^j, w = e^{-2 pi i / N}
            if constexpr (R == 2) {
                u[1] = cmul(u[1], w1);
            } else {
                const C w2 = cmul(w1, w1);
                u[1] = cmul(u[1], w1);
                u[2] = cmul(u[2], w2);
                u[3] = cmul(u[3], cmul(w2, w1));
            }
            dft_small<R>(u);
        }
        // element j + 512 r = tid + T (q + r NB): reorder to v[q + r NB]
        C t[8];
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) t[q + r * NB] = v[q * R + r];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = t[k];
    }
}

// Three waves per SIMD for lines that fit one wavefront (the kernel is latency
// bound; the register cap costs at most a few spilled dwords); four for an IO
// policy that declares `kFourWaves` (its instance fits 128 registers without
// spills, and it reads the chirp spectrum from global memory so that four
// work-groups fit a CU's LDS).
template <class T, class = void>
struct FourWaves : std::false_type {};
template <class T>
struct FourWaves<T, std::void_t<decltype(T::kFourWaves)>>
    : std::integral_constant<bool, T::kFourWaves> {};
template <class T, class = void>
struct LoadPrio : std::false_type {};
template <class T>
struct LoadPrio<T, std::void_t<decltype(T::kLoadPrio)>>
    : std::integral_constant<bool, T::kLoadPrio> {};

// The chirp spectrum is copied to LDS (once per work-group) up to P = 1024;
// at 2048 only for a policy that declares `kVhLds2048` — elsewhere the copy's
// LDS would cost work-groups per CU.
template <class T, class = void>
struct VhLds2048 : std::false_type {};
template <class T>
struct VhLds2048<T, std::void_t<decltype(T::kVhLds2048)>>
    : std::integral_constant<bool, T::kVhLds2048> {};

template <int P, class IO>
struct VhLds {
    static constexpr bool v =
        (P <= 1024 && !FourWaves<IO>::value) || (P == 2048 && VhLds2048<IO>::value);
};

template <int P, class IO>
struct WavesFor {
    static constexpr bool f32 = sizeof(real_t<typename IO::C>) == 4;
    static constexpr int v = P <= 1024   ? (FourWaves<IO>::value ? 4 : 3)
                             : !f32      ? 2
                             : P == 4096 ? 5
                                         : 2;
};

template <int P, class IO>
__global__ __launch_bounds__(R16<P>::WG, (WavesFor<P, IO>::v)) void k_blue_r16(
    IO io, int nlines, BlueT<typename IO::C> B) {
    using C = typename IO::C;
    using R = real_t<C>;
    constexpr int T = R16<P>::T, WG = R16<P>::WG, LINES = R16<P>::LINES, LW = R16<P>::LW;
    extern __shared__ __align__(16) char smem_raw[];
    R *smem_d = reinterpret_cast<R *>(smem_raw);
    const int li = threadIdx.x / T, tid = threadIdx.x % T;
    const int line0 = xcd_group(blockIdx.x, gridDim.x) * LINES;
    if constexpr (HasLive<IO>::value) {
        bool any = false;  // uniform over the work-group
        for (int i = 0; i < LINES; ++i) any = any || (line0 + i < nlines && io.live(line0 + i));
        if (!any) return;
    }
    const int line = line0 + li;
    R *lds = smem_d + li * LW;
    // The chirp spectrum is read by every line between the two FFTs: one copy
    // in LDS per work-group instead of a cache-missing global read per line
    // (where the copy does not cost occupancy, see VhLds).
    constexpr bool kVhLds = VhLds<P, IO>::v;
    const C *vh = B.vhat;
    if constexpr (kVhLds) {
        C *v2 = reinterpret_cast<C *>(smem_d + LINES * LW);
        for (int i = threadIdx.x; i < P; i += WG) v2[i] = B.vhat[i];
        __syncthreads();
        vh = v2;
    }
    C v[16];
    // Raised wave priority while the line's loads are issued (complex128
    // policies that declare `kLoadPrio`, FFT sizes up to 1024): waves in their
    // load phase get their requests out ahead of waves computing.
    constexpr bool kPrio = LoadPrio<IO>::value && sizeof(R) == 8 && P <= 1024;
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(2);
    constexpr bool kOI = OddIn<IO>::value, kOO = OddOut<IO>::value;
    static_assert(!(kOI || kOO) || (P >= 1024 && P <= 4096),
                  "odd-input / odd-output paths need 1024 <= P <= 4096");
    // Every load of a line is issued before any is used: indices are clamped
    // into the window and out-of-window elements zeroed afterwards, so no
    // load waits behind a branch (the IO policies' loads are branch-free too).
    if constexpr (kOI) {
        // inputs only at odd t = 2u + 1 < P/2: the FFT of the window is
        // FFT_P(a)(k) = W^k FFT_{P/2}(a'')(k mod P/2), a''_u = a_{2u+1},
        // W = e^{-2 pi i / P}.  Load a''_u at u = tid + T s, s < 8.
        static_assert(IO::kLoad == IO_DIRECT, "odd-input path loads directly");
        C u8[8];
        if (line < nlines) {
            const auto c = io.at(line);
#pragma unroll
            for (int h = 0; h < 8; h += 4) {
                if (2 * T * h >= B.Kin) {  // past the input (uniform)
#pragma unroll
                    for (int e = 0; e < 4; ++e) u8[h + e] = C{0, 0};
                    continue;
                }
                C raw[4], pw[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int t = 2 * (tid + T * (h + e)) + 1;
                    const int tc = t < B.Kin ? t : B.Kin - 1;
                    raw[e] = io.load(c, B.j0 + tc);
                    pw[e] = B.pre[tc];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int t = 2 * (tid + T * (h + e)) + 1;
                    u8[h + e] = cscale(cmul(raw[e], pw[e]), (real_t<C>)(t < B.Kin ? 1 : 0));
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) u8[e] = C{0, 0};
        }
        if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
        fft_r8_half<P>(u8, lds, B.tw, tid);
        // v[s] = W^k Y''(k mod P/2), k = tid + T s; W^{k + P/2} = -W^k
        twiddle_stride16th(u8, B.tw[tid]);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            v[e] = u8[e];
            v[e + 8] = C{-u8[e].x, -u8[e].y};
        }
    } else if constexpr (IO::kLoad == IO_DIRECT) {
        if (line < nlines) {
            const auto c = io.at(line);
#pragma unroll
            for (int h8 = 0; h8 < 16; h8 += IO::kBatch) {
                if (T * h8 >= B.Kin) {  // the whole batch lies past the input (uniform)
#pragma unroll
                    for (int e = 0; e < IO::kBatch; ++e) v[h8 + e] = C{0, 0};
                    continue;
                }
                C raw[IO::kBatch], pw[IO::kBatch];
#pragma unroll
                for (int e = 0; e < IO::kBatch; ++e) {
                    const int t = tid + T * (h8 + e);
                    const int tc = t < B.Kin ? t : B.Kin - 1;
                    raw[e] = io.load(c, B.j0 + tc);
                    pw[e] = B.pre[tc];
                }
#pragma unroll
                for (int e = 0; e < IO::kBatch; ++e) {
                    const int t = tid + T * (h8 + e);
                    v[h8 + e] = cscale(cmul(raw[e], pw[e]), (real_t<C>)(t < B.Kin ? 1 : 0));
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < 16; ++s) v[s] = C{0, 0};
        }
    } else {
        // Staged through the LDS lines viewed as complex (Kin <= P/2 fits).
        // WG is a multiple of LINES, so each thread always stages the same line.
        // Each line has WG / LINES = T staging threads, 16 elements each.
        const int ls = threadIdx.x % LINES, lns = line0 + ls, tl = threadIdx.x / LINES;
        C *dst = reinterpret_cast<C *>(smem_d + ls * LW);
        if (lns < nlines) {
            const auto c = io.at(lns);
#pragma unroll
            for (int h8 = 0; h8 < 16; h8 += IO::kBatch) {
                if (T * h8 >= B.Kin) break;  // past the input (uniform)
                C raw[IO::kBatch], pw[IO::kBatch];
#pragma unroll
                for (int e = 0; e < IO::kBatch; ++e) {
                    const int t = tl + T * (h8 + e);
                    const int tc = t < B.Kin ? t : B.Kin - 1;
                    raw[e] = io.load(c, B.j0 + tc);
                    pw[e] = B.pre[tc];
                }
#pragma unroll
                for (int e = 0; e < IO::kBatch; ++e) {
                    materialize(raw[e]);
                    materialize(pw[e]);
                }
#pragma unroll
                for (int e = 0; e < IO::kBatch; ++e) {
                    const int t = tl + T * (h8 + e);
                    if (t < B.Kin) dst[t] = cmul(raw[e], pw[e]);
                }
            }
        }
        __syncthreads();
        const C *src = reinterpret_cast<const C *>(lds);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int t = tid + T * s;
            v[s] = (t < B.Kin && line < nlines) ? src[t] : C{0, 0};
        }
        __syncthreads();
    }
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
    if constexpr (!kOI) fft_r16<P>(v, lds, B.tw, tid);
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = cconj(cmul(v[s], vh[tid + T * s]));
    if constexpr (kOO) {
        // only odd outputs q = 2 v' + 1 are read: FFT_P(c)(2v'+1) =
        // FFT_{P/2}(d)(v'), d_j = (c_j - c_{j+P/2}) W^j; v[s] then holds
        // output 2 (tid + T s) + 1 for s < 8
        C u8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) u8[e] = csub(v[e], v[e + 8]);
        twiddle_stride16th(u8, B.tw[tid]);
        fft_r8_half<P>(u8, lds, B.tw, tid);
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = u8[e];
    } else {
        fft_r16<P>(v, lds, B.tw, tid);
    }
    // v[s] = conj(c[q]), q = tid + T*s: output k = k0 + q for q < Kout.
    // Post-chirp factors: loaded 8 at a time (clamped indices), so that a
    // half line's loads are in flight together without doubling the
    // registers; a half past the outputs is skipped (with Kout <= P/2, the
    // usual case, one half and one round trip).
    if constexpr (IO::kStore == IO_DIRECT) {
        static_assert(!kOO, "odd-output path stores through LDS");
        if (line < nlines) {
            const auto c = io.at(line);
#pragma unroll
            for (int h8 = 0; h8 < 16; h8 += 8) {
                if (T * h8 >= B.Kout) break;  // uniform
                C pq[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int q = tid + T * (h8 + e);
                    pq[e] = B.post[q < B.Kout ? q : B.Kout - 1];
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) materialize(pq[e]);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int q = tid + T * (h8 + e);
                    if (q < B.Kout) io.store(c, B.k0 + q, cmul(cconj(v[h8 + e]), pq[e]));
                }
            }
        }
    } else {
        // Kout <= P/2 complex fit in the line viewed as complex.
        C *buf = reinterpret_cast<C *>(lds);
        line_sync<P>();
        if constexpr (kOO) {  // odd positions q = 2 (tid + T e) + 1 only
            C pq[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int q = 2 * (tid + T * e) + 1;
                pq[e] = B.post[q < B.Kout ? q : B.Kout - 1];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) materialize(pq[e]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int q = 2 * (tid + T * e) + 1;
                if (q < B.Kout) buf[q] = cmul(cconj(v[e]), pq[e]);
            }
        } else {
#pragma unroll
            for (int h8 = 0; h8 < 16; h8 += 8) {
                if (T * h8 >= B.Kout) break;  // uniform
                C pq[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int q = tid + T * (h8 + e);
                    pq[e] = B.post[q < B.Kout ? q : B.Kout - 1];
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) materialize(pq[e]);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int q = tid + T * (h8 + e);
                    if (q < B.Kout) buf[q] = cmul(cconj(v[h8 + e]), pq[e]);
                }
            }
        }
        __syncthreads();
        if constexpr (IO::kStore == IO_STAGED) {
            const int ls = threadIdx.x % LINES, lns = line0 + ls;
            if (lns < nlines) {
                const auto c = io.at(lns);
                const C *src = reinterpret_cast<const C *>(smem_d + ls * LW);
                for (int t = threadIdx.x / LINES; t < B.Kout; t += WG / LINES)
                    io.store(c, B.k0 + t, src[t]);
            }
        } else if constexpr (IO::kStore == IO_STAGED_PAIR) {
            const int ls = threadIdx.x % LINES, lns = line0 + ls;
            if (lns < nlines) {
                const auto c = io.at(lns);
                const C *src = reinterpret_cast<const C *>(smem_d + ls * LW);
                const int K = -B.k0;
                for (int k = threadIdx.x / LINES; k <= K; k += WG / LINES)
                    io.store_pair(c, k, src[k + K], src[K - k]);
            }
        } else {  // IO_PAIR: outputs k in [-K, K], K = -k0; pairs (k, -k)
            if (line < nlines) {
                const auto c = io.at(line);
                const int K = -B.k0;
                for (int k = tid; k <= K; k += T) io.store_pair(c, k, buf[k + K], buf[K - k]);
            }
        }
    }
}

template <int P, class IO>
static hipError_t launch_r16(const IO &io, int nlines, const BlueT<typename IO::C> &B,
                             hipStream_t st) {
    using G = R16<P>;
    const size_t lds = (size_t)G::LINES * G::LW * sizeof(real_t<typename IO::C>) +
                       (VhLds<P, IO>::v ? (size_t)P * sizeof(typename IO::C) : 0);
    if (lds > 65536) {
        static bool attr_set = false;
        if (!attr_set) {
            hipError_t e = hipFuncSetAttribute((const void *)k_blue_r16<P, IO>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            attr_set = true;
        }
    }
    const int grid = (nlines + G::LINES - 1) / G::LINES;
    hipLaunchKernelGGL((k_blue_r16<P, IO>), dim3(grid), dim3(G::WG), lds, st, io, nlines, B);
    return hipGetLastError();
}

template <class IO>
static hipError_t run_bluestein_r16(const IO &io, int nlines, const BlueT<typename IO::C> &B,
                                    hipStream_t st) {
    if (nlines <= 0) return hipSuccess;
    switch (B.P) {
        case 256: return launch_r16<256>(io, nlines, B, st);
        case 512: return launch_r16<512>(io, nlines, B, st);
        case 1024: return launch_r16<1024>(io, nlines, B, st);
        case 2048: return launch_r16<2048>(io, nlines, B, st);
        case 4096: return launch_r16<4096>(io, nlines, B, st);
        default: return hipErrorInvalidValue;
    }
}

template <class IO>
static hipError_t run_bluestein(const IO &io, int nlines, const BlueT<typename IO::C> &B,
                                hipStream_t st) {
    if (nlines <= 0) return hipSuccess;
#define CVL_BLUE_CASE(PP)                                                              \
    case PP: {                                                                          \
        constexpr int LN = LinesFor<PP>::v;                                             \
        const int grid = (nlines + LN - 1) / LN;                                        \
        hipLaunchKernelGGL((k_bluestein<PP, LN, IO>), dim3(grid), dim3(256),            \
                           LN * PP * sizeof(typename IO::C), st, io, nlines, B);        \
        return hipGetLastError();                                                       \
    }
    switch (B.P) {
        CVL_BLUE_CASE(8)
        CVL_BLUE_CASE(16)
        CVL_BLUE_CASE(32)
        CVL_BLUE_CASE(64)
        CVL_BLUE_CASE(128)
        default:
            return run_bluestein_r16(io, nlines, B, st);
    }
#undef CVL_BLUE_CASE
}

// ---------------------------------------------------------------------------
// Curvelet (real map, even n) stage IO.
// Cube / plane layouts: X, W1, V2, Z: [r][m][nn] with m in [0, L), nn = n/2 + h,
// row length Nep.  W2: [b][a][k], k = n/2 in [0, h].  V1: [b][a][nn].  The
// grid, [a][b][g], holds the real coefficients either as reals (G = real_t<C>)
// or as complex numbers with a zero imaginary part (G = C).
// ---------------------------------------------------------------------------

// Grid elements are written once per analysis and read by nothing else in
// it: non-temporal (streaming) stores, which do not keep the lines in the
// caches for the stages that follow.
typedef double cvl_d2v __attribute__((ext_vector_type(2)));
typedef float cvl_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void grid_put(double *p, double x) { __builtin_nontemporal_store(x, p); }
__device__ __forceinline__ void grid_put(float *p, float x) { __builtin_nontemporal_store(x, p); }
__device__ __forceinline__ void grid_put(cd *p, double x) {
    __builtin_nontemporal_store(cvl_d2v{x, 0.0}, reinterpret_cast<cvl_d2v *>(p));
}
__device__ __forceinline__ void grid_put(cf *p, float x) {
    __builtin_nontemporal_store(cvl_f2v{x, 0.0f}, reinterpret_cast<cvl_f2v *>(p));
}
// ... and read once per synthesis: non-temporal loads.
__device__ __forceinline__ double grid_get(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float grid_get(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double grid_get(const cd *p) {
    return __builtin_nontemporal_load(&p->x);
}
__device__ __forceinline__ float grid_get(const cf *p) {
    return __builtin_nontemporal_load(&p->x);
}

// alpha DFT of the analysis: line (b, k >= 0); input over m in (-L, L) with the
// reality condition W1(b, -m, -n) = conj W1(b, m, n); output a in [0, 2L-1).
template <class C_>
struct InvAlphaIO {
    using C = C_;
    static constexpr bool kLoadPrio = true;  // (complex128, P <= 1024)
    static constexpr int kLoad = IO_STAGED, kStore = IO_STAGED;
    static constexpr int kBatch = 8;  // inputs fill at most half the line (Kin <= P/2)
    const C *W1;
    C *W2;
    int L, h, Nep, Nm;
    struct Ctx {
        const C *pos, *neg;  // W1[b][m][h+k], W1[b][m][h-k] at m = 0
        C *out;              // W2[b][a][k] at a = 0
    };
    __device__ Ctx at(int line) const {
        const int b = line / (h + 1), k = line % (h + 1);
        const C *base = W1 + (size_t)b * L * Nep + h;
        return Ctx{base + k, base - k, W2 + (size_t)b * Nm * (h + 1) + k};
    }
    __device__ C load(const Ctx &c, int m) const {
        const bool pos = m >= 0;
        const C v = pos ? c.pos[(size_t)m * Nep] : c.neg[(size_t)(-m) * Nep];
        return C{v.x, pos ? v.y : -v.y};
    }
    __device__ void store(const Ctx &c, int a, C v) const { c.out[(size_t)a * (h + 1)] = v; }
};

// gamma DFT of the analysis, one real line (a, b) of the grid per transform.
// Coefficients: even n from W2 (n < 0 by conjugation), odd n zero.
template <class C_, class G>
struct InvGammaIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const C *W2;
    G *grid;
    int L, h, Nm;
    struct Ctx {
        const C *src;
        G *dst;
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        return Ctx{W2 + ((size_t)b * Nm + a) * (h + 1), grid + (size_t)line * Nm};
    }
    __device__ C load(const Ctx &c, int n) const {
        const C v = c.src[(n < 0 ? -n : n) >> 1];
        const real_t<C> keep = (n & 1) ? 0 : 1, sg = n < 0 ? -keep : keep;
        return C{keep * v.x, sg * v.y};
    }
    __device__ void store(const Ctx &c, int g, C v) const { grid_put(c.dst + g, v.x); }
};

// gamma DFT of the analysis, two real lines (2p, 2p+1) per complex transform:
// z_n = c1_n + i c2_n; line 2p is the real, line 2p+1 the imaginary part.
template <class C_, class G>
struct InvGammaPackIO {
    using C = C_;
    static constexpr bool kLoadPrio = true;  // (complex128, P <= 1024)
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // two loads per element
    const C *W2;
    G *grid;
    int L, h, Nm, nreal;
    struct Ctx {
        const C *s1, *s2;
        G *d1, *d2;
        bool two;
    };
    __device__ Ctx at(int p) const {
        const int l1 = 2 * p, l2 = 2 * p + 1;
        const bool two = l2 < nreal;
        const int a1 = l1 / L, b1 = l1 % L;
        const int a2 = two ? l2 / L : a1, b2 = two ? l2 % L : b1;
        return Ctx{W2 + ((size_t)b1 * Nm + a1) * (h + 1), W2 + ((size_t)b2 * Nm + a2) * (h + 1),
                   grid + (size_t)l1 * Nm, grid + (size_t)(two ? l2 : l1) * Nm, two};
    }
    __device__ C load(const Ctx &c, int n) const {
        // s2 is a valid pointer even for a lone last line (it then repeats s1)
        const int k = (n < 0 ? -n : n) >> 1;
        const C c1 = c.s1[k], c2 = c.s2[k];
        const real_t<C> keep = (n & 1) ? 0 : 1;        // odd n: zero
        const real_t<C> w2 = c.two ? keep : 0;         // no second line: zero
        const real_t<C> sg = n < 0 ? -1 : 1;           // conjugate both for n < 0
        return C{keep * c1.x - sg * w2 * c2.y, sg * keep * c1.y + w2 * c2.x};
    }
    __device__ void store(const Ctx &c, int g, C v) const {
        grid_put(c.d1 + g, v.x);
        if (c.two) grid_put(c.d2 + g, v.y);
    }
};

// gamma DFT of the synthesis on line (a, b) of the real grid, so
// c_-n = conj c_n: only even n >= 0 are kept, V1[b][a][n/2].
template <class C_, class G>
struct FwdGammaIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const G *grid;
    C *V1;
    int L, h, Nm;
    struct Ctx {
        const G *src;
        C *dst;  // V1[b][a][0]
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        return Ctx{grid + (size_t)line * Nm, V1 + ((size_t)b * Nm + a) * (h + 1)};
    }
    __device__ C load(const Ctx &c, int g) const { return C{grid_get(c.src + g), 0}; }
    __device__ void store(const Ctx &c, int n, C v) const {
        if ((n & 1) || n < 0) return;
        c.dst[n / 2] = v;
    }
};

// gamma DFT of the synthesis, real lines (2p, 2p+1) of the grid packed as
// z = w1 + i w2; with Z_n its DFT, c1_n = (Z_n + conj Z_-n)/2 and
// c2_n = (Z_n - conj Z_-n)/(2i); even n >= 0 kept.
template <class C_, class G>
struct FwdGammaPackIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_PAIR;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const G *grid;
    C *V1;
    int L, h, Nm, nreal;
    struct Ctx {
        const G *s1, *s2;
        C *d1, *d2;  // V1[b][a][0] of both lines
        bool two;
    };
    __device__ Ctx at(int p) const {
        const int l1 = 2 * p, l2 = 2 * p + 1;
        const bool two = l2 < nreal;
        const int a1 = l1 / L, b1 = l1 % L;
        const int a2 = two ? l2 / L : a1, b2 = two ? l2 % L : b1;
        return Ctx{grid + (size_t)l1 * Nm, grid + (size_t)(two ? l2 : l1) * Nm,
                   V1 + ((size_t)b1 * Nm + a1) * (h + 1), V1 + ((size_t)b2 * Nm + a2) * (h + 1),
                   two};
    }
    __device__ C load(const Ctx &c, int g) const {
        // s2 is a valid pointer even for a lone last line (it then repeats s1)
        const real_t<C> a = grid_get(c.s1 + g), b = grid_get(c.s2 + g);
        return C{a, (real_t<C>)(c.two ? 1 : 0) * b};
    }
    __device__ void store_pair(const Ctx &c, int n, C zn, C zmn) const {
        if (n & 1) return;
        const C czm = cconj(zmn);
        const C s = cadd(zn, czm), d = csub(zn, czm);
        c.d1[n / 2] = C{s.x * (real_t<C>)0.5, s.y * (real_t<C>)0.5};
        if (c.two) c.d2[n / 2] = C{d.y * (real_t<C>)0.5, d.x * (real_t<C>)-0.5};
    }
};

// The two packed gamma stages at an even band-limit L with 1024 <= P <= 4096: the
// analysis window (n = t - (L-1)) holds non-zero coefficients (even n) only
// at odd t, and the synthesis reads only the outputs of even n, at odd
// positions q = n + L - 1; each then runs one of its two FFTs at half length.
template <class C_, class G>
struct InvGammaPackOddIO : InvGammaPackIO<C_, G> {
    static constexpr bool kOddIn = true;
};
template <class C_, class G>
struct FwdGammaPackOddIO : FwdGammaPackIO<C_, G> {
    static constexpr bool kOddOut = true;
    static constexpr bool kFourWaves = true;
};

// alpha DFT of the synthesis: line (b, k), k = n/2 >= 0, all m in (-L, L).
// The grid is real, so the line of -n is the conjugate of the line of n and
// its transform at m is the conjugate of this one's at -m:
//   V2[b][m][h+k] = out(m),  V2[b][m][h-k] = conj out(-m),  m >= 0.
template <class C_>
struct FwdAlphaIO {
    using C = C_;
    static constexpr bool kLoadPrio = true;  // (complex128, P <= 1024)
    static constexpr int kLoad = IO_STAGED, kStore = IO_STAGED;
    static constexpr int kBatch = 8;  // inputs fill at most half the line (Kin <= P/2)
    const C *V1;
    C *V2;
    int L, h, Nm, Nep;
    struct Ctx {
        const C *src;
        C *pos, *neg;  // V2[b][0][h+k], V2[b][0][h-k]
        bool mirror;
    };
    __device__ Ctx at(int line) const {
        const int b = line / (h + 1), k = line % (h + 1);
        C *base = V2 + (size_t)b * L * Nep + h;
        return Ctx{V1 + (size_t)b * Nm * (h + 1) + k, base + k, base - k, k > 0};
    }
    __device__ C load(const Ctx &c, int a) const { return c.src[(size_t)a * (h + 1)]; }
    __device__ void store(const Ctx &c, int m, C v) const {
        if (m >= 0) c.pos[(size_t)m * Nep] = v;
        if (m <= 0 && c.mirror) c.neg[(size_t)(-m) * Nep] = cconj(v);
    }
};

// beta DFT of the analysis (replaces the parity-folded GEMM at large L_j).
// With beta_b = pi + 2 pi k'/(2L-1), k' = b - (L-1), the sum over m' in
// (-L, L) of X[m'] e^{i m' beta_b} is a plain DFT of (-1)^{m'} X[m'] at k'.
// The cube holds m' >= 0 with X[-m'] = (-1)^{m+n} X[m'] (n even), so a line of
// even m is even in m' and one of odd m odd: line (p, nn) transforms
// z = X_{2p} + X_{2p+1} and splits the result by parity of beta ->
// -beta (k' -> -k'):  W1_e(beta) = (Z(beta) + Z(-beta))/2,
// W1_o(beta) = (Z(beta) - Z(-beta))/2, stored for b = L-1-k, k = 0..L-1.
// X, W1: [row][m][nn] with row m' (input) or b (output): `rows` (= L) cube
// rows of Nep per plane, plane stride `plane` (= L*Nep).
template <class C_>
struct BetaInvPairIO {
    using C = C_;
    static constexpr bool kVhLds2048 = sizeof(real_t<C_>) == 4;  // complex64 only
    static constexpr bool kLoadPrio = true;  // (complex128, P <= 1024)
    static constexpr int kLoad = IO_STAGED, kStore = IO_STAGED_PAIR;
    static constexpr int kBatch = 8;  // two loads per element
    const C *X;
    C *W1;
    int L, Ne, Nep, rows;
    size_t plane;
    struct Ctx {
        const C *xe, *xo;  // X[0][2p][nn], X[0][2p+1][nn]
        C *we, *wo;        // W1[0][2p][nn], W1[0][2p+1][nn] (wo null past the last m)
        real_t<C> wo_on;   // 1, or 0 when there is no odd partner
    };
    __device__ Ctx at(int line) const {
        const int p = line / Ne, nn = line % Ne;
        const int me = 2 * p, mo = 2 * p + 1;
        const size_t oe = (size_t)me * Nep + nn, oo = (size_t)mo * Nep + nn;
        // a lone last (even) m reads its own row as the odd partner, weighted 0
        return Ctx{X + oe, X + (mo < rows ? oo : oe), W1 + oe, mo < rows ? W1 + oo : nullptr,
                   (real_t<C>)(mo < rows ? 1 : 0)};
    }
    __device__ C load(const Ctx &c, int j) const {
        const int mp = j < 0 ? -j : j;
        const size_t row = (size_t)mp * plane;
        const C e = c.xe[row], o = c.xo[row];
        const real_t<C> se = (mp & 1) ? -1 : 1;
        const real_t<C> so = (j < 0 ? -c.wo_on : c.wo_on) * se;
        return C{se * e.x + so * o.x, se * e.y + so * o.y};
    }
    __device__ void store_pair(const Ctx &c, int k, C zk, C zmk) const {
        const size_t row = (size_t)(L - 1 - k) * plane;  // b = L-1-k: Z(beta_b) = zmk
        const real_t<C> h = (real_t<C>)0.5;
        c.we[row] = C{(zmk.x + zk.x) * h, (zmk.y + zk.y) * h};
        if (c.wo) c.wo[row] = C{(zmk.x - zk.x) * h, (zmk.y - zk.y) * h};
    }
};

// The same analysis beta DFT writing each line's outputs contiguously in b,
// T[(m Nep + nn) L + b] (line-major), for a tiled transpose into W1 after it.
// At P = 4096 a work-group holds one line, and its stores one element per b
// plane (8 MB apart at L = 1024 in complex64) merged so poorly in the L2 that
// the kernel wrote 3.4 times its output bytes; written line-major they are
// whole cache lines.
template <class C_>
struct BetaInvLineIO : BetaInvPairIO<C_> {
    using C = C_;
    using Ctx = typename BetaInvPairIO<C_>::Ctx;
    __device__ Ctx at(int line) const {
        Ctx c = BetaInvPairIO<C_>::at(line);
        const int p = line / this->Ne, nn = line % this->Ne;
        const int me = 2 * p, mo = 2 * p + 1;
        c.we = this->W1 + ((size_t)me * this->Nep + nn) * this->L;
        c.wo = mo < this->rows ? this->W1 + ((size_t)mo * this->Nep + nn) * this->L : nullptr;
        return c;
    }
    __device__ void store_pair(const Ctx &c, int k, C zk, C zmk) const {
        const int b = this->L - 1 - k;  // Z(beta_b) = zmk
        const real_t<C> h = (real_t<C>)0.5;
        c.we[b] = C{(zmk.x + zk.x) * h, (zmk.y + zk.y) * h};
        if (c.wo) c.wo[b] = C{(zmk.x - zk.x) * h, (zmk.y - zk.y) * h};
    }
};

// W1[b][m][nn] = T[(m Nep + nn) L + b] for nn < Ne (the padding columns of W1
// are not read).  Work-group: one m, 32 nn x 64 b through LDS; reads of T rows
// and writes of W1 rows both contiguous.
template <class C>
__global__ __launch_bounds__(256) void k_lines_to_planes(const C *__restrict__ T,
                                                         C *__restrict__ W1, int L, int Ne,
                                                         int Nep) {
    __shared__ C tile[32][65];
    const int nn0 = blockIdx.x * 32, b0 = blockIdx.y * 64, m = blockIdx.z;
    const int tid = threadIdx.x;
    {
        const int cb = tid & 63, r0 = tid >> 6;
        const int b = b0 + cb;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int nn = nn0 + r0 + 4 * i;
            if (nn < Ne && b < L) tile[r0 + 4 * i][cb] = T[((size_t)m * Nep + nn) * L + b];
        }
    }
    __syncthreads();
    const int cn = tid & 31, rb = tid >> 5;
    const int nn = nn0 + cn;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int b = b0 + rb + 8 * i;
        if (b < L && nn < Ne) W1[((size_t)b * L + m) * Nep + nn] = tile[cn][rb + 8 * i];
    }
}

// ---------------------------------------------------------------------------
// Unrotated curvelets (every n in (-L, L)).  Cube rows per unrot_off; W2 and
// V1 planes [b][a][n] with n in [0, L): the grid is real, so the coefficient
// of -n is the conjugate of that of n, and the cube of m < 0 follows from
// W1(b, -m, -n) = conj W1(b, m, n).
// ---------------------------------------------------------------------------

// alpha DFT of the analysis: line (b, n >= 0), input m in (-L, L), output a.
template <class C_>
struct UnrotInvAlphaIO {
    using C = C_;
    static constexpr int kLoad = IO_STAGED, kStore = IO_STAGED;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const C *W1;
    C *W2;
    ScaleGeom g;
    struct Ctx {
        const C *plane;  // W1[b]
        C *out;          // W2[b][0][n]
        int n;
    };
    __device__ Ctx at(int line) const {
        const int b = line / g.L, n = line % g.L;
        return Ctx{W1 + (size_t)b * 2 * g.L * g.Nep, W2 + (size_t)b * g.Nm * g.L + n, n};
    }
    __device__ C load(const Ctx &c, int m) const {
        // W1(b, m, n) = 0 for |m| > |n| (every cube term has m <= l = |n|);
        // those entries need not have been written
        const bool pos = m >= 0;
        const bool nz = (pos ? m : -m) <= c.n;
        const C v = nz ? c.plane[pos ? unrot_off(g, m, c.n) : unrot_off(g, -m, -c.n)] : C{0, 0};
        return C{v.x, pos ? v.y : -v.y};
    }
    __device__ void store(const Ctx &c, int a, C v) const { c.out[(size_t)a * g.L] = v; }
};

// beta DFT of the analysis on the unrotated cube (the pairing of
// BetaInvPairIO: rows 2m and 2m + 1, the two parities of m + n, share a
// column).  Only the structurally non-zero entries are read (m' <= l and
// m <= l, l = |n|: the others are not written by the contraction); a line
// whose two rows are both zero is dead, and its output is never read.
template <class C_>
struct UnrotBetaInvPairIO {
    using C = C_;
    static constexpr int kLoad = IO_STAGED, kStore = IO_STAGED_PAIR;
    static constexpr int kBatch = 8;  // two loads per element
    const C *X;
    C *W1;
    ScaleGeom g;
    int ne;  // columns in use per row
    struct Ctx {
        const C *xe, *xo;  // X[0][2m][nn], X[0][2m+1][nn]
        C *we, *wo;
        int ke, ko;        // largest m' with a non-zero entry in each row, or -1
    };
    // l = |n| of column nn in row (m, s) when that entry can be non-zero, else -1
    __device__ int lim(int m, int s, int nn) const {
        const int pn = (s + m) & 1, ho = g.L >> 1;
        if (pn ? nn >= 2 * ho : nn > 2 * g.h) return -1;
        const int n = pn ? 2 * (nn - ho) + 1 : 2 * (nn - g.h);
        const int l = n < 0 ? -n : n;
        return m <= l ? l : -1;
    }
    __device__ bool live(int line) const {
        const int m = line / ne, nn = line % ne;
        return lim(m, 0, nn) >= 0 || lim(m, 1, nn) >= 0;
    }
    __device__ Ctx at(int line) const {
        const int m = line / ne, nn = line % ne;
        const size_t oe = (size_t)2 * m * g.Nep + nn, oo = oe + g.Nep;
        return Ctx{X + oe, X + oo, W1 + oe, W1 + oo, lim(m, 0, nn), lim(m, 1, nn)};
    }
    __device__ C load(const Ctx &c, int j) const {
        const int mp = j < 0 ? -j : j;
        const size_t row = (size_t)mp * 2 * g.L * g.Nep;
        const C e = mp <= c.ke ? c.xe[row] : C{0, 0};
        const C o = mp <= c.ko ? c.xo[row] : C{0, 0};
        const real_t<C> se = (mp & 1) ? -1 : 1;
        const real_t<C> so = j < 0 ? -se : se;
        return C{se * e.x + so * o.x, se * e.y + so * o.y};
    }
    __device__ void store_pair(const Ctx &c, int k, C zk, C zmk) const {
        const size_t row = (size_t)(g.L - 1 - k) * 2 * g.L * g.Nep;  // b = L-1-k
        const real_t<C> h = (real_t<C>)0.5;
        c.we[row] = C{(zmk.x + zk.x) * h, (zmk.y + zk.y) * h};
        c.wo[row] = C{(zmk.x - zk.x) * h, (zmk.y - zk.y) * h};
    }
};

// gamma DFT of the analysis, one real line (a, b) of the grid.
template <class C_, class G>
struct UnrotInvGammaIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const C *W2;
    G *grid;
    int L, Nm;
    struct Ctx {
        const C *src;
        G *dst;
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        return Ctx{W2 + ((size_t)b * Nm + a) * L, grid + (size_t)line * Nm};
    }
    __device__ C load(const Ctx &c, int n) const {
        const C v = c.src[n < 0 ? -n : n];
        return C{v.x, n < 0 ? -v.y : v.y};
    }
    __device__ void store(const Ctx &c, int g, C v) const { grid_put(c.dst + g, v.x); }
};

// gamma DFT of the analysis, two real lines (2p, 2p+1) per complex transform
// (z_n = c1_n + i c2_n; real part to line 2p, imaginary part to line 2p+1).
template <class C_, class G>
struct UnrotInvGammaPackIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // two loads per element
    const C *W2;
    G *grid;
    int L, Nm, nreal;
    struct Ctx {
        const C *s1, *s2;
        G *d1, *d2;
        bool two;
    };
    __device__ Ctx at(int p) const {
        const int l1 = 2 * p, l2 = 2 * p + 1;
        const bool two = l2 < nreal;
        const int a1 = l1 / L, b1 = l1 % L;
        const int a2 = two ? l2 / L : a1, b2 = two ? l2 % L : b1;
        return Ctx{W2 + ((size_t)b1 * Nm + a1) * L, W2 + ((size_t)b2 * Nm + a2) * L,
                   grid + (size_t)l1 * Nm, grid + (size_t)(two ? l2 : l1) * Nm, two};
    }
    __device__ C load(const Ctx &c, int n) const {
        // s2 is a valid pointer even for a lone last line (it then repeats s1)
        const int k = n < 0 ? -n : n;
        const C c1 = c.s1[k], c2 = c.s2[k];
        const real_t<C> w2 = c.two ? 1 : 0;   // no second line: zero
        const real_t<C> sg = n < 0 ? -1 : 1;  // conjugate both for n < 0
        return C{c1.x - sg * w2 * c2.y, sg * c1.y + w2 * c2.x};
    }
    __device__ void store(const Ctx &c, int g, C v) const {
        grid_put(c.d1 + g, v.x);
        if (c.two) grid_put(c.d2 + g, v.y);
    }
};

// gamma DFT of the synthesis on line (a, b) of the real grid: n >= 0 kept.
template <class C_, class G>
struct UnrotFwdGammaIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const G *grid;
    C *V1;
    int L, Nm;
    struct Ctx {
        const G *src;
        C *dst;  // V1[b][a][0]
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        return Ctx{grid + (size_t)line * Nm, V1 + ((size_t)b * Nm + a) * L};
    }
    __device__ C load(const Ctx &c, int g) const { return C{grid_get(c.src + g), 0}; }
    __device__ void store(const Ctx &c, int n, C v) const {
        if (n >= 0) c.dst[n] = v;
    }
};

// gamma DFT of the synthesis, real lines (2p, 2p+1) packed as z = w1 + i w2
// and separated as c1_n = (Z_n + conj Z_-n)/2, c2_n = (Z_n - conj Z_-n)/(2i).
template <class C_, class G>
struct UnrotFwdGammaPackIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_PAIR;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const G *grid;
    C *V1;
    int L, Nm, nreal;
    struct Ctx {
        const G *s1, *s2;
        C *d1, *d2;  // V1[b][a][0] of both lines
        bool two;
    };
    __device__ Ctx at(int p) const {
        const int l1 = 2 * p, l2 = 2 * p + 1;
        const bool two = l2 < nreal;
        const int a1 = l1 / L, b1 = l1 % L;
        const int a2 = two ? l2 / L : a1, b2 = two ? l2 % L : b1;
        return Ctx{grid + (size_t)l1 * Nm, grid + (size_t)(two ? l2 : l1) * Nm,
                   V1 + ((size_t)b1 * Nm + a1) * L, V1 + ((size_t)b2 * Nm + a2) * L, two};
    }
    __device__ C load(const Ctx &c, int g) const {
        // s2 is a valid pointer even for a lone last line (it then repeats s1)
        const real_t<C> a = grid_get(c.s1 + g), b = grid_get(c.s2 + g);
        return C{a, (real_t<C>)(c.two ? 1 : 0) * b};
    }
    __device__ void store_pair(const Ctx &c, int n, C zn, C zmn) const {
        const C czm = cconj(zmn);
        const C s = cadd(zn, czm), d = csub(zn, czm);
        c.d1[n] = C{s.x * (real_t<C>)0.5, s.y * (real_t<C>)0.5};
        if (c.two) c.d2[n] = C{d.y * (real_t<C>)0.5, d.x * (real_t<C>)-0.5};
    }
};

// alpha DFT of the synthesis: line (b, n >= 0), all m in (-L, L); m >= 0 to
// (m, n), m <= 0 mirrored as conj to (-m, -n) (n > 0).
template <class C_>
struct UnrotFwdAlphaIO {
    using C = C_;
    static constexpr int kLoad = IO_STAGED, kStore = IO_STAGED;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const C *V1;
    C *V2;
    ScaleGeom g;
    struct Ctx {
        const C *src;  // V1[b][0][n]
        C *plane;      // V2[b]
        int n;
    };
    __device__ Ctx at(int line) const {
        const int b = line / g.L, n = line % g.L;
        return Ctx{V1 + (size_t)b * g.Nm * g.L + n, V2 + (size_t)b * 2 * g.L * g.Nep, n};
    }
    __device__ C load(const Ctx &c, int a) const { return c.src[(size_t)a * g.L]; }
    // only |m| <= |n| is stored: the synthesis contraction reads (m, +-l) with
    // m <= l, and the beta GEMM between keeps columns apart
    __device__ void store(const Ctx &c, int m, C v) const {
        if (m >= 0 && m <= c.n) c.plane[unrot_off(g, m, c.n)] = v;
        if (m <= 0 && -m <= c.n && c.n > 0) c.plane[unrot_off(g, -m, -c.n)] = cconj(v);
    }
};

// ---------------------------------------------------------------------------
// Complex signals.  A complex map f = f_a + i f_b is analysed as its two real
// parts' coefficient sets a_lm, b_lm (each with the reality condition), run
// through the real-signal stages up to the gamma DFT, where the two enter one
// complex transform per grid line: W(a, b, g) = W_a + i W_b, whose gamma
// coefficients are z_n = A_n + i B_n with A_-n = conj A_n, B_-n = conj B_n.
// The synthesis splits a complex grid line the same way:
// A_n = (Z_n + conj Z_-n)/2, B_n = (Z_n - conj Z_-n)/(2i).
// ---------------------------------------------------------------------------

// gamma DFT of the analysis: line (a, b); even n of W2a (A) and W2b (B).
template <class C_>
struct InvGammaCplxIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // two loads per element
    const C *W2a, *W2b;
    C *grid;
    int L, h, Nm;
    struct Ctx {
        const C *sa, *sb;
        C *d;
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        const size_t o = ((size_t)b * Nm + a) * (h + 1);
        return Ctx{W2a + o, W2b + o, grid + (size_t)line * Nm};
    }
    __device__ C load(const Ctx &c, int n) const {
        const int k = (n < 0 ? -n : n) >> 1;
        const C A = c.sa[k], B = c.sb[k];
        const real_t<C> keep = (n & 1) ? 0 : 1;   // odd n: zero
        const real_t<C> sg = n < 0 ? -1 : 1;      // conjugate both for n < 0
        return C{keep * (A.x - sg * B.y), keep * (sg * A.y + B.x)};
    }
    __device__ void store(const Ctx &c, int g, C v) const { c.d[g] = v; }
};

// gamma DFT of the synthesis: line (a, b) of a complex grid split into the
// even n >= 0 coefficients of its two real parts, V1a and V1b [b][a][n/2].
template <class C_>
struct FwdGammaCplxIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_PAIR;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const C *grid;
    C *V1a, *V1b;
    int L, h, Nm;
    struct Ctx {
        const C *src;
        C *da, *db;
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        const size_t o = ((size_t)b * Nm + a) * (h + 1);
        return Ctx{grid + (size_t)line * Nm, V1a + o, V1b + o};
    }
    __device__ C load(const Ctx &c, int g) const { return c.src[g]; }
    __device__ void store_pair(const Ctx &c, int n, C zn, C zmn) const {
        if (n & 1) return;
        const C czm = cconj(zmn);
        const C s = cadd(zn, czm), d = csub(zn, czm);
        c.da[n / 2] = C{s.x * (real_t<C>)0.5, s.y * (real_t<C>)0.5};
        c.db[n / 2] = C{d.y * (real_t<C>)0.5, d.x * (real_t<C>)-0.5};
    }
};

// The same two stages for the unrotated curvelets (every n; W2 / V1 rows of
// L entries, n in [0, L)).
template <class C_>
struct UnrotInvGammaCplxIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // two loads per element
    const C *W2a, *W2b;
    C *grid;
    int L, Nm;
    struct Ctx {
        const C *sa, *sb;
        C *d;
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        const size_t o = ((size_t)b * Nm + a) * L;
        return Ctx{W2a + o, W2b + o, grid + (size_t)line * Nm};
    }
    __device__ C load(const Ctx &c, int n) const {
        const int k = n < 0 ? -n : n;
        const C A = c.sa[k], B = c.sb[k];
        const real_t<C> sg = n < 0 ? -1 : 1;
        return C{A.x - sg * B.y, sg * A.y + B.x};
    }
    __device__ void store(const Ctx &c, int g, C v) const { c.d[g] = v; }
};

template <class C_>
struct UnrotFwdGammaCplxIO {
    using C = C_;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_PAIR;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const C *grid;
    C *V1a, *V1b;
    int L, Nm;
    struct Ctx {
        const C *src;
        C *da, *db;
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        const size_t o = ((size_t)b * Nm + a) * L;
        return Ctx{grid + (size_t)line * Nm, V1a + o, V1b + o};
    }
    __device__ C load(const Ctx &c, int g) const { return c.src[g]; }
    __device__ void store_pair(const Ctx &c, int n, C zn, C zmn) const {
        const C czm = cconj(zmn);
        const C s = cadd(zn, czm), d = csub(zn, czm);
        c.da[n] = C{s.x * (real_t<C>)0.5, s.y * (real_t<C>)0.5};
        c.db[n] = C{d.y * (real_t<C>)0.5, d.x * (real_t<C>)-0.5};
    }
};

// phi DFTs of the SHT of a complex map (every m, column m + L - 1).
struct ShtInvPhiCplxIO {
    using C = cd;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const cd *G;
    cd *map;
    int L, Nm;
    struct Ctx {
        const cd *src;
        cd *dst;
    };
    __device__ Ctx at(int t) const {
        return Ctx{G + (size_t)t * Nm + (L - 1), map + (size_t)t * Nm};
    }
    __device__ cd load(const Ctx &c, int m) const { return c.src[m]; }
    __device__ void store(const Ctx &c, int p, cd v) const { c.dst[p] = v; }
};

struct ShtFwdPhiCplxIO {
    using C = cd;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const cd *map;
    cd *F1;
    int L, Nm;
    struct Ctx {
        const cd *src;
        cd *dst;
    };
    __device__ Ctx at(int t) const {
        return Ctx{map + (size_t)t * Nm, F1 + (size_t)t * Nm + (L - 1)};
    }
    __device__ cd load(const Ctx &c, int p) const { return c.src[p]; }
    __device__ void store(const Ctx &c, int m, cd v) const { c.dst[m] = v; }
};

struct ShtInvPhiIO {
    using C = cd;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const cd *G;
    double *map;
    int L, Nm;
    struct Ctx {
        const cd *src;
        double *dst;
    };
    __device__ Ctx at(int t) const { return Ctx{G + (size_t)t * L, map + (size_t)t * Nm}; }
    __device__ cd load(const Ctx &c, int m) const {
        const cd v = c.src[m < 0 ? -m : m];
        return cd{v.x, m < 0 ? -v.y : v.y};
    }
    __device__ void store(const Ctx &c, int p, cd v) const { c.dst[p] = v.x; }
};

struct ShtFwdPhiIO {
    using C = cd;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const double *map;
    cd *F1;
    int L, Nm;
    struct Ctx {
        const double *src;
        cd *dst;
    };
    __device__ Ctx at(int t) const { return Ctx{map + (size_t)t * Nm, F1 + (size_t)t * L}; }
    __device__ cd load(const Ctx &c, int p) const { return cd{c.src[p], 0.0}; }
    __device__ void store(const Ctx &c, int m, cd v) const { c.dst[m] = v; }
};

template <class C>
static hipError_t inv_alpha_t(const ScaleGeom &g, const BlueT<C> &B, const C *W1, C *W2,
                              hipStream_t st) {
    InvAlphaIO<C> io{W1, W2, g.L, g.h, g.Nep, g.Nm};
    return run_bluestein(io, g.L * (g.h + 1), B, st);
}
template <class C, class G>
static hipError_t inv_gamma_t(const ScaleGeom &g, const BlueT<C> &B, const C *W2, G *grid,
                              hipStream_t st) {
    const int nreal = g.Nm * g.L;
    if (B.P >= 1024 && B.P <= 4096 && (g.L & 1) == 0) {
        InvGammaPackOddIO<C, G> io{{W2, grid, g.L, g.h, g.Nm, nreal}};
        const int n = (nreal + 1) / 2;
        return B.P == 1024 ? launch_r16<1024>(io, n, B, st)
               : B.P == 2048 ? launch_r16<2048>(io, n, B, st)
                             : launch_r16<4096>(io, n, B, st);
    }
    if (B.P >= 256) {
        InvGammaPackIO<C, G> io{W2, grid, g.L, g.h, g.Nm, nreal};
        return run_bluestein_r16(io, (nreal + 1) / 2, B, st);
    }
    InvGammaIO<C, G> io{W2, grid, g.L, g.h, g.Nm};
    return run_bluestein(io, nreal, B, st);
}
template <class C, class G>
static hipError_t fwd_gamma_t(const ScaleGeom &g, const BlueT<C> &B, const G *grid, C *V1,
                              hipStream_t st) {
    const int nreal = g.Nm * g.L;
    if ((B.P == 1024 || B.P == 2048 || B.P == 4096) && (g.L & 1) == 0) {
        FwdGammaPackOddIO<C, G> io{{grid, V1, g.L, g.h, g.Nm, nreal}};
        const int n = (nreal + 1) / 2;
        return B.P == 1024   ? launch_r16<1024>(io, n, B, st)
               : B.P == 2048 ? launch_r16<2048>(io, n, B, st)
                             : launch_r16<4096>(io, n, B, st);
    }
    if (B.P >= 256) {
        FwdGammaPackIO<C, G> io{grid, V1, g.L, g.h, g.Nm, nreal};
        return run_bluestein_r16(io, (nreal + 1) / 2, B, st);
    }
    FwdGammaIO<C, G> io{grid, V1, g.L, g.h, g.Nm};
    return run_bluestein(io, nreal, B, st);
}
template <class C>
static hipError_t fwd_alpha_t(const ScaleGeom &g, const BlueT<C> &B, const C *V1, C *V2,
                              hipStream_t st) {
    FwdAlphaIO<C> io{V1, V2, g.L, g.h, g.Nm, g.Nep};
    return run_bluestein(io, g.L * (g.h + 1), B, st);
}

template <class C>
static hipError_t inv_beta_t(const ScaleGeom &g, const BlueT<C> &B, const C *X, C *W1,
                             hipStream_t st) {
    BetaInvPairIO<C> io{X, W1, g.L, g.Ne, g.Nep, g.L, (size_t)g.L * g.Nep};
    return run_bluestein(io, ((g.L + 1) / 2) * g.Ne, B, st);
}
hipError_t launch_inv_beta_dft(const ScaleGeom &g, const BluesteinDev &B, const cd *X, cd *W1,
                               hipStream_t st) {
    return inv_beta_t(g, B, X, W1, st);
}
hipError_t launch_inv_beta_dft(const ScaleGeom &g, const BluesteinF &B, const cf *X, cf *W1,
                               hipStream_t st) {
    return inv_beta_t(g, B, X, W1, st);
}
template <class C>
static hipError_t inv_beta_lines_t(const ScaleGeom &g, const BlueT<C> &B, const C *X, C *T,
                                   hipStream_t st) {
    BetaInvLineIO<C> io{{X, T, g.L, g.Ne, g.Nep, g.L, (size_t)g.L * g.Nep}};
    return run_bluestein(io, ((g.L + 1) / 2) * g.Ne, B, st);
}
hipError_t launch_inv_beta_dft_lines(const ScaleGeom &g, const BluesteinDev &B, const cd *X,
                                     cd *T, hipStream_t st) {
    return inv_beta_lines_t(g, B, X, T, st);
}
hipError_t launch_inv_beta_dft_lines(const ScaleGeom &g, const BluesteinF &B, const cf *X,
                                     cf *T, hipStream_t st) {
    return inv_beta_lines_t(g, B, X, T, st);
}
template <class C>
static hipError_t lines_to_planes_t(const ScaleGeom &g, const C *T, C *W1, hipStream_t st) {
    dim3 grid((g.Ne + 31) / 32, (g.L + 63) / 64, g.L);
    hipLaunchKernelGGL(k_lines_to_planes<C>, grid, dim3(256), 0, st, T, W1, g.L, g.Ne, g.Nep);
    return hipGetLastError();
}
hipError_t launch_beta_lines_to_planes(const ScaleGeom &g, const cd *T, cd *W1, hipStream_t st) {
    return lines_to_planes_t(g, T, W1, st);
}
hipError_t launch_beta_lines_to_planes(const ScaleGeom &g, const cf *T, cf *W1, hipStream_t st) {
    return lines_to_planes_t(g, T, W1, st);
}

hipError_t launch_inv_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *W1, cd *W2,
                            hipStream_t st) {
    return inv_alpha_t(g, B, W1, W2, st);
}
hipError_t launch_inv_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *W2, cd *grid,
                            hipStream_t st) {
    return inv_gamma_t(g, B, W2, grid, st);
}
hipError_t launch_inv_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *W2,
                            double *grid, hipStream_t st) {
    return inv_gamma_t(g, B, W2, grid, st);
}
hipError_t launch_fwd_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *grid, cd *V1,
                            hipStream_t st) {
    return fwd_gamma_t(g, B, grid, V1, st);
}
hipError_t launch_fwd_gamma(const ScaleGeom &g, const BluesteinDev &B, const double *grid,
                            cd *V1, hipStream_t st) {
    return fwd_gamma_t(g, B, grid, V1, st);
}
hipError_t launch_fwd_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *V1, cd *V2,
                            hipStream_t st) {
    return fwd_alpha_t(g, B, V1, V2, st);
}
hipError_t launch_inv_alpha(const ScaleGeom &g, const BluesteinF &B, const cf *W1, cf *W2,
                            hipStream_t st) {
    return inv_alpha_t(g, B, W1, W2, st);
}
hipError_t launch_inv_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *W2, cf *grid,
                            hipStream_t st) {
    return inv_gamma_t(g, B, W2, grid, st);
}
hipError_t launch_inv_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *W2,
                            float *grid, hipStream_t st) {
    return inv_gamma_t(g, B, W2, grid, st);
}
hipError_t launch_fwd_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *grid, cf *V1,
                            hipStream_t st) {
    return fwd_gamma_t(g, B, grid, V1, st);
}
hipError_t launch_fwd_gamma(const ScaleGeom &g, const BluesteinF &B, const float *grid,
                            cf *V1, hipStream_t st) {
    return fwd_gamma_t(g, B, grid, V1, st);
}
hipError_t launch_fwd_alpha(const ScaleGeom &g, const BluesteinF &B, const cf *V1, cf *V2,
                            hipStream_t st) {
    return fwd_alpha_t(g, B, V1, V2, st);
}
// ---- unrotated curvelet stages ----
template <class C>
static hipError_t unrot_inv_beta_t(const ScaleGeom &g, const BlueT<C> &B, const C *X, C *W1,
                                   hipStream_t st) {
    const int ne = unrot_cols(g);
    UnrotBetaInvPairIO<C> io{X, W1, g, ne};
    return run_bluestein(io, g.L * ne, B, st);
}
template <class C>
static hipError_t unrot_inv_alpha_t(const ScaleGeom &g, const BlueT<C> &B, const C *W1, C *W2,
                                    hipStream_t st) {
    UnrotInvAlphaIO<C> io{W1, W2, g};
    return run_bluestein(io, g.L * g.L, B, st);
}
template <class C, class G>
static hipError_t unrot_inv_gamma_t(const ScaleGeom &g, const BlueT<C> &B, const C *W2, G *grid,
                                    hipStream_t st) {
    const int nreal = g.Nm * g.L;
    if (B.P >= 256) {
        UnrotInvGammaPackIO<C, G> io{W2, grid, g.L, g.Nm, nreal};
        return run_bluestein_r16(io, (nreal + 1) / 2, B, st);
    }
    UnrotInvGammaIO<C, G> io{W2, grid, g.L, g.Nm};
    return run_bluestein(io, nreal, B, st);
}
template <class C, class G>
static hipError_t unrot_fwd_gamma_t(const ScaleGeom &g, const BlueT<C> &B, const G *grid, C *V1,
                                    hipStream_t st) {
    const int nreal = g.Nm * g.L;
    if (B.P >= 256) {
        UnrotFwdGammaPackIO<C, G> io{grid, V1, g.L, g.Nm, nreal};
        return run_bluestein_r16(io, (nreal + 1) / 2, B, st);
    }
    UnrotFwdGammaIO<C, G> io{grid, V1, g.L, g.Nm};
    return run_bluestein(io, nreal, B, st);
}
template <class C>
static hipError_t unrot_fwd_alpha_t(const ScaleGeom &g, const BlueT<C> &B, const C *V1, C *V2,
                                    hipStream_t st) {
    UnrotFwdAlphaIO<C> io{V1, V2, g};
    return run_bluestein(io, g.L * g.L, B, st);
}
hipError_t launch_unrot_inv_beta_dft(const ScaleGeom &g, const BluesteinDev &B, const cd *X,
                                     cd *W1, hipStream_t st) {
    return unrot_inv_beta_t(g, B, X, W1, st);
}
hipError_t launch_unrot_inv_beta_dft(const ScaleGeom &g, const BluesteinF &B, const cf *X,
                                     cf *W1, hipStream_t st) {
    return unrot_inv_beta_t(g, B, X, W1, st);
}
hipError_t launch_unrot_inv_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *W1,
                                  cd *W2, hipStream_t st) {
    return unrot_inv_alpha_t(g, B, W1, W2, st);
}
hipError_t launch_unrot_inv_alpha(const ScaleGeom &g, const BluesteinF &B, const cf *W1,
                                  cf *W2, hipStream_t st) {
    return unrot_inv_alpha_t(g, B, W1, W2, st);
}
hipError_t launch_unrot_inv_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *W2,
                                  cd *grid, hipStream_t st) {
    return unrot_inv_gamma_t(g, B, W2, grid, st);
}
hipError_t launch_unrot_inv_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *W2,
                                  double *grid, hipStream_t st) {
    return unrot_inv_gamma_t(g, B, W2, grid, st);
}
hipError_t launch_unrot_inv_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *W2,
                                  cf *grid, hipStream_t st) {
    return unrot_inv_gamma_t(g, B, W2, grid, st);
}
hipError_t launch_unrot_inv_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *W2,
                                  float *grid, hipStream_t st) {
    return unrot_inv_gamma_t(g, B, W2, grid, st);
}
hipError_t launch_unrot_fwd_gamma(const ScaleGeom &g, const BluesteinDev &B, const cd *grid,
                                  cd *V1, hipStream_t st) {
    return unrot_fwd_gamma_t(g, B, grid, V1, st);
}
hipError_t launch_unrot_fwd_gamma(const ScaleGeom &g, const BluesteinDev &B,
                                  const double *grid, cd *V1, hipStream_t st) {
    return unrot_fwd_gamma_t(g, B, grid, V1, st);
}
hipError_t launch_unrot_fwd_gamma(const ScaleGeom &g, const BluesteinF &B, const cf *grid,
                                  cf *V1, hipStream_t st) {
    return unrot_fwd_gamma_t(g, B, grid, V1, st);
}
hipError_t launch_unrot_fwd_gamma(const ScaleGeom &g, const BluesteinF &B, const float *grid,
                                  cf *V1, hipStream_t st) {
    return unrot_fwd_gamma_t(g, B, grid, V1, st);
}
hipError_t launch_unrot_fwd_alpha(const ScaleGeom &g, const BluesteinDev &B, const cd *V1,
                                  cd *V2, hipStream_t st) {
    return unrot_fwd_alpha_t(g, B, V1, V2, st);
}
hipError_t launch_unrot_fwd_alpha(const ScaleGeom &g, const BluesteinF &B, const cf *V1,
                                  cf *V2, hipStream_t st) {
    return unrot_fwd_alpha_t(g, B, V1, V2, st);
}

// ---- complex signals ----
template <class C>
static hipError_t inv_gamma_cplx_t(const ScaleGeom &g, const BlueT<C> &B, const C *W2a,
                                   const C *W2b, C *grid, hipStream_t st) {
    InvGammaCplxIO<C> io{W2a, W2b, grid, g.L, g.h, g.Nm};
    return run_bluestein(io, g.Nm * g.L, B, st);
}
template <class C>
static hipError_t fwd_gamma_cplx_t(const ScaleGeom &g, const BlueT<C> &B, const C *grid, C *V1a,
                                   C *V1b, hipStream_t st) {
    FwdGammaCplxIO<C> io{grid, V1a, V1b, g.L, g.h, g.Nm};
    return run_bluestein(io, g.Nm * g.L, B, st);
}
template <class C>
static hipError_t unrot_inv_gamma_cplx_t(const ScaleGeom &g, const BlueT<C> &B, const C *W2a,
                                         const C *W2b, C *grid, hipStream_t st) {
    UnrotInvGammaCplxIO<C> io{W2a, W2b, grid, g.L, g.Nm};
    return run_bluestein(io, g.Nm * g.L, B, st);
}
template <class C>
static hipError_t unrot_fwd_gamma_cplx_t(const ScaleGeom &g, const BlueT<C> &B, const C *grid,
                                         C *V1a, C *V1b, hipStream_t st) {
    UnrotFwdGammaCplxIO<C> io{grid, V1a, V1b, g.L, g.Nm};
    return run_bluestein(io, g.Nm * g.L, B, st);
}
hipError_t launch_inv_gamma_cplx(const ScaleGeom &g, const BluesteinDev &B, const cd *W2a,
                                 const cd *W2b, cd *grid, hipStream_t st) {
    return inv_gamma_cplx_t(g, B, W2a, W2b, grid, st);
}
hipError_t launch_inv_gamma_cplx(const ScaleGeom &g, const BluesteinF &B, const cf *W2a,
                                 const cf *W2b, cf *grid, hipStream_t st) {
    return inv_gamma_cplx_t(g, B, W2a, W2b, grid, st);
}
hipError_t launch_fwd_gamma_cplx(const ScaleGeom &g, const BluesteinDev &B, const cd *grid,
                                 cd *V1a, cd *V1b, hipStream_t st) {
    return fwd_gamma_cplx_t(g, B, grid, V1a, V1b, st);
}
hipError_t launch_fwd_gamma_cplx(const ScaleGeom &g, const BluesteinF &B, const cf *grid,
                                 cf *V1a, cf *V1b, hipStream_t st) {
    return fwd_gamma_cplx_t(g, B, grid, V1a, V1b, st);
}
hipError_t launch_unrot_inv_gamma_cplx(const ScaleGeom &g, const BluesteinDev &B,
                                       const cd *W2a, const cd *W2b, cd *grid, hipStream_t st) {
    return unrot_inv_gamma_cplx_t(g, B, W2a, W2b, grid, st);
}
hipError_t launch_unrot_inv_gamma_cplx(const ScaleGeom &g, const BluesteinF &B,
                                       const cf *W2a, const cf *W2b, cf *grid, hipStream_t st) {
    return unrot_inv_gamma_cplx_t(g, B, W2a, W2b, grid, st);
}
hipError_t launch_unrot_fwd_gamma_cplx(const ScaleGeom &g, const BluesteinDev &B,
                                       const cd *grid, cd *V1a, cd *V1b, hipStream_t st) {
    return unrot_fwd_gamma_cplx_t(g, B, grid, V1a, V1b, st);
}
hipError_t launch_unrot_fwd_gamma_cplx(const ScaleGeom &g, const BluesteinF &B,
                                       const cf *grid, cf *V1a, cf *V1b, hipStream_t st) {
    return unrot_fwd_gamma_cplx_t(g, B, grid, V1a, V1b, st);
}
hipError_t launch_sht_inv_phi_cplx(int L, const BluesteinDev &B, const cd *G, cd *map,
                                   hipStream_t st) {
    ShtInvPhiCplxIO io{G, map, L, 2 * L - 1};
    return run_bluestein(io, L, B, st);
}
hipError_t launch_sht_fwd_phi_cplx(int L, const BluesteinDev &B, const cd *map, cd *F1,
                                   hipStream_t st) {
    ShtFwdPhiCplxIO io{map, F1, L, 2 * L - 1};
    return run_bluestein(io, L, B, st);
}

hipError_t launch_sht_inv_phi(int L, const BluesteinDev &B, const cd *G, double *map,
                              hipStream_t st) {
    ShtInvPhiIO io{G, map, L, 2 * L - 1};
    return run_bluestein(io, L, B, st);
}
hipError_t launch_sht_fwd_phi(int L, const BluesteinDev &B, const double *map, cd *F1,
                              hipStream_t st) {
    ShtFwdPhiIO io{map, F1, L, 2 * L - 1};
    return run_bluestein(io, L, B, st);
}

// ---------------------------------------------------------------------------
// General complex Wigner transforms: all m in (-L, L), all n in (-N, N).
// Cube / plane layouts: [r][m + L - 1][n + N - 1] with row length Nnp.
// ---------------------------------------------------------------------------
static inline int nnp_of(int N) { return ((2 * N - 1) + 31) / 32 * 32; }

struct GenInvAlphaIO {  // line (b, n); in m; out a
    using C = cd;
    static constexpr int kLoad = IO_STAGED, kStore = IO_STAGED;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const cd *W1;
    cd *W2;
    int L, Nn, Nnp, Nm;
    struct Ctx {
        const cd *src;
        cd *dst;
    };
    __device__ Ctx at(int line) const {
        const int b = line / Nn, n = line % Nn;
        return Ctx{W1 + ((size_t)b * Nm + (L - 1)) * Nnp + n, W2 + (size_t)b * Nm * Nnp + n};
    }
    __device__ cd load(const Ctx &c, int m) const { return c.src[(ptrdiff_t)m * Nnp]; }
    __device__ void store(const Ctx &c, int a, cd v) const { c.dst[(size_t)a * Nnp] = v; }
};
struct GenInvGammaIO {  // line (a, b); in n; out g
    using C = cd;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const cd *W2;
    cd *grid;
    int L, N, Nnp, Nm, Ng;
    struct Ctx {
        const cd *src;
        cd *dst;
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        return Ctx{W2 + ((size_t)b * Nm + a) * Nnp + (N - 1), grid + (size_t)line * Ng};
    }
    __device__ cd load(const Ctx &c, int n) const { return c.src[n]; }
    __device__ void store(const Ctx &c, int g, cd v) const { c.dst[g] = v; }
};
struct GenFwdGammaIO {  // line (a, b); in g; out n
    using C = cd;
    static constexpr int kLoad = IO_DIRECT, kStore = IO_DIRECT;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const cd *grid;
    cd *V1;
    int L, N, Nnp, Nm, Ng;
    struct Ctx {
        const cd *src;
        cd *dst;
    };
    __device__ Ctx at(int line) const {
        const int a = line / L, b = line % L;
        return Ctx{grid + (size_t)line * Ng, V1 + ((size_t)b * Nm + a) * Nnp + (N - 1)};
    }
    __device__ cd load(const Ctx &c, int g) const { return c.src[g]; }
    __device__ void store(const Ctx &c, int n, cd v) const { c.dst[n] = v; }
};
struct GenFwdAlphaIO {  // line (b, n); in a; out m
    using C = cd;
    static constexpr int kLoad = IO_STAGED, kStore = IO_STAGED;
    static constexpr int kBatch = 8;  // inputs fill at most about half the line
    const cd *V1;
    cd *V2;
    int L, Nn, Nnp, Nm;
    struct Ctx {
        const cd *src;
        cd *dst;
    };
    __device__ Ctx at(int line) const {
        const int b = line / Nn, n = line % Nn;
        return Ctx{V1 + (size_t)b * Nm * Nnp + n, V2 + ((size_t)b * Nm + (L - 1)) * Nnp + n};
    }
    __device__ cd load(const Ctx &c, int a) const { return c.src[(size_t)a * Nnp]; }
    __device__ void store(const Ctx &c, int m, cd v) const { c.dst[(ptrdiff_t)m * Nnp] = v; }
};

hipError_t launch_gen_inv_alpha(int L, int N, const BluesteinDev &B, const cd *W1,
                                cd *W2, hipStream_t st) {
    GenInvAlphaIO io{W1, W2, L, 2 * N - 1, nnp_of(N), 2 * L - 1};
    return run_bluestein(io, L * (2 * N - 1), B, st);
}
hipError_t launch_gen_inv_gamma(int L, int N, const BluesteinDev &B, const cd *W2,
                                cd *grid, hipStream_t st) {
    GenInvGammaIO io{W2, grid, L, N, nnp_of(N), 2 * L - 1, 2 * N - 1};
    return run_bluestein(io, (2 * L - 1) * L, B, st);
}
hipError_t launch_gen_fwd_gamma(int L, int N, const BluesteinDev &B, const cd *grid,
                                cd *V1, hipStream_t st) {
    GenFwdGammaIO io{grid, V1, L, N, nnp_of(N), 2 * L - 1, 2 * N - 1};
    return run_bluestein(io, (2 * L - 1) * L, B, st);
}
hipError_t launch_gen_fwd_alpha(int L, int N, const BluesteinDev &B, const cd *V1,
                                cd *V2, hipStream_t st) {
    GenFwdAlphaIO io{V1, V2, L, 2 * N - 1, nnp_of(N), 2 * L - 1};
    return run_bluestein(io, L * (2 * N - 1), B, st);
}

}  // namespace cvl
