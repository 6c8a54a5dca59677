// Host-side tables: curvelet kernels (Sec. II-B), parity-folded beta matrices
// (Sec. III-A-2) and Bluestein chirp tables for the odd-length MW DFTs.
#include "host_tables.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <map>
#include <thread>

namespace cvl {
namespace host {

namespace {

using ld = long double;
const ld kPiL = 3.141592653589793238462643383279502884L;

// 20-point Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration.
struct GL20 {
    ld x[20], w[20];
    GL20() {
        const int n = 20;
        for (int i = 0; i < n; ++i) {
            ld z = std::cos(kPiL * (i + 0.75L) / (n + 0.5L));
            for (int it = 0; it < 100; ++it) {
                ld p0 = 1, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                ld dp = n * (z * p1 - p0) / (z * z - 1);
                ld dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-19L) break;
            }
            ld p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            ld dp = n * (z * p1 - p0) / (z * z - 1);
            x[i] = z;
            w[i] = 2 / ((1 - z * z) * dp * dp);
        }
    }
};
const GL20 &gl20() {
    static GL20 g;
    return g;
}

// s_lambda(u)^2 / u with s(x) = exp(-1/(1-x^2)) on (-1, 1).
ld integrand(ld u, ld lam) {
    ld x = 2 * lam / (lam - 1) * (u - 1 / lam) - 1;
    if (x <= -1 || x >= 1) return 0;
    return std::exp(-2 / (1 - x * x)) / u;
}

ld integral(ld a, ld b, ld lam) {
    if (b <= a) return 0;
    const GL20 &g = gl20();
    const int panels = 64;
    ld h = (b - a) / panels, s = 0;
    for (int p = 0; p < panels; ++p) {
        ld c = a + (p + 0.5L) * h, r = 0.5L * h;
        ld acc = 0;
        for (int i = 0; i < 20; ++i) acc += g.w[i] * integrand(c + r * g.x[i], lam);
        s += acc * r;
    }
    return s;
}

}  // namespace

double k_lambda(double t, double lam) {
    if (t <= 1.0 / lam) return 1.0;
    if (t >= 1.0) return 0.0;
    static std::mutex mu;
    static std::map<double, ld> den_cache;
    ld den;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = den_cache.find(lam);
        if (it == den_cache.end()) {
            den = integral(1 / (ld)lam, 1, lam);
            den_cache[lam] = den;
        } else {
            den = it->second;
        }
    }
    return (double)(integral(t, 1, lam) / den);
}

std::vector<double> kappa_table(int L, double lam, int J0, int J) {
    std::vector<double> out((size_t)(J - J0 + 1) * L, 0.0);
    for (int j = J0; j <= J; ++j) {
        double lo = std::pow(lam, j), hi = std::pow(lam, j + 1);
        for (int l = 0; l < L; ++l) {
            double v = k_lambda(l / hi, lam) - k_lambda(l / lo, lam);
            out[(size_t)(j - J0) * L + l] = v > 0 ? std::sqrt(v) : 0.0;
        }
    }
    return out;
}

std::vector<double> phi_table(int L, double lam, int J0) {
    std::vector<double> out(L);
    double s = std::pow(lam, J0);
    for (int l = 0; l < L; ++l)
        out[l] = std::sqrt((2.0 * l + 1) / (4 * M_PI)) * std::sqrt(k_lambda(l / s, lam));
    return out;
}

std::vector<double> delta_col_l(int L) {
    // a_l(0) = prod_{i<=l} sqrt((2i-1)/(2i)); a_l(n+1) = a_l(n) sqrt((l-n)/(l+n+1)).
    std::vector<double> out((size_t)L * L, 0.0);
    ld a0 = 1;
    for (int l = 0; l < L; ++l) {
        if (l > 0) a0 *= std::sqrt((ld)(2 * l - 1) / (ld)(2 * l));
        ld a = a0;
        for (int n = 0; n <= l; ++n) {
            out[(size_t)l * L + n] = (double)a;
            a *= std::sqrt((ld)(l - n) / (ld)(l + n + 1));
        }
    }
    return out;
}

std::vector<double> zeta_rotated(int L, double theta) {
    const int Nm = 2 * L - 1;
    std::vector<double> z((size_t)L * Nm, 0.0);
    const ld sh = std::sin((ld)theta / 2), ch = std::cos((ld)theta / 2);
    // b^e in log space (0^0 = 1, 0^e = 0 for e > 0)
    auto lpow = [](ld b, int e, bool *zero) -> ld {
        if (e == 0) return 0.0L;
        if (b <= 0.0L) {
            *zero = true;
            return 0.0L;
        }
        return (ld)e * std::log(b);
    };
    for (int l = 0; l < L; ++l) {
        for (int n = -l; n <= l; ++n) {
            const ld lb = 0.5L * (std::lgamma((ld)(2 * l + 1)) - std::lgamma((ld)(l + n + 1)) -
                                  std::lgamma((ld)(l - n + 1)));
            bool z1 = false, z2 = false;
            const ld e1 = lb + lpow(sh, l - n, &z1) + lpow(ch, l + n, &z1);
            const ld e2 = lb + lpow(sh, l + n, &z2) + lpow(ch, l - n, &z2);
            const ld t1 = z1 ? 0.0L : std::exp(e1);
            const ld t2 = z2 ? 0.0L : std::exp(e2) * ((n & 1) ? -1.0L : 1.0L);
            z[(size_t)l * Nm + n + L - 1] = (double)((t1 + t2) / std::sqrt(2.0L));
        }
    }
    return z;
}

void beta_inverse_mats(int L, std::vector<double> &C, std::vector<double> &S) {
    const long Nm = 2L * L - 1;
    C.assign((size_t)L * L, 0.0);
    S.assign((size_t)L * L, 0.0);
    for (int b = 0; b < L; ++b) {
        for (int mp = 0; mp < L; ++mp) {
            // m' beta_b = pi * m'(2b+1) / Nm, reduced mod 2 pi exactly
            long q = ((long)mp * (2 * b + 1)) % (2 * Nm);
            ld ang = kPiL * (ld)q / (ld)Nm;
            C[(size_t)b * L + mp] = mp ? (double)(2 * std::cos(ang)) : 1.0;
            S[(size_t)b * L + mp] = mp ? (double)(2 * std::sin(ang)) : 0.0;
        }
    }
}

namespace {
// w(p) = int_0^pi sin(b) e^{ipb} db
std::complex<double> wgt(long p) {
    if (p == 1) return {0.0, M_PI / 2};
    if (p == -1) return {0.0, -M_PI / 2};
    if (p % 2 == 0) return {2.0 / (1.0 - (double)p * (double)p), 0.0};
    return {0.0, 0.0};
}
}  // namespace

void beta_forward_mats(int L, double factor, std::vector<double> &Qp,
                       std::vector<double> &Qs) {
    const long Nm = 2L * L - 1;
    Qp.assign((size_t)L * L, 0.0);
    Qs.assign((size_t)L * L, 0.0);
    // phase table e^{i pi q / Nm}, q < 2 Nm
    std::vector<std::complex<double>> ph(2 * Nm);
    for (long q = 0; q < 2 * Nm; ++q) {
        ld a = kPiL * (ld)q / (ld)Nm;
        ph[q] = {(double)std::cos(a), (double)std::sin(a)};
    }
    auto work = [&](int b0, int b1) {
        for (int b = b0; b < b1; ++b) {
            const double cb = (b < L - 1) ? 1.0 : 0.0;
            for (int mp = 0; mp < L; ++mp) {
                std::complex<double> acc_p(0, 0), acc_m(0, 0);
                for (long mpp = -(L - 1); mpp <= L - 1; ++mpp) {
                    long q = ((mpp * (2 * b + 1)) % (2 * Nm) + 2 * Nm) % (2 * Nm);
                    std::complex<double> eplus = ph[q];          // e^{+i m'' beta_b}
                    std::complex<double> eminus = std::conj(eplus);
                    std::complex<double> Kp, Km;
                    if (mp == 0) {
                        Kp = wgt(mpp);
                        Km = 0.0;
                    } else {
                        Kp = wgt(mpp - mp) + wgt(mpp + mp);
                        Km = wgt(mpp - mp) - wgt(mpp + mp);
                    }
                    if (Kp != 0.0) acc_p += Kp * (eminus + cb * eplus);
                    if (Km != 0.0) acc_m += Km * (eminus - cb * eplus);
                }
                Qp[(size_t)mp * L + b] = factor / Nm * acc_p.real();
                Qs[(size_t)mp * L + b] = factor / Nm * acc_m.imag();
            }
        }
    };
    int nthr = (int)std::thread::hardware_concurrency();
    if (nthr < 1) nthr = 1;
    if (nthr > 16) nthr = 16;
    if ((long)L * L * L < 4000000L) nthr = 1;
    std::vector<std::thread> th;
    int per = (L + nthr - 1) / nthr;
    for (int t = 0; t < nthr; ++t) {
        int b0 = t * per, b1 = std::min(L, b0 + per);
        if (b0 < b1) th.emplace_back(work, b0, b1);
    }
    for (auto &t : th) t.join();
}

int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

namespace {
void fft_ld(std::vector<std::complex<ld>> &a) {
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        for (size_t i = 0; i < n; i += len) {
            for (size_t k = 0; k < len / 2; ++k) {
                ld ang = -2 * kPiL * (ld)k / (ld)len;
                std::complex<ld> w(std::cos(ang), std::sin(ang));
                std::complex<ld> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
        }
    }
}

std::complex<double> chirp(long x, long Nd, int sigma) {
    long q = (x * x) % (2 * Nd);
    ld a = sigma * kPiL * (ld)q / (ld)Nd;
    return {(double)std::cos(a), (double)std::sin(a)};
}
}  // namespace

Bluestein make_bluestein(int Nd, int Kin, int j0, int Kout, int k0, int sigma,
                         double scale) {
    Bluestein B;
    B.Nd = Nd;
    B.Kin = Kin;
    B.j0 = j0;
    B.Kout = Kout;
    B.k0 = k0;
    B.sigma = sigma;
    B.P = next_pow2(Kin + Kout - 1);
    if (B.P < 8) B.P = 8;
    // The register engine (P >= 256) stages a line's inputs and outputs in one
    // padded LDS line of P + P/16 reals: a window wider than half of that
    // (an SHT's 2L - 1 samples to L outputs, say) takes the next size.
    while (B.P >= 256 && 2 * std::max(Kin, Kout) > B.P + B.P / 16) B.P *= 2;
    B.pre.resize(Kin);
    B.post.resize(Kout);
    for (int t = 0; t < Kin; ++t) B.pre[t] = chirp(j0 + t, Nd, sigma);
    for (int t = 0; t < Kout; ++t) B.post[t] = chirp(k0 + t, Nd, sigma);
    // Chirp kernel at lags s - (Kin - 1) = k - j - (k0 - j0), s < Kin + Kout - 1,
    // stored circularly at its lag: output k0 + q then lands at position q.
    const long dmin = (long)k0 - j0 - (Kin - 1);
    std::vector<std::complex<ld>> v(B.P, 0);
    for (int s = 0; s < Kin + Kout - 1; ++s) {
        long x = s + dmin;
        long q = (x * x) % (2L * Nd);
        ld a = -sigma * kPiL * (ld)q / (ld)Nd;
        v[(s - (Kin - 1) + B.P) % B.P] = std::complex<ld>(std::cos(a), std::sin(a));
    }
    fft_ld(v);
    B.vhat.resize(B.P);
    for (int p = 0; p < B.P; ++p)
        B.vhat[p] = std::complex<double>((double)(v[p].real() * scale / B.P),
                                         (double)(v[p].imag() * scale / B.P));
    return B;
}

std::vector<std::complex<double>> twiddles(int P) {
    std::vector<std::complex<double>> t(P);
    for (int x = 0; x < P; ++x) {
        ld a = -2 * kPiL * (ld)x / (ld)P;
        t[x] = {(double)std::cos(a), (double)std::sin(a)};
    }
    return t;
}

}  // namespace host
}  // namespace cvl
