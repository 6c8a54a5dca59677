// Host-side (CPU, FP64 / long double) tables of the curvelet transform.
// Pure C++: no HIP types, testable without a GPU.
#pragma once
#include <complex>
#include <vector>

namespace cvl {
namespace host {

// k_lambda(t) of Sec. II-B: ratio of int_t^1 s_lambda(u)^2/u du to
// int_{1/lambda}^1 s_lambda(u)^2/u du, 1 below 1/lambda, 0 above 1.
// Composite 20-point Gauss-Legendre over 64 panels.
double k_lambda(double t, double lam);

// kappa^(j)(l) = sqrt(k(l/lambda^(j+1)) - k(l/lambda^j)) for j in [J0, J], l < L:
// out[(j - J0) * L + l].
std::vector<double> kappa_table(int L, double lam, int J0, int J);

// Phi_l0 = sqrt((2l+1)/4pi) sqrt(k(l/lambda^J0)), l < L.
std::vector<double> phi_table(int L, double lam, int J0);

// a_l(n) = sqrt(C(2l, l+n)) / 2^l = Delta^l_{n,l} = d^l_{n,l}(pi/2) for 0 <= n <= l,
// out[l * L + n] (zero for n > l).
std::vector<double> delta_col_l(int L);

// Directional component of spin-s curvelets rotated by rho* = (0, theta, 0)
// (Sec. II-B): z[l * (2L - 1) + n + L - 1] = zeta_ln for 0 <= l < L, |n| <= l,
// zeta_ln = (d^l_{n,l}(theta) + (-1)^l d^l_{n,-l}(theta)) / sqrt 2 from the
// one-term edge cases of the factorial sum of d^l (Sec. II-A):
// d^l_{n,l} = sqrt(C(2l, l+n)) sin(t/2)^(l-n) cos(t/2)^(l+n) and
// d^l_{n,-l} = (-1)^(l-n) sqrt(C(2l, l+n)) sin(t/2)^(l+n) cos(t/2)^(l-n).
std::vector<double> zeta_rotated(int L, double theta);

// MW beta nodes of band-limit L: angles pi(2b+1)/(2L-1), as exact phases.
// Inverse beta matrices (rows b, columns m' >= 0), parity-folded:
//   C[b][m'] = (m' ? 2 : 1) cos(m' beta_b),  S[b][m'] = 2 sin(m' beta_b).
void beta_inverse_mats(int L, std::vector<double> &C, std::vector<double> &S);

// Forward beta matrices (rows m' >= 0, columns b): the beta extension,
// the length-(2L-1) beta DFT and the correlation with the weights
// w(p) = int_0^pi sin(b) e^{ipb} db, composed and folded over +-m':
//   Z_m' = sum_b Q^s[m'][b] X(beta_b) with s = +-1 the beta-parity;
// Q^+ is real (returned in Qp), Q^- is purely imaginary (i * Qs returned).
// `factor` is (2pi)^2 for Wigner transforms, 2pi for the SHT.
void beta_forward_mats(int L, double factor, std::vector<double> &Qp,
                       std::vector<double> &Qs);

// Bluestein (chirp-z) tables for
//   out[k] = scale * sum_{j=j0}^{j0+Kin-1} in[j] exp(sigma 2 pi i j k / Nd),
//   k in [k0, k0 + Kout),
// evaluated as a circular convolution of length P (power of two >= Kin+Kout-1)
// whose position q holds output k0 + q.
struct Bluestein {
    int Nd = 0, P = 0, Kin = 0, j0 = 0, Kout = 0, k0 = 0, sigma = 0;
    std::vector<std::complex<double>> pre;   // Kin:  exp(sigma i pi (j0+t)^2 / Nd)
    std::vector<std::complex<double>> post;  // Kout: exp(sigma i pi (k0+t)^2 / Nd)
    std::vector<std::complex<double>> vhat;  // P:    FFT_P(v) * scale / P
};
Bluestein make_bluestein(int Nd, int Kin, int j0, int Kout, int k0, int sigma,
                         double scale);

// tw[x] = exp(-2 pi i x / P), x < P.
std::vector<std::complex<double>> twiddles(int P);

int next_pow2(int x);

}  // namespace host
}  // namespace cvl
