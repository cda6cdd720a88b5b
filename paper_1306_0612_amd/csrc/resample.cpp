// Arclength-equispaced resampling of a sampled closed curve on the sphere
// (host; lbs_resample_curve_host in include/lbs.h).
//
// Section 6, Example 2 smooths coastline samples and resamples them at
// equally spaced points in arclength, with the trapezoidal rule of
// eq. disc_sphere then running over the arclength parameter.  Steps:
//  1. project the samples from the antipode of the inside point c:
//     zeta = (x.e1 + i x.e2) / (1 + x.c), a conformal map with
//     |dx| = 2 |d zeta| / (1 + |zeta|^2);
//  2. Fourier coefficients of the trigonometric interpolant (modes
//     |k| <= K, by FFT; Bluestein's chirp transform for any sample count);
//  3. zeta, zeta', zeta'' on a fine grid of F points (zero-padded inverse
//     FFTs, F a power of two with F >= 32 max(2K + 1, n_out)); the speed and
//     its running integral s(tau) (spectral integration), L = s(2 pi);
//  4. tau_j with s(tau_j) = j L / n_out by Newton steps on ten-point
//     Lagrange interpolants of the fine tables (error ~ (2 pi K / F)^10 / 10!,
//     below 1e-16 at this F);
//  5. x, x_t, x_tt at tau_j for t = 2 pi s / L by the chain rule and the
//     inverse projection x = (2 Re zeta e1 + 2 Im zeta e2 + (1 - |zeta|^2) c)
//     / (1 + |zeta|^2).
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "lbs_internal.h"

namespace lbs {
namespace {

using cd = std::complex<double>;

// In-place radix-2 FFT (n a power of two); inv: exp(+i ...) without scaling.
void fft_pow2(std::vector<cd> &a, bool inv) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    const double ang = 2.0 * M_PI / (double)len * (inv ? 1.0 : -1.0);
    const size_t half = len >> 1;
    std::vector<cd> w(half);
    for (size_t k = 0; k < half; ++k) w[k] = cd(std::cos(ang * (double)k), std::sin(ang * (double)k));
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < half; ++k) {
        const cd u = a[i + k], v = a[i + k + half] * w[k];
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
  }
}

size_t pow2_at_least(size_t n) {
  size_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

// DFT of any length (forward, exp(-i 2 pi jk / n)) by Bluestein's chirp
// z-transform: X_k = conj(w_k) sum_j (x_j conj(w_j)) w_{k-j}, w_m =
// exp(i pi m^2 / n), as a convolution of power-of-two length.
std::vector<cd> dft(const std::vector<cd> &x) {
  const size_t n = x.size();
  if ((n & (n - 1)) == 0) {
    std::vector<cd> a = x;
    fft_pow2(a, false);
    return a;
  }
  std::vector<cd> w(n);
  for (size_t m = 0; m < n; ++m) {
    // m^2 mod 2n keeps the angle small and exact
    const unsigned long long q = ((unsigned long long)m * m) % (2ull * n);
    const double ang = M_PI * (double)q / (double)n;
    w[m] = cd(std::cos(ang), std::sin(ang));
  }
  const size_t L = pow2_at_least(2 * n - 1);
  std::vector<cd> a(L, cd(0, 0)), b(L, cd(0, 0));
  for (size_t j = 0; j < n; ++j) a[j] = x[j] * std::conj(w[j]);
  b[0] = w[0];
  for (size_t m = 1; m < n; ++m) b[m] = b[L - m] = w[m];
  fft_pow2(a, false);
  fft_pow2(b, false);
  for (size_t i = 0; i < L; ++i) a[i] *= b[i];
  fft_pow2(a, true);
  std::vector<cd> out(n);
  for (size_t k = 0; k < n; ++k) out[k] = std::conj(w[k]) * a[k] / (double)L;
  return out;
}

// Ten-point Lagrange interpolation of the periodic table f (F entries over
// [0, 2 pi)) at tau; `lin` is added per period crossed (the running
// arclength grows by L per turn).
template <typename T>
T lagrange(const std::vector<T> &f, double tau, double lin = 0.0) {
  const int64_t F = (int64_t)f.size();
  const double u = tau * (double)F / (2.0 * M_PI);
  const int64_t m0 = (int64_t)std::floor(u) - 4;
  T acc = T(0);
  for (int i = 0; i < 10; ++i) {
    double wgt = 1.0;
    for (int l = 0; l < 10; ++l)
      if (l != i) wgt *= (u - (double)(m0 + l)) / (double)(i - l);
    const int64_t m = m0 + i;
    const int64_t wrap = (m >= 0) ? m / F : -((-m + F - 1) / F);
    acc += wgt * (f[(size_t)(m - wrap * F)] + T(lin * (double)wrap));
  }
  return acc;
}

}  // namespace
}  // namespace lbs

using namespace lbs;

extern "C" lbs_status lbs_resample_curve_host(int32_t n_in, const double *x_in,
                                              const double *center, int32_t n_modes,
                                              int32_t n_out, double *x_out, double *xt_out,
                                              double *xtt_out, double *length_out) {
  try {
    if (!x_in || !center || !x_out || !xt_out || !xtt_out)
      throw ApiError{LBS_ERR_INVALID_ARG, "null pointer argument"};
    if (n_in < 8 || n_out < 8) throw ApiError{LBS_ERR_INVALID_ARG, "fewer than 8 points"};
    const int K = n_modes > 0 ? n_modes : (n_in - 1) / 2;
    if (2 * K + 1 > n_in) throw ApiError{LBS_ERR_INVALID_ARG, "n_modes must be below n_in / 2"};
    const double c[3] = {center[0], center[1], center[2]};
    const double cn = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    if (!(std::fabs(cn - 1.0) < 1e-10)) throw ApiError{LBS_ERR_GEOMETRY, "center is not a unit vector"};
    // frame: e1 = normalize(z x c) (x when c is on the z axis), e2 = e1 x c
    double e1[3] = {-c[1], c[0], 0.0};
    if (std::hypot(e1[0], e1[1]) < 1e-12) {
      e1[0] = 1.0;
      e1[1] = 0.0;
    }
    {
      const double d = e1[0] * c[0] + e1[1] * c[1] + e1[2] * c[2];
      for (int a = 0; a < 3; ++a) e1[a] -= d * c[a];
      const double nn = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
      for (int a = 0; a < 3; ++a) e1[a] /= nn;
    }
    const double e2[3] = {e1[1] * c[2] - e1[2] * c[1], e1[2] * c[0] - e1[0] * c[2],
                          e1[0] * c[1] - e1[1] * c[0]};
    std::vector<cd> z(n_in);
    for (int j = 0; j < n_in; ++j) {
      const double *x = x_in + 3 * (size_t)j;
      const double a = x[0] * e1[0] + x[1] * e1[1] + x[2] * e1[2];
      const double b = x[0] * e2[0] + x[1] * e2[1] + x[2] * e2[2];
      const double h = x[0] * c[0] + x[1] * c[1] + x[2] * c[2];
      if (!std::isfinite(a) || !std::isfinite(b) || !(1.0 + h > 1e-8))
        throw ApiError{LBS_ERR_GEOMETRY, "sample " + std::to_string(j) +
                                             " is not finite or opposite the centre"};
      z[j] = cd(a, b) / (1.0 + h);
    }
    const std::vector<cd> Z = dft(z);
    // fine tables of zeta, zeta', zeta''
    const size_t F = pow2_at_least(32 * (size_t)std::max(2 * K + 1, (int)n_out));
    std::vector<cd> f0(F, 0.0), f1(F, 0.0), f2(F, 0.0);
    for (int k = -K; k <= K; ++k) {
      const cd ck = Z[(size_t)((k + n_in) % n_in)] / (double)n_in;
      const size_t at = (size_t)((k + (int64_t)F) % (int64_t)F);
      f0[at] = ck;
      f1[at] = ck * cd(0.0, (double)k);
      f2[at] = ck * (-(double)k * (double)k);
    }
    fft_pow2(f0, true);
    fft_pow2(f1, true);
    fft_pow2(f2, true);
    std::vector<double> sp(F);
    double L = 0.0;
    for (size_t m = 0; m < F; ++m) {
      sp[m] = 2.0 * std::abs(f1[m]) / (1.0 + std::norm(f0[m]));
      L += sp[m];
    }
    L *= 2.0 * M_PI / (double)F;
    // running arclength s(tau_m) = (L / 2 pi) tau_m + sum_{k != 0} S_k (e^{ik tau} - 1) / (ik)
    std::vector<cd> S(F);
    for (size_t m = 0; m < F; ++m) S[m] = sp[m];
    fft_pow2(S, false);
    const int64_t Fi = (int64_t)F;
    for (int64_t q = 0; q < Fi; ++q) {
      const int64_t k = q <= Fi / 2 ? q : q - Fi;
      if (k == 0 || k == Fi / 2) S[(size_t)q] = 0.0;
      else S[(size_t)q] = S[(size_t)q] / ((double)F * cd(0.0, (double)k));
    }
    cd s0 = 0.0;
    for (size_t q = 0; q < F; ++q) s0 += S[q];
    fft_pow2(S, true);
    std::vector<double> sv(F);
    for (size_t m = 0; m < F; ++m)
      sv[m] = L * (double)m / (double)F + (S[m] - s0).real();
    sv[0] = 0.0;
    const double cL = L / (2.0 * M_PI);
    for (int j = 0; j < n_out; ++j) {
      const double target = L * (double)j / (double)n_out;
      // bracket on the table, then Newton on the interpolants
      const size_t ub = (size_t)(std::upper_bound(sv.begin(), sv.end(), target) - sv.begin());
      const size_t m = ub > 0 ? ub - 1 : 0;
      double tau = 2.0 * M_PI * (double)m / (double)F + (target - sv[m]) / sp[m];
      for (int it = 0; it < 4; ++it)
        tau -= (lagrange(sv, tau, L) - target) / lagrange(sp, tau);
      const cd zz = lagrange(f0, tau), z1 = lagrange(f1, tau), z2 = lagrange(f2, tau);
      const double q0 = 1.0 + std::norm(zz), a1 = std::abs(z1);
      const double spd = 2.0 * a1 / q0;
      const double dsp = 2.0 * (std::conj(z1) * z2).real() / (a1 * q0) -
                         4.0 * a1 * (std::conj(zz) * z1).real() / (q0 * q0);
      const double tt = cL / spd, ttt = -(dsp / spd) * tt * tt;
      const cd zt = z1 * tt, ztt = z2 * tt * tt + z1 * ttt;
      const double qt = 2.0 * (std::conj(zz) * zt).real();
      const double qtt = 2.0 * (std::conj(zz) * ztt).real() + 2.0 * std::norm(zt);
      const double p = q0;
      const cd w = 2.0 * zz / p;
      const cd wt = 2.0 * zt / p - 2.0 * zz * qt / (p * p);
      const cd wtt = 2.0 * ztt / p - 4.0 * zt * qt / (p * p) - 2.0 * zz * qtt / (p * p) +
                     4.0 * zz * qt * qt / (p * p * p);
      const double h = 2.0 / p - 1.0, ht = -2.0 * qt / (p * p),
                   htt = -2.0 * qtt / (p * p) + 4.0 * qt * qt / (p * p * p);
      for (int a = 0; a < 3; ++a) {
        x_out[3 * (size_t)j + a] = w.real() * e1[a] + w.imag() * e2[a] + h * c[a];
        xt_out[3 * (size_t)j + a] = wt.real() * e1[a] + wt.imag() * e2[a] + ht * c[a];
        xtt_out[3 * (size_t)j + a] = wtt.real() * e1[a] + wtt.imag() * e2[a] + htt * c[a];
      }
    }
    if (length_out) *length_out = L;
    return LBS_OK;
  } catch (const ApiError &e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_last_error("host allocation failed");
    return LBS_ERR_OUT_OF_MEMORY;
  }
}
