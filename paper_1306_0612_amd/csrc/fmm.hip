// 2D Coulomb FMM for the Cauchy part of the double-layer operator.
//
// The operator of Section 5 (eq. disc_sphere) splits, for target node i, as
//   (K sigma)_i = Re sum_{j != i} p_j / (xi_i - xi_j) + tau_i sigma_i + gamma
// with complex strengths p_j = -i q_j, q_j = (s h / pi) xi'_j sigma_j.
// The sum is the planar Coulomb/Cauchy potential that the paper evaluates
// with the 2D FMM (Section 5).  Expansions are stored scaled by the box
// half-width r so that same-level translations are level independent:
//   multipole  Psi(z) = sum_{k=1..P} a_k (r / (z - c))^k,
//              a_k = (1/r) sum_j p_j ((z_j - c)/r)^(k-1)
//   local      Psi(z) = sum_{l=0..P-1} b_l ((z - c)/r)^l
// Translations (binomial series of 1/(z - z_j)):
//   M2M  child c1 (half-width r/2) -> parent c0: d = c1 - c0 = (r/2) delta,
//        A_l = sum_{k<=l} a_k C(l-1,k-1) delta^(l-k) 2^-l
//   M2L  same-level, c_s - c_t = r tau, tau = 2 (dx + i dy):
//        b_l = tau^-l sum_k (-1)^k C(k+l-1,l) tau^-k a_k
//   L2L  parent c0 -> child c1 = c0 + (r/2) delta:
//        b'_m = sum_{l>=m} b_l C(l,m) delta^(l-m) 2^-l
//   P2L  b_l = -sum_j (p_j/u_j) (r/u_j)^l, u_j = z_j - c
//   M2P  Psi(z) = sum_k a_k (r_w/(z - c_w))^k
#include <cmath>
#include <type_traits>
#include <vector>

#include "cplx.h"
#include "lbs_internal.h"

namespace lbs {

// ----------------------------------------------------------------- tables
static double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
  return std::round(r);
}

static void cpow_host(double x, double y, int n, double &ox, double &oy) {
  double rx = 1, ry = 0;
  for (int i = 0; i < n; ++i) {
    double t = rx * x - ry * y;
    ry = rx * y + ry * x;
    rx = t;
  }
  ox = rx;
  oy = ry;
}

void build_tables(Tables &t, int P, hipStream_t s) {
  t.P = P;
  // M2M and L2L factorized as scale x Pascal x scale (quadrant offset
  // delta = (+-1, +-1), |delta|^2 = 2):
  //   M2M: A_lo = 1/2 (delta/2)^lo sum_{k <= lo} C(lo, k) (conj(delta)/2)^k a_k
  //   L2L: b'_m = (conj(delta)/2)^m sum_{l >= m} C(l, m) (delta/2)^l b_l
  // Tables: C (P x P, zero above the diagonal), pre[q][n] =
  // (conj(delta_q)/2)^n and post[q][n] = (delta_q/2)^n.
  std::vector<double> bc(P * P, 0.0), pre(4 * P * 2), post(4 * P * 2);
  for (int n = 0; n < P; ++n)
    for (int k = 0; k <= n; ++k) bc[n * P + k] = binom(n, k);
  for (int q = 0; q < 4; ++q) {
    const double dx = (q & 1) ? 1.0 : -1.0, dy = (q & 2) ? 1.0 : -1.0;
    for (int n = 0; n < P; ++n) {
      double ax, ay, bx, by;
      cpow_host(0.5 * dx, -0.5 * dy, n, ax, ay);
      cpow_host(0.5 * dx, 0.5 * dy, n, bx, by);
      pre[2 * (q * P + n)] = ax;
      pre[2 * (q * P + n) + 1] = ay;
      post[2 * (q * P + n)] = bx;
      post[2 * (q * P + n) + 1] = by;
    }
  }
  std::vector<double> h(P * P);
  for (int l = 0; l < P; ++l)
    for (int ki = 0; ki < P; ++ki) {
      int k = ki + 1;
      h[l * P + ki] = ((k & 1) ? -1.0 : 1.0) * binom(k + l - 1, l);
    }
  const int NP = 2 * P + 1;
  std::vector<double> itp(49 * NP * 2, 0.0);
  for (int code = 0; code < 49; ++code) {
    int dx = code / 7 - 3, dy = code % 7 - 3;
    if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
    double tx = 2.0 * dx, ty = 2.0 * dy, d = tx * tx + ty * ty;
    double ix = tx / d, iy = -ty / d;  // 1 / tau
    for (int n = 0; n < NP; ++n) {
      double px, py;
      cpow_host(ix, iy, n, px, py);
      itp[(code * NP + n) * 2] = px;
      itp[(code * NP + n) * 2 + 1] = py;
    }
  }
  auto to32 = [](const std::vector<double> &v) {
    return std::vector<float>(v.begin(), v.end());
  };
  t.bc64.upload(bc, s);
  t.pre64.upload(pre, s);
  t.post64.upload(post, s);
  t.h64.upload(h, s);
  t.itp64.upload(itp, s);
  t.bc32.upload(to32(bc), s);
  t.pre32.upload(to32(pre), s);
  t.post32.upload(to32(post), s);
  t.h32.upload(to32(h), s);
  t.itp32.upload(to32(itp), s);
  LBS_HIP(hipStreamSynchronize(s));
}

// ----------------------------------------------------------------- kernels
// v[0 .. NV) summed over the 64 lanes of a wave by recursive halving: at
// step s (partner lane ^ (32 >> s)) a lane keeps the upper half of its
// values when that lane bit is set, else the lower half, and adds its
// partner's copy of the half it keeps; once a single value is left the
// remaining steps add it whole.  Lane i returns the total of value
// i >> (6 - log2 NV); NV - 1 + 6 - log2 NV shuffles in all.
// One halving step at lane offset 32 or 16 for the pair (a, b): the
// permlane swaps exchange the upper 32 lanes of a with the lower 32 of b
// (the odd 16-lane rows of a with the even rows of b), after which a + b is,
// in every lane, its own plus its partner's copy of the value it keeps.
template <int O>
__device__ __forceinline__ float swap_add(float a, float b) {
  static_assert(O == 32 || O == 16, "lane offsets with a swap instruction");
  const auto r = O == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false)
                         : __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

template <typename T, int NV, bool SWAP, int S = 0>
__device__ __forceinline__ void halving_steps(T (&v)[NV], int lane) {
  if constexpr (S < 6) {
    constexpr int o = 32 >> S, h = NV >> (S + 1);
    if constexpr (SWAP && h >= 1 && sizeof(T) == 4 && o >= 16) {
#pragma unroll
      for (int k = 0; k < h; ++k) v[k] = swap_add<o>(v[k], v[k + h]);
    } else if constexpr (h >= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int k = 0; k < h; ++k) {
        const T send = up ? v[k] : v[k + h];
        const T keep = up ? v[k + h] : v[k];
        v[k] = keep + __shfl_xor(send, o, 64);
      }
    } else {
      v[0] += __shfl_xor(v[0], o, 64);
    }
    halving_steps<T, NV, SWAP, S + 1>(v, lane);
  }
}

// SWAP: the steps at lane offsets 32 and 16 of FP32 values by permlane
// swaps (swap_add) instead of selects and a cross-lane read.
template <typename T, int NV, bool SWAP = true>
__device__ __forceinline__ T halving_sum(T (&v)[NV], int lane) {
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0,
                "a power of two up to the wave size");
  halving_steps<T, NV, SWAP>(v, lane);
  return v[0];
}

constexpr int pow2_ceil(int n) { return n <= 1 ? 1 : 2 * pow2_ceil((n + 1) / 2); }
constexpr int log2_exact(int n) { return n <= 1 ? 0 : 1 + log2_exact(n / 2); }

// Coefficients per register pass of the P2M and P2L sums: 2 KB real
// accumulators per lane (KB of 16 FP64 or 32 FP32 terms keeps them within
// 64 registers); an order above KB takes several passes over the sources.
template <typename T, int P>
constexpr int kChunk() {
  return P < (sizeof(T) == 8 ? 16 : 32) ? P : (sizeof(T) == 8 ? 16 : 32);
}

// P2L sum of one box (centre (cxb, cyb), half-width rb) over the sources
// of its X list, xf_idx[x0 .. x0 + total) (concatenated at set-up), for
// coefficients K0 .. K0 + KB - 1: lane q accumulates t_q (r/u_q)^l,
// t_q = -p_q / u_q, u_q = z_q - c, for sources q, q + 64, ... in registers
// (parts of coefficient K0 + l as values 2l, 2l + 1); one halving sum.
// Lane i returns the total of value i >> (6 - log2 NV), NV = pow2 >= 2 KB.
template <typename T, int P, int K0, int KB>
__device__ __forceinline__ T p2l_sum(int64_t x0, int total,
                                     const int32_t *__restrict__ xf_idx,
                                     double cxb, double cyb, T rb,
                                     const double *__restrict__ sx,
                                     const double *__restrict__ sy,
                                     const cx<T> *__restrict__ pr, int lane) {
  constexpr int NV = pow2_ceil(2 * KB);
  T acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = T(0);
  for (int q = lane; q < total; q += 64) {
    const int64_t j = xf_idx[x0 + q];
    const cx<T> u{T(sx[j] - cxb), T(sy[j] - cyb)};
    cx<T> iu;
    if constexpr (sizeof(T) == 4) {  // FP32 expansions: hardware reciprocal
      const float d = __builtin_amdgcn_rcpf(u.x * u.x + u.y * u.y);
      iu = cx<T>{u.x * d, -u.y * d};
    } else {
      iu = cinv(u);
    }
    const cx<T> rho = rb * iu;
    cx<T> t = pr[j] * iu;
    t = cx<T>{-t.x, -t.y};
    if (K0 > 0) t = t * cpow(rho, K0);
#pragma unroll
    for (int l = 0; l < KB; ++l) {
      if (K0 + l < P) {
        acc[2 * l] += t.x;
        acc[2 * l + 1] += t.y;
        t = t * rho;
      }
    }
  }
  return halving_sum<T, NV>(acc, lane);
}

// Where the leaf multipole pass finds its strengths: with sigma set it
// forms p_j = -i q_j sigma_j itself (q-factor qfac_t in tree order, sigma in
// API order through perm, stride ldx per right-hand side) and stores them
// for the near field and P2L; otherwise it reads p as given.
struct StrengthSrc {
  const int64_t *perm = nullptr;
  const double *qfac_t = nullptr;
  const double *sigma = nullptr;
  int64_t ldx = 0;
  // with gpart set: gpart[r * (#leaves) + leaf] = sum over the leaf's
  // sources of gw_t[j] sigma_j (FP64), for GammaFused
  const double *gw_t = nullptr;
  double *gpart = nullptr;
  // optional, for the FP32 leaf multipoles: -i q_j as (Im q_j, -Re q_j)
  // rounded to FP32 and the permutation as 32-bit indices (half the bytes
  // of qfac_t and perm)
  const float2 *qm32 = nullptr;
  const int32_t *perm32 = nullptr;
};

// Leaf multipoles, one wave per leaf (every source lies in one leaf): lane
// j accumulates p_j w_j^k of sources j, j + 64, ... in registers, KB
// coefficients per pass (real and imaginary parts as values 2k, 2k + 1 of
// NV = pow2 >= 2 KB), and one halving sum per pass leaves the parts of
// coefficient k in lanes (2k + c) << SH.  The first pass forms the
// strengths (when asked to); later passes read them back.
template <typename T, int P>
__global__ void __launch_bounds__(64)
    k_p2m(const int32_t *__restrict__ leaves,
          const int64_t *__restrict__ ls_rng,
          const double4 *__restrict__ ls_geo,
          const double *__restrict__ sx, const double *__restrict__ sy,
          cx<T> *__restrict__ p, int64_t ns, cx<T> *__restrict__ M,
          int nbox, StrengthSrc ss) {
  constexpr int KB = kChunk<T, P>(), NV = pow2_ceil(2 * KB),
                SH = 6 - log2_exact(NV);
  // the leaf's source range and frame by work-group (one load level less
  // than through its box id, which only the final store needs)
  const int b = leaves[blockIdx.x];
  const int r = blockIdx.y;
  const int lane = threadIdx.x;
  const double4 geo = ls_geo[blockIdx.x];
  const double c_x = geo.x, c_y = geo.y, ir = geo.z;
  cx<T> *pr = p + (int64_t)r * ns;
  double gsum = 0.0;
  const int64_t e0 = ls_rng[2 * blockIdx.x], e1 = ls_rng[2 * blockIdx.x + 1];
  if (e1 == e0 && !ss.gpart) return;  // an empty range: the whole wave, M left as it is
  const int vi = lane >> SH;
  const bool writer = (lane & ((1 << SH) - 1)) == 0;
#pragma unroll
  for (int k0 = 0; k0 < P; k0 += KB) {
    T acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = T(0);
    for (int64_t j = e0 + lane; j < e1; j += 64) {
      const cx<T> w{T((sx[j] - c_x) * ir), T((sy[j] - c_y) * ir)};
      cx<T> pw;
      if (k0 == 0 && ss.sigma) {  // form the strength: p_j = -i q_j sigma_j
        const double sg = ss.sigma[(int64_t)r * ss.ldx + ss.perm[j]];
        const double qx = ss.qfac_t[2 * j], qy = ss.qfac_t[2 * j + 1];
        pw = cx<T>{T(qy * sg), T(-qx * sg)};
        pr[j] = pw;
        if (ss.gpart) gsum += ss.gw_t[j] * sg;
      } else {
        pw = pr[j];
      }
      if (k0 > 0) pw = pw * cpow(w, k0);
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (k0 + k < P) {
          acc[2 * k] += pw.x;
          acc[2 * k + 1] += pw.y;
          pw = pw * w;
        }
      }
    }
    const T tot = halving_sum<T, NV, false>(acc, lane);
    T *Mb = reinterpret_cast<T *>(M + ((int64_t)r * nbox + b) * P);
    if (writer && vi < 2 * KB && 2 * k0 + vi < 2 * P) Mb[2 * k0 + vi] = T(ir) * tot;
  }
  if (ss.gpart) {  // block-uniform
    for (int o = 32; o > 0; o >>= 1) gsum += __shfl_xor(gsum, o, 64);
    if (lane == 0) ss.gpart[(int64_t)r * gridDim.x + blockIdx.x] = gsum;
  }
}

// The FP32 leaf multipoles of two leaves per wave (list entries 2 w and
// 2 w + 1 on lanes 0-31 and 32-63): as k_p2m, with every source loop
// striding by 32 and the halving sum run inside each half (lane offsets
// 16 .. 1), so that the sum's fixed cost is shared by two leaves.  One
// pass: P <= 32 coefficients, NV = 2 P values.
template <typename T, int NV, int S = 0>
__device__ __forceinline__ void halving_steps_half(T (&v)[NV], int lane) {
  if constexpr (S < 5) {
    constexpr int o = 16 >> S, h = NV >> (S + 1);
    if constexpr (h >= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int k = 0; k < h; ++k) {
        const T send = up ? v[k] : v[k + h];
        const T keep = up ? v[k + h] : v[k];
        v[k] = keep + __shfl_xor(send, o, 64);
      }
    } else {
      v[0] += __shfl_xor(v[0], o, 64);
    }
    halving_steps_half<T, NV, S + 1>(v, lane);
  }
}

template <int P>
__global__ void __launch_bounds__(64)
    k_p2m_pair(const int32_t *__restrict__ leaves, int nleaf,
               const int64_t *__restrict__ ls_rng,
               const double4 *__restrict__ ls_geo,
               const double *__restrict__ sx, const double *__restrict__ sy,
               const float2 *__restrict__ w32,
               cx<float> *__restrict__ p, int64_t ns, cx<float> *__restrict__ M,
               int nbox, StrengthSrc ss) {
  constexpr int NV = pow2_ceil(2 * P), SH = 5 - log2_exact(NV);
  static_assert(P <= 16, "one pass of at most 32 values per lane");
  const int lane = threadIdx.x, half = lane >> 5, hl = lane & 31;
  const int e = 2 * blockIdx.x + half;  // this half's list entry
  const bool has = e < nleaf;           // uniform within the half
  const int r = blockIdx.y;
  cx<float> *pr = p + (int64_t)r * ns;
  float acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.f;
  double gsum = 0.0;
  int b = 0;
  double ir = 0.0;
  if (has) {
    b = leaves[e];
    const double4 geo = ls_geo[e];
    const double c_x = geo.x, c_y = geo.y;
    ir = geo.z;
    const int64_t e0 = ls_rng[2 * e], e1 = ls_rng[2 * e + 1];
    if (w32 && ss.sigma && ss.qm32) {  // uniform
      // sources j and j + 32 of this lane per step, every load issued
      // before the dependent gathers of sigma, the terms added in source
      // order as below
      const double *sgr = ss.sigma + (int64_t)r * ss.ldx;
      for (int64_t j = e0 + hl; j < e1; j += 64) {
        const bool two = j + 32 < e1;
        const int64_t jb = two ? j + 32 : j;
        const int ia = ss.perm32[j], ib = ss.perm32[jb];
        const float2 wa = w32[j], wb = w32[jb];
        const float2 qa = ss.qm32[j], qb = ss.qm32[jb];
        double ga = 0.0, gb = 0.0;
        if (ss.gpart) {
          ga = ss.gw_t[j];
          gb = ss.gw_t[jb];
        }
        const double sa = sgr[ia], sb = sgr[ib];
        cx<float> pa{float((double)qa.x * sa), float((double)qa.y * sa)};
        cx<float> pb{float((double)qb.x * sb), float((double)qb.y * sb)};
        pr[j] = pa;
        if (ss.gpart) gsum += ga * sa;
        if (two) {
          pr[jb] = pb;
          if (ss.gpart) gsum += gb * sb;
        } else {
          pb = cx<float>{0.f, 0.f};
        }
        const cx<float> wca{wa.x, wa.y}, wcb{wb.x, wb.y};
#pragma unroll
        for (int k = 0; k < P; ++k) {
          acc[2 * k] += pa.x;
          acc[2 * k + 1] += pa.y;
          pa = pa * wca;
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
          acc[2 * k] += pb.x;
          acc[2 * k + 1] += pb.y;
          pb = pb * wcb;
        }
      }
    } else
    for (int64_t j = e0 + hl; j < e1; j += 32) {
      cx<float> w;
      if (w32) {  // uniform: the leaf-relative positions of set-up
        const float2 t = w32[j];
        w = cx<float>{t.x, t.y};
      } else {
        w = cx<float>{float((sx[j] - c_x) * ir), float((sy[j] - c_y) * ir)};
      }
      cx<float> pw;
      if (ss.sigma) {  // form the strength: p_j = -i q_j sigma_j
        if (ss.qm32) {  // uniform
          const double sg = ss.sigma[(int64_t)r * ss.ldx + ss.perm32[j]];
          const float2 q = ss.qm32[j];
          pw = cx<float>{float((double)q.x * sg), float((double)q.y * sg)};
          if (ss.gpart) gsum += ss.gw_t[j] * sg;
        } else {
          const double sg = ss.sigma[(int64_t)r * ss.ldx + ss.perm[j]];
          const double qx = ss.qfac_t[2 * j], qy = ss.qfac_t[2 * j + 1];
          pw = cx<float>{float(qy * sg), float(-qx * sg)};
          if (ss.gpart) gsum += ss.gw_t[j] * sg;
        }
        pr[j] = pw;
      } else {
        pw = pr[j];
      }
#pragma unroll
      for (int k = 0; k < P; ++k) {
        acc[2 * k] += pw.x;
        acc[2 * k + 1] += pw.y;
        pw = pw * w;
      }
    }
  }
  halving_steps_half<float, NV>(acc, lane);
  const int vi = hl >> SH;
  if (has && (hl & ((1 << SH) - 1)) == 0 && vi < 2 * P) {
    float *Mb = reinterpret_cast<float *>(M + ((int64_t)r * nbox + b) * P);
    Mb[vi] = float(ir) * acc[0];
  }
  if (ss.gpart) {  // block-uniform
    for (int o = 16; o > 0; o >>= 1) gsum += __shfl_xor(gsum, o, 64);
    if (has && hl == 0) ss.gpart[(int64_t)r * nleaf + e] = gsum;
  }
}

// The FP64 leaf multipoles of two leaves per wave (list entries 2 w and
// 2 w + 1 on lanes 0-31 and 32-63): as k_p2m, KB coefficients per pass
// over the sources (the first pass forms the strengths, later passes read
// them back), every source loop striding by 32 and one halving sum per
// pass inside each half, so that the sums' fixed cost is shared by two
// leaves.
template <int P>
__global__ void __launch_bounds__(64)
    k_p2m_pair64(const int32_t *__restrict__ leaves, int nleaf,
                 const int64_t *__restrict__ ls_rng,
                 const double4 *__restrict__ ls_geo,
                 const double *__restrict__ sx, const double *__restrict__ sy,
                 cx<double> *__restrict__ p, int64_t ns, cx<double> *__restrict__ M,
                 int nbox, StrengthSrc ss) {
  constexpr int KB = kChunk<double, P>(), NV = pow2_ceil(2 * KB), SH = 5 - log2_exact(NV);
  static_assert(NV <= 32, "at most one value per lane of a half after the halving sum");
  const int lane = threadIdx.x, half = lane >> 5, hl = lane & 31;
  const int e = 2 * blockIdx.x + half;  // this half's list entry
  const bool has = e < nleaf;           // uniform within the half
  const int r = blockIdx.y;
  cx<double> *pr = p + (int64_t)r * ns;
  double gsum = 0.0, c_x = 0.0, c_y = 0.0, ir = 0.0;
  int b = 0;
  int64_t e0 = 0, e1 = 0;
  if (has) {
    b = leaves[e];
    const double4 geo = ls_geo[e];
    c_x = geo.x;
    c_y = geo.y;
    ir = geo.z;
    e0 = ls_rng[2 * e];
    e1 = ls_rng[2 * e + 1];
  }
  const int vi = hl >> SH;
  const bool writer = has && (hl & ((1 << SH) - 1)) == 0;
#pragma unroll
  for (int k0 = 0; k0 < P; k0 += KB) {
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int64_t j = e0 + hl; j < e1; j += 32) {
      const cx<double> w{(sx[j] - c_x) * ir, (sy[j] - c_y) * ir};
      cx<double> pw;
      if (k0 == 0 && ss.sigma) {  // form the strength: p_j = -i q_j sigma_j
        const double sg = ss.sigma[(int64_t)r * ss.ldx + ss.perm[j]];
        const double qx = ss.qfac_t[2 * j], qy = ss.qfac_t[2 * j + 1];
        pw = cx<double>{qy * sg, -qx * sg};
        pr[j] = pw;
        if (ss.gpart) gsum += ss.gw_t[j] * sg;
      } else {
        pw = pr[j];
      }
      if (k0 > 0) pw = pw * cpow(w, k0);
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (k0 + k < P) {
          acc[2 * k] += pw.x;
          acc[2 * k + 1] += pw.y;
          pw = pw * w;
        }
      }
    }
    halving_steps_half<double, NV>(acc, lane);
    if (writer && vi < 2 * KB && 2 * k0 + vi < 2 * P) {
      double *Mb = reinterpret_cast<double *>(M + ((int64_t)r * nbox + b) * P);
      Mb[2 * k0 + vi] = ir * acc[0];
    }
  }
  if (ss.gpart) {  // block-uniform
    for (int o = 16; o > 0; o >>= 1) gsum += __shfl_xor(gsum, o, 64);
    if (has && hl == 0) ss.gpart[(int64_t)r * nleaf + e] = gsum;
  }
}

// gamma[r G + g] = the sum of the partial sums of geometry g's source
// leaves, positions gl_ptr[g] .. gl_ptr[g + 1] of the plan's leaf list.
// Block (c, g, r) sums chunk c of that range into csum; the last block of
// (g, r) to finish (a device-scope counter) adds the chunk sums in index
// order and resets the counter for the next application, so the result
// does not depend on the order in which blocks run.
constexpr int kGammaChunk = 2048;
__device__ __forceinline__ void gamma_chunk(int c, int g, int r, int nch,
                                            const int32_t *__restrict__ gl_ptr,
                                            const double *__restrict__ gpart,
                                            int nls, int G,
                                            double *__restrict__ csum,
                                            int32_t *__restrict__ cnt,
                                            double *__restrict__ gamma) {
  __shared__ double red[4];
  __shared__ bool last;
  const int tid = threadIdx.x, slot = r * G + g;
  const int a = gl_ptr[g] + c * kGammaChunk, b = min(gl_ptr[g + 1], a + kGammaChunk);
  double v = 0.0;
  for (int e = a + tid; e < b; e += 256) v += gpart[(int64_t)r * nls + e];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    csum[(int64_t)slot * nch + c] = red[0] + red[1] + red[2] + red[3];
    __threadfence();
    last = atomicAdd(&cnt[slot], 1) == nch - 1;
  }
  __syncthreads();
  if (last && tid == 0) {
    __threadfence();
    double t = 0.0;
    for (int k = 0; k < nch; ++k)
      t += __hip_atomic_load(&csum[(int64_t)slot * nch + k], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    gamma[slot] = t;
    cnt[slot] = 0;
  }
}

__global__ void __launch_bounds__(256)
    k_gamma_reduce(const int32_t *__restrict__ gl_ptr,
                   const double *__restrict__ gpart, int nls, int G,
                   double *__restrict__ csum, int32_t *__restrict__ cnt,
                   double *__restrict__ gamma) {
  gamma_chunk(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, gl_ptr, gpart,
              nls, G, csum, cnt, gamma);
}

// The correction sums of GammaFused for a kernel that takes them as extra
// work-groups: group x >= first (x - first = g nchunk + c) reduces chunk c
// of geometry g for right-hand side blockIdx.y.
struct GammaGroups {
  const int32_t *gl_ptr = nullptr;
  const double *gpart = nullptr;
  double *csum = nullptr;
  int32_t *cnt = nullptr;
  double *gamma = nullptr;
  int nls = 0, G = 0, nchunk = 0, first = 0;
};

// ------------------------------------------------ upward / downward passes
template <typename T>
struct Chunk16;
template <>
struct Chunk16<float> {
  using type = float4;
};
template <>
struct Chunk16<double> {
  using type = double2;
};

// v (coefficients k, k + 1 in FP32; k in FP64) times tab[k], tab[k + 1]
template <typename T>
__device__ __forceinline__ void scale_chunk(typename Chunk16<T>::type &v, const cx<T> *tab,
                                            int k) {
  if constexpr (sizeof(T) == 4) {
    const cx<T> a = cx<T>{v.x, v.y} * tab[k], b = cx<T>{v.z, v.w} * tab[k + 1];
    v = make_float4(a.x, a.y, b.x, b.y);
  } else {
    const cx<T> a = cx<T>{v.x, v.y} * tab[k];
    v = make_double2(a.x, a.y);
  }
}

// One component of a pass program per work-group (PassProgram in tree.h),
// for right-hand side blockIdx.y.  Its inputs are staged in LDS with every
// load in flight at once, scaled as the program says; then its work boxes
// are finished level by level from LDS only, each also written to E:
//   upward    A_lo = 1/2 sum_q post[q][lo] sum_{k <= lo} C(lo, k) a~_{q,k},
//             a~ a child's multipole times pre[q_child]; the result is kept
//             times pre[q_box] for the box's parent
//   downward  b_m = own_m + pre[q][m] sum_{l >= m} C(l, m) c_l, c the
//             parent's local times post[q]; the result is passed on times
//             post[q_child] to each child of the component
// (C is zero off its triangle, so the fixed-length sums add exact zeros).
// Upward, an absent child reads a slot of zeros (slot CAP), so that the
// four quadrant sums run side by side without branches.
constexpr int kPassThreads = 1024;
template <typename T, int P, bool DOWN>
__global__ void __launch_bounds__(kPassThreads)
    k_pass(const int32_t *__restrict__ hdr, const int2 *__restrict__ ext,
           const int4 *__restrict__ par, const int32_t *__restrict__ stp,
           const T *__restrict__ Cb, const cx<T> *__restrict__ Pre,
           const cx<T> *__restrict__ Post, cx<T> *__restrict__ E, int nbox) {
  using V = typename Chunk16<T>::type;
  constexpr int NT = kPassThreads, CAP = pass_cap(P, (int)sizeof(cx<T>));
  static_assert(P * (int)sizeof(cx<T>) % 16 == 0, "expansions of whole 16-byte chunks");
  constexpr int CH = P * (int)sizeof(cx<T>) / 16, IT = (CAP * CH + NT - 1) / NT;
  constexpr int CPC = 16 / (int)sizeof(cx<T>);  // coefficients per chunk
  __shared__ __align__(16) cx<T> sl[(CAP + 1) * P];  // expansion slots + zeros
  __shared__ int4 spd[CAP];                          // work boxes in step order
  __shared__ int32_t sst[kPassMaxSteps + 1];
  __shared__ T sC[P * P];  // upward C(lo, k) at k P + lo; downward C(l, m) at l P + m
  __shared__ cx<T> sPre[4 * P], sPost[4 * P];
  const int tid = threadIdx.x;
  const int32_t *h = hdr + 8 * (int64_t)blockIdx.x;
  const int ne = h[1], p0 = h[2], np = h[3], s0 = h[4], ns = h[5];
  cx<T> *Er = E + (int64_t)blockIdx.y * nbox * P;
  int2 d[IT];
  V v[IT];
  // ext: this component's CAP input slots (box -1 past #ext), read
  // without waiting for the header
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT;
    d[i] = e < CAP * CH ? ext[(int64_t)blockIdx.x * CAP + e / CH] : make_int2(-1, 0);
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT;
    if (d[i].x >= 0) v[i] = reinterpret_cast<const V *>(Er + (int64_t)d[i].x * P)[e % CH];
  }
  for (int i = tid; i < np; i += NT) spd[i] = par[p0 + i];
  for (int i = tid; i <= ns; i += NT) sst[i] = stp[s0 + i];
  for (int i = tid; i < P * P; i += NT) sC[i] = DOWN ? Cb[i] : Cb[(i % P) * P + i / P];
  for (int i = tid; i < 4 * P; i += NT) {
    sPre[i] = Pre[i];
    sPost[i] = Post[i];
  }
  if (tid < P) sl[CAP * P + tid] = cx<T>{T(0), T(0)};
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT;
    if (e < ne * CH) {  // slot e / CH, chunk e % CH
      const int mode = d[i].y & 3, q = d[i].y >> 2, k = (e % CH) * CPC;
      if (mode == 1) scale_chunk<T>(v[i], sPre + q * P, k);
      else if (mode == 2) scale_chunk<T>(v[i], sPost + q * P, k);
      reinterpret_cast<V *>(sl)[e] = v[i];
    }
  }
  __syncthreads();
  for (int st = 0; st < ns; ++st) {
    const int a = sst[st], b = sst[st + 1];
    if constexpr (!DOWN) {
      if ((b - a) * P * 4 <= NT) {  // uniform
        // a step of few boxes: four lanes per (box, coefficient), one child
        // quadrant each, so that the chain per lane is short; the quadrant
        // sums meet by two cross-lane steps (it & 3 = tid & 3: NT is a
        // multiple of 4, and the four lanes of a group are active together)
        for (int it = tid; it < (b - a) * P * 4; it += NT) {
          const int qq = it & 3, jm = it >> 2;
          const int j = a + jm / P, m = jm % P;
          const int4 pd = spd[j];
          const int box = pd.x & 0x3FFFFFFF, q = (int)((uint32_t)pd.x >> 30);
          const int w = qq < 2 ? pd.z : pd.w;
          const int sq = (qq & 1) ? (int)((uint32_t)w >> 16) : (w & 0xFFFF);
          const cx<T> *ak = sl + (sq == kPassNone ? CAP : sq) * P;
          cx<T> sum{T(0), T(0)};
#pragma unroll
          for (int k = 0; k < P; ++k) sum = sum + sC[k * P + m] * ak[k];
          cx<T> acc = sPost[qq * P + m] * sum;
          acc.x += __shfl_xor(acc.x, 1, 64);
          acc.y += __shfl_xor(acc.y, 1, 64);
          acc.x += __shfl_xor(acc.x, 2, 64);
          acc.y += __shfl_xor(acc.y, 2, 64);
          if (qq == 0) {
            const cx<T> A = T(0.5) * acc;
            Er[(int64_t)box * P + m] = A;
            sl[(ne + j) * P + m] = A * sPre[q * P + m];
          }
        }
      } else {
        // one lane per (box, coefficient), the four quadrant sums side by side
        for (int it = tid; it < (b - a) * P; it += NT) {
          const int j = a + it / P, m = it % P;
          const int4 pd = spd[j];
          const int box = pd.x & 0x3FFFFFFF, q = (int)((uint32_t)pd.x >> 30);
          const int s4[4] = {pd.z & 0xFFFF, (int)((uint32_t)pd.z >> 16), pd.w & 0xFFFF,
                             (int)((uint32_t)pd.w >> 16)};
          cx<T> sum[4];
          const cx<T> *ak[4];
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            ak[qq] = sl + (s4[qq] == kPassNone ? CAP : s4[qq]) * P;
            sum[qq] = cx<T>{T(0), T(0)};
          }
#pragma unroll
          for (int k = 0; k < P; ++k) {
            const T c = sC[k * P + m];
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) sum[qq] = sum[qq] + c * ak[qq][k];
          }
          // the quadrant terms added as the four-lane form adds them
          const cx<T> t0 = sPost[m] * sum[0], t1 = sPost[P + m] * sum[1];
          const cx<T> t2 = sPost[2 * P + m] * sum[2], t3 = sPost[3 * P + m] * sum[3];
          const cx<T> A = T(0.5) * ((t0 + t1) + (t2 + t3));
          Er[(int64_t)box * P + m] = A;
          sl[(ne + j) * P + m] = A * sPre[q * P + m];
        }
      }
    } else {
      for (int it = tid; it < (b - a) * P; it += NT) {
        const int j = a + it / P, m = it % P;
        const int4 pd = spd[j];
        const int box = pd.x & 0x3FFFFFFF, q = (int)((uint32_t)pd.x >> 30);
        const int s4[4] = {pd.z & 0xFFFF, (int)((uint32_t)pd.z >> 16), pd.w & 0xFFFF,
                           (int)((uint32_t)pd.w >> 16)};
        const int own = pd.y & 0xFFFF, ver = (int)((uint32_t)pd.y >> 16);
        cx<T> val = sl[own * P + m];
        if (ver != kPassNone) {
          const cx<T> *cl = sl + ver * P;
          cx<T> s2[2] = {cx<T>{T(0), T(0)}, cx<T>{T(0), T(0)}};
#pragma unroll
          for (int l = 0; l < P; ++l) s2[l & 1] = s2[l & 1] + sC[l * P + m] * cl[l];
          val = val + sPre[q * P + m] * (s2[0] + s2[1]);
        }
        Er[(int64_t)box * P + m] = val;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          if (s4[qq] != kPassNone) sl[s4[qq] * P + m] = sPost[qq * P + m] * val;
      }
    }
    __syncthreads();
  }
}

// The rounds of a pass program, one launch each.
template <typename T, int P, bool DOWN>
static void run_pass(const DevPass &pg, const T *bc, const cx<T> *pre, const cx<T> *post,
                     cx<T> *E, int nbox, int nrhs, hipStream_t s) {
  if (pg.cap != pass_cap(P, (int)sizeof(cx<T>)))
    throw ApiError{LBS_ERR_UNSUPPORTED, "pass program built for another expansion order"};
  for (size_t k = 0; k + 1 < pg.round_ptr.size(); ++k) {
    const int a = pg.round_ptr[k], n = pg.round_ptr[k + 1] - a;
    if (n <= 0) continue;
    hipLaunchKernelGGL((k_pass<T, P, DOWN>), dim3(n, nrhs), dim3(kPassThreads), 0, s,
                       pg.hdr.p + 8 * (int64_t)a,
                       reinterpret_cast<const int2 *>(pg.ext.p) + (int64_t)a * pg.cap,
                       reinterpret_cast<const int4 *>(pg.par.p), pg.stp.p, bc, pre, post, E,
                       nbox);
  }
}

template <int P>
struct Groups {
  static constexpr int G = 64 / P;
};

// P2L parts of one box's local expansion into px (values 2k, 2k + 1 of
// coefficient k), KB coefficients per pass (p2l_sum).
template <typename T, int P, int K0>
__device__ __forceinline__ void p2l_pass_lds(int64_t xf0, int total,
                                             const int32_t *__restrict__ xf_idx,
                                             double cxb, double cyb, T rb,
                                             const double *__restrict__ sx,
                                             const double *__restrict__ sy,
                                             const cx<T> *__restrict__ pr, T *px, int lane) {
  if constexpr (K0 < P) {
    constexpr int KB = kChunk<T, P>(), NV = pow2_ceil(2 * KB),
                  SH = 6 - log2_exact(NV);
    const T tot = p2l_sum<T, P, K0, KB>(xf0, total, xf_idx, cxb, cyb, rb, sx,
                                        sy, pr, lane);
    const int vi = lane >> SH;
    if ((lane & ((1 << SH) - 1)) == 0 && vi < 2 * KB && 2 * K0 + vi < 2 * P)
      px[2 * K0 + vi] = tot;
    p2l_pass_lds<T, P, K0 + KB>(xf0, total, xf_idx, cxb, cyb, rb, sx, sy, pr, px, lane);
  }
}

// M2L over the V list of every box with targets at level >= 2 (vector
// ALU).  One 64-lane block per box; lane (g, l) accumulates coefficient l
// from every G-th list entry with the factorized translation
// b_l += tau^-l sum_k H[l][k] (tau^-k a_k), H[l][k] = (-1)^k C(k+l-1, l).
// The box's P2L sum over its X list (every box with an X list whose local
// expansion is used is one of these boxes) follows in the same block and
// is added to the M2L result before the one store.
template <typename T, int P>
__global__ void __launch_bounds__(64)
    k_m2l(const int32_t *__restrict__ boxes,
          const int32_t *__restrict__ v_ptr, const int32_t *__restrict__ v_src,
          const uint8_t *__restrict__ v_code, const T *__restrict__ H,
          const cx<T> *__restrict__ itp, const cx<T> *__restrict__ M,
          cx<T> *__restrict__ L, int nbox, const int64_t *__restrict__ xf_ptr,
          const int32_t *__restrict__ xf_idx, const double *__restrict__ cxv,
          const double *__restrict__ cyv, const double *__restrict__ rad,
          const double *__restrict__ sx, const double *__restrict__ sy,
          const cx<T> *__restrict__ p, int64_t ns) {
  constexpr int G = Groups<P>::G;
  constexpr int NP = 2 * P + 1;
  __shared__ cx<T> ybuf[G][P];
  __shared__ cx<T> red[G][P];
  __shared__ T px[2 * P];
  const int b = boxes[blockIdx.x];
  const int r = blockIdx.y;
  const int lane = threadIdx.x;
  const int g = lane / P, l = lane % P;
  const bool act = g < G;
  T hrow[P];
#pragma unroll
  for (int k = 0; k < P; ++k) hrow[k] = act ? H[l * P + k] : T(0);
  cx<T> acc{T(0), T(0)};
  const cx<T> *Mr = M + (int64_t)r * nbox * P;
  const int vb = v_ptr[b], nv = v_ptr[b + 1] - vb;
  for (int base = 0; base < nv; base += G) {
    const int v = base + g;
    const bool ok = act && v < nv;
    int code = 0;
    if (ok) {
      const int src = v_src[vb + v];
      code = v_code[vb + v];
      ybuf[g][l] = itp[code * NP + l + 1] * Mr[(int64_t)src * P + l];
    }
    __syncthreads();
    if (ok) {
      cx<T> z{T(0), T(0)};
#pragma unroll
      for (int k = 0; k < P; ++k) z = z + hrow[k] * ybuf[g][k];
      acc = acc + itp[code * NP + l] * z;
    }
    __syncthreads();
  }
  if (act) red[g][l] = acc;
  // (xf_ptr null: no P2L here)
  const int64_t xf0 = xf_ptr ? xf_ptr[b] : 0;
  const int nx = xf_ptr ? (int)(xf_ptr[b + 1] - xf0) : 0;  // block-uniform
  if (nx > 0)
    p2l_pass_lds<T, P, 0>(xf0, nx, xf_idx, cxv[b], cyv[b], T(rad[b]), sx, sy,
                          p + (int64_t)r * ns, px, lane);
  __syncthreads();
  if (act && g == 0) {
    cx<T> s = red[0][l];
#pragma unroll
    for (int gg = 1; gg < G; ++gg) s = s + red[gg][l];
    if (nx > 0) s = s + cx<T>{px[2 * l], px[2 * l + 1]};
    L[((int64_t)r * nbox + b) * P + l] = s;
  }
}

// M2L for FP32 expansions of 16 terms on the matrix cores, followed by the
// box's P2L sum (p2l_sum).  One wave per target box.  For 8 V-list sources
// at a time the wave forms
// Y[k][2v + part] = part(tau_v^-(k+1) a_{v,k+1}) (16 x 16), multiplies
// Z = H Y with four v_mfma_f32_16x16x4f32 (H: 16 x 16, real), then scales
// column pair (2v, 2v+1) of Z by tau_v^-l and accumulates.  Lane layout of
// the 16x16x4 instruction: A[i][k] in lane i + 16 k, B[k][j] in lane
// j + 16 k, D[i][j] in lane j + 16 (i / 4), register i % 4.
typedef float v4f __attribute__((ext_vector_type(4)));

// The X-list sources of the boxes for the P2L sums folded into the FP32
// M2L (per-box ranges xf_ptr into the concatenated source indices xf_idx;
// box centres (bx, by) and half-widths rad).
struct XListSrc {
  const int64_t *xf_ptr;
  const int32_t *xf_idx;
  const double *bx, *by, *rad, *sx, *sy;
  const cx<float> *p;
  int64_t ns;
};

__global__ void __launch_bounds__(256)
    k_m2l_mfma16(int nb, const int32_t *__restrict__ boxes,
                 const int32_t *__restrict__ v_ptr,
                 const int32_t *__restrict__ v_src,
                 const uint8_t *__restrict__ v_code,
                 const float *__restrict__ H, const cx<float> *__restrict__ itp,
                 const cx<float> *__restrict__ M, cx<float> *__restrict__ L,
                 int nbox, XListSrc xs, GammaGroups gg) {
  constexpr int P = 16, NP = 2 * P + 1;
  if ((int)blockIdx.x >= gg.first) {  // block-uniform: a correction chunk
    const int x = blockIdx.x - gg.first;
    gamma_chunk(x % gg.nchunk, x / gg.nchunk, blockIdx.y, gg.nchunk, gg.gl_ptr,
                gg.gpart, gg.nls, gg.G, gg.csum, gg.cnt, gg.gamma);
    return;
  }
  // the 49 x (2P + 1) table of tau^-n, read by every pair, in LDS
  __shared__ cx<float> sItp[49 * NP];
  for (int i = threadIdx.x; i < 49 * NP; i += 256) sItp[i] = itp[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.y;
  const int col = lane & 15, kq = lane >> 4;
  const int vslot = col >> 1, part = col & 1;
  float a[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) a[s] = H[col * P + 4 * s + kq];
  // each wave takes every (4 x #M2L groups)-th box, so that the table
  // above is read once per block for several boxes; the next box's id and
  // list offsets are loaded while this box is worked on (box ids two
  // ahead, offsets one ahead; past the end, box 0 stands in)
  const int stride = 4 * gg.first;
  int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  int b = wv < nb ? boxes[wv] : 0;
  int bn = wv + stride < nb ? boxes[wv + stride] : 0;
  int vb = v_ptr[b], ve = v_ptr[b + 1];
  int64_t xb0 = xs.xf_ptr[b], xb1 = xs.xf_ptr[b + 1];
  for (; wv < nb; wv += stride) {
    const int nv = ve - vb;
    const int64_t x0 = xb0;
    const int xt = (int)(xb1 - xb0);
    const int bc = b;
    b = bn;
    bn = wv + 2 * stride < nb ? boxes[wv + 2 * stride] : 0;
    const int vbc = vb;
    vb = v_ptr[b];
    ve = v_ptr[b + 1];
    xb0 = xs.xf_ptr[b];
    xb1 = xs.xf_ptr[b + 1];
    const cx<float> *Mr = M + (int64_t)r * nbox * P;
    // the box's list entries, lane e holding entry e (a V list has at most
    // 27 entries; any beyond 64 are read directly)
    int esrc = 0, ecode = 0;
    if (lane < nv) {
      esrc = v_src[vbc + lane];
      ecode = v_code[vbc + lane];
    }
    // multipole coefficients k = 4 s + kq of the batch's source vslot
    auto fetch = [&](int base, cx<float> (&mv)[4], int &code, bool &ok) {
      const int v = base + vslot;
      ok = v < nv;
      int src = __shfl(esrc, v & 63, 64);
      code = __shfl(ecode, v & 63, 64);
      if (ok && v >= 64) {
        src = v_src[vbc + v];
        code = v_code[vbc + v];
      }
      if (!ok) src = code = 0;
      const cx<float> *ms = Mr + (int64_t)src * P;
#pragma unroll
      for (int s = 0; s < 4; ++s) mv[s] = ok ? ms[4 * s + kq] : cx<float>{0.f, 0.f};
    };
    float accr[4] = {0.f, 0.f, 0.f, 0.f}, acci[4] = {0.f, 0.f, 0.f, 0.f};
    cx<float> mcur[4], mnxt[4];
    int ccur, cnxt = 0;
    bool okc, oknx = false;
    fetch(0, mcur, ccur, okc);
    for (int base = 0; base < nv; base += 8) {
      // the next batch's loads go out before this batch's products
      if (base + 8 < nv) fetch(base + 8, mnxt, cnxt, oknx);  // wave-uniform
      const bool ok = okc;
      const cx<float> *ip = sItp + ccur * NP;
      v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + kq;
        const cx<float> y = ip[k + 1] * mcur[s];
        const float bv = ok ? (part ? y.y : y.x) : 0.f;
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bv, d, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float mine = d[j];
        const float other = __shfl_xor(mine, 1, 64);
        if (ok && part == 0) {
          const cx<float> t = ip[4 * kq + j] * cx<float>{mine, other};
          accr[j] += t.x;
          acci[j] += t.y;
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) mcur[s] = mnxt[s];
      ccur = cnxt;
      okc = oknx;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      for (int off = 2; off < 16; off <<= 1) {
        accr[j] += __shfl_xor(accr[j], off, 64);
        acci[j] += __shfl_xor(acci[j], off, 64);
      }
    }
    // P2L over the box's X list: the real part of coefficient l ends in
    // lane 4 l, the imaginary part in lane 4 l + 2
    if (xt > 0) {  // wave-uniform
      const float v = p2l_sum<float, P, 0, P>(x0, xt, xs.xf_idx, xs.bx[bc],
                                              xs.by[bc], float(xs.rad[bc]),
                                              xs.sx, xs.sy,
                                              xs.p + (int64_t)r * xs.ns, lane);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        accr[j] += __shfl(v, (lane & 48) + 4 * j, 64);
        acci[j] += __shfl(v, (lane & 48) + 4 * j + 2, 64);
      }
    }
    if (col == 0) {
      cx<float> *dst = L + ((int64_t)r * nbox + bc) * P + 4 * kq;
#pragma unroll
      for (int j = 0; j < 4; ++j) dst[j] = cx<float>{accr[j], acci[j]};
    }
  }
}

// P2L over the X list of one box per wave (p2l_sum, KB coefficients per
// pass), added to the M2L result.
template <typename T, int P, int K0>
__device__ __forceinline__ void p2l_pass(int64_t xf0, int total,
                                         const int32_t *__restrict__ xf_idx,
                                         double cxb, double cyb, T rb,
                                         const double *__restrict__ sx,
                                         const double *__restrict__ sy,
                                         const cx<T> *__restrict__ pr,
                                         T *__restrict__ Lb, int lane) {
  if constexpr (K0 < P) {
    constexpr int KB = kChunk<T, P>(), NV = pow2_ceil(2 * KB),
                  SH = 6 - log2_exact(NV);
    const T tot = p2l_sum<T, P, K0, KB>(xf0, total, xf_idx, cxb, cyb, rb, sx,
                                        sy, pr, lane);
    const int vi = lane >> SH;
    if ((lane & ((1 << SH) - 1)) == 0 && vi < 2 * KB && 2 * K0 + vi < 2 * P)
      Lb[2 * K0 + vi] += tot;
    p2l_pass<T, P, K0 + KB>(xf0, total, xf_idx, cxb, cyb, rb, sx, sy, pr, Lb,
                            lane);
  }
}

template <typename T, int P>
__global__ void __launch_bounds__(64)
    k_p2l(const int32_t *__restrict__ boxes, const int64_t *__restrict__ xf_ptr,
          const int32_t *__restrict__ xf_idx, const double *__restrict__ cxv,
          const double *__restrict__ cyv, const double *__restrict__ rad,
          const double *__restrict__ sx, const double *__restrict__ sy,
          const cx<T> *__restrict__ p, int64_t ns, cx<T> *__restrict__ L,
          int nbox) {
  const int b = boxes[blockIdx.x];
  const int r = blockIdx.y;
  const int64_t xf0 = xf_ptr[b];
  if (xf_ptr[b + 1] == xf0) return;  // nothing to add (the whole wave)
  p2l_pass<T, P, 0>(xf0, (int)(xf_ptr[b + 1] - xf0), xf_idx, cxv[b], cyv[b],
                    T(rad[b]), sx, sy, p + (int64_t)r * ns,
                    reinterpret_cast<T *>(L + ((int64_t)r * nbox + b) * P),
                    (int)threadIdx.x);
}

__device__ __forceinline__ double rcp64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ int pow2_at_least(int n) {
  int t = 1;
  while (t < n) t <<= 1;
  return t;
}

constexpr int kStage = 128;  // U-list sources staged in LDS per pass

// Potential at the targets of one leaf (one 64-lane block).  Lanes are
// (target, slice): with tp = pow2 >= #targets (<= 32) the block has
// S = 64 / tp slices, each taking every S-th staged source, W-list box and
// ancestor; slices are summed by shuffles.  Work: the local expansions of
// the leaf and its ancestors (level >= 2), M2P over its W list, the direct
// sum over the gathered sources of its U list (self pair excluded by
// d == 0), then the operator row assembly in API order.  FP64 version.
template <int P>
__global__ void __launch_bounds__(64, 8)
    k_leaf64(const LeafHdr *__restrict__ hdr,
             const double *__restrict__ cxv, const double *__restrict__ cyv,
             const double *__restrict__ rad,
             const double *__restrict__ tx, const double *__restrict__ ty,
             const int64_t *__restrict__ tperm,
             const int32_t *__restrict__ uf_idx,
             const int32_t *__restrict__ w_src,
             const double *__restrict__ sx, const double *__restrict__ sy,
             const cx<double> *__restrict__ p, int64_t ns,
             const cx<double> *__restrict__ M,
             const cx<double> *__restrict__ L, int nbox,
             double *__restrict__ out, int64_t ldy, double scale,
             Assembly as) {
  __shared__ double2 sz[kStage];
  __shared__ double2 sp[kStage];
  constexpr int NC = 2;  // sub-chunks of <= 32 targets per pass over U
  const LeafHdr &hd = hdr[blockIdx.x];
  const int b = hd.b;
  const int r = blockIdx.y;
  const int lane = threadIdx.x;
  const cx<double> *pr = p + (int64_t)r * ns;
  const cx<double> *Mr = M + (int64_t)r * nbox * P;
  const cx<double> *Lr = L + (int64_t)r * nbox * P;
  const int64_t tb0 = hd.t0, ntb = hd.nt;
  const int64_t uf0 = hd.uf0;
  const int utot = (int)(hd.uf1 - uf0);  // U-list sources of the leaf
  const int wb = hd.wb, we = hd.we;
  const bool has_local = hd.lev >= 2;
  const double ir_b = hd.ir, cx_b = hd.cx, cy_b = hd.cy;
  for (int64_t tc0 = 0; tc0 < ntb; tc0 += 32 * NC) {
    const int nt = (int)min<int64_t>(32 * NC, ntb - tc0);
    const int nch = (nt + 31) / 32;
    // sub-chunk c: targets [32 c, min(32 c + 32, nt)) on tp_c lanes times
    // S_c = 64 / tp_c source slices, tp_c = min(32, next power of two)
    int S[NC], sl[NC], ti[NC];
    bool act[NC];
    double zxs[NC], zys[NC], fld[NC];
    int Smax = 1;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      S[c] = 64;
      sl[c] = 0;
      act[c] = false;
      ti[c] = 0;
      zxs[c] = zys[c] = fld[c] = 0.0;
      if (c >= nch) continue;  // uniform
      const int rem = nt - 32 * c;
      const int tp = rem >= 32 ? 32 : pow2_at_least(rem);
      const int lg = __builtin_ctz(tp);  // tp is a power of two
      S[c] = 64 >> lg;
      Smax = max(Smax, S[c]);
      const int tl = lane & (tp - 1);
      sl[c] = lane >> lg;
      act[c] = 32 * c + tl < nt;
      ti[c] = (int)tc0 + 32 * c + tl;
      if (!act[c]) continue;
      const int64_t i = tb0 + ti[c];
      const double zx = tx[i], zy = ty[i];
      zxs[c] = zx;
      zys[c] = zy;
      double field = 0.0;
      if (sl[c] == 0 && has_local) {
        const cx<double> w{(zx - cx_b) * ir_b, (zy - cy_b) * ir_b};
        const cx<double> *La = Lr + (int64_t)b * P;
        cx<double> acc = La[P - 1];
        for (int l = P - 2; l >= 0; --l) acc = cfma(acc, w, La[l]);
        field += acc.x;
      }
      for (int e = wb + sl[c]; e < we; e += S[c]) {
        const int cw = w_src[e];
        cx<double> d{zx - cxv[cw], zy - cyv[cw]};
        cx<double> rho = rad[cw] * cinv(d);
        const cx<double> *a = Mr + (int64_t)cw * P;
        cx<double> acc = a[P - 1];
        for (int k = P - 2; k >= 0; --k) acc = cfma(acc, rho, a[k]);
        field += (acc * rho).x;
      }
      fld[c] = field;
    }
    {  // the leaf's U-list sources, kStage at a time
      const int total = utot;
      for (int q0 = 0; q0 < total; q0 += kStage) {
        const int take = min(kStage, total - q0);
        // pad to a multiple of Smax with sources of zero strength at the
        // origin: they add 0 * rcp(|z|^2 + 1e-300) = 0
        const int tpad = (take + Smax - 1) & ~(Smax - 1);  // Smax: power of two
        for (int q = lane; q < tpad; q += 64) {
          if (q < take) {
            const int64_t j = uf_idx[uf0 + q0 + q];
            sz[q] = make_double2(sx[j], sy[j]);
            const cx<double> pj = pr[j];
            sp[q] = make_double2(pj.x, pj.y);
          } else {
            sz[q] = make_double2(0.0, 0.0);
            sp[q] = make_double2(0.0, 0.0);
          }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c >= nch) continue;  // uniform
          const int Sc = S[c], niter = tpad >> __builtin_ctz(Sc);
          const double zx = zxs[c], zy = zys[c];
          double f = fld[c];
          const double2 *zq = sz + sl[c];
          const double2 *pq = sp + sl[c];
#pragma unroll 2
          for (int it = 0; it < niter; ++it) {
            const double2 s2 = zq[it * Sc];
            const double2 p2 = pq[it * Sc];
            const double dx = zx - s2.x, dy = zy - s2.y;
            // |d|^2 + 1e-300: a target's own source (d = 0) contributes
            // 0 * rcp(1e-300) = 0; any other |d|^2 above 1e-284 is unchanged
            const double d2 = fma(dx, dx, fma(dy, dy, 1e-300));
            f += fma(p2.x, dx, p2.y * dy) * rcp64(d2);
          }
          fld[c] = f;
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (c >= nch) continue;  // uniform
      double field = fld[c];
      for (int o = 64 >> __builtin_ctz(S[c]); o < 64; o <<= 1) field += __shfl_xor(field, o, 64);
      if (act[c] && sl[c] == 0) {
        const int64_t api = tperm[tb0 + ti[c]];
        double val = scale * field;
        if (as.sigma) {
          const double sg = as.sigma[(int64_t)r * as.ldx + api];
          val += (as.ident + as.tau[api]) * sg +
                 as.gamma[r * as.G + (as.geo ? as.geo[api] : 0)];
        }
        out[(int64_t)r * ldy + api] = val;
      }
    }
  }
}

// A staged U-list source of the FP32 leaf kernel: position (FP64) and the
// FP32 strengths of RB right-hand sides, 16-byte aligned so that one
// address serves both reads.
template <int RB>
struct alignas(16) Src32 {
  double2 z;
  float2 p[RB];
};

// Direct sums of one target lane over the staged sources zq[0], zq[S],
// ..., zq[(niter - 1) S] (S compile-time, so the unrolled reads take
// immediate offsets): f[q] += Re(p_q conj(d)) / |d|^2, d = z_t - z_j formed
// in FP64 and rounded once.  |d|^2 + 1e-30: a target's own source (d = 0)
// contributes 0 * rcp(1e-30) = 0; the bias leaves any |d|^2 above 2e-23
// (node spacings above 5e-12) unchanged in FP32.
template <int S, int RB>
__device__ __forceinline__ void near_sums32(const Src32<RB> *__restrict__ zq,
                                            int niter, double ax, double ay,
                                            float (&f)[RB]) {
  if constexpr (RB == 1) {
#pragma unroll 4
    for (int it = 0; it < niter; ++it) {
      const Src32<1> &e = zq[it * S];
      const float dx = (float)(ax - e.z.x);
      const float dy = (float)(ay - e.z.y);
      const float d2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
      f[0] += fmaf(e.p[0].x, dx, e.p[0].y * dy) * __builtin_amdgcn_rcpf(d2);
    }
  } else {
#pragma unroll 2
    for (int it = 0; it < niter; ++it) {
      const Src32<RB> &e = zq[it * S];
      const float dx = (float)(ax - e.z.x);
      const float dy = (float)(ay - e.z.y);
      const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, fmaf(dy, dy, 1e-30f)));
      const float ux = dx * inv, uy = dy * inv;
#pragma unroll
      for (int q = 0; q < RB; ++q) f[q] = fmaf(e.p[q].x, ux, fmaf(e.p[q].y, uy, f[q]));
    }
  }
}

// FP32 variant: each pair's difference d = z_i - z_j is formed in FP64
// and rounded once to FP32 (one FP64 add and one conversion per
// coordinate, at the FP32 rate on this chip), the rest in FP32.  A block
// handles
// RB right-hand sides (blockIdx.y * RB + 0 .. RB - 1, those < nrhs): each
// pair's difference and reciprocal are formed once and applied to every
// right-hand side of the block.
template <int P, int RB>
__global__ void __launch_bounds__(64, RB == 1 ? 8 : 1)
    k_leaf32(const LeafHdr *__restrict__ hdr,
             const double *__restrict__ cxv, const double *__restrict__ cyv,
             const double *__restrict__ rad,
             const double *__restrict__ tx, const double *__restrict__ ty,
             const int64_t *__restrict__ tperm,
             const int32_t *__restrict__ uf_idx,
             const int32_t *__restrict__ w_src,
             const double *__restrict__ sx, const double *__restrict__ sy,
             const cx<float> *__restrict__ p, int64_t ns,
             const cx<float> *__restrict__ M, const cx<float> *__restrict__ L,
             int nbox, int nrhs, double *__restrict__ out, int64_t ldy,
             double scale, Assembly as) {
  __shared__ Src32<RB> sz[kStage];
  constexpr int NC = 2;  // sub-chunks of <= 32 targets per pass over U
  const LeafHdr &hd = hdr[blockIdx.x];
  const int b = hd.b;
  const int r0 = blockIdx.y * RB, nr = min(RB, nrhs - r0);
  const int lane = threadIdx.x;
  const int64_t tb0 = hd.t0, ntb = hd.nt;
  const int64_t uf0 = hd.uf0;
  const int utot = (int)(hd.uf1 - uf0);  // U-list sources of the leaf
  const int wb = hd.wb, we = hd.we;
  const bool has_local = hd.lev >= 2;
  const double ir_b = hd.ir, cx_b = hd.cx, cy_b = hd.cy;
  for (int64_t tc0 = 0; tc0 < ntb; tc0 += 32 * NC) {
    const int nt = (int)min<int64_t>(32 * NC, ntb - tc0);
    const int nch = (nt + 31) / 32;
    // sub-chunk c: targets [32 c, min(32 c + 32, nt)) on tp_c lanes times
    // S_c = 64 / tp_c source slices, tp_c = min(32, next power of two)
    int S[NC], sl[NC], ti[NC];
    bool act[NC];
    float fld[NC][RB];
    double zxd[NC], zyd[NC];
    int Smax = 1;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      S[c] = 64;
      sl[c] = 0;
      act[c] = false;
      ti[c] = 0;
      zxd[c] = zyd[c] = 0.0;
#pragma unroll
      for (int q = 0; q < RB; ++q) fld[c][q] = 0.f;
      if (c >= nch) continue;  // uniform
      const int rem = nt - 32 * c;
      const int tp = rem >= 32 ? 32 : pow2_at_least(rem);
      const int lg = __builtin_ctz(tp);  // tp is a power of two
      S[c] = 64 >> lg;
      Smax = max(Smax, S[c]);
      const int tl = lane & (tp - 1);
      sl[c] = lane >> lg;
      act[c] = 32 * c + tl < nt;
      ti[c] = (int)tc0 + 32 * c + tl;
      if (!act[c]) continue;
      const int64_t i = tb0 + ti[c];
      zxd[c] = tx[i];
      zyd[c] = ty[i];
    }
    {  // the leaf's U-list sources, kStage at a time
      const int total = utot;
      for (int q0 = 0; q0 < total; q0 += kStage) {
        const int take = min(kStage, total - q0);
        // pad to a multiple of Smax (<= 64, divides kStage) with sources of
        // zero strength at the origin: they add 0 * rcp(|z|^2 + 1e-30) = 0
        const int tpad = (take + Smax - 1) & ~(Smax - 1);  // Smax: power of two
        for (int q = lane; q < tpad; q += 64) {
          if (q < take) {
            const int64_t j = uf_idx[uf0 + q0 + q];
            sz[q].z = make_double2(sx[j], sy[j]);
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
              const cx<float> pj = rr < nr ? p[(int64_t)(r0 + rr) * ns + j]
                                           : cx<float>{0.f, 0.f};
              sz[q].p[rr] = make_float2(pj.x, pj.y);
            }
          } else {
            sz[q].z = make_double2(0.0, 0.0);
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) sz[q].p[rr] = make_float2(0.f, 0.f);
          }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c >= nch) continue;  // uniform
          const int Sc = S[c], niter = tpad >> __builtin_ctz(Sc);
          const double ax = zxd[c], ay = zyd[c];
          float f[RB];
#pragma unroll
          for (int q = 0; q < RB; ++q) f[q] = fld[c][q];
          const Src32<RB> *zq = sz + sl[c];
          switch (Sc) {  // wave-uniform
            case 2: near_sums32<2, RB>(zq, niter, ax, ay, f); break;
            case 4: near_sums32<4, RB>(zq, niter, ax, ay, f); break;
            case 8: near_sums32<8, RB>(zq, niter, ax, ay, f); break;
            case 16: near_sums32<16, RB>(zq, niter, ax, ay, f); break;
            case 32: near_sums32<32, RB>(zq, niter, ax, ay, f); break;
            default: near_sums32<64, RB>(zq, niter, ax, ay, f); break;
          }
#pragma unroll
          for (int q = 0; q < RB; ++q) fld[c][q] = f[q];
        }
        __syncthreads();
      }
    }
    // per right-hand side: L2P (slice 0) and this slice's share of M2P,
    // the sum over slices, the assembled row; the accumulators of the
    // next right-hand side rotate into fld[c][0] (constant register indices)
#pragma unroll 1
    for (int q = 0; q < nr; ++q) {
      const int r = r0 + q;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (c >= nch) continue;  // uniform
        float field = fld[c][0];
        if (act[c]) {
          const double zx = zxd[c], zy = zyd[c];
          if (sl[c] == 0 && has_local) {
            const cx<float> w{float((zx - cx_b) * ir_b), float((zy - cy_b) * ir_b)};
            const cx<float> *La = L + ((int64_t)r * nbox + b) * P;
            cx<float> acc = La[P - 1];
            for (int l = P - 2; l >= 0; --l) acc = cfma(acc, w, La[l]);
            field += acc.x;
          }
          for (int e = wb + sl[c]; e < we; e += S[c]) {
            const int cw = w_src[e];
            const double dx = zx - cxv[cw], dy = zy - cyv[cw];
            const double id = rad[cw] / (dx * dx + dy * dy);
            const cx<float> rho{float(dx * id), float(-dy * id)};
            const cx<float> *a = M + ((int64_t)r * nbox + cw) * P;
            cx<float> acc = a[P - 1];
            for (int k = P - 2; k >= 0; --k) acc = cfma(acc, rho, a[k]);
            field += (acc * rho).x;
          }
        }
        for (int o = 64 >> __builtin_ctz(S[c]); o < 64; o <<= 1) field += __shfl_xor(field, o, 64);
        if (act[c] && sl[c] == 0) {
          const int64_t api = tperm[tb0 + ti[c]];
          double val = scale * (double)field;
          if (as.sigma) {
            const double sg = as.sigma[(int64_t)r * as.ldx + api];
            val += (as.ident + as.tau[api]) * sg +
                   as.gamma[r * as.G + (as.geo ? as.geo[api] : 0)];
          }
          out[(int64_t)r * ldy + api] = val;
        }
#pragma unroll
        for (int k = 0; k + 1 < RB; ++k) fld[c][k] = fld[c][k + 1];
      }
    }
  }
}

// Set-up of the FP32 leaf multipoles' inputs: w32[j] = (z_j - c) / r of
// source j's leaf, rounded once to FP32 as the multipole pass forms it, and
// perm32[j] = src_perm[j]; one wave per source leaf.
__global__ void __launch_bounds__(64)
    k_p2m_inputs32(int nleaf, const int64_t *__restrict__ ls_rng,
                   const double4 *__restrict__ ls_geo, const double *__restrict__ sx,
                   const double *__restrict__ sy, const int64_t *__restrict__ perm,
                   float2 *__restrict__ w32, int32_t *__restrict__ perm32) {
  const int e = blockIdx.x;
  if (e >= nleaf) return;
  const double4 geo = ls_geo[e];
  const int64_t e0 = ls_rng[2 * e], e1 = ls_rng[2 * e + 1];
  for (int64_t j = e0 + threadIdx.x; j < e1; j += 64) {
    w32[j] = make_float2(float((sx[j] - geo.x) * geo.z), float((sy[j] - geo.y) * geo.z));
    perm32[j] = (int32_t)perm[j];
  }
}

void build_p2m_inputs32(DevPlan &pl, hipStream_t s) {
  if (pl.ns > INT32_MAX)
    throw ApiError{LBS_ERR_UNSUPPORTED, "more than 2^31 - 1 sources in one plan"};
  pl.w32.alloc((size_t)pl.ns);
  pl.perm32.alloc((size_t)pl.ns);
  if (pl.n_leaf_s > 0)
    hipLaunchKernelGGL(k_p2m_inputs32, dim3(pl.n_leaf_s), dim3(64), 0, s, pl.n_leaf_s,
                       pl.ls_rng.p, pl.ls_geo.p, pl.sx.p, pl.sy.p, pl.src_perm.p, pl.w32.p,
                       pl.perm32.p);
  LBS_HIP(hipGetLastError());
}

// qm32[j] = (Im q_j, -Re q_j) in FP32 (so that -i q_j sigma = qm32 sigma),
// q = qfac_t interleaved complex
__global__ void k_qm32(int64_t n, const double *__restrict__ qfac_t, float2 *__restrict__ qm32) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < n) qm32[j] = make_float2(float(qfac_t[2 * j + 1]), float(-qfac_t[2 * j]));
}

void launch_qm32(int64_t n, const double *qfac_t, float2 *qm32, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_qm32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, qfac_t,
                     qm32);
  LBS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- drivers
// Returns whether the correction sums of gf were formed too (by the FP32
// MFMA M2L launch).
template <typename T, int P>
static bool far_field(const DevPlan &pl, const Tables &tb, Workspace &ws,
                      cx<T> *p, cx<T> *M, cx<T> *L, int nrhs,
                      hipStream_t s, StrengthSrc ss = StrengthSrc{},
                      const GammaFused *gf = nullptr) {
  bool gamma_done = false;
  StageTimer *tm = ws.timer;
  const cx<T> *itp, *pre, *post;
  const T *H, *bc;
  if constexpr (sizeof(T) == 8) {
    itp = (const cx<T> *)tb.itp64.p;
    H = (const T *)tb.h64.p;
    bc = (const T *)tb.bc64.p;
    pre = (const cx<T> *)tb.pre64.p;
    post = (const cx<T> *)tb.post64.p;
  } else {
    itp = (const cx<T> *)tb.itp32.p;
    H = (const T *)tb.h32.p;
    bc = (const T *)tb.bc32.p;
    pre = (const cx<T> *)tb.pre32.p;
    post = (const cx<T> *)tb.post32.p;
  }
  {
    TimerScope ts(tm, ST_UPWARD, s);
    if (pl.n_leaf_s > 0)
    {
      if constexpr (sizeof(T) == 4 && P <= 16)  // two leaves per wave
        hipLaunchKernelGGL((k_p2m_pair<P>), dim3((pl.n_leaf_s + 1) / 2, nrhs), dim3(64), 0, s,
                           pl.leaf_s.p, pl.n_leaf_s, pl.ls_rng.p, pl.ls_geo.p, pl.sx.p,
                           pl.sy.p, pl.w32.n ? pl.w32.p : nullptr, p, pl.ns, M, pl.nbox, ss);
      else if constexpr (sizeof(T) == 8)  // two leaves per wave
        hipLaunchKernelGGL((k_p2m_pair64<P>), dim3((pl.n_leaf_s + 1) / 2, nrhs), dim3(64), 0,
                           s, pl.leaf_s.p, pl.n_leaf_s, pl.ls_rng.p, pl.ls_geo.p, pl.sx.p,
                           pl.sy.p, (cx<double> *)p, pl.ns, (cx<double> *)M, pl.nbox, ss);
      else
        hipLaunchKernelGGL((k_p2m<T, P>), dim3(pl.n_leaf_s, nrhs), dim3(64), 0,
                           s, pl.leaf_s.p, pl.ls_rng.p, pl.ls_geo.p, pl.sx.p,
                           pl.sy.p, p, pl.ns, M, pl.nbox, ss);
    }
    run_pass<T, P, false>(pl.up[sizeof(T) == 8], bc, pre, post, M, pl.nbox, nrhs, s);
  }
  // the FP32 MFMA M2L also forms the P2L sums of its boxes: every box with
  // an X list whose local expansion is used (level >= 2, with targets) is
  // one of its boxes
  constexpr bool p2l_in_m2l = sizeof(T) == 4 && P == 16;
  if (pl.n_m2l > 0) {
    TimerScope ts(tm, ST_M2L, s);
    if constexpr (p2l_in_m2l) {
      const XListSrc xs{pl.xf_ptr.p, pl.xf_idx.p, pl.cx.p, pl.cy.p, pl.rad.p,
                        pl.sx.p, pl.sy.p, (const cx<float> *)p, pl.ns};
      GammaGroups gg;
      gg.first = std::min((pl.n_m2l + 3) / 4, pl.m2l_groups);
      int groups = gg.first;
      if (gf && pl.n_leaf_s > 0) {  // the correction sums ride along
        gg = GammaGroups{gf->gl_ptr, ws.gpart.p, ws.gcsum.p, ws.gcnt.p, gf->gamma,
                         pl.n_leaf_s, gf->G, gf->nchunk, gg.first};
        groups += gf->nchunk * gf->G;
        gamma_done = true;
      }
      hipLaunchKernelGGL(k_m2l_mfma16, dim3(groups, nrhs), dim3(256), 0, s,
                         pl.n_m2l, pl.m2l_wave.p, pl.v_ptr.p, pl.v_src.p,
                         pl.v_code.p, H, itp, (const cx<T> *)M, L, pl.nbox, xs,
                         gg);
    } else {
      hipLaunchKernelGGL((k_m2l<T, P>), dim3(pl.n_m2l, nrhs), dim3(64), 0, s,
                         pl.m2l_box.p, pl.v_ptr.p, pl.v_src.p, pl.v_code.p, H,
                         itp, (const cx<T> *)M, L, pl.nbox, pl.xf_ptr.p, pl.xf_idx.p,
                         pl.cx.p, pl.cy.p, pl.rad.p, pl.sx.p, pl.sy.p, (const cx<T> *)p,
                         pl.ns);
    }
  }
  TimerScope ts(tm, ST_L2L, s);
  run_pass<T, P, true>(pl.dn[sizeof(T) == 8], bc, pre, post, L, pl.nbox, nrhs, s);
  return gamma_done;
}

template <int P>
static void run64(const DevPlan &pl, const Tables &tb, Workspace &ws,
                  int nrhs, double *out, int64_t ldy, double scale,
                  const Assembly &as, hipStream_t s, const StrengthSrc &ss,
                  const GammaFused *gf) {
  auto *p = (cx<double> *)ws.pstr64.p;
  auto *M = (cx<double> *)ws.mult64.p;
  auto *L = (cx<double> *)ws.loc64.p;
  far_field<double, P>(pl, tb, ws, p, M, L, nrhs, s, ss);
  if (gf && pl.n_leaf_s > 0) {
    TimerScope ts(ws.timer, ST_GAMMA, s);
    hipLaunchKernelGGL(k_gamma_reduce, dim3(gf->nchunk, gf->G, nrhs), dim3(256), 0,
                       s, gf->gl_ptr, ws.gpart.p, pl.n_leaf_s, gf->G, ws.gcsum.p,
                       ws.gcnt.p, gf->gamma);
  }
  if (pl.n_leaf_t > 0) {
    TimerScope ts(ws.timer, ST_LEAF, s);
    hipLaunchKernelGGL((k_leaf64<P>), dim3(pl.n_leaf_t, nrhs), dim3(64), 0, s,
                       pl.lt_hdr.p, pl.cx.p, pl.cy.p, pl.rad.p,
                       pl.tx.p, pl.ty.p, pl.tgt_perm.p, pl.uf_idx.p,
                       pl.w_src.p, pl.sx.p, pl.sy.p,
                       (const cx<double> *)p, pl.ns, (const cx<double> *)M,
                       (const cx<double> *)L, pl.nbox, out, ldy, scale, as);
  }
}

template <int P>
static void run32(const DevPlan &pl, const Tables &tb, Workspace &ws,
                  int nrhs, double *out, int64_t ldy, double scale,
                  const Assembly &as, hipStream_t s, const StrengthSrc &ss,
                  const GammaFused *gf) {
  auto *p = (cx<float> *)ws.pstr32.p;
  auto *M = (cx<float> *)ws.mult32.p;
  auto *L = (cx<float> *)ws.loc32.p;
  const bool gamma_done = far_field<float, P>(pl, tb, ws, p, M, L, nrhs, s, ss, gf);
  if (gf && pl.n_leaf_s > 0 && !gamma_done) {
    TimerScope ts(ws.timer, ST_GAMMA, s);
    hipLaunchKernelGGL(k_gamma_reduce, dim3(gf->nchunk, gf->G, nrhs), dim3(256), 0,
                       s, gf->gl_ptr, ws.gpart.p, pl.n_leaf_s, gf->G, ws.gcsum.p,
                       ws.gcnt.p, gf->gamma);
  }
  if (pl.n_leaf_t > 0) {
    TimerScope ts(ws.timer, ST_LEAF, s);
    auto launch = [&](auto kern, int rb) {
      hipLaunchKernelGGL(kern, dim3(pl.n_leaf_t, (nrhs + rb - 1) / rb), dim3(64),
                         0, s, pl.lt_hdr.p, pl.cx.p, pl.cy.p, pl.rad.p, pl.tx.p,
                         pl.ty.p,
                         pl.tgt_perm.p,
                         pl.uf_idx.p, pl.w_src.p,
                         pl.sx.p, pl.sy.p,
                         (const cx<float> *)p, pl.ns, (const cx<float> *)M,
                         (const cx<float> *)L, pl.nbox, nrhs, out, ldy, scale,
                         as);
    };
    // one right-hand side per block, or blocks of 4 sharing each pair
    if (nrhs == 1) launch(k_leaf32<P, 1>, 1);
    else launch(k_leaf32<P, 4>, 4);
  }
}

void fmm_apply64(const DevPlan &pl, const Tables &tb, Workspace &ws,
                 const double *qfac_t, const double *sigma, int64_t ldx,
                 int nrhs, double *out, int64_t ldy, double scale,
                 const Assembly &as, hipStream_t s, const GammaFused *gf) {
  // the strengths p_j = -i q_j sigma_j (and with gf the partial gamma
  // sums) are formed by the leaf multipole pass
  const StrengthSrc ss{pl.src_perm.p, qfac_t, sigma, ldx, gf ? gf->gw_t : nullptr,
                       gf ? ws.gpart.p : nullptr};
  switch (tb.P) {
    case 20: run64<20>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    case 24: run64<24>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    case 30: run64<30>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    case 36: run64<36>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    case 40: run64<40>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    case 48: run64<48>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    default:
      throw ApiError{LBS_ERR_UNSUPPORTED,
                     "p64 must be one of 20, 24, 30, 36, 40, 48"};
  }
  LBS_HIP(hipGetLastError());
}

void fmm_far64(const DevPlan &pl, const Tables &tb, Workspace &ws, const double *qfac_t,
               const double *sigma, int64_t ldx, int nrhs, hipStream_t s) {
  const StrengthSrc ss{pl.src_perm.p, qfac_t, sigma, ldx, nullptr, nullptr};
  auto *p = (cx<double> *)ws.pstr64.p;
  auto *M = (cx<double> *)ws.mult64.p;
  auto *L = (cx<double> *)ws.loc64.p;
  switch (tb.P) {
    case 20: far_field<double, 20>(pl, tb, ws, p, M, L, nrhs, s, ss); break;
    case 24: far_field<double, 24>(pl, tb, ws, p, M, L, nrhs, s, ss); break;
    case 30: far_field<double, 30>(pl, tb, ws, p, M, L, nrhs, s, ss); break;
    case 36: far_field<double, 36>(pl, tb, ws, p, M, L, nrhs, s, ss); break;
    case 40: far_field<double, 40>(pl, tb, ws, p, M, L, nrhs, s, ss); break;
    case 48: far_field<double, 48>(pl, tb, ws, p, M, L, nrhs, s, ss); break;
    default:
      throw ApiError{LBS_ERR_UNSUPPORTED,
                     "p64 must be one of 20, 24, 30, 36, 40, 48"};
  }
  LBS_HIP(hipGetLastError());
}

void fmm_apply32(const DevPlan &pl, const Tables &tb, Workspace &ws,
                 const double *qfac_t, const float2 *qm32, const double *sigma, int64_t ldx,
                 int nrhs, double *out, int64_t ldy, double scale,
                 const Assembly &as, hipStream_t s, const GammaFused *gf) {
  // the strengths p_j = -i q_j sigma_j (and with gf the partial gamma
  // sums) are formed by the leaf multipole pass
  const StrengthSrc ss{pl.src_perm.p, qfac_t, sigma, ldx, gf ? gf->gw_t : nullptr,
                       gf ? ws.gpart.p : nullptr,
                       qm32 && pl.perm32.n ? qm32 : nullptr,
                       qm32 && pl.perm32.n ? pl.perm32.p : nullptr};
  switch (tb.P) {
    case 12: run32<12>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    case 16: run32<16>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    case 20: run32<20>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    case 24: run32<24>(pl, tb, ws, nrhs, out, ldy, scale, as, s, ss, gf); break;
    default:
      throw ApiError{LBS_ERR_UNSUPPORTED, "p32 must be one of 12, 16, 20, 24"};
  }
  LBS_HIP(hipGetLastError());
}


// ------------------------------------------------- full complex output
// Psi(z) = sum_j p_j / (z - z_j) and Psi'(z) at the targets, complex, FP64,
// for given complex strengths (API order of the plan's sources).  Used by
// the transposed operator and the shape derivatives.
__global__ void k_strengths_given(int64_t ns, const int64_t *__restrict__ perm,
                                  const double *__restrict__ pin,
                                  cx<double> *__restrict__ p) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ns) return;
  const int64_t a = perm[j];
  p[j] = cx<double>{pin[2 * a], pin[2 * a + 1]};
}

// Psi and (DERIV) Psi' at the targets of one leaf (one 64-lane block):
// lanes are (target, slice) as in the FP32 kernels, tp = pow2 >= #targets
// (64 above 32 targets) lanes per slice and S = 64 / tp slices, each taking
// every S-th W-list box and staged source; slices are summed by shuffles.
// Reciprocals by rcp64 (hardware estimate and two Newton-Raphson steps).
template <int P, bool DERIV>
__global__ void __launch_bounds__(64)
    k_leaf64_full(const int32_t *__restrict__ leaves,
                  const int32_t *__restrict__ lev,
                  const int64_t *__restrict__ t0, const int64_t *__restrict__ t1,
                  const int64_t *__restrict__ s0, const int64_t *__restrict__ s1,
                  const double *__restrict__ cxv, const double *__restrict__ cyv,
                  const double *__restrict__ rad,
                  const double *__restrict__ tx, const double *__restrict__ ty,
                  const int64_t *__restrict__ tperm,
                  const int64_t *__restrict__ uf_ptr,
                  const int32_t *__restrict__ uf_idx,
                  const int32_t *__restrict__ w_ptr,
                  const int32_t *__restrict__ w_src,
                  const double *__restrict__ sx, const double *__restrict__ sy,
                  const cx<double> *__restrict__ p,
                  const cx<double> *__restrict__ M,
                  const cx<double> *__restrict__ L,
                  double *__restrict__ psi, double *__restrict__ dpsi) {
  __shared__ double2 sz[kStage];
  __shared__ double2 sp[kStage];
  const int b = leaves[blockIdx.x];
  const int lane = threadIdx.x;
  const int64_t tb0 = t0[b], ntb = t1[b] - tb0;
  const int tp = ntb <= 32 ? pow2_at_least((int)ntb) : 64;
  const int S = 64 / tp, tl = lane % tp, sl = lane / tp;
  const int64_t uf0 = uf_ptr[b];
  const int utot = (int)(uf_ptr[b + 1] - uf0);  // U-list sources of the leaf
  const int wb = w_ptr[b], we = w_ptr[b + 1];
  for (int64_t tc = 0; tc < ntb; tc += tp) {
    const int64_t i = tb0 + tc + tl;
    const bool act = tc + tl < ntb;
    const double zx = act ? tx[i] : 0.0, zy = act ? ty[i] : 0.0;
    cx<double> f{0.0, 0.0}, df{0.0, 0.0};
    if (act) {
      if (sl == 0 && lev[b] >= 2) {
        const double ir = 1.0 / rad[b];
        const cx<double> w{(zx - cxv[b]) * ir, (zy - cyv[b]) * ir};
        const cx<double> *Lb = L + (int64_t)b * P;
        cx<double> acc = Lb[P - 1], dacc = (double)(P - 1) * Lb[P - 1];
        for (int l = P - 2; l >= 1; --l) {
          acc = cfma(acc, w, Lb[l]);
          if constexpr (DERIV) dacc = dacc * w + (double)l * Lb[l];
        }
        acc = cfma(acc, w, Lb[0]);
        f = f + acc;
        if constexpr (DERIV) df = df + ir * dacc;
      }
      for (int e = wb + sl; e < we; e += S) {
        const int c = w_src[e];
        const double dx = zx - cxv[c], dy = zy - cyv[c];
        const double r2 = rcp64(fma(dx, dx, dy * dy));
        const cx<double> iz{dx * r2, -dy * r2};
        const cx<double> rho = rad[c] * iz;
        const cx<double> *a = M + (int64_t)c * P;
        cx<double> acc = a[P - 1], dacc = (double)P * a[P - 1];
        for (int k = P - 2; k >= 0; --k) {
          acc = cfma(acc, rho, a[k]);
          if constexpr (DERIV) dacc = dacc * rho + (double)(k + 1) * a[k];
        }
        f = f + acc * rho;
        if constexpr (DERIV) df = df - (dacc * rho) * iz;
      }
    }
    {  // the leaf's U-list sources, kStage at a time
      const int total = utot;
      for (int q0 = 0; q0 < total; q0 += kStage) {
        const int take = min(kStage, total - q0);
        for (int q = lane; q < take; q += 64) {
          const int64_t j = uf_idx[uf0 + q0 + q];
          sz[q] = make_double2(sx[j], sy[j]);
          sp[q] = make_double2(p[j].x, p[j].y);
        }
        __syncthreads();
        if (act) {
          for (int q = sl; q < take; q += S) {
            const double dx = zx - sz[q].x, dy = zy - sz[q].y;
            // 1 / d = conj(d) / |d|^2; the bias makes a source at the
            // target (d = 0) contribute 0
            const double r2 = rcp64(fma(dx, dx, fma(dy, dy, 1e-300)));
            const cx<double> iv{dx * r2, -dy * r2};
            const cx<double> t = cx<double>{sp[q].x, sp[q].y} * iv;
            f = f + t;
            if constexpr (DERIV) df = df - t * iv;
          }
        }
        __syncthreads();
      }
    }
    for (int o = tp; o < 64; o <<= 1) {
      f.x += __shfl_xor(f.x, o, 64);
      f.y += __shfl_xor(f.y, o, 64);
      if constexpr (DERIV) {
        df.x += __shfl_xor(df.x, o, 64);
        df.y += __shfl_xor(df.y, o, 64);
      }
    }
    if (act && sl == 0) {
      const int64_t api = tperm[i];
      psi[2 * api] = f.x;
      psi[2 * api + 1] = f.y;
      if constexpr (DERIV) {
        dpsi[2 * api] = df.x;
        dpsi[2 * api + 1] = df.y;
      }
    }
  }
}

template <int P>
static void run64_full(const DevPlan &pl, const Tables &tb, Workspace &ws,
                       double *psi, double *dpsi, hipStream_t s) {
  auto *p = (cx<double> *)ws.pstr64.p;
  auto *M = (cx<double> *)ws.mult64.p;
  auto *L = (cx<double> *)ws.loc64.p;
  far_field<double, P>(pl, tb, ws, p, M, L, 1, s);
  if (pl.n_leaf_t > 0) {
    auto k = dpsi ? k_leaf64_full<P, true> : k_leaf64_full<P, false>;
    hipLaunchKernelGGL(k, dim3(pl.n_leaf_t), dim3(64), 0, s,
                       pl.leaf_t.p, pl.lev.p, pl.t0.p, pl.t1.p, pl.s0.p,
                       pl.s1.p, pl.cx.p, pl.cy.p, pl.rad.p, pl.tx.p, pl.ty.p,
                       pl.tgt_perm.p, pl.uf_ptr.p, pl.uf_idx.p, pl.w_ptr.p,
                       pl.w_src.p, pl.sx.p, pl.sy.p, (const cx<double> *)p,
                       (const cx<double> *)M, (const cx<double> *)L, psi,
                       dpsi);
  }
}

void fmm_apply64_full(const DevPlan &pl, const Tables &tb, Workspace &ws,
                      const double *pin, double *psi, double *dpsi,
                      hipStream_t s) {
  if (pl.ns > 0)
    hipLaunchKernelGGL(k_strengths_given, dim3((unsigned)((pl.ns + 255) / 256)),
                       dim3(256), 0, s, pl.ns, pl.src_perm.p, pin,
                       (cx<double> *)ws.pstr64.p);
  switch (tb.P) {
    case 20: run64_full<20>(pl, tb, ws, psi, dpsi, s); break;
    case 24: run64_full<24>(pl, tb, ws, psi, dpsi, s); break;
    case 30: run64_full<30>(pl, tb, ws, psi, dpsi, s); break;
    case 36: run64_full<36>(pl, tb, ws, psi, dpsi, s); break;
    case 40: run64_full<40>(pl, tb, ws, psi, dpsi, s); break;
    case 48: run64_full<48>(pl, tb, ws, psi, dpsi, s); break;
    default:
      throw ApiError{LBS_ERR_UNSUPPORTED,
                     "p64 must be one of 20, 24, 30, 36, 40, 48"};
  }
  LBS_HIP(hipGetLastError());
}

// M[list[e]] = the sum of the partial multipoles of entry e's chunks
// [ptr[e], ptr[e + 1]), in chunk order; one thread per (entry, coefficient).
template <int P>
__global__ void __launch_bounds__(256)
    k_sum_chunks(int n, const int32_t *__restrict__ list, const uint32_t *__restrict__ ptr,
                 const cx<double> *__restrict__ part, cx<double> *__restrict__ M) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)n * P) return;
  const int e = (int)(id / P), k = (int)(id % P);
  cx<double> a{0.0, 0.0};
  for (uint32_t c = ptr[e]; c < ptr[e + 1]; ++c) a = a + part[(int64_t)c * P + k];
  M[(int64_t)list[e] * P + k] = a;
}

template <int P>
static void run64_sources(const DevPlan &pl, const Tables &tb, Workspace &ws,
                          PointSources &ps, const cx<double> *pin, double *psi, double *dpsi,
                          hipStream_t s) {
  auto *M = (cx<double> *)ws.mult64.p;
  auto *L = (cx<double> *)ws.loc64.p;
  const auto *H = (const double *)tb.h64.p;
  const auto *itp = (const cx<double> *)tb.itp64.p;
  // multipoles of every box of level >= 2 from the points it holds: the
  // partial multipoles of chunks of at most kSrcChunk pairs, added per box
  // (boxes without points get zeros)
  launch_gather_cx(ps.nm, ps.m_t.p, (const double *)pin, ps.m_p.p, s);
  auto *part = (cx<double> *)ps.c_part.p;
  if (ps.n_c > 0)
    hipLaunchKernelGGL((k_p2m<double, P>), dim3(ps.n_c, 1), dim3(64), 0, s, ps.c_iota.p,
                       ps.c_rng.p, ps.c_geo.p, ps.m_x.p, ps.m_y.p, (cx<double> *)ps.m_p.p,
                       ps.nm, part, ps.n_c, StrengthSrc{});
  if (ps.n_m > 0)
    hipLaunchKernelGGL((k_sum_chunks<P>), dim3((unsigned)(((int64_t)ps.n_m * P + 255) / 256)),
                       dim3(256), 0, s, ps.n_m, ps.m_list.p, ps.c_ptr.p, part, M);
  // the tree's V lists, then the points' own local-expansion terms
  if (pl.n_m2l > 0)
    hipLaunchKernelGGL((k_m2l<double, P>), dim3(pl.n_m2l, 1), dim3(64), 0, s, pl.m2l_box.p,
                       pl.v_ptr.p, pl.v_src.p, pl.v_code.p, H, itp, (const cx<double> *)M, L,
                       pl.nbox, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                       nullptr, int64_t(0));
  if (ps.n_m > 0)
    hipLaunchKernelGGL((k_p2l<double, P>), dim3(ps.n_m, 1), dim3(64), 0, s, ps.m_list.p,
                       ps.l_ptr.p, ps.l_t.p, pl.cx.p, pl.cy.p, pl.rad.p, ps.x, ps.y, pin, ps.n,
                       L, pl.nbox);
  run_pass<double, P, true>(pl.dn[1], (const double *)tb.bc64.p, (const cx<double> *)tb.pre64.p,
                            (const cx<double> *)tb.post64.p, L, pl.nbox, 1, s);
  // at the plan's targets: local expansions, W lists, direct sums
  if (pl.n_leaf_t > 0) {
    auto k = dpsi ? k_leaf64_full<P, true> : k_leaf64_full<P, false>;
    hipLaunchKernelGGL(k, dim3(pl.n_leaf_t), dim3(64), 0, s, pl.leaf_t.p,
                       pl.lev.p, pl.t0.p, pl.t1.p, pl.s0.p, pl.s1.p, pl.cx.p, pl.cy.p, pl.rad.p,
                       pl.tx.p, pl.ty.p, pl.tgt_perm.p, ps.d_ptr.p, ps.d_t.p, pl.w_ptr.p,
                       pl.w_src.p, ps.x, ps.y, pin, (const cx<double> *)M,
                       (const cx<double> *)L, psi, dpsi);
  }
}

void fmm_sources64_full(const DevPlan &pl, const Tables &tb, Workspace &ws, PointSources &ps,
                        const double *pin, double *psi, double *dpsi, hipStream_t s) {
  const auto *pc = (const cx<double> *)pin;
  switch (tb.P) {
    case 20: run64_sources<20>(pl, tb, ws, ps, pc, psi, dpsi, s); break;
    case 24: run64_sources<24>(pl, tb, ws, ps, pc, psi, dpsi, s); break;
    case 30: run64_sources<30>(pl, tb, ws, ps, pc, psi, dpsi, s); break;
    case 36: run64_sources<36>(pl, tb, ws, ps, pc, psi, dpsi, s); break;
    case 40: run64_sources<40>(pl, tb, ws, ps, pc, psi, dpsi, s); break;
    case 48: run64_sources<48>(pl, tb, ws, ps, pc, psi, dpsi, s); break;
    default:
      throw ApiError{LBS_ERR_UNSUPPORTED,
                     "p64 must be one of 20, 24, 30, 36, 40, 48"};
  }
  LBS_HIP(hipGetLastError());
}

// FP32 counterpart for the transposed operator (field only): strengths in
// FP32, near-field differences formed in FP64 as in k_leaf32.
__global__ void k_strengths_given32(int64_t ns, const int64_t *__restrict__ perm,
                                    const double *__restrict__ pin,
                                    cx<float> *__restrict__ p) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ns) return;
  const int64_t a = perm[j];
  p[j] = cx<float>{float(pin[2 * a]), float(pin[2 * a + 1])};
}

template <int P>
__global__ void __launch_bounds__(64)
    k_leaf32_full(const int32_t *__restrict__ leaves,
                  const int32_t *__restrict__ lev,
                  const int64_t *__restrict__ t0, const int64_t *__restrict__ t1,
                  const int64_t *__restrict__ s0, const int64_t *__restrict__ s1,
                  const double *__restrict__ cxv, const double *__restrict__ cyv,
                  const double *__restrict__ rad,
                  const double *__restrict__ tx, const double *__restrict__ ty,
                  const int64_t *__restrict__ tperm,
                  const int64_t *__restrict__ uf_ptr,
                  const int32_t *__restrict__ uf_idx,
                  const int32_t *__restrict__ w_ptr,
                  const int32_t *__restrict__ w_src,
                  const double *__restrict__ sx, const double *__restrict__ sy,
                  const cx<float> *__restrict__ p,
                  const cx<float> *__restrict__ M,
                  const cx<float> *__restrict__ L, double *__restrict__ psi) {
  __shared__ double2 sz[kStage];
  __shared__ float2 sp[kStage];
  const int b = leaves[blockIdx.x];
  const int lane = threadIdx.x;
  const int64_t tb0 = t0[b], ntb = t1[b] - tb0;
  const int tp = ntb <= 32 ? pow2_at_least((int)ntb) : 64;
  const int S = 64 / tp, tl = lane % tp, sl = lane / tp;
  const int64_t uf0 = uf_ptr[b];
  const int utot = (int)(uf_ptr[b + 1] - uf0);  // U-list sources of the leaf
  const int wb = w_ptr[b], we = w_ptr[b + 1];
  for (int64_t tc = 0; tc < ntb; tc += tp) {
    const int64_t i = tb0 + tc + tl;
    const bool act = tc + tl < ntb;
    const double zx = act ? tx[i] : 0.0, zy = act ? ty[i] : 0.0;
    cx<float> f{0.f, 0.f};
    if (act) {
      if (sl == 0 && lev[b] >= 2) {
        const double ir = 1.0 / rad[b];
        const cx<float> w{float((zx - cxv[b]) * ir), float((zy - cyv[b]) * ir)};
        const cx<float> *La = L + (int64_t)b * P;
        cx<float> acc = La[P - 1];
        for (int l = P - 2; l >= 0; --l) acc = cfma(acc, w, La[l]);
        f = f + acc;
      }
      for (int e = wb + sl; e < we; e += S) {
        const int c = w_src[e];
        const double dx = zx - cxv[c], dy = zy - cyv[c];
        const double id = rad[c] / (dx * dx + dy * dy);
        const cx<float> rho{float(dx * id), float(-dy * id)};
        const cx<float> *a = M + (int64_t)c * P;
        cx<float> acc = a[P - 1];
        for (int k = P - 2; k >= 0; --k) acc = cfma(acc, rho, a[k]);
        f = f + acc * rho;
      }
    }
    {  // the leaf's U-list sources, kStage at a time
      const int total = utot;
      for (int q0 = 0; q0 < total; q0 += kStage) {
        const int take = min(kStage, total - q0);
        for (int q = lane; q < take; q += 64) {
          const int64_t j = uf_idx[uf0 + q0 + q];
          sz[q] = make_double2(sx[j], sy[j]);
          const cx<float> pj = p[j];
          sp[q] = make_float2(pj.x, pj.y);
        }
        __syncthreads();
        if (act) {
          for (int q = sl; q < take; q += S) {
            const double2 s2 = sz[q];
            const float2 p2 = sp[q];
            const float dx = (float)(zx - s2.x);
            const float dy = (float)(zy - s2.y);
            // p / d = p conj(d) / |d|^2; the 1e-30 bias makes a target's own
            // source (d = 0, in a self plan) contribute 0
            const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, fmaf(dy, dy, 1e-30f)));
            f.x += fmaf(p2.x, dx, p2.y * dy) * inv;
            f.y += fmaf(p2.y, dx, -p2.x * dy) * inv;
          }
        }
        __syncthreads();
      }
    }
    for (int o = tp; o < 64; o <<= 1) {
      f.x += __shfl_xor(f.x, o, 64);
      f.y += __shfl_xor(f.y, o, 64);
    }
    if (act && sl == 0) {
      const int64_t api = tperm[i];
      psi[2 * api] = f.x;
      psi[2 * api + 1] = f.y;
    }
  }
}

template <int P>
static void run32_full(const DevPlan &pl, const Tables &tb, Workspace &ws,
                       double *psi, hipStream_t s) {
  auto *p = (cx<float> *)ws.pstr32.p;
  auto *M = (cx<float> *)ws.mult32.p;
  auto *L = (cx<float> *)ws.loc32.p;
  far_field<float, P>(pl, tb, ws, p, M, L, 1, s);
  if (pl.n_leaf_t > 0)
    hipLaunchKernelGGL((k_leaf32_full<P>), dim3(pl.n_leaf_t), dim3(64), 0, s,
                       pl.leaf_t.p, pl.lev.p, pl.t0.p, pl.t1.p, pl.s0.p,
                       pl.s1.p, pl.cx.p, pl.cy.p, pl.rad.p, pl.tx.p, pl.ty.p,
                       pl.tgt_perm.p,
                       pl.uf_ptr.p, pl.uf_idx.p, pl.w_ptr.p, pl.w_src.p,
                       pl.sx.p, pl.sy.p,
                       (const cx<float> *)p, (const cx<float> *)M,
                       (const cx<float> *)L, psi);
}

void fmm_apply32_full(const DevPlan &pl, const Tables &tb, Workspace &ws,
                      const double *pin, double *psi, hipStream_t s) {
  if (pl.ns > 0)
    hipLaunchKernelGGL(k_strengths_given32, dim3((unsigned)((pl.ns + 255) / 256)),
                       dim3(256), 0, s, pl.ns, pl.src_perm.p, pin,
                       (cx<float> *)ws.pstr32.p);
  switch (tb.P) {
    case 12: run32_full<12>(pl, tb, ws, psi, s); break;
    case 16: run32_full<16>(pl, tb, ws, psi, s); break;
    case 20: run32_full<20>(pl, tb, ws, psi, s); break;
    case 24: run32_full<24>(pl, tb, ws, psi, s); break;
    default:
      throw ApiError{LBS_ERR_UNSUPPORTED, "p32 must be one of 12, 16, 20, 24"};
  }
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
