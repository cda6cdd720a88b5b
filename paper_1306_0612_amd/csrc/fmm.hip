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
  std::vector<double> m2m(4 * P * P * 2, 0.0), l2l(4 * P * P * 2, 0.0);
  for (int q = 0; q < 4; ++q) {
    double dx = (q & 1) ? 1.0 : -1.0, dy = (q & 2) ? 1.0 : -1.0;
    for (int lo = 0; lo < P; ++lo)
      for (int ki = 0; ki <= lo; ++ki) {
        double px, py;
        cpow_host(dx, dy, lo - ki, px, py);
        double c = binom(lo, ki) * std::ldexp(1.0, -(lo + 1));
        size_t at = ((size_t)(q * P + lo) * P + ki) * 2;
        m2m[at] = c * px;
        m2m[at + 1] = c * py;
      }
    for (int m = 0; m < P; ++m)
      for (int l = m; l < P; ++l) {
        double px, py;
        cpow_host(dx, dy, l - m, px, py);
        double c = binom(l, m) * std::ldexp(1.0, -l);
        size_t at = ((size_t)(q * P + m) * P + l) * 2;
        l2l[at] = c * px;
        l2l[at + 1] = c * py;
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
  t.m2m64.upload(m2m, s);
  t.l2l64.upload(l2l, s);
  t.h64.upload(h, s);
  t.itp64.upload(itp, s);
  t.m2m32.upload(to32(m2m), s);
  t.l2l32.upload(to32(l2l), s);
  t.h32.upload(to32(h), s);
  t.itp32.upload(to32(itp), s);
  LBS_HIP(hipStreamSynchronize(s));
}

// ----------------------------------------------------------------- kernels
// Strengths in tree order: p_j = -i qfac_j sigma_j.
template <typename T>
__global__ void k_strengths(int64_t ns, const int64_t *__restrict__ perm,
                            const double *__restrict__ qfac_t,
                            const double *__restrict__ sigma, int64_t ldx,
                            cx<T> *__restrict__ p) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (j >= ns) return;
  double s = sigma[(int64_t)r * ldx + perm[j]];
  double qx = qfac_t[2 * j], qy = qfac_t[2 * j + 1];
  // -i (qx + i qy) s = (qy - i qx) s
  p[(int64_t)r * ns + j] = cx<T>{T(qy * s), T(-qx * s)};
}

template <typename T, int P>
__global__ void k_p2m(int nl, const int32_t *__restrict__ leaves,
                      const int64_t *__restrict__ s0,
                      const int64_t *__restrict__ s1,
                      const double *__restrict__ cxv,
                      const double *__restrict__ cyv,
                      const double *__restrict__ rad,
                      const double *__restrict__ sx,
                      const double *__restrict__ sy,
                      const cx<T> *__restrict__ p, int64_t ns,
                      cx<T> *__restrict__ M, int nbox) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (t >= nl) return;
  int b = leaves[t];
  double c_x = cxv[b], c_y = cyv[b], ir = 1.0 / rad[b];
  cx<T> acc[P];
#pragma unroll
  for (int k = 0; k < P; ++k) acc[k] = cx<T>{T(0), T(0)};
  const cx<T> *pr = p + (int64_t)r * ns;
  for (int64_t j = s0[b]; j < s1[b]; ++j) {
    cx<T> w{T((sx[j] - c_x) * ir), T((sy[j] - c_y) * ir)};
    cx<T> pw = pr[j];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      acc[k] = acc[k] + pw;
      pw = pw * w;
    }
  }
  cx<T> *out = M + ((int64_t)r * nbox + b) * P;
  T s = T(ir);
#pragma unroll
  for (int k = 0; k < P; ++k) out[k] = s * acc[k];
}

template <typename T, int P>
__global__ void k_m2m(int b0, int b1, const uint8_t *__restrict__ leaf,
                      const int32_t *__restrict__ child0,
                      const int32_t *__restrict__ nchild,
                      const int32_t *__restrict__ quad,
                      const int64_t *__restrict__ s0,
                      const int64_t *__restrict__ s1,
                      const cx<T> *__restrict__ tab, cx<T> *__restrict__ M,
                      int nbox) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  int b = b0 + gid / P, lo = gid % P;
  int r = blockIdx.y;
  if (b >= b1) return;
  if (leaf[b] || s1[b] == s0[b]) return;
  cx<T> acc{T(0), T(0)};
  for (int c = child0[b]; c < child0[b] + nchild[b]; ++c) {
    if (s1[c] == s0[c]) continue;
    const cx<T> *a = M + ((int64_t)r * nbox + c) * P;
    const cx<T> *row = tab + ((size_t)quad[c] * P + lo) * P;
    for (int ki = 0; ki <= lo; ++ki) acc = acc + row[ki] * a[ki];
  }
  M[((int64_t)r * nbox + b) * P + lo] = acc;
}

template <int P>
struct Groups {
  static constexpr int G = 64 / P;
};

// Local expansion of every box with targets at level >= 2: M2L over its V
// list and P2L over its X list.  One 64-lane block per box; lane (g, l)
// accumulates coefficient l from every G-th list entry.
template <typename T, int P>
__global__ void __launch_bounds__(64)
    k_m2l(int nb, const int32_t *__restrict__ boxes,
          const int32_t *__restrict__ v_ptr, const int32_t *__restrict__ v_src,
          const uint8_t *__restrict__ v_code,
          const int32_t *__restrict__ x_ptr, const int32_t *__restrict__ x_src,
          const double *__restrict__ cxv, const double *__restrict__ cyv,
          const double *__restrict__ rad, const int64_t *__restrict__ s0,
          const int64_t *__restrict__ s1, const double *__restrict__ sx,
          const double *__restrict__ sy, const cx<T> *__restrict__ p,
          int64_t ns, const T *__restrict__ H, const cx<T> *__restrict__ itp,
          const cx<T> *__restrict__ M, cx<T> *__restrict__ L, int nbox) {
  constexpr int G = Groups<P>::G;
  constexpr int NP = 2 * P + 1;
  __shared__ cx<T> ybuf[G][P];
  __shared__ cx<T> red[G][P];
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
  if (act) {
    const double cxb = cxv[b], cyb = cyv[b];
    const T rb = T(rad[b]);
    const cx<T> *pr = p + (int64_t)r * ns;
    for (int e = x_ptr[b]; e < x_ptr[b + 1]; ++e) {
      const int c = x_src[e];
      for (int64_t j = s0[c] + g; j < s1[c]; j += G) {
        cx<T> u{T(sx[j] - cxb), T(sy[j] - cyb)};
        cx<T> iu = cinv(u);
        cx<T> rho = rb * iu;
        cx<T> term = (pr[j] * iu) * cpow(rho, l);
        acc = acc - term;
      }
    }
    red[g][l] = acc;
  }
  __syncthreads();
  if (act && g == 0) {
    cx<T> s = red[0][l];
#pragma unroll
    for (int gg = 1; gg < G; ++gg) s = s + red[gg][l];
    L[((int64_t)r * nbox + b) * P + l] = s;
  }
}

template <typename T, int P>
__global__ void k_l2l(int b0, int b1, const int32_t *__restrict__ parent,
                      const int32_t *__restrict__ quad,
                      const uint8_t *__restrict__ has_tgt,
                      const cx<T> *__restrict__ tab, cx<T> *__restrict__ L,
                      int nbox) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  int b = b0 + gid / P, m = gid % P;
  int r = blockIdx.y;
  if (b >= b1) return;
  if (!has_tgt[b]) return;
  const int pb = parent[b];
  const cx<T> *bp = L + ((int64_t)r * nbox + pb) * P;
  const cx<T> *row = tab + ((size_t)quad[b] * P + m) * P;
  cx<T> acc{T(0), T(0)};
  for (int l = m; l < P; ++l) acc = acc + row[l] * bp[l];
  cx<T> *dst = L + ((int64_t)r * nbox + b) * P + m;
  *dst = *dst + acc;
}

__device__ __forceinline__ double rcp64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Far and near field at the targets of one leaf (one 64-lane block):
// L2P of the leaf's local expansion, M2P over its W list and the direct
// sum over the sources of its U list (self pair excluded by d == 0), then
// the assembly of the operator row in API order.
template <int P>
__global__ void __launch_bounds__(64)
    k_leaf64(const int32_t *__restrict__ leaves,
             const int64_t *__restrict__ t0, const int64_t *__restrict__ t1,
             const int64_t *__restrict__ s0, const int64_t *__restrict__ s1,
             const double *__restrict__ cxv, const double *__restrict__ cyv,
             const double *__restrict__ rad, const int32_t *__restrict__ lev,
             const double *__restrict__ tx, const double *__restrict__ ty,
             const int64_t *__restrict__ tperm,
             const int32_t *__restrict__ u_ptr,
             const int32_t *__restrict__ u_src,
             const int32_t *__restrict__ w_ptr,
             const int32_t *__restrict__ w_src,
             const double *__restrict__ sx, const double *__restrict__ sy,
             const cx<double> *__restrict__ p, int64_t ns,
             const cx<double> *__restrict__ M,
             const cx<double> *__restrict__ L, int nbox,
             double *__restrict__ out, int64_t ldy, double scale,
             Assembly as) {
  __shared__ double lx[64], ly[64];
  __shared__ cx<double> lp[64];
  const int b = leaves[blockIdx.x];
  const int r = blockIdx.y;
  const int lane = threadIdx.x;
  const cx<double> *pr = p + (int64_t)r * ns;
  const cx<double> *Mr = M + (int64_t)r * nbox * P;
  const cx<double> *Lb = L + ((int64_t)r * nbox + b) * P;
  for (int64_t tb = t0[b]; tb < t1[b]; tb += 64) {
    const int64_t i = tb + lane;
    const bool act = i < t1[b];
    const double zx = act ? tx[i] : 0.0, zy = act ? ty[i] : 0.0;
    double field = 0.0;
    if (act && lev[b] >= 2) {
      const double ir = 1.0 / rad[b];
      cx<double> w{(zx - cxv[b]) * ir, (zy - cyv[b]) * ir};
      cx<double> acc = Lb[P - 1];
      for (int l = P - 2; l >= 0; --l) acc = acc * w + Lb[l];
      field += acc.x;
    }
    if (act) {
      for (int e = w_ptr[b]; e < w_ptr[b + 1]; ++e) {
        const int c = w_src[e];
        cx<double> d{zx - cxv[c], zy - cyv[c]};
        cx<double> rho = rad[c] * cinv(d);
        const cx<double> *a = Mr + (int64_t)c * P;
        cx<double> acc = a[P - 1];
        for (int k = P - 2; k >= 0; --k) acc = acc * rho + a[k];
        field += (acc * rho).x;
      }
    }
    for (int e = u_ptr[b]; e < u_ptr[b + 1]; ++e) {
      const int c = u_src[e];
      for (int64_t jb = s0[c]; jb < s1[c]; jb += 64) {
        const int64_t j = jb + lane;
        const int cnt = (int)min<int64_t>(64, s1[c] - jb);
        __syncthreads();
        if (lane < cnt) {
          lx[lane] = sx[j];
          ly[lane] = sy[j];
          lp[lane] = pr[j];
        }
        __syncthreads();
        if (act) {
          for (int q = 0; q < cnt; ++q) {
            const double dx = zx - lx[q], dy = zy - ly[q];
            const double d2 = dx * dx + dy * dy;
            const double inv = d2 > 0.0 ? rcp64(d2) : 0.0;
            field += (lp[q].x * dx + lp[q].y * dy) * inv;
          }
        }
      }
    }
    if (act) {
      const int64_t api = tperm[i];
      double val = scale * field;
      if (as.sigma) {
        const double sg = as.sigma[(int64_t)r * as.ldx + api];
        val += (as.ident + as.tau[api]) * sg + as.gamma[r];
      }
      out[(int64_t)r * ldy + api] = val;
    }
  }
}

// FP32 variant: near-field differences on hi/lo coordinate pairs,
// d = (hi_i - hi_j) + (lo_i - lo_j), arithmetic in FP32.
template <int P>
__global__ void __launch_bounds__(64)
    k_leaf32(const int32_t *__restrict__ leaves,
             const int64_t *__restrict__ t0, const int64_t *__restrict__ t1,
             const int64_t *__restrict__ s0, const int64_t *__restrict__ s1,
             const double *__restrict__ cxv, const double *__restrict__ cyv,
             const double *__restrict__ rad, const int32_t *__restrict__ lev,
             const double *__restrict__ tx, const double *__restrict__ ty,
             const float *__restrict__ txh, const float *__restrict__ txl,
             const float *__restrict__ tyh, const float *__restrict__ tyl,
             const int64_t *__restrict__ tperm,
             const int32_t *__restrict__ u_ptr,
             const int32_t *__restrict__ u_src,
             const int32_t *__restrict__ w_ptr,
             const int32_t *__restrict__ w_src,
             const float *__restrict__ sxh, const float *__restrict__ sxl,
             const float *__restrict__ syh, const float *__restrict__ syl,
             const cx<float> *__restrict__ p, int64_t ns,
             const cx<float> *__restrict__ M, const cx<float> *__restrict__ L,
             int nbox, double *__restrict__ out, int64_t ldy, double scale,
             Assembly as) {
  __shared__ float lxh[64], lxl[64], lyh[64], lyl[64];
  __shared__ cx<float> lp[64];
  const int b = leaves[blockIdx.x];
  const int r = blockIdx.y;
  const int lane = threadIdx.x;
  const cx<float> *pr = p + (int64_t)r * ns;
  const cx<float> *Mr = M + (int64_t)r * nbox * P;
  const cx<float> *Lb = L + ((int64_t)r * nbox + b) * P;
  for (int64_t tb = t0[b]; tb < t1[b]; tb += 64) {
    const int64_t i = tb + lane;
    const bool act = i < t1[b];
    const double zx = act ? tx[i] : 0.0, zy = act ? ty[i] : 0.0;
    const float zxh = act ? txh[i] : 0.f, zxl = act ? txl[i] : 0.f;
    const float zyh = act ? tyh[i] : 0.f, zyl = act ? tyl[i] : 0.f;
    float field = 0.f;
    if (act && lev[b] >= 2) {
      const double ir = 1.0 / rad[b];
      cx<float> w{float((zx - cxv[b]) * ir), float((zy - cyv[b]) * ir)};
      cx<float> acc = Lb[P - 1];
      for (int l = P - 2; l >= 0; --l) acc = acc * w + Lb[l];
      field += acc.x;
    }
    if (act) {
      for (int e = w_ptr[b]; e < w_ptr[b + 1]; ++e) {
        const int c = w_src[e];
        const double dx = zx - cxv[c], dy = zy - cyv[c];
        const double id = rad[c] / (dx * dx + dy * dy);
        cx<float> rho{float(dx * id), float(-dy * id)};
        const cx<float> *a = Mr + (int64_t)c * P;
        cx<float> acc = a[P - 1];
        for (int k = P - 2; k >= 0; --k) acc = acc * rho + a[k];
        field += (acc * rho).x;
      }
    }
    for (int e = u_ptr[b]; e < u_ptr[b + 1]; ++e) {
      const int c = u_src[e];
      for (int64_t jb = s0[c]; jb < s1[c]; jb += 64) {
        const int64_t j = jb + lane;
        const int cnt = (int)min<int64_t>(64, s1[c] - jb);
        __syncthreads();
        if (lane < cnt) {
          lxh[lane] = sxh[j];
          lxl[lane] = sxl[j];
          lyh[lane] = syh[j];
          lyl[lane] = syl[j];
          lp[lane] = pr[j];
        }
        __syncthreads();
        if (act) {
          for (int q = 0; q < cnt; ++q) {
            const float dx = (zxh - lxh[q]) + (zxl - lxl[q]);
            const float dy = (zyh - lyh[q]) + (zyl - lyl[q]);
            const float d2 = dx * dx + dy * dy;
            const float inv = d2 > 0.f ? __builtin_amdgcn_rcpf(d2) : 0.f;
            field += (lp[q].x * dx + lp[q].y * dy) * inv;
          }
        }
      }
    }
    if (act) {
      const int64_t api = tperm[i];
      double val = scale * (double)field;
      if (as.sigma) {
        const double sg = as.sigma[(int64_t)r * as.ldx + api];
        val += (as.ident + as.tau[api]) * sg + as.gamma[r];
      }
      out[(int64_t)r * ldy + api] = val;
    }
  }
}

// ---------------------------------------------------------------- drivers
template <typename T, int P>
static void upward_downward(const DevPlan &pl, const Tables &tb,
                            const cx<T> *p, cx<T> *M, cx<T> *L, int nrhs,
                            StageTimer *tm, hipStream_t s) {
  const cx<T> *m2m, *l2l, *itp;
  const T *H;
  if constexpr (sizeof(T) == 8) {
    m2m = (const cx<T> *)tb.m2m64.p;
    l2l = (const cx<T> *)tb.l2l64.p;
    itp = (const cx<T> *)tb.itp64.p;
    H = (const T *)tb.h64.p;
  } else {
    m2m = (const cx<T> *)tb.m2m32.p;
    l2l = (const cx<T> *)tb.l2l32.p;
    itp = (const cx<T> *)tb.itp32.p;
    H = (const T *)tb.h32.p;
  }
  if (pl.n_leaf_s > 0) {
    TimerScope ts(tm, ST_P2M, s);
    dim3 grid((pl.n_leaf_s + 63) / 64, nrhs);
    hipLaunchKernelGGL((k_p2m<T, P>), grid, dim3(64), 0, s, pl.n_leaf_s,
                       pl.leaf_s.p, pl.s0.p, pl.s1.p, pl.cx.p, pl.cy.p,
                       pl.rad.p, pl.sx.p, pl.sy.p, p, pl.ns, M, pl.nbox);
  }
  {
  TimerScope ts(tm, ST_M2M, s);
  for (int l = pl.nlevels - 2; l >= 2; --l) {
    int b0 = pl.level_ptr[l], b1 = pl.level_ptr[l + 1];
    int threads = (b1 - b0) * P;
    if (threads <= 0) continue;
    dim3 grid((threads + 255) / 256, nrhs);
    hipLaunchKernelGGL((k_m2m<T, P>), grid, dim3(256), 0, s, b0, b1,
                       pl.leaf.p, pl.child0.p, pl.nchild.p, pl.quad.p,
                       pl.s0.p, pl.s1.p, m2m, M, pl.nbox);
  }
  }
  if (pl.n_m2l > 0) {
    TimerScope ts(tm, ST_M2L, s);
    dim3 grid(pl.n_m2l, nrhs);
    hipLaunchKernelGGL((k_m2l<T, P>), grid, dim3(64), 0, s, pl.n_m2l,
                       pl.m2l_box.p, pl.v_ptr.p, pl.v_src.p, pl.v_code.p,
                       pl.x_ptr.p, pl.x_src.p, pl.cx.p, pl.cy.p, pl.rad.p,
                       pl.s0.p, pl.s1.p, pl.sx.p, pl.sy.p, p, pl.ns, H, itp,
                       (const cx<T> *)M, L, pl.nbox);
  }
  TimerScope ts(tm, ST_L2L, s);
  for (int l = 3; l < pl.nlevels; ++l) {
    int b0 = pl.level_ptr[l], b1 = pl.level_ptr[l + 1];
    int threads = (b1 - b0) * P;
    if (threads <= 0) continue;
    dim3 grid((threads + 255) / 256, nrhs);
    hipLaunchKernelGGL((k_l2l<T, P>), grid, dim3(256), 0, s, b0, b1,
                       pl.parent.p, pl.quad.p, pl.has_tgt.p, l2l, L,
                       pl.nbox);
  }
}

template <int P>
static void run64(const DevPlan &pl, const Tables &tb, Workspace &ws,
                  int nrhs, double *out, int64_t ldy, double scale,
                  const Assembly &as, hipStream_t s) {
  auto *p = (cx<double> *)ws.pstr64.p;
  auto *M = (cx<double> *)ws.mult64.p;
  auto *L = (cx<double> *)ws.loc64.p;
  upward_downward<double, P>(pl, tb, p, M, L, nrhs, ws.timer, s);
  if (pl.n_leaf_t > 0) {
    TimerScope ts(ws.timer, ST_LEAF, s);
    dim3 grid(pl.n_leaf_t, nrhs);
    hipLaunchKernelGGL((k_leaf64<P>), grid, dim3(64), 0, s, pl.leaf_t.p,
                       pl.t0.p, pl.t1.p, pl.s0.p, pl.s1.p, pl.cx.p, pl.cy.p,
                       pl.rad.p, pl.lev.p, pl.tx.p, pl.ty.p,
                       pl.tgt_perm.p, pl.u_ptr.p, pl.u_src.p, pl.w_ptr.p,
                       pl.w_src.p, pl.sx.p, pl.sy.p, (const cx<double> *)p,
                       pl.ns, (const cx<double> *)M, (const cx<double> *)L,
                       pl.nbox, out, ldy, scale, as);
  }
}

template <int P>
static void run32(const DevPlan &pl, const Tables &tb, Workspace &ws,
                  int nrhs, double *out, int64_t ldy, double scale,
                  const Assembly &as, hipStream_t s) {
  auto *p = (cx<float> *)ws.pstr32.p;
  auto *M = (cx<float> *)ws.mult32.p;
  auto *L = (cx<float> *)ws.loc32.p;
  upward_downward<float, P>(pl, tb, p, M, L, nrhs, ws.timer, s);
  if (pl.n_leaf_t > 0) {
    TimerScope ts(ws.timer, ST_LEAF, s);
    dim3 grid(pl.n_leaf_t, nrhs);
    hipLaunchKernelGGL((k_leaf32<P>), grid, dim3(64), 0, s, pl.leaf_t.p,
                       pl.t0.p, pl.t1.p, pl.s0.p, pl.s1.p, pl.cx.p, pl.cy.p,
                       pl.rad.p, pl.lev.p, pl.tx.p, pl.ty.p, pl.txh.p,
                       pl.txl.p, pl.tyh.p, pl.tyl.p, pl.tgt_perm.p,
                       pl.u_ptr.p, pl.u_src.p, pl.w_ptr.p, pl.w_src.p,
                       pl.sxh.p, pl.sxl.p, pl.syh.p, pl.syl.p,
                       (const cx<float> *)p, pl.ns, (const cx<float> *)M,
                       (const cx<float> *)L, pl.nbox, out, ldy, scale, as);
  }
}

void fmm_apply64(const DevPlan &pl, const Tables &tb, Workspace &ws,
                 const double *qfac_t, const double *sigma, int64_t ldx,
                 int nrhs, double *out, int64_t ldy, double scale,
                 const Assembly &as, hipStream_t s) {
  if (pl.ns > 0) {
    TimerScope ts(ws.timer, ST_STRENGTHS, s);
    dim3 grid((unsigned)((pl.ns + 255) / 256), nrhs);
    hipLaunchKernelGGL((k_strengths<double>), grid, dim3(256), 0, s, pl.ns,
                       pl.src_perm.p, qfac_t, sigma, ldx,
                       (cx<double> *)ws.pstr64.p);
  }
  switch (tb.P) {
    case 20: run64<20>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    case 24: run64<24>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    case 30: run64<30>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    case 36: run64<36>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    case 40: run64<40>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    case 48: run64<48>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    default:
      throw ApiError{LBS_ERR_UNSUPPORTED,
                     "p64 must be one of 20, 24, 30, 36, 40, 48"};
  }
  LBS_HIP(hipGetLastError());
}

void fmm_apply32(const DevPlan &pl, const Tables &tb, Workspace &ws,
                 const double *qfac_t, const double *sigma, int64_t ldx,
                 int nrhs, double *out, int64_t ldy, double scale,
                 const Assembly &as, hipStream_t s) {
  if (pl.ns > 0) {
    TimerScope ts(ws.timer, ST_STRENGTHS, s);
    dim3 grid((unsigned)((pl.ns + 255) / 256), nrhs);
    hipLaunchKernelGGL((k_strengths<float>), grid, dim3(256), 0, s, pl.ns,
                       pl.src_perm.p, qfac_t, sigma, ldx,
                       (cx<float> *)ws.pstr32.p);
  }
  switch (tb.P) {
    case 12: run32<12>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    case 16: run32<16>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    case 20: run32<20>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    case 24: run32<24>(pl, tb, ws, nrhs, out, ldy, scale, as, s); break;
    default:
      throw ApiError{LBS_ERR_UNSUPPORTED, "p32 must be one of 12, 16, 20, 24"};
  }
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
