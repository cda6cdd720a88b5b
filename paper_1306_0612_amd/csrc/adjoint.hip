// Transposed operators and the shape derivative of a target misfit
// (adjoint of the method of Section 5).  All FP64.
//
// With the system A(beta) x = [2g; 0] (eq. matrix_eqns) and the evaluation
// u = T(beta) x (eq. eqn:u_multi), the misfit L = 1/2 |u - u*|^2 has
//   dL/dg = 2 lambda_sigma,     A^T lambda = T^T w,  w = u - u*,
//   dL/dbeta = w^T (dT/dbeta) x - lambda^T (dA/dbeta) x.
// beta are the Fourier coefficients of the island radii; they move the
// nodes, hence xi, xi', xi'' (Section 3) of the kernel and the node
// positions of the log-source rows.  Complex cotangents g of a complex
// quantity z are defined by d(Phi) = Re(g dz).
#include <cmath>

#include "cplx.h"
#include "lbs_internal.h"

namespace lbs {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInvPi_ = 0.31830988618379067154;
constexpr double kLog2_ = 0.69314718055994530942;

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ bool in_sorted(const int32_t *a, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < n && a[lo] == x;
}

// out_j = ident y_j + Re(i q_j F_j) + tau_j y_j + gw_j Y_geo(j), the rows of
// (I + K)^T y: q_j = (s h / pi) xi'_j, F_j = sum_{i != j} y_i / (xi_j - xi_i),
// Y = sum of y over the geometry.
__global__ void k_kT_assemble(int64_t N, const double *__restrict__ y,
                              const double *__restrict__ F,
                              const double *__restrict__ qfac,
                              const double *__restrict__ tau,
                              const double *__restrict__ gw,
                              const int32_t *__restrict__ geo,
                              const double *__restrict__ ysum, double ident,
                              double *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double qx = qfac[2 * j], qy = qfac[2 * j + 1];
  const double fx = F[2 * j], fy = F[2 * j + 1];
  // Re(i (q F)) = -Im(q F)
  const double t = -(qx * fy + qy * fx);
  out[j] = ident * y[j] + t + tau[j] * y[j] + gw[j] * ysum[geo[j]];
}

void launch_kT_assemble(const Geometry &g, const double *y, const double *F,
                        const double *ysum, double ident, double *out,
                        hipStream_t s) {
  if (g.N == 0) return;
  hipLaunchKernelGGL(k_kT_assemble, dim3((unsigned)((g.N + 255) / 256)),
                     dim3(256), 0, s, g.N, y, F, g.qfac.p, g.tau.p, g.gw.p,
                     g.node_geo.p, ysum, ident, out);
  LBS_HIP(hipGetLastError());
}

// complex strengths from a real vector: out = (y, 0)
__global__ void k_real_to_complex(int64_t n, const double *__restrict__ y,
                                  double *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    out[2 * j] = y[j];
    out[2 * j + 1] = 0.0;
  }
}

void launch_real_to_complex(int64_t n, const double *y, double *out,
                            hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_real_to_complex, dim3((unsigned)((n + 255) / 256)),
                     dim3(256), 0, s, n, y, out);
  LBS_HIP(hipGetLastError());
}

// out = (y[idx[q]], 0) for q < n
__global__ void k_gather_complex(int64_t n, const int64_t *__restrict__ idx,
                                 const double *__restrict__ y,
                                 double *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) {
    out[2 * q] = y[idx[q]];
    out[2 * q + 1] = 0.0;
  }
}

void launch_gather_complex(int64_t n, const int64_t *idx, const double *y,
                           double *out, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_complex, dim3((unsigned)((n + 255) / 256)),
                     dim3(256), 0, s, n, idx, y, out);
  LBS_HIP(hipGetLastError());
}

// out[0] = sum of x (one block)
__global__ void __launch_bounds__(1024)
    k_sum(int64_t n, const double *__restrict__ x, double *__restrict__ out) {
  __shared__ double red[16];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) a += x[i];
  a = wsum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += red[q];
    out[0] = t;
  }
}

void launch_sum(int64_t n, const double *x, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, n, x, out);
  LBS_HIP(hipGetLastError());
}

// the double-layer strengths p_j = -i qfac_j sigma_j (API order)
__global__ void k_dl_strengths(int64_t n, const double *__restrict__ qfac,
                               const double *__restrict__ sigma,
                               double *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    out[2 * j] = qfac[2 * j + 1] * sigma[j];
    out[2 * j + 1] = -qfac[2 * j] * sigma[j];
  }
}

void launch_dl_strengths(const Geometry &g, const double *sigma, double *out,
                         hipStream_t s) {
  if (g.N == 0) return;
  hipLaunchKernelGGL(k_dl_strengths, dim3((unsigned)((g.N + 255) / 256)),
                     dim3(256), 0, s, g.N, g.qfac.p, sigma, out);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------------ E^T
// (E^T y)_m = sum_i 2 G(x_i, c_m) y_i over the nodes of m's geometry.  In
// island k's own frame (xi' = projection from the antipode of c_k, the frame
// of the forward log-source product), for m not among k's near centres,
//   sum_{i in k} y_i log|x_i - c_m| = Y_k log|c_k - c_m|
//       - Re sum_l q^l Q_k[l] / l - ELL_k / 2,
// q = 2 rho'_k (a - i b) / |c_k - c_m|^2 (a, b: c_m on k's frame vectors),
// Q_k[l] = sum_i y_i (xi'_i / rho'_k)^l, Y_k = sum_i y_i,
// ELL_k = sum_i y_i log(1 + |xi'_i|^2); near islands directly in 3D.
//
// Moments are stored slot-major, mom[s * M + k], so that lanes over islands
// read them coalesced: slots 2 (l - 1), 2 (l - 1) + 1 hold Q_k[l] / l
// (l = 1..P), slot 2 P holds Y_k and slot 2 P + 1 ELL_k.  One wave per
// (island, half of the series): half h sums the powers h P/2 + 1 .. (h + 1)
// P/2, starting from u^(h P/2 + 1) by repeated squaring; half 0 also forms
// Y_k and ELL_k.
__global__ void __launch_bounds__(64)
    k_island_moments(int M, const int64_t *__restrict__ offs,
                     const double *__restrict__ xil,
                     const double *__restrict__ elll,
                     const double *__restrict__ rhol,
                     const double *__restrict__ y, double *__restrict__ mom) {
  constexpr int P = kPlog, PH = P / 2;
  static_assert(2 * PH == P, "the series splits in two halves");
  const int k = blockIdx.x, h = blockIdx.y, ln = threadIdx.x;
  const int l0 = h * PH;
  const double ir = 1.0 / rhol[k];
  cx<double> acc[PH];
#pragma unroll
  for (int l = 0; l < PH; ++l) acc[l] = cx<double>{0.0, 0.0};
  double ys = 0.0, ys_ell = 0.0;
  for (int64_t i = offs[k] + ln; i < offs[k + 1]; i += 64) {
    const double yi = y[i];
    const cx<double> u{xil[2 * i] * ir, xil[2 * i + 1] * ir};
    cx<double> pw = yi * u;
    if (h == 0) {
      ys += yi;
      ys_ell += yi * elll[i];
    } else {
      cx<double> base = u;  // pw = y_i u^(l0 + 1)
      for (int e = l0; e > 0; e >>= 1) {
        if (e & 1) pw = pw * base;
        base = base * base;
      }
    }
#pragma unroll
    for (int l = 0; l < PH; ++l) {
      acc[l] = acc[l] + pw;
      pw = pw * u;
    }
  }
#pragma unroll
  for (int l = 0; l < PH; ++l) {
    const double inv = 1.0 / (double)(l0 + l + 1);
    const double vx = wsum(acc[l].x), vy = wsum(acc[l].y);
    if (ln == 0) {
      mom[(int64_t)(2 * (l0 + l)) * M + k] = vx * inv;
      mom[(int64_t)(2 * (l0 + l) + 1) * M + k] = vy * inv;
    }
  }
  if (h == 0) {
    ys = wsum(ys);
    ys_ell = wsum(ys_ell);
    if (ln == 0) {
      mom[(int64_t)(2 * P) * M + k] = ys;
      mom[(int64_t)(2 * P + 1) * M + k] = ys_ell;
    }
  }
}

// (E^T y)_m for a tile of TM consecutive centres m per block: threads over
// the islands k of the geometry, the series ratios q_km and h_km formed from
// the centres and k's frame, each moment Q_k[l] read once and applied to the
// TM Horner chains; k near m (m's transposed near list, ascending) is left
// to the direct sum over its nodes.
template <int TM>
__global__ void __launch_bounds__(256)
    k_logsrc_T(int M, const int32_t *__restrict__ isl_geo,
               const int32_t *__restrict__ gisl,
               const int64_t *__restrict__ offs,
               const double *__restrict__ cxyz,
               const double *__restrict__ xyz,
               const int32_t *__restrict__ nearT_ptr,
               const int32_t *__restrict__ nearT_idx,
               const double *__restrict__ frame,
               const double *__restrict__ rhol,
               const double *__restrict__ mom, const double *__restrict__ y,
               double alpha, double *__restrict__ out) {
  constexpr int P = kPlog;
  __shared__ double red[4][2 * TM];
  const int mb = blockIdx.x * TM;
  const int tid = threadIdx.x, ln = tid & 63, wv = tid >> 6;
  // the tile's centres: geometry ranges, table rows, near-list cursors
  int ka[TM], kb[TM], np[TM], ne[TM];
  double cm[TM][3];
  int klo = M, khi = 0;
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int m = mb + t;
    if (m < M) {
      const int g = isl_geo[m];
      ka[t] = gisl[g];
      kb[t] = gisl[g + 1];
      np[t] = nearT_ptr[m];
      ne[t] = nearT_ptr[m + 1];
      klo = min(klo, ka[t]);
      khi = max(khi, kb[t]);
    } else {
      ka[t] = kb[t] = 0;
      np[t] = ne[t] = 0;
    }
  }
  double tot[TM], ysum[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    tot[t] = ysum[t] = 0.0;
    const int m = mb + t < M ? mb + t : M - 1;
    cm[t][0] = cxyz[3 * m];
    cm[t][1] = cxyz[3 * m + 1];
    cm[t][2] = cxyz[3 * m + 2];
  }
  for (int k = klo + tid; k < khi; k += 256) {
    const double *mk = mom + k;
    const double Yk = mk[(int64_t)(2 * P) * M], Ek = mk[(int64_t)(2 * P + 1) * M];
    // k's centre and frame: q_km = 2 rho'_k (a - i b) / |c_k - c_m|^2 and
    // log|c_k - c_m| are formed here, for the tile's centres c_m
    const double ck0 = cxyz[3 * k], ck1 = cxyz[3 * k + 1], ck2 = cxyz[3 * k + 2];
    const double *fk = frame + 6 * k;
    const double f0 = fk[0], f1 = fk[1], f2 = fk[2], f3 = fk[3], f4 = fk[4], f5 = fk[5];
    const double rk2 = 2.0 * rhol[k];
    cx<double> q[TM], ser[TM];
    double hk[TM], w[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const bool in = k >= ka[t] && k < kb[t];
      if (in) ysum[t] += Yk;
      while (np[t] < ne[t] && nearT_idx[np[t]] < k) ++np[t];
      const bool far = in && !(np[t] < ne[t] && nearT_idx[np[t]] == k);
      const double x0 = cm[t][0], x1 = cm[t][1], x2 = cm[t][2];
      const double d0 = x0 - ck0, d1 = x1 - ck1, d2 = x2 - ck2;
      const double dd = far ? d0 * d0 + d1 * d1 + d2 * d2 : 1.0;  // far pairs: dd > 0
      const double ff = rk2 / dd;
      q[t] = far ? cx<double>{(x0 * f0 + x1 * f1 + x2 * f2) * ff,
                              -(x0 * f3 + x1 * f4 + x2 * f5) * ff}
                 : cx<double>{0.0, 0.0};
      hk[t] = far ? 0.5 * log(dd) : 0.0;
      w[t] = far ? 1.0 : 0.0;
      ser[t] = cx<double>{mk[(int64_t)(2 * (P - 1)) * M], mk[(int64_t)(2 * (P - 1) + 1) * M]};
    }
    // sum_l q^l Q_k[l] / l by Horner's rule over the scaled moments
#pragma unroll
    for (int l = P - 1; l >= 1; --l) {
      const cx<double> Ql{mk[(int64_t)(2 * (l - 1)) * M], mk[(int64_t)(2 * (l - 1) + 1) * M]};
#pragma unroll
      for (int t = 0; t < TM; ++t) ser[t] = cfma(ser[t], q[t], Ql);
    }
#pragma unroll
    for (int t = 0; t < TM; ++t)
      tot[t] += w[t] * (Yk * hk[t] - (ser[t] * q[t]).x - 0.5 * Ek);
  }
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const double a = wsum(tot[t]), b = wsum(ysum[t]);
    if (ln == 0) {
      red[wv][2 * t] = a;
      red[wv][2 * t + 1] = b;
    }
  }
  __syncthreads();
  // near islands directly, one centre after another
#pragma unroll 1
  for (int t = 0; t < TM; ++t) {
    const int m = mb + t;
    if (m >= M) break;  // block-uniform
    const double x0 = cxyz[3 * m], x1 = cxyz[3 * m + 1], x2 = cxyz[3 * m + 2];
    double acc = 0.0;
    for (int e = nearT_ptr[m]; e < nearT_ptr[m + 1]; ++e) {
      const int k = nearT_idx[e];
      for (int64_t i = offs[k] + tid; i < offs[k + 1]; i += 256) {
        const double d0 = xyz[3 * i] - x0, d1 = xyz[3 * i + 1] - x1,
                     d2 = xyz[3 * i + 2] - x2;
        acc += y[i] * 0.5 * log(d0 * d0 + d1 * d1 + d2 * d2);
      }
    }
    acc = wsum(acc);
    __shared__ double rn[4];
    if (ln == 0) rn[wv] = acc;
    __syncthreads();
    if (tid == 0) {
      const double t4 = red[0][2 * t] + red[1][2 * t] + red[2][2 * t] + red[3][2 * t] +
                        rn[0] + rn[1] + rn[2] + rn[3];
      const double ys4 = red[0][2 * t + 1] + red[1][2 * t + 1] + red[2][2 * t + 1] +
                         red[3][2 * t + 1];
      out[m] = alpha * (-kInvPi_ * t4 + 0.5 * kInvPi_ * kLog2_ * ys4);
    }
    __syncthreads();
  }
}

void launch_logsrc_T(const Geometry &g, const double *y, double *mom,
                     double alpha, double *out, hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_island_moments, dim3(g.M, 2), dim3(64), 0, s, g.M,
                     g.doffs.p, g.xil.p, g.elll.p, g.rhol.p, y, mom);
  constexpr int TM = 4;
  hipLaunchKernelGGL(k_logsrc_T<TM>, dim3((g.M + TM - 1) / TM), dim3(256), 0, s,
                     g.M, g.isl_geo.p, g.dgisl.p, g.doffs.p, g.dcenter.p,
                     g.xyz.p, g.nearRT_ptr.p, g.nearRT_idx.p, g.frame.p, g.rhol.p, mom, y,
                     alpha, out);
  LBS_HIP(hipGetLastError());
}

// F^T z: node i gets z of its island unless the island is its geometry's
// first (which carries the row sum(A) = 0 instead of a constraint).
// out_i = a * x_i + b * (F^T z)_i
__global__ void k_FT(int64_t N, const int32_t *__restrict__ island,
                     const int32_t *__restrict__ isl_geo,
                     const int32_t *__restrict__ gisl,
                     const double *__restrict__ z, double a,
                     const double *__restrict__ x, double b,
                     double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int k = island[i];
  const double f = (k == gisl[isl_geo[k]]) ? 0.0 : z[k];
  out[i] = a * x[i] + b * f;
}

void launch_FT(const Geometry &g, const double *z, double a, const double *x,
               double b, double *out, hipStream_t s) {
  if (g.N == 0) return;
  hipLaunchKernelGGL(k_FT, dim3((unsigned)((g.N + 255) / 256)), dim3(256), 0,
                     s, g.N, g.island.p, g.isl_geo.p, g.dgisl.p, z, a, x, b,
                     out);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------------ T^T
// (T^T w)_a[m] = sum_t w_t G(x_t, c_m) (direct), in tiles: a work-group
// takes kTIsl islands (centres in LDS) and kTTgt targets (8 per thread, read
// once per tile), sums per island over its targets and writes one partial
// per (island, target chunk); a second kernel adds each island's partials
// in chunk order.  Chunk c of tile row 0 also writes the chunk's sum of w.
constexpr int kTIsl = 16;
constexpr int kTTgt = 2048;
__global__ void __launch_bounds__(256)
    k_evalT_logsrc_tile(int64_t T, const double *__restrict__ txyz,
                        const double *__restrict__ w, int M,
                        const double *__restrict__ cxyz, int nch,
                        double *__restrict__ part, double *__restrict__ wpart) {
  __shared__ double sc[kTIsl][3];
  __shared__ double red[4][kTIsl + 1];
  const int tid = threadIdx.x, ln = tid & 63, wv = tid >> 6;
  const int ch = blockIdx.x, m0 = blockIdx.y * kTIsl;
  if (tid < kTIsl * 3) {
    const int i = tid / 3, c = tid % 3;
    sc[i][c] = m0 + i < M ? cxyz[3 * (m0 + i) + c] : 0.0;
  }
  __syncthreads();
  double acc[kTIsl], ws = 0.0;
#pragma unroll
  for (int i = 0; i < kTIsl; ++i) acc[i] = 0.0;
  const int64_t t0 = (int64_t)ch * kTTgt;
  for (int j = 0; j < kTTgt / 256; ++j) {
    const int64_t t = t0 + tid + 256 * j;
    if (t >= T) break;
    const double x0 = txyz[3 * t], x1 = txyz[3 * t + 1], x2 = txyz[3 * t + 2], wt = w[t];
    ws += wt;
#pragma unroll
    for (int i = 0; i < kTIsl; ++i) {
      const double d0 = x0 - sc[i][0], d1 = x1 - sc[i][1], d2 = x2 - sc[i][2];
      acc[i] += wt * log(d0 * d0 + d1 * d1 + d2 * d2);
    }
  }
#pragma unroll
  for (int i = 0; i < kTIsl; ++i) {
    const double v = wsum(acc[i]);
    if (ln == 0) red[wv][i] = v;
  }
  {
    const double v = wsum(ws);
    if (ln == 0) red[wv][kTIsl] = v;
  }
  __syncthreads();
  if (tid < kTIsl && m0 + tid < M)
    part[(int64_t)(m0 + tid) * nch + ch] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
  if (tid == 0 && blockIdx.y == 0)
    wpart[ch] = red[0][kTIsl] + red[1][kTIsl] + red[2][kTIsl] + red[3][kTIsl];
}

__global__ void __launch_bounds__(64)
    k_evalT_logsrc_sum(int M, int nch, const double *__restrict__ part,
                       const double *__restrict__ wpart, double *__restrict__ out) {
  const int m = blockIdx.x, ln = threadIdx.x;
  double a = 0.0, ws = 0.0;
  for (int c = ln; c < nch; c += 64) {
    a += part[(int64_t)m * nch + c];
    ws += wpart[c];
  }
  a = wsum(a);
  ws = wsum(ws);
  // G = -(1/4pi) log|d|^2 + log2/4pi
  if (ln == 0) out[m] = -0.25 * kInvPi_ * a + 0.25 * kInvPi_ * kLog2_ * ws;
}

void launch_evalT_logsrc(const Geometry &g, int64_t T, const double *txyz,
                         const double *w, double *out, DBuf<double> &scratch, hipStream_t s) {
  if (g.M == 0) return;
  const int nch = (int)std::max<int64_t>(1, (T + kTTgt - 1) / kTTgt);
  const size_t need = (size_t)g.M * nch + nch;
  if (scratch.n < need) scratch.alloc(need);
  double *part = scratch.p, *wpart = part + (size_t)g.M * nch;
  if (T == 0) {
    launch_fill((int64_t)need, 0.0, scratch.p, s);
  } else {
    hipLaunchKernelGGL(k_evalT_logsrc_tile, dim3(nch, (g.M + kTIsl - 1) / kTIsl), dim3(256), 0, s,
                       T, txyz, w, g.M, g.dcenter.p, nch, part, wpart);
  }
  hipLaunchKernelGGL(k_evalT_logsrc_sum, dim3(g.M), dim3(64), 0, s, g.M, nch, part, wpart, out);
  LBS_HIP(hipGetLastError());
}

// (T^T w)_sigma[j] = 1/2 Re(i q_j F^T_j) + 1/2 gw_j W
__global__ void k_evalT_sigma(int64_t N, const double *__restrict__ FT,
                              const double *__restrict__ qfac,
                              const double *__restrict__ gw,
                              const double *__restrict__ wsum_dev,
                              double *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double qx = qfac[2 * j], qy = qfac[2 * j + 1];
  const double fx = FT[2 * j], fy = FT[2 * j + 1];
  out[j] = 0.5 * (-(qx * fy + qy * fx)) + 0.5 * gw[j] * wsum_dev[0];
}

void launch_evalT_sigma(const Geometry &g, const double *FT,
                        const double *wsum_dev, double *out, hipStream_t s) {
  if (g.N == 0) return;
  hipLaunchKernelGGL(k_evalT_sigma, dim3((unsigned)((g.N + 255) / 256)),
                     dim3(256), 0, s, g.N, FT, g.qfac.p, g.gw.p, wsum_dev,
                     out);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------------ shape VJP
// Dual numbers with three tangent directions (r, r', r'').
struct D3 {
  double v, d0, d1, d2;
};
__device__ __forceinline__ D3 dc(double v) { return D3{v, 0, 0, 0}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) {
  return D3{a.v + b.v, a.d0 + b.d0, a.d1 + b.d1, a.d2 + b.d2};
}
__device__ __forceinline__ D3 operator-(D3 a, D3 b) {
  return D3{a.v - b.v, a.d0 - b.d0, a.d1 - b.d1, a.d2 - b.d2};
}
__device__ __forceinline__ D3 operator*(D3 a, D3 b) {
  return D3{a.v * b.v, a.d0 * b.v + a.v * b.d0, a.d1 * b.v + a.v * b.d1,
            a.d2 * b.v + a.v * b.d2};
}
__device__ __forceinline__ D3 operator*(double s, D3 a) {
  return D3{s * a.v, s * a.d0, s * a.d1, s * a.d2};
}
__device__ __forceinline__ D3 inv(D3 a) {
  const double i = 1.0 / a.v, i2 = -i * i;
  return D3{i, a.d0 * i2, a.d1 * i2, a.d2 * i2};
}
__device__ __forceinline__ D3 dsin(D3 a) {
  const double s = sin(a.v), c = cos(a.v);
  return D3{s, c * a.d0, c * a.d1, c * a.d2};
}
__device__ __forceinline__ D3 dcos(D3 a) {
  const double s = sin(a.v), c = cos(a.v);
  return D3{c, -s * a.d0, -s * a.d1, -s * a.d2};
}

// Per node: cotangents of (xi, xi', xi'') of
//   Phi = w^T T x - lambda^T A x   (x = [sigma; A])
// pulled back through the curve and projection formulas to r, r', r'' and
// then to the 16 radius coefficients; summed per island (one block each).
__global__ void __launch_bounds__(256)
    k_shape_vjp(const lbs_island *__restrict__ isl,
                const int64_t *__restrict__ offs,
                const int32_t *__restrict__ isl_geo,
                const double *__restrict__ sign,
                const double *__restrict__ xi, const double *__restrict__ dxi,
                const double *__restrict__ ddxi,
                const double *__restrict__ sigma,
                const double *__restrict__ lam,
                const double *__restrict__ Fl, const double *__restrict__ dFl,
                const double *__restrict__ dFp, const double *__restrict__ Fw,
                const double *__restrict__ dFw, const double *__restrict__ LSd,
                const double *__restrict__ lam_sum,
                const double *__restrict__ a_sum,
                const double *__restrict__ w_sum,
                double *__restrict__ dcoef) {
  __shared__ double red[4][16];
  const int k = blockIdx.x;
  const int tid = threadIdx.x, ln = tid & 63, wv = tid >> 6;
  const int g = isl_geo[k];
  const lbs_island I = isl[k];
  const int64_t n = offs[k + 1] - offs[k];
  const double h = 2.0 * kPi / (double)n;
  const double c = sign[k] * h / kPi;
  const double Lam = lam_sum[g], As = a_sum[g], W = w_sum[0];
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int64_t i = offs[k] + tid; i < offs[k + 1]; i += 256) {
    const int64_t j = i - offs[k];
    const double t = (2.0 * kPi * (double)j) / (double)n;
    const cx<double> z{xi[2 * i], xi[2 * i + 1]};
    const cx<double> zd{dxi[2 * i], dxi[2 * i + 1]};
    const cx<double> zdd{ddxi[2 * i], ddxi[2 * i + 1]};
    const double sg = sigma[i], lm = lam[i];
    const cx<double> I1{0.0, 1.0};
    const double a2 = z.x * z.x + z.y * z.y, den = 1.0 / (1.0 + a2);
    const cx<double> zbar{z.x, -z.y};
    const cx<double> p = cx<double>{0.0, -c * sg} * zd;   // -i c sigma xi'
    const cx<double> izd = cinv(zd);
    // d(xi'): Kernel (A), diagonal (B), correction (C), eval (T)
    const cx<double> F{Fl[2 * i], Fl[2 * i + 1]};
    const cx<double> Fw_{Fw[2 * i], Fw[2 * i + 1]};
    cx<double> g_d = (c * sg) * (I1 * F);
    g_d = g_d + (-0.5 * c * lm * sg) * (I1 * zdd * izd * izd);
    const cx<double> corr_d = (c * sg * den) * (cx<double>{0.0, -1.0} * zbar);
    g_d = g_d + Lam * corr_d;
    const cx<double> gT_d = (0.5 * c * sg) * (I1 * Fw_) + (0.5 * W) * corr_d;
    // d(xi'')
    const cx<double> g_dd = (0.5 * c * lm * sg) * (I1 * izd);
    // d(xi)
    const cx<double> H{-dFl[2 * i], -dFl[2 * i + 1]};   // sum lam/(z-z_i)^2
    const cx<double> D{-dFp[2 * i], -dFp[2 * i + 1]};   // sum p/(z-z_j)^2
    const cx<double> HT{-dFw[2 * i], -dFw[2 * i + 1]};
    cx<double> g_z = (-lm) * D + p * H;
    const cx<double> alpha = (den * den) * zd;
    const cx<double> beta = (-den * den) * (zbar * zbar * zd);
    const cx<double> corr_z =
        (c * sg) * (cx<double>{0.0, -1.0} * (beta - cx<double>{alpha.x, -alpha.y}));
    g_z = g_z + Lam * corr_z;
    const cx<double> LS{LSd[2 * i], LSd[2 * i + 1]};
    g_z = g_z + (-kInvPi_ * lm) * (LS - (As * den) * zbar);
    const cx<double> gT_z = (0.5) * (p * HT) + (0.5 * W) * corr_z;
    // total cotangents of Phi = Phi_T - Phi_A
    const cx<double> Gz = gT_z - g_z, Gd = gT_d - g_d;
    const cx<double> Gdd = cx<double>{-g_dd.x, -g_dd.y};
    // xi, xi', xi'' as functions of (r, r', r'') at this t
    double rr = 1.0, rt = 0.0, rtt = 0.0;
    double cs[8], sn[8];
    for (int m = 1; m <= 8; ++m) {
      sincos((double)m * t, &sn[m - 1], &cs[m - 1]);
      const double am = I.coef[m - 1], bm = I.coef[7 + m];
      rr += am * cs[m - 1] + bm * sn[m - 1];
      rt += (double)m * (-am * sn[m - 1] + bm * cs[m - 1]);
      rtt += (double)(m * m) * (-am * cs[m - 1] - bm * sn[m - 1]);
    }
    const D3 R{I.r0 * rr, 1, 0, 0}, Rt{I.r0 * rt, 0, 1, 0},
        Rtt{I.r0 * rtt, 0, 0, 1};
    double st, ct;
    sincos(t, &st, &ct);
    const double *cc = I.center, *e1 = I.e1;
    const double e2[3] = {e1[1] * cc[2] - e1[2] * cc[1],
                          e1[2] * cc[0] - e1[0] * cc[2],
                          e1[0] * cc[1] - e1[1] * cc[0]};
    double u[3], v[3];
    for (int a = 0; a < 3; ++a) {
      u[a] = ct * e1[a] + st * e2[a];
      v[a] = -st * e1[a] + ct * e2[a];
    }
    const D3 sr = dsin(R), cr = dcos(R);
    D3 X[3], Xt[3], Xtt[3];
    const D3 pc = dc(-1.0) * Rt * sr, pu = Rt * cr;
    const D3 qc = dc(-1.0) * (Rtt * sr + Rt * Rt * cr);
    const D3 qu = Rtt * cr - Rt * Rt * sr - sr, qv = 2.0 * (Rt * cr);
    for (int a = 0; a < 3; ++a) {
      X[a] = cc[a] * cr + u[a] * sr;
      Xt[a] = cc[a] * pc + u[a] * pu + v[a] * sr;
      Xtt[a] = cc[a] * qc + u[a] * qu + v[a] * qv;
    }
    const D3 id = inv(dc(1.0) - X[2]);
    const D3 id2 = id * id, id3 = id2 * id;
    // xi = w id, xi' = w' id + w x3' id^2,
    // xi'' = w'' id + 2 w' x3' id^2 + w x3'' id^2 + 2 w x3'^2 id^3
    D3 zr[3][2];  // [quantity][re, im]
    for (int part = 0; part < 2; ++part) {
      const D3 w = X[part], wt = Xt[part], wtt = Xtt[part];
      zr[0][part] = w * id;
      zr[1][part] = wt * id + w * Xt[2] * id2;
      zr[2][part] = wtt * id + 2.0 * (wt * Xt[2] * id2) + w * Xtt[2] * id2 +
                    2.0 * (w * Xt[2] * Xt[2] * id3);
    }
    // dPhi/d(r, r', r'') = Re(G_z dxi + G_d dxi' + G_dd dxi'')
    auto contract = [&](int dir) {
      auto dv = [&](const D3 &x) {
        return dir == 0 ? x.d0 : (dir == 1 ? x.d1 : x.d2);
      };
      const cx<double> Gs[3] = {Gz, Gd, Gdd};
      double s = 0.0;
      for (int q = 0; q < 3; ++q) s += Gs[q].x * dv(zr[q][0]) - Gs[q].y * dv(zr[q][1]);
      return s;
    };
    const double dr = contract(0), drt = contract(1), drtt = contract(2);
    for (int m = 1; m <= 8; ++m) {
      const double fm = (double)m;
      acc[m - 1] += I.r0 * (dr * cs[m - 1] - drt * fm * sn[m - 1] -
                            drtt * fm * fm * cs[m - 1]);
      acc[7 + m] += I.r0 * (dr * sn[m - 1] + drt * fm * cs[m - 1] -
                            drtt * fm * fm * sn[m - 1]);
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double v = wsum(acc[q]);
    if (ln == 0) red[wv][q] = v;
  }
  __syncthreads();
  if (tid < 16)
    dcoef[(int64_t)k * 16 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

void launch_shape_vjp(const Geometry &g, const double *sigma,
                      const double *lam, const double *Fl, const double *dFl,
                      const double *dFp, const double *Fw, const double *dFw,
                      const double *LSd, const double *lam_sum,
                      const double *a_sum, const double *w_sum, double *dcoef,
                      hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_shape_vjp, dim3(g.M), dim3(256), 0, s, g.disl.p,
                     g.doffs.p, g.isl_geo.p, g.dsign.p, g.xi.p, g.dxi.p,
                     g.ddxi.p, sigma, lam, Fl, dFl, dFp, Fw, dFw, LSd,
                     lam_sum, a_sum, w_sum, dcoef);
  LBS_HIP(hipGetLastError());
}

// Sum_m A_m / (xi_n - eta_m) over m's geometry: derivative of the
// per-island log-source expansion (far centres, coefficients of
// k_logsrc_local for z = A) plus the near centres directly.
__global__ void k_logsrc_deriv(int64_t N, int M, const int32_t *__restrict__ island,
                               const double *__restrict__ xi,
                               const double *__restrict__ eta,
                               const double *__restrict__ rho,
                               const int32_t *__restrict__ near_ptr,
                               const int32_t *__restrict__ near_idx,
                               const double *__restrict__ A,
                               const double *__restrict__ Lc,
                               double *__restrict__ out) {
  constexpr int P = kPlog;
  constexpr int stride = 2 * (kPlog + 1) + 2;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int k = island[i];
  const double *L = Lc + (int64_t)k * stride;
  const double ir = 1.0 / rho[k];
  const cx<double> z{xi[2 * i], xi[2 * i + 1]};
  const cx<double> u{(z.x - eta[2 * k]) * ir, (z.y - eta[2 * k + 1]) * ir};
  cx<double> d = (double)P * cx<double>{L[2 * P], L[2 * P + 1]};
  for (int l = P - 1; l >= 1; --l)
    d = d * u + (double)l * cx<double>{L[2 * l], L[2 * l + 1]};
  d = ir * d;
  for (int e = near_ptr[k]; e < near_ptr[k + 1]; ++e) {
    const int m = near_idx[e];
    d = d + A[m] * cinv(cx<double>{z.x - eta[2 * m], z.y - eta[2 * m + 1]});
  }
  out[2 * i] = d.x;
  out[2 * i + 1] = d.y;
  (void)M;
}

void launch_logsrc_deriv(const Geometry &g, Workspace &ws, const double *A,
                         double *out, hipStream_t s) {
  if (g.N == 0) return;
  // expansion coefficients of the far centres for z = A
  launch_logsrc_local(g, ws, A, s);
  hipLaunchKernelGGL(k_logsrc_deriv, dim3((unsigned)((g.N + 255) / 256)),
                     dim3(256), 0, s, g.N, g.M, g.island.p, g.xi.p, g.deta.p,
                     g.drho.p, g.near_ptr.p, g.near_idx.p, A, ws.logL.p, out);
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
