// Log-source and constraint rows of the block system (Section 5,
// eqs. matrix_eqns and matrix_eqns_c), the Schur complement of the block
// preconditioner, and the GMRES building blocks.  All FP64.
#include <cmath>

#include "cplx.h"
#include "lbs_internal.h"

namespace lbs {

constexpr double kInvPi = 0.31830988618379067154;
constexpr double kLog2 = 0.69314718055994530942;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------ log sources
// (E z)_i = sum_m 2 z_m G(x_i, c_m),  G(x, y) = -(1/2pi) log|x - y| + log2/4pi
// (Section 1.1, eq. eqn:greens_func).  For target island k and a centre m
// with |eta_m - eta_k| > 3 rho_k ("far"), the planar identity
//   log|x - c| = log 2 + log|xi - eta| - ell(xi)/2 - ell(eta)/2,
//   ell(z) = log(1 + |z|^2),
// and the series log(1 - u q) = -sum_l (u q)^l / l with u = (xi - eta_k)/rho_k,
// q = rho_k / (eta_m - eta_k), |u| <= 1, |q| < 1/3 give
//   sum_far z_m log|x_i - c_m| = Re sum_l L_k[l] u^l - Z_k ell_i / 2,
//   L_k[0] = sum_far z_m (log 2 + log|eta_k - eta_m| - ell(eta_m)/2),
//   L_k[l] = -sum_far z_m q^l / l,   Z_k = sum_far z_m.
// Near centres (own centre included) are summed directly in 3D.
constexpr int kLogStride = 2 * (kPlog + 1) + 2;

__device__ __forceinline__ bool in_sorted(const int32_t *a, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < n && a[lo] == x;
}

__global__ void __launch_bounds__(256)
    k_logsrc_local(int M, const double *__restrict__ eta,
                   const double *__restrict__ rho,
                   const double *__restrict__ ellc,
                   const int32_t *__restrict__ near_ptr,
                   const int32_t *__restrict__ near_idx,
                   const double *__restrict__ z, int64_t ldz,
                   double *__restrict__ Lout) {
  constexpr int P = kPlog;
  __shared__ double red[4][2 * (P + 1) + 2];
  const int k = blockIdx.x, r = blockIdx.y;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const double ex = eta[2 * k], ey = eta[2 * k + 1], rk = rho[k];
  const int32_t *nl = near_idx + near_ptr[k];
  const int nn = near_ptr[k + 1] - near_ptr[k];
  const double *zr = z + (int64_t)r * ldz;
  cx<double> acc[P];
#pragma unroll
  for (int l = 0; l < P; ++l) acc[l] = cx<double>{0.0, 0.0};
  double a0 = 0.0, zf = 0.0, zt = 0.0;
  for (int m = tid; m < M; m += 256) {
    const double zm = zr[m];
    zt += zm;
    if (in_sorted(nl, nn, m)) continue;
    const double dx = eta[2 * m] - ex, dy = eta[2 * m + 1] - ey;
    const double d2 = dx * dx + dy * dy;
    zf += zm;
    a0 += zm * (kLog2 + 0.5 * log(d2) - 0.5 * ellc[m]);
    const double f = rk / d2;
    const cx<double> q{dx * f, -dy * f};   // rho_k / (eta_m - eta_k)
    cx<double> pw = zm * q;
#pragma unroll
    for (int l = 0; l < P; ++l) {
      acc[l] = acc[l] + pw;
      pw = pw * q;
    }
  }
  // reduce: wave sums, then across the 4 waves
  auto put = [&](int slot, double v) {
    v = wave_sum(v);
    if (ln == 0) red[wv][slot] = v;
  };
  put(0, a0);
  put(1, 0.0);
#pragma unroll
  for (int l = 0; l < P; ++l) {
    put(2 * (l + 1), acc[l].x);
    put(2 * (l + 1) + 1, acc[l].y);
  }
  put(2 * (P + 1), zf);
  put(2 * (P + 1) + 1, zt);
  __syncthreads();
  double *out = Lout + ((int64_t)r * M + k) * kLogStride;
  for (int s = tid; s < kLogStride; s += 256) {
    double v = red[0][s] + red[1][s] + red[2][s] + red[3][s];
    if (s >= 2 && s < 2 * (P + 1)) v *= -1.0 / (double)(s / 2);  // -q^l / l
    out[s] = v;
  }
}

__global__ void k_logsrc_node(int64_t N, int M, const int32_t *__restrict__ island,
                              const double *__restrict__ xi,
                              const double *__restrict__ xyz,
                              const double *__restrict__ ell,
                              const double *__restrict__ eta,
                              const double *__restrict__ rho,
                              const double *__restrict__ cxyz,
                              const int32_t *__restrict__ near_ptr,
                              const int32_t *__restrict__ near_idx,
                              const double *__restrict__ z, int64_t ldz,
                              const double *__restrict__ Lc,
                              double *__restrict__ out, int64_t ldo,
                              double alpha) {
  constexpr int P = kPlog;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  const int k = island[i];
  const double *L = Lc + ((int64_t)r * M + k) * kLogStride;
  const double ir = 1.0 / rho[k];
  const cx<double> u{(xi[2 * i] - eta[2 * k]) * ir,
                     (xi[2 * i + 1] - eta[2 * k + 1]) * ir};
  cx<double> s{L[2 * P], L[2 * P + 1]};
  for (int l = P - 1; l >= 0; --l) s = s * u + cx<double>{L[2 * l], L[2 * l + 1]};
  double tot = s.x - 0.5 * L[2 * (P + 1)] * ell[i];
  const double x0 = xyz[3 * i], x1 = xyz[3 * i + 1], x2 = xyz[3 * i + 2];
  const double *zr = z + (int64_t)r * ldz;
  for (int e = near_ptr[k]; e < near_ptr[k + 1]; ++e) {
    const int m = near_idx[e];
    const double d0 = x0 - cxyz[3 * m], d1 = x1 - cxyz[3 * m + 1],
                 d2 = x2 - cxyz[3 * m + 2];
    tot += zr[m] * 0.5 * log(d0 * d0 + d1 * d1 + d2 * d2);
  }
  const double ez = -kInvPi * tot + kLog2 * 0.5 * kInvPi * L[2 * (P + 1) + 1];
  out[(int64_t)r * ldo + i] += alpha * ez;
}

void launch_logsrc_apply(const Geometry &g, Workspace &ws, const double *z,
                         int64_t ldz, int nrhs, double *out, int64_t ldo,
                         double alpha, hipStream_t s) {
  if (g.M == 0 || g.N == 0) return;
  hipLaunchKernelGGL(k_logsrc_local, dim3(g.M, nrhs), dim3(256), 0, s, g.M,
                     g.deta.p, g.drho.p, g.dellc.p, g.near_ptr.p,
                     g.near_idx.p, z, ldz, ws.logL.p);
  hipLaunchKernelGGL(k_logsrc_node, dim3((unsigned)((g.N + 255) / 256), nrhs),
                     dim3(256), 0, s, g.N, g.M, g.island.p, g.xi.p, g.xyz.p,
                     g.ell.p, g.deta.p, g.drho.p, g.dcenter.p, g.near_ptr.p,
                     g.near_idx.p, z, ldz, ws.logL.p, out, ldo, alpha);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------ constraint rows
// out[k] = sum over island k of y (k >= 1); out[0] = a0 (row of sum(A)).
__global__ void __launch_bounds__(256)
    k_island_sums(int M, const int64_t *__restrict__ offs,
                  const double *__restrict__ y, int64_t ldy,
                  const double *__restrict__ arow, int64_t lda,
                  double *__restrict__ out, int64_t ldo) {
  __shared__ double red[4];
  const int k = blockIdx.x, r = blockIdx.y;
  const double *yr = y + (int64_t)r * ldy;
  double acc = 0.0;
  if (k == 0) {
    if (arow)
      for (int m = threadIdx.x; m < M; m += 256) acc += arow[(int64_t)r * lda + m];
  } else {
    for (int64_t i = offs[k] + threadIdx.x; i < offs[k + 1]; i += 256)
      acc += yr[i];
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    out[(int64_t)r * ldo + k] = red[0] + red[1] + red[2] + red[3];
}

void launch_island_sums(const Geometry &g, const double *y, int64_t ldy,
                        int nrhs, double *out, int64_t ldo, hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_island_sums, dim3(g.M, nrhs), dim3(256), 0, s, g.M,
                     g.doffs.p, y, ldy, (const double *)nullptr, (int64_t)0,
                     out, ldo);
  LBS_HIP(hipGetLastError());
}

void launch_constraint_rows(const Geometry &g, const double *sigma,
                            int64_t ldx, const double *A, int64_t lda,
                            int nrhs, double *out, int64_t ldo,
                            hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_island_sums, dim3(g.M, nrhs), dim3(256), 0, s, g.M,
                     g.doffs.p, sigma, ldx, A, lda, out, ldo);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------ Schur complement
// S = D - F E: row 0 is (1, ..., 1) (sum(A) = 0 has no sigma part); row
// k >= 1 is -sum_{i in island k} 2 G(x_i, c_m).
__global__ void k_build_schur(int M, const int64_t *__restrict__ offs,
                              const double *__restrict__ xyz,
                              const double *__restrict__ cxyz,
                              double *__restrict__ S) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (m >= M) return;
  if (k == 0) {
    S[m] = 1.0;
    return;
  }
  const double c0 = cxyz[3 * m], c1 = cxyz[3 * m + 1], c2 = cxyz[3 * m + 2];
  double acc = 0.0;
  int64_t n = offs[k + 1] - offs[k];
  for (int64_t i = offs[k]; i < offs[k + 1]; ++i) {
    const double d0 = xyz[3 * i] - c0, d1 = xyz[3 * i + 1] - c1,
                 d2 = xyz[3 * i + 2] - c2;
    acc += log(d0 * d0 + d1 * d1 + d2 * d2);
  }
  // 2 G = -(1/2pi) log|d|^2 + log2 / 2pi
  const double sum2g = -0.5 * kInvPi * acc + 0.5 * kInvPi * kLog2 * (double)n;
  S[(int64_t)k * M + m] = -sum2g;
}

void launch_build_schur(const Geometry &g, double *S, hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_build_schur, dim3((g.M + 255) / 256, g.M), dim3(256),
                     0, s, g.M, g.doffs.p, g.xyz.p, g.dcenter.p, S);
  LBS_HIP(hipGetLastError());
}

// Gauss-Jordan elimination with partial pivoting on [S | I].
__global__ void __launch_bounds__(256)
    k_gj_pivot(int M, int c, const double *__restrict__ A, int *__restrict__ piv) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  double best = -1.0;
  int at = c;
  for (int r = c + threadIdx.x; r < M; r += 256) {
    double v = fabs(A[(int64_t)r * M + c]);
    if (v > best) { best = v; at = r; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = at;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      double o = bv[threadIdx.x + w];
      int oi = bi[threadIdx.x + w];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) piv[0] = bi[0];
}

__global__ void k_gj_swap_scale(int M, int c, double *__restrict__ A,
                                double *__restrict__ B,
                                const int *__restrict__ piv,
                                double *__restrict__ f) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = piv[0];
  if (j < M) {
    if (p != c) {
      double t = A[(int64_t)c * M + j];
      A[(int64_t)c * M + j] = A[(int64_t)p * M + j];
      A[(int64_t)p * M + j] = t;
      t = B[(int64_t)c * M + j];
      B[(int64_t)c * M + j] = B[(int64_t)p * M + j];
      B[(int64_t)p * M + j] = t;
    }
  }
}

__global__ void k_gj_norm(int M, int c, double *__restrict__ A,
                          double *__restrict__ B, double *__restrict__ f) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const double inv = 1.0 / A[(int64_t)c * M + c];
  __syncthreads();
  if (j < M) {
    // factors of the other rows (column c before elimination)
    f[j] = (j == c) ? 0.0 : A[(int64_t)j * M + c];
  }
  if (j < M && j != c) {
    A[(int64_t)c * M + j] *= inv;
  }
  if (j < M) B[(int64_t)c * M + j] *= inv;
}

__global__ void k_gj_fix_pivot(int M, int c, double *__restrict__ A) {
  A[(int64_t)c * M + c] = 1.0;
}

__global__ void k_gj_eliminate(int M, int c, double *__restrict__ A,
                               double *__restrict__ B,
                               const double *__restrict__ f) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= M || r == c) return;
  const double fr = f[r];
  if (fr == 0.0) return;
  if (j > c) A[(int64_t)r * M + j] -= fr * A[(int64_t)c * M + j];
  B[(int64_t)r * M + j] -= fr * B[(int64_t)c * M + j];
}

__global__ void k_gj_zero_col(int M, int c, double *__restrict__ A) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < M && r != c) A[(int64_t)r * M + c] = 0.0;
}

__global__ void k_identity(int M, double *__restrict__ B) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (j < M) B[(int64_t)r * M + j] = (r == j) ? 1.0 : 0.0;
}

void invert_dense(int M, double *S, double *Sinv, hipStream_t s) {
  if (M == 0) return;
  DBuf<int> piv;
  piv.alloc(1);
  DBuf<double> f;
  f.alloc(M);
  const unsigned nb = (M + 255) / 256;
  hipLaunchKernelGGL(k_identity, dim3(nb, M), dim3(256), 0, s, M, Sinv);
  for (int c = 0; c < M; ++c) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, M, c, S, piv.p);
    hipLaunchKernelGGL(k_gj_swap_scale, dim3(nb), dim3(256), 0, s, M, c, S,
                       Sinv, piv.p, f.p);
    // f must be read from the swapped matrix before the pivot row is scaled:
    // k_gj_norm reads column c of every row (pivot row excluded) and scales
    // the pivot row except its diagonal entry, which k_gj_fix_pivot sets.
    hipLaunchKernelGGL(k_gj_norm, dim3(nb), dim3(256), 0, s, M, c, S, Sinv,
                       f.p);
    hipLaunchKernelGGL(k_gj_fix_pivot, dim3(1), dim3(1), 0, s, M, c, S);
    hipLaunchKernelGGL(k_gj_eliminate, dim3(nb, M), dim3(256), 0, s, M, c, S,
                       Sinv, f.p);
    hipLaunchKernelGGL(k_gj_zero_col, dim3(nb), dim3(256), 0, s, M, c, S);
  }
  LBS_HIP(hipGetLastError());
  LBS_HIP(hipStreamSynchronize(s));
}

// y = alpha A x (A: M x M row-major), one wave per row.
__global__ void __launch_bounds__(256)
    k_gemv(int M, const double *__restrict__ A, const double *__restrict__ x,
           int64_t ldx, double *__restrict__ y, int64_t ldy, double alpha) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ln = threadIdx.x & 63;
  const int r = blockIdx.y;
  if (row >= M) return;
  const double *xr = x + (int64_t)r * ldx;
  const double *a = A + (int64_t)row * M;
  double acc = 0.0;
  for (int j = ln; j < M; j += 64) acc += a[j] * xr[j];
  acc = wave_sum(acc);
  if (ln == 0) y[(int64_t)r * ldy + row] = alpha * acc;
}

void launch_gemv(int M, const double *A, const double *x, int64_t ldx,
                 int nrhs, double *y, int64_t ldy, double alpha,
                 hipStream_t s) {
  if (M == 0) return;
  hipLaunchKernelGGL(k_gemv, dim3((M + 3) / 4, nrhs), dim3(256), 0, s, M, A,
                     x, ldx, y, ldy, alpha);
  LBS_HIP(hipGetLastError());
}

// u_t += sum_m A_m G(x_t, c_m) + add[r]  (direct, one thread per target)
__global__ void __launch_bounds__(256)
    k_eval_logsrc(int64_t T, const double *__restrict__ txyz, int M,
                  const double *__restrict__ cxyz,
                  const double *__restrict__ A, int64_t lda,
                  const double *__restrict__ add, double *__restrict__ u,
                  int64_t ldu) {
  __shared__ double c[256][3];
  __shared__ double a[256];
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  const bool act = t < T;
  const double x0 = act ? txyz[3 * t] : 0.0, x1 = act ? txyz[3 * t + 1] : 0.0,
               x2 = act ? txyz[3 * t + 2] : 0.0;
  double acc = 0.0, asum = 0.0;
  for (int mb = 0; mb < M; mb += 256) {
    __syncthreads();
    const int m = mb + threadIdx.x;
    if (m < M) {
      c[threadIdx.x][0] = cxyz[3 * m];
      c[threadIdx.x][1] = cxyz[3 * m + 1];
      c[threadIdx.x][2] = cxyz[3 * m + 2];
      a[threadIdx.x] = A[(int64_t)r * lda + m];
    }
    __syncthreads();
    const int cnt = min(256, M - mb);
    for (int q = 0; q < cnt; ++q) {
      const double d0 = x0 - c[q][0], d1 = x1 - c[q][1], d2 = x2 - c[q][2];
      acc += a[q] * log(d0 * d0 + d1 * d1 + d2 * d2);
      asum += a[q];
    }
  }
  if (!act) return;
  // G = -(1/4pi) log|d|^2 + log2/4pi
  u[(int64_t)r * ldu + t] += -0.25 * kInvPi * acc + 0.25 * kInvPi * kLog2 * asum +
                             add[r];
}

void launch_eval_logsrc(int64_t T, const double *txyz, int M,
                        const double *cxyz, const double *A, int64_t lda,
                        int nrhs, const double *add, double *u, int64_t ldu,
                        hipStream_t s) {
  if (T == 0) return;
  hipLaunchKernelGGL(k_eval_logsrc, dim3((unsigned)((T + 255) / 256), nrhs),
                     dim3(256), 0, s, T, txyz, M, cxyz, A, lda, add, u, ldu);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------------ GMRES parts
// w -= sum_{j < k1} h[j] V_j ; optionally hacc[j] += h[j]
__global__ void k_maxpy(int64_t n, int k1, const double *__restrict__ V,
                        int64_t ldv, const double *__restrict__ h,
                        double *__restrict__ w, double *__restrict__ hacc) {
  __shared__ double hs[128];
  for (int j = threadIdx.x; j < k1; j += blockDim.x) hs[j] = h[j];
  __syncthreads();
  if (hacc && blockIdx.x == 0)
    for (int j = threadIdx.x; j < k1; j += blockDim.x) hacc[j] += hs[j];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < k1; ++j) acc += hs[j] * V[(int64_t)j * ldv + i];
  w[i] -= acc;
}

void launch_maxpy(int64_t n, int k1, const double *V, int64_t ldv,
                  const double *h, double *w, double *hacc, hipStream_t s) {
  hipLaunchKernelGGL(k_maxpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     s, n, k1, V, ldv, h, w, hacc);
  LBS_HIP(hipGetLastError());
}

// x += sum_{j < k} y[j] V_j
__global__ void k_update(int64_t n, int k, const double *__restrict__ V,
                         int64_t ldv, const double *__restrict__ y,
                         double *__restrict__ x) {
  __shared__ double ys[128];
  for (int j = threadIdx.x; j < k; j += blockDim.x) ys[j] = y[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc += ys[j] * V[(int64_t)j * ldv + i];
  x[i] += acc;
}

void launch_update(int64_t n, int k, const double *V, int64_t ldv,
                   const double *y, double *x, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     s, n, k, V, ldv, y, x);
  LBS_HIP(hipGetLastError());
}

// v = w / sqrt(nrm2) and hout = sqrt(nrm2) (v = 0 on breakdown)
__global__ void k_normalize(int64_t n, const double *__restrict__ nrm2,
                            const double *__restrict__ w,
                            double *__restrict__ v, double *__restrict__ hout) {
  const double s = sqrt(fmax(nrm2[0], 0.0));
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && hout) hout[0] = s;
  if (i < n) v[i] = s > 0.0 ? w[i] / s : 0.0;
}

void launch_normalize(int64_t n, const double *nrm2, const double *w,
                      double *v, double *hout, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, dim3((unsigned)((n + 255) / 256)), dim3(256),
                     0, s, n, nrm2, w, v, hout);
  LBS_HIP(hipGetLastError());
}

// y = a x + b y
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x,
                        double b, double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

void launch_axpby(int64_t n, double a, const double *x, double b, double *y,
                  hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     s, n, a, x, b, y);
  LBS_HIP(hipGetLastError());
}

__global__ void k_fill(int64_t n, double v, double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

void launch_fill(int64_t n, double v, double *x, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     s, n, v, x);
  LBS_HIP(hipGetLastError());
}

// Givens step k of GMRES(m): H is column-major with leading dimension
// m + 1; column k holds h_{0..k+1, k}.  Applies the previous rotations,
// forms rotation k, updates g and writes |g_{k+1}| to resid.
__global__ void k_givens(int k, int m, double *__restrict__ H,
                         double *__restrict__ cs, double *__restrict__ sn,
                         double *__restrict__ g, double *__restrict__ resid) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double *h = H + (int64_t)k * (m + 1);
  for (int j = 0; j < k; ++j) {
    const double t = cs[j] * h[j] + sn[j] * h[j + 1];
    h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1];
    h[j] = t;
  }
  const double a = h[k], b = h[k + 1];
  const double den = hypot(a, b);
  double c = 1.0, s = 0.0;
  if (den > 0.0) {
    c = a / den;
    s = b / den;
  }
  cs[k] = c;
  sn[k] = s;
  h[k] = den;
  h[k + 1] = 0.0;
  g[k + 1] = -s * g[k];
  g[k] = c * g[k];
  resid[0] = fabs(g[k + 1]);
}

void launch_givens(int k, int m, double *H, double *cs, double *sn,
                   double *gvec, double *resid, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, k, m, H, cs, sn, gvec,
                     resid);
  LBS_HIP(hipGetLastError());
}

// Solve the k x k upper triangle of H for y (H y = g).
__global__ void k_backsolve(int k, int m, const double *__restrict__ H,
                            const double *__restrict__ g,
                            double *__restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double acc = g[i];
    for (int j = i + 1; j < k; ++j) acc -= H[(int64_t)j * (m + 1) + i] * y[j];
    const double d = H[(int64_t)i * (m + 1) + i];
    y[i] = d != 0.0 ? acc / d : 0.0;
  }
}

void launch_backsolve(int k, int m, const double *H, const double *gvec,
                      double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, s, k, m, H, gvec, y);
  LBS_HIP(hipGetLastError());
}

// g = (beta, 0, ..., 0) with beta = sqrt(nrm2)
__global__ void k_init_g(int m, const double *__restrict__ nrm2,
                         double *__restrict__ g) {
  const int j = threadIdx.x;
  if (j <= m) g[j] = (j == 0) ? sqrt(fmax(nrm2[0], 0.0)) : 0.0;
}

void launch_init_g(int m, const double *nrm2, double *g, hipStream_t s) {
  hipLaunchKernelGGL(k_init_g, dim3(1), dim3(128), 0, s, m, nrm2, g);
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
