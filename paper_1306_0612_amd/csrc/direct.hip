// Direct O(N^2) evaluation of the Cauchy part of the double-layer operator
// (Section 5, eq. disc_sphere) in FP64, and block reductions.
#include "cplx.h"
#include "lbs_internal.h"

namespace lbs {

constexpr int kTile = 256;

// field_i = Re sum_{j != i} p_j / (xi_i - xi_j), p_j = -i qfac_j sigma_j,
// over the nodes themselves (txi == nullptr) or separate targets.
__global__ void __launch_bounds__(kTile)
    k_direct(int64_t N, const double *__restrict__ xi,
             const double *__restrict__ qfac, const double *__restrict__ sigma,
             int64_t ldx, int64_t T, const double *__restrict__ txi,
             const uint8_t *__restrict__ pole, double *__restrict__ out,
             int64_t ldy, double scale, Assembly as) {
  __shared__ double sx[kTile], sy[kTile], px[kTile], py[kTile];
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kTile + threadIdx.x;
  const bool act = i < T;
  const double *tz = txi ? txi : xi;
  const double zx = act ? tz[2 * i] : 0.0, zy = act ? tz[2 * i + 1] : 0.0;
  const double *sg = sigma + (int64_t)r * ldx;
  double acc = 0.0;
  for (int64_t jb = 0; jb < N; jb += kTile) {
    const int64_t j = jb + threadIdx.x;
    __syncthreads();
    if (j < N) {
      sx[threadIdx.x] = xi[2 * j];
      sy[threadIdx.x] = xi[2 * j + 1];
      const double s = sg[j];
      px[threadIdx.x] = qfac[2 * j + 1] * s;   // p = -i q s
      py[threadIdx.x] = -qfac[2 * j] * s;
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(kTile, N - jb);
    for (int q = 0; q < cnt; ++q) {
      const double dx = zx - sx[q], dy = zy - sy[q];
      const double d2 = dx * dx + dy * dy;
      if (d2 > 0.0) acc += (px[q] * dx + py[q] * dy) / d2;
    }
  }
  if (!act) return;
  if (pole && pole[i]) acc = 0.0;
  double val = scale * acc;
  if (as.sigma) {
    const double s = as.sigma[(int64_t)r * as.ldx + i];
    val += (as.ident + as.tau[i]) * s + as.gamma[r];
  }
  out[(int64_t)r * ldy + i] = val;
}

void direct_apply64(int64_t N, const double *xi, const double *qfac,
                    const double *sigma, int64_t ldx, int nrhs, double *out,
                    int64_t ldy, const Assembly &as, hipStream_t s) {
  if (N == 0) return;
  dim3 grid((unsigned)((N + kTile - 1) / kTile), nrhs);
  hipLaunchKernelGGL(k_direct, grid, dim3(kTile), 0, s, N, xi, qfac, sigma,
                     ldx, N, (const double *)nullptr,
                     (const uint8_t *)nullptr, out, ldy, 1.0, as);
  LBS_HIP(hipGetLastError());
}

void direct_eval64(int64_t N, const double *xi, const double *qfac,
                   const double *sigma, int64_t ldx, int64_t T,
                   const double *txi, const uint8_t *pole, int nrhs,
                   double *out, int64_t ldy, double scale, hipStream_t s) {
  if (T == 0) return;
  dim3 grid((unsigned)((T + kTile - 1) / kTile), nrhs);
  hipLaunchKernelGGL(k_direct, grid, dim3(kTile), 0, s, N, xi, qfac, sigma,
                     ldx, T, txi, pole, out, ldy, scale, Assembly{});
  LBS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- dots
constexpr int kRedBlocks = 512;

__global__ void __launch_bounds__(256)
    k_dot_partial(int64_t n, const double *__restrict__ a, int64_t lda,
                  const double *__restrict__ b, int64_t ldb,
                  double *__restrict__ part) {
  __shared__ double red[256];
  const int r = blockIdx.y;
  const double *ar = a + (int64_t)r * lda, *br = b + (int64_t)r * ldb;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    acc += ar[i] * br[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)r * gridDim.x + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256)
    k_sum_partial(int nb, const double *__restrict__ part,
                  double *__restrict__ out) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) acc += part[(int64_t)r * nb + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = red[0];
}

void launch_dots(int64_t n, int nrhs, const double *a, int64_t lda,
                 const double *b, int64_t ldb, double *out, double *scratch,
                 hipStream_t s) {
  int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_dot_partial, dim3(nb, nrhs), dim3(256), 0, s, n, a,
                     lda, b, ldb, scratch);
  hipLaunchKernelGGL(k_sum_partial, dim3(nrhs), dim3(256), 0, s, nb, scratch,
                     out);
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
