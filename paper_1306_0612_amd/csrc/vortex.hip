// Point vortices in the domain (Section 6, Example 2): the stream function
// is psi = psi* + sum_j Gamma_j G(x, v_j), G the generalized fundamental
// solution of Section 1.1 (eq. eqn:greens_func), and psi* solves the
// Dirichlet problem with the data g - sum_j Gamma_j G(x, v_j).  This file
// sums the vortex field directly, O(points x vortices) in FP64: the
// paper's example has 72 vortices, for which the sum costs a small
// fraction of one FMM application.
#include <cmath>

#include "lbs_internal.h"

namespace lbs {
namespace {

constexpr double kInv4Pi = 0.07957747154594766788;
constexpr double kLog2v = 0.69314718055994530942;

// out[r ldo + i] = beta in[r ldi + i] + alpha sum_j gamma[r nv + j] G(x_i, v_j)
// for the points x_i (n x 3) and vortices v_j (nv x 3); vortices staged
// through LDS in tiles of 256.  in may be null (beta ignored).
__global__ void __launch_bounds__(256)
    k_vortex_field(int64_t n, const double *__restrict__ x, int nv,
                   const double *__restrict__ v,
                   const double *__restrict__ gamma, double alpha,
                   const double *__restrict__ in, int64_t ldi, double beta,
                   double *__restrict__ out, int64_t ldo) {
  __shared__ double vx[256], vy[256], vz[256], vg[256];
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = i < n;
  double x0 = 0.0, x1 = 0.0, x2 = 0.0;
  if (live) {
    x0 = x[3 * i];
    x1 = x[3 * i + 1];
    x2 = x[3 * i + 2];
  }
  double acc = 0.0, gsum = 0.0;
  for (int j0 = 0; j0 < nv; j0 += 256) {
    __syncthreads();
    const int jl = j0 + threadIdx.x;
    if (jl < nv) {
      vx[threadIdx.x] = v[3 * jl];
      vy[threadIdx.x] = v[3 * jl + 1];
      vz[threadIdx.x] = v[3 * jl + 2];
      vg[threadIdx.x] = gamma[(int64_t)r * nv + jl];
    }
    __syncthreads();
    const int jn = min(256, nv - j0);
    for (int jj = 0; jj < jn; ++jj) {
      const double d0 = x0 - vx[jj], d1 = x1 - vy[jj], d2 = x2 - vz[jj];
      acc += vg[jj] * log(d0 * d0 + d1 * d1 + d2 * d2);
      gsum += vg[jj];
    }
  }
  if (!live) return;
  // G = -(1/4 pi) log|x - v|^2 + (1/4 pi) log 2
  const double f = kInv4Pi * (kLog2v * gsum - acc);
  const double base = in ? beta * in[(int64_t)r * ldi + i] : 0.0;
  out[(int64_t)r * ldo + i] = base + alpha * f;
}

}  // namespace

void launch_vortex_field(int64_t n, const double *x, int nv, const double *v,
                         const double *gamma, int nrhs, double alpha,
                         const double *in, int64_t ldi, double beta,
                         double *out, int64_t ldo, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_vortex_field, dim3((unsigned)((n + 255) / 256), nrhs),
                     dim3(256), 0, s, n, x, nv, v, gamma, alpha, in, ldi, beta,
                     out, ldo);
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
