// Nodes of the island curves on the sphere and their stereographic images
// (Section 3), with the per-node coefficients of the Nystrom operator
// (Section 5, eq. disc_sphere).
#include <cmath>

#include "lbs_internal.h"

namespace lbs {

// Stereographic image xi = w / d, w = x1 + i x2, d = 1 - x3, of a curve
// point and its first two parameter derivatives by the quotient rule.
__device__ __forceinline__ void stereo_derivs(
    double x0, double x1, double x2, double xt0, double xt1, double xt2,
    double xtt0, double xtt1, double xtt2, double *xi, double *dxi,
    double *ddxi) {
  const double d = 1.0 - x2, id = 1.0 / d;
  const double wr = x0, wi = x1, wtr = xt0, wti = xt1, wttr = xtt0,
               wtti = xtt1;
  const double z3t = xt2, z3tt = xtt2;
  xi[0] = wr * id;
  xi[1] = wi * id;
  const double id2 = id * id, id3 = id2 * id;
  dxi[0] = wtr * id + wr * z3t * id2;
  dxi[1] = wti * id + wi * z3t * id2;
  ddxi[0] = wttr * id + 2.0 * wtr * z3t * id2 + wr * z3tt * id2 +
            2.0 * wr * z3t * z3t * id3;
  ddxi[1] = wtti * id + 2.0 * wti * z3t * id2 + wi * z3tt * id2 +
            2.0 * wi * z3t * z3t * id3;
}

// One thread per node.  Island k's node j sits at t = 2 pi j / N_k on the
// curve x(t) = cos r c + sin r u(t), u = cos t e1 + sin t e2, e2 = e1 x c,
// r(t) = r0 (1 + sum_n a_n cos nt + b_n sin nt).  Outputs x, and
// xi = w / d, w = x1 + i x2, d = 1 - x3, with xi' and xi'' by the quotient
// rule.
__global__ void k_geometry(const lbs_island *__restrict__ isl,
                           const int64_t *__restrict__ offs,
                           const int32_t *__restrict__ island, int64_t N,
                           double *__restrict__ xyz, double *__restrict__ xi,
                           double *__restrict__ dxi,
                           double *__restrict__ ddxi) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int k = island[i];
  const int64_t j = i - offs[k], n = offs[k + 1] - offs[k];
  const double t = (2.0 * M_PI * (double)j) / (double)n;
  const lbs_island I = isl[k];
  const double c0 = I.center[0], c1 = I.center[1], c2 = I.center[2];
  const double a0 = I.e1[0], a1 = I.e1[1], a2 = I.e1[2];
  // e2 = e1 x c
  const double b0 = a1 * c2 - a2 * c1, b1 = a2 * c0 - a0 * c2,
               b2 = a0 * c1 - a1 * c0;
  double r = 1.0, rt = 0.0, rtt = 0.0;
  for (int m = 1; m <= 8; ++m) {
    double sn, cs;
    sincos((double)m * t, &sn, &cs);
    const double am = I.coef[m - 1], bm = I.coef[7 + m];
    r += am * cs + bm * sn;
    rt += (double)m * (-am * sn + bm * cs);
    rtt += (double)(m * m) * (-am * cs - bm * sn);
  }
  r *= I.r0;
  rt *= I.r0;
  rtt *= I.r0;
  double st, ct;
  sincos(t, &st, &ct);
  const double u0 = ct * a0 + st * b0, u1 = ct * a1 + st * b1,
               u2 = ct * a2 + st * b2;
  const double v0 = -st * a0 + ct * b0, v1 = -st * a1 + ct * b1,
               v2 = -st * a2 + ct * b2;
  double sr, cr;
  sincos(r, &sr, &cr);
  // x, x', x''
  const double x0 = cr * c0 + sr * u0, x1 = cr * c1 + sr * u1,
               x2 = cr * c2 + sr * u2;
  const double pc = -rt * sr, pu = rt * cr, pv = sr;
  const double xt0 = pc * c0 + pu * u0 + pv * v0,
               xt1 = pc * c1 + pu * u1 + pv * v1,
               xt2 = pc * c2 + pu * u2 + pv * v2;
  const double qc = -(rtt * sr + rt * rt * cr),
               qu = rtt * cr - rt * rt * sr - sr, qv = 2.0 * rt * cr;
  const double xtt0 = qc * c0 + qu * u0 + qv * v0,
               xtt1 = qc * c1 + qu * u1 + qv * v1,
               xtt2 = qc * c2 + qu * u2 + qv * v2;
  xyz[3 * i] = x0;
  xyz[3 * i + 1] = x1;
  xyz[3 * i + 2] = x2;
  stereo_derivs(x0, x1, x2, xt0, xt1, xt2, xtt0, xtt1, xtt2, xi + 2 * i,
                dxi + 2 * i, ddxi + 2 * i);
}

// Nodes given as samples x, x', x'' (N x 3 each): copy x, and the
// stereographic image with its derivatives.
__global__ void k_geometry_sampled(int64_t N, const double *__restrict__ x,
                                   const double *__restrict__ xt,
                                   const double *__restrict__ xtt,
                                   double *__restrict__ xyz,
                                   double *__restrict__ xi,
                                   double *__restrict__ dxi,
                                   double *__restrict__ ddxi) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double *p = x + 3 * i, *q = xt + 3 * i, *r = xtt + 3 * i;
  xyz[3 * i] = p[0];
  xyz[3 * i + 1] = p[1];
  xyz[3 * i + 2] = p[2];
  stereo_derivs(p[0], p[1], p[2], q[0], q[1], q[2], r[0], r[1], r[2],
                xi + 2 * i, dxi + 2 * i, ddxi + 2 * i);
}

void launch_geometry_sampled(int64_t N, const double *x, const double *xt,
                             const double *xtt, double *xyz, double *xi,
                             double *dxi, double *ddxi, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_geometry_sampled, dim3((unsigned)((N + 255) / 256)),
                     dim3(256), 0, s, N, x, xt, xtt, xyz, xi, dxi, ddxi);
  LBS_HIP(hipGetLastError());
}

void launch_geometry(const lbs_island *isl_dev, int M,
                     const int64_t *offs_dev, const int32_t *island_dev,
                     int64_t N, double *xyz, double *xi, double *dxi,
                     double *ddxi, hipStream_t s) {
  (void)M;
  if (N == 0) return;
  hipLaunchKernelGGL(k_geometry, dim3((unsigned)((N + 255) / 256)),
                     dim3(256), 0, s, isl_dev, offs_dev, island_dev, N, xyz,
                     xi, dxi, ddxi);
  LBS_HIP(hipGetLastError());
}

// Per-node operator coefficients with the island orientation sign s_k:
//   qfac = (s h / pi) xi'          (strength factor of the Cauchy sum)
//   tau  = -(s h / 2 pi) Im(xi''/xi')  (diagonal: self-limit of the
//                                       Cauchy term, times 2h)
//   gw   = (s h / pi) Im(conj(xi) xi' / (1 + |xi|^2))  (correction term)
//   ell  = log(1 + |xi|^2)
__global__ void k_node_coeffs(int64_t N, const int32_t *__restrict__ island,
                              const double *__restrict__ sign,
                              const int64_t *__restrict__ offs,
                              const double *__restrict__ xi,
                              const double *__restrict__ dxi,
                              const double *__restrict__ ddxi,
                              double *__restrict__ qfac,
                              double *__restrict__ tau,
                              double *__restrict__ gw,
                              double *__restrict__ ell) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int k = island[i];
  const double h = 2.0 * M_PI / (double)(offs[k + 1] - offs[k]);
  const double f = sign[k] * h / M_PI;
  const double zr = xi[2 * i], zi = xi[2 * i + 1];
  const double dr = dxi[2 * i], di = dxi[2 * i + 1];
  const double er = ddxi[2 * i], ei = ddxi[2 * i + 1];
  qfac[2 * i] = f * dr;
  qfac[2 * i + 1] = f * di;
  // Im(xi''/xi') = (ei dr - er di) / |xi'|^2
  tau[i] = -0.5 * f * (ei * dr - er * di) / (dr * dr + di * di);
  const double a2 = zr * zr + zi * zi;
  // Im(conj(xi) xi') = zr di - zi dr
  gw[i] = f * (zr * di - zi * dr) / (1.0 + a2);
  ell[i] = log1p(a2);
}

void launch_node_coeffs(int64_t N, const int32_t *island, const double *sign,
                        const int64_t *offs, const double *xi,
                        const double *dxi, const double *ddxi, double *qfac,
                        double *tau, double *gw, double *ell, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_node_coeffs, dim3((unsigned)((N + 255) / 256)),
                     dim3(256), 0, s, N, island, sign, offs, xi, dxi, ddxi,
                     qfac, tau, gw, ell);
  LBS_HIP(hipGetLastError());
}

// Node images in their own island's frame (log-source expansions): with
// a = x.e1, b = x.e2, h = x.c of island k, the stereographic projection from
// the antipode -c maps x to xi' = (a + i b)/(1 + h), the island centre to 0
// and keeps the chord identity
//   |x - y|^2 = 4 |xi'_x - xi'_y|^2 / ((1 + |xi'_x|^2)(1 + |xi'_y|^2)).
// Outputs xi' (complex) and ell' = log(1 + |xi'|^2).
__global__ void k_local_frame(int64_t N, const int32_t *__restrict__ island,
                              const lbs_island *__restrict__ isl,
                              const double *__restrict__ xyz,
                              double *__restrict__ xil,
                              double *__restrict__ elll) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const lbs_island &I = isl[island[i]];
  const double *c = I.center, *e1 = I.e1;
  const double e2[3] = {e1[1] * c[2] - e1[2] * c[1], e1[2] * c[0] - e1[0] * c[2],
                        e1[0] * c[1] - e1[1] * c[0]};
  const double x0 = xyz[3 * i], x1 = xyz[3 * i + 1], x2 = xyz[3 * i + 2];
  const double a = x0 * e1[0] + x1 * e1[1] + x2 * e1[2];
  const double b = x0 * e2[0] + x1 * e2[1] + x2 * e2[2];
  const double h = x0 * c[0] + x1 * c[1] + x2 * c[2];
  const double inv = 1.0 / (1.0 + h);
  xil[2 * i] = a * inv;
  xil[2 * i + 1] = b * inv;
  elll[i] = log1p((a * a + b * b) * inv * inv);
}

void launch_local_frame(int64_t N, const int32_t *island,
                        const lbs_island *isl, const double *xyz, double *xil,
                        double *elll, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_local_frame, dim3((unsigned)((N + 255) / 256)),
                     dim3(256), 0, s, N, island, isl, xyz, xil, elll);
  LBS_HIP(hipGetLastError());
}

__global__ void k_permute_complex(int64_t n, const int64_t *__restrict__ perm,
                                  const double *__restrict__ in,
                                  double *__restrict__ out) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t a = perm[j];
  out[2 * j] = in[2 * a];
  out[2 * j + 1] = in[2 * a + 1];
}

void launch_permute_complex(int64_t n, const int64_t *perm, const double *in,
                            double *out, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_permute_complex, dim3((unsigned)((n + 255) / 256)),
                     dim3(256), 0, s, n, perm, in, out);
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
