// Close evaluation of the representation of eq. eqn:u_multi (Section 4.1)
// at targets near a curve.
//
// The trapezoidal rule that discretizes the double layer (Section 5) loses
// its accuracy within a few node spacings of a curve.  For every
// (target, island) pair in the island's close zone, island k's Cauchy part
// -s_k Re v(z), v(z) = (1/2 pi i) sum_j sigma_j a_j, a_j = h xi'_j / (xi_j - z),
// is replaced by the globally compensated rule for exterior Cauchy
// integrals (Ioakimidis, Papadakis and Perdios 1991; Helsing and Ojala
// 2008; Barnett, Wu and Veerapaneni 2015):
//
//   v(z) = sum_j V_j a_j / (sum_j a_j - 2 pi i s_k),
//
// with V the exterior boundary values of v, which the Plemelj formulas give
// as the smooth integral
//
//   V_i = (1/2 pi i) [ sum_{j != i} h (sigma_j - sigma_i) xi'_j / (xi_j - xi_i)
//                      + h sigma'_i ],
//
// sigma' the derivative of sigma's trigonometric interpolant (spectral
// differentiation matrix (1/2) (-1)^(i-j) cot((t_i - t_j)/2) for even N,
// csc for odd N).  The evaluation pass has already summed the trapezoidal
// v at every target, so each pair adds -s_k Re(v_close - v_trap).  FP64.
#include <cmath>

#include "cplx.h"
#include "lbs_internal.h"

namespace lbs {

namespace {

constexpr double kTwoPi = 6.28318530717958647692;

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// V for the nodes of island act[blockIdx.x], column blockIdx.y; node data
// staged through LDS in tiles of 256.
__global__ void __launch_bounds__(256)
    k_close_bvals(const int32_t *__restrict__ act,
                  const int64_t *__restrict__ offs,
                  const double *__restrict__ xi, const double *__restrict__ dxi,
                  const double *__restrict__ sigma, int64_t ldx,
                  double *__restrict__ V, int64_t ldv) {
  __shared__ double ts[256], tx[256], ty[256], tdx[256], tdy[256];
  const int k = act[blockIdx.x];
  const int r = blockIdx.y;
  const int64_t a = offs[k];
  const int n = (int)(offs[k + 1] - a);
  const double h = kTwoPi / (double)n;
  const double *sg = sigma + (int64_t)r * ldx + a;
  const bool even = (n & 1) == 0;
  for (int i0 = 0; i0 < n; i0 += 256) {
    const int i = i0 + threadIdx.x;
    const bool live = i < n;
    double si = 0.0, xr = 0.0, xim = 0.0;
    if (live) {
      si = sg[i];
      xr = xi[2 * (a + i)];
      xim = xi[2 * (a + i) + 1];
    }
    double ds = 0.0;           // spectral derivative of sigma at node i
    double vr = 0.0, vi = 0.0; // sum of (sigma_j - sigma_i) xi'_j / (xi_j - xi_i)
    for (int j0 = 0; j0 < n; j0 += 256) {
      __syncthreads();
      const int jl = j0 + threadIdx.x;
      if (jl < n) {
        ts[threadIdx.x] = sg[jl];
        tx[threadIdx.x] = xi[2 * (a + jl)];
        ty[threadIdx.x] = xi[2 * (a + jl) + 1];
        tdx[threadIdx.x] = dxi[2 * (a + jl)];
        tdy[threadIdx.x] = dxi[2 * (a + jl) + 1];
      }
      __syncthreads();
      if (!live) continue;
      const int jn = min(256, n - j0);
      for (int jj = 0; jj < jn; ++jj) {
        const int j = j0 + jj;
        if (j == i) continue;
        const int m = i - j;
        double sn, cs;
        sincospi((double)m / (double)n, &sn, &cs);
        const double sgn = (m & 1) ? -0.5 : 0.5;
        ds += sgn * (even ? cs / sn : 1.0 / sn) * ts[jj];
        const double dx = tx[jj] - xr, dy = ty[jj] - xim;
        const double inv = 1.0 / (dx * dx + dy * dy);
        const double ds_j = ts[jj] - si;
        // (dxi_j / (xi_j - xi_i)) = dxi_j * conj(d) / |d|^2
        const double qr = (tdx[jj] * dx + tdy[jj] * dy) * inv;
        const double qi = (tdy[jj] * dx - tdx[jj] * dy) * inv;
        vr += ds_j * qr;
        vi += ds_j * qi;
      }
    }
    if (live) {
      // V = h (sum + ds) / (2 pi i) = -i h (sum + ds) / (2 pi)
      const double sr = vr + ds, sim = vi;
      const double f = h / kTwoPi;
      V[2 * ((int64_t)r * ldv + a + i)] = f * sim;
      V[2 * ((int64_t)r * ldv + a + i) + 1] = -f * sr;
    }
  }
}

// One wave per close target: for each of its close islands the sums
// S_a = sum a_j, S_V = sum V_j a_j, S_s = sum sigma_j a_j over the island's
// nodes, then u += -s_k Re(S_V / (S_a - 2 pi i s_k) - S_s / (2 pi i)).
__global__ void __launch_bounds__(256)
    k_close_correct(int ntgt, const double *__restrict__ zt,
                    const int64_t *__restrict__ out_idx,
                    const int32_t *__restrict__ cptr,
                    const int32_t *__restrict__ cisl,
                    const int64_t *__restrict__ offs,
                    const double *__restrict__ sign,
                    const double *__restrict__ xi, const double *__restrict__ dxi,
                    const double *__restrict__ sigma, int64_t ldx,
                    const double *__restrict__ V, int64_t ldv,
                    double *__restrict__ u, int64_t ldu) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ln = threadIdx.x & 63;
  const int r = blockIdx.y;
  if (t >= ntgt) return;
  const double zx = zt[2 * t], zy = zt[2 * t + 1];
  const double *sg = sigma + (int64_t)r * ldx;
  const double *Vr = V + 2 * (int64_t)r * ldv;
  double add = 0.0;
  for (int e = cptr[t]; e < cptr[t + 1]; ++e) {
    const int k = cisl[e];
    const int64_t a = offs[k], b = offs[k + 1];
    const double h = kTwoPi / (double)(b - a);
    double sar = 0.0, sai = 0.0, svr = 0.0, svi = 0.0, ssr = 0.0, ssi = 0.0;
    for (int64_t j = a + ln; j < b; j += 64) {
      const double dx = xi[2 * j] - zx, dy = xi[2 * j + 1] - zy;
      const double inv = h / (dx * dx + dy * dy);
      // a_j = h dxi_j conj(d) / |d|^2
      const double ar = (dxi[2 * j] * dx + dxi[2 * j + 1] * dy) * inv;
      const double ai = (dxi[2 * j + 1] * dx - dxi[2 * j] * dy) * inv;
      const double vr = Vr[2 * j], vi = Vr[2 * j + 1], s = sg[j];
      sar += ar;
      sai += ai;
      svr += vr * ar - vi * ai;
      svi += vr * ai + vi * ar;
      ssr += s * ar;
      ssi += s * ai;
    }
    sar = wsum(sar);
    sai = wsum(sai);
    svr = wsum(svr);
    svi = wsum(svi);
    ssr = wsum(ssr);
    ssi = wsum(ssi);
    const double sk = sign[k];
    // v_close = S_V / (S_a - 2 pi i s_k)
    const double dr = sar, di = sai - kTwoPi * sk;
    const double dd = 1.0 / (dr * dr + di * di);
    const double vc = (svr * dr + svi * di) * dd;
    // v_trap = S_s / (2 pi i): real part Im(S_s) / (2 pi)
    const double vt = ssi / kTwoPi;
    add += -sk * (vc - vt);
  }
  if (ln == 0) u[(int64_t)r * ldu + out_idx[t]] += add;
}

}  // namespace

void launch_close_eval(const Geometry &g, const ClosePlan &cp, int nrhs,
                       const double *sigma, int64_t ldx, double *V,
                       double *u, int64_t ldu, hipStream_t s) {
  if (cp.n_tgt == 0) return;
  hipLaunchKernelGGL(k_close_bvals, dim3(cp.n_act, nrhs), dim3(256), 0, s,
                     cp.act.p, g.doffs.p, g.xi.p, g.dxi.p, sigma, ldx, V, g.N);
  hipLaunchKernelGGL(k_close_correct, dim3((cp.n_tgt + 3) / 4, nrhs),
                     dim3(256), 0, s, cp.n_tgt, cp.z.p, cp.out.p, cp.ptr.p,
                     cp.isl.p, g.doffs.p, g.dsign.p, g.xi.p, g.dxi.p, sigma,
                     ldx, V, g.N, u, ldu);
  LBS_HIP(hipGetLastError());
}


// ----------------------------------------------------------- close pairs
// The (target, island) pairs of an evaluation whose island's close zone
// holds the target, found on the device: islands are binned by the cell of
// their centre in a uniform 3D grid (cell side >= every zone's chord
// radius, keys (geometry << 48 | ix << 32 | iy << 16 | iz) sorted), and a
// target looks at the 27 cells around its own.
namespace {

__device__ __forceinline__ int64_t find_cell(const uint64_t *keys, int nk, uint64_t key) {
  int a = 0, b = nk;
  while (a < b) {
    const int m = (a + b) >> 1;
    if (keys[m] < key) a = m + 1;
    else b = m;
  }
  return (a < nk && keys[a] == key) ? a : -1;
}

// The islands whose zone holds target position q, ascending in out[0:n]
// (n <= kCloseMax, else the count only); returns the count.
constexpr int kCloseMax = 32;
template <bool FILL>
__device__ int close_islands(const double *x, int geo, const CloseGridView &G, int *out) {
  int n = 0;
  const int64_t cx = (int64_t)floor((x[0] + 1.0) / G.cell);
  const int64_t cy = (int64_t)floor((x[1] + 1.0) / G.cell);
  const int64_t cz = (int64_t)floor((x[2] + 1.0) / G.cell);
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        const int64_t ix = cx + dx, iy = cy + dy, iz = cz + dz;
        if (ix < 0 || iy < 0 || iz < 0) continue;
        const uint64_t key = ((uint64_t)geo << 48) | ((uint64_t)ix << 32) | ((uint64_t)iy << 16) |
                             (uint64_t)iz;
        const int64_t c = find_cell(G.keys, G.nkeys, key);
        if (c < 0) continue;
        for (int e = G.ptr[c]; e < G.ptr[c + 1]; ++e) {
          const int k = G.isl[e];
          const double *ck = G.center + 3 * k;
          if (x[0] * ck[0] + x[1] * ck[1] + x[2] * ck[2] > G.zone_cos[k]) {
            if (FILL && n < kCloseMax) {  // insertion in ascending order
              int j = n;
              while (j > 0 && out[j - 1] > k) {
                out[j] = out[j - 1];
                --j;
              }
              out[j] = k;
            }
            ++n;
          }
        }
      }
  return n;
}

__global__ void __launch_bounds__(256)
    k_close_count(int64_t n, const int64_t *__restrict__ idx, const double *__restrict__ txyz,
                  const int32_t *__restrict__ tgeo, CloseGridView G, int32_t *__restrict__ cnt) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const int64_t t = idx[q];
  cnt[q] = close_islands<false>(txyz + 3 * t, tgeo[t], G, nullptr);
}

// close target q (pos[q] >= 0): its image, output row and islands
__global__ void __launch_bounds__(256)
    k_close_fill(int64_t n, const int64_t *__restrict__ idx, const double *__restrict__ txyz,
                 const int32_t *__restrict__ tgeo, const double *__restrict__ tx,
                 const double *__restrict__ ty, const int32_t *__restrict__ pos,
                 const int32_t *__restrict__ ptr, CloseGridView G, double *__restrict__ z,
                 int64_t *__restrict__ out, int32_t *__restrict__ isl,
                 uint8_t *__restrict__ used) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n || pos[q] < 0) return;
  const int64_t t = idx[q];
  int list[kCloseMax];
  const int m = close_islands<true>(txyz + 3 * t, tgeo[t], G, list);
  const int p = pos[q];
  z[2 * p] = tx[q];
  z[2 * p + 1] = ty[q];
  out[p] = t;
  for (int i = 0; i < m && i < kCloseMax; ++i) {
    isl[ptr[p] + i] = list[i];
    used[list[i]] = 1;  // every writer stores the same value
  }
}

}  // namespace

void launch_close_count(int64_t n, const int64_t *idx, const double *txyz, const int32_t *tgeo,
                        const CloseGridView &G, int32_t *cnt, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_close_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx,
                     txyz, tgeo, G, cnt);
  LBS_HIP(hipGetLastError());
}

void launch_close_fill(int64_t n, const int64_t *idx, const double *txyz, const int32_t *tgeo,
                       const double *tx, const double *ty, const int32_t *pos, const int32_t *ptr,
                       const CloseGridView &G, double *z, int64_t *out, int32_t *isl,
                       uint8_t *used, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_close_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx,
                     txyz, tgeo, tx, ty, pos, ptr, G, z, out, isl, used);
  LBS_HIP(hipGetLastError());
}

int close_list_max() { return kCloseMax; }

}  // namespace lbs
