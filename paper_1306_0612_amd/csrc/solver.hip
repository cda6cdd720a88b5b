// Log-source and constraint rows of the block system (Section 5,
// eqs. matrix_eqns and matrix_eqns_c), the Schur complement of the block
// preconditioner, and the GMRES building blocks.  All FP64.
//
// A handle may hold G independent geometries: nodes and islands are
// numbered geometry-major, and every operator below acts on each geometry
// separately (a block-diagonal system).
#include <cmath>
#include <type_traits>

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
// (Section 1.1, eq. eqn:greens_func), m over the islands of i's geometry.
//
// Expansions in each island's own frame.  For target island k with centre c,
// frame (e1, e2 = e1 x c) and node images xi' = (x.e1 + i x.e2)/(1 + x.c)
// (the stereographic projection from -c, which sends c to 0), a centre m has
// eta' = (a + i b)/(1 + h), a = c_m.e1, b = c_m.e2, h = c_m.c, and the chord
// identity gives
//   log|x_i - c_m| = log|c - c_m| + Re log(1 - u q) - ell'_i / 2,
//   u = xi'_i / rho'_k,  q = rho'_k / eta' = 2 rho'_k (a - i b) / |c - c_m|^2,
// ell'_i = log(1 + |xi'_i|^2), rho'_k = max |xi'| over the island.  For
// |eta'| > 3 rho'_k ("far") the series log(1 - u q) = -sum_l (u q)^l / l
// converges with |u q| < 1/3, so
//   sum_far z_m log|x_i - c_m| = Re sum_l L_k[l] u^l - Z_k ell'_i / 2,
//   L_k[0] = sum_far z_m log|c - c_m|,  L_k[l] = -sum_far z_m q^l / l,
//   Z_k = sum_far z_m.
// Near centres (own centre included) are summed directly in 3D.  In this
// frame an island is a disk of radius about tan(r/2) at the origin, so the
// near lists hold only the neighbouring islands wherever the island lies
// on the sphere.
//
// kPlog = 30 terms ((1/3)^30 ~ 5e-15), in FP64: the block preconditioner
// multiplies E by z = S^-1 (...), whose entries are large and cancel in
// E z, so FP32 sums here perturb P^-1 well beyond FP32 rounding (measured:
// more refinement steps).  Per island the coefficients are stored as
// [L0, 0, L1, ..., LP, Z_far, Z_total] (2 (P + 1) + 2 doubles).
template <int P>
constexpr int log_stride() { return 2 * (P + 1) + 2; }

__device__ __forceinline__ bool in_sorted(const int32_t *a, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < n && a[lo] == x;
}

// L_k for every island k from its far list (Geometry::far_*: the pairs,
// q = rho'_k / eta' and log|c_k - c_m|, sorted by |q|, largest first).
// One wave per (island, half of the series): half h sums the terms
// h P/2 + 1 .. (h + 1) P/2 of every chunk whose |q| needs them, starting
// from z q^(h P/2 + 1) by repeated squaring; half 0 also forms L0, Z_far
// and Z_total.  A chunk needs the terms that keep the series tail below
// the bound of the full P terms at the far limit |q| = 1/3.
__global__ void __launch_bounds__(64)
    k_logsrc_local(int M, const int32_t *__restrict__ isl_geo,
                   const int32_t *__restrict__ gisl,
                   const int64_t *__restrict__ far_ptr,
                   const int64_t *__restrict__ far_cptr,
                   const int32_t *__restrict__ far_nt,
                   const int32_t *__restrict__ far_idx,
                   const double *__restrict__ far_q,
                   const double *__restrict__ far_h,
                   const double *__restrict__ z, int64_t ldz,
                   double *__restrict__ Lout) {
  constexpr int P = kPlog, PH = P / 2, stride = log_stride<P>();
  static_assert(2 * PH == P, "the series splits in two halves");
  const int k = blockIdx.x, r = blockIdx.y, h = blockIdx.z;
  const int ln = threadIdx.x;
  const int l0 = h * PH;  // this half: powers l0 + 1 .. l0 + PH
  const double *zr = z + (int64_t)r * ldz;
  double *out = Lout + ((int64_t)r * M + k) * stride;
  const int64_t e0 = far_ptr[k], e1 = far_ptr[k + 1];
  const int32_t *ntc = far_nt + far_cptr[k];
  if (h > 0 && (e1 == e0 || ntc[0] <= l0)) {  // no chunk reaches this half
    if (ln < PH) {
      out[2 * (l0 + ln + 1)] = 0.0;
      out[2 * (l0 + ln + 1) + 1] = 0.0;
    }
    return;
  }
  cx<double> acc[PH];
#pragma unroll
  for (int l = 0; l < PH; ++l) acc[l] = cx<double>{0.0, 0.0};
  double a0 = 0.0, zf = 0.0;
  const int nch = (int)((e1 - e0 + kLogChunk - 1) / kLogChunk);
  // U chunks per step, their loads issued before any of them is used (4:
  // few enough registers for four waves per SIMD)
  constexpr int U = 4;
  for (int c0 = 0; c0 < nch; c0 += U) {
    int nt[U];
    cx<double> q[U];
    double hh[U], zm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // indices clamped into the list (nch >= 1 here); entries past the
      // end or of chunks without terms for this half get zero weight
      const int64_t j = e0 + (int64_t)(c0 + u) * kLogChunk + ln;
      const int64_t jc = j < e1 ? j : e1 - 1;
      const int nc = ntc[c0 + u < nch ? c0 + u : nch - 1] - l0;
      nt[u] = c0 + u < nch ? nc : 0;  // wave-uniform
      const bool ok = nt[u] > 0 && j < e1;
      const int mi = far_idx[jc];
      const cx<double> qi{far_q[2 * jc], far_q[2 * jc + 1]};
      const double hi = far_h[jc], zi = zr[mi];
      q[u] = ok ? qi : cx<double>{0.0, 0.0};
      hh[u] = ok ? hi : 0.0;
      zm[u] = ok ? zi : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (nt[u] <= 0) continue;  // wave-uniform
      cx<double> pw = zm[u] * q[u];
      if (h == 0) {
        zf += zm[u];
        a0 += zm[u] * hh[u];
      } else {
        cx<double> base = q[u];
        for (int p = l0; p > 0; p >>= 1) {
          if (p & 1) pw = pw * base;
          base = base * base;
        }
      }
#pragma unroll
      for (int l = 0; l < PH; ++l) {
        if (l < nt[u]) {
          acc[l] = acc[l] + pw;
          pw = pw * q[u];
        }
      }
    }
    if (nt[U - 1] <= 0) break;  // later chunks need no more terms
  }
#pragma unroll
  for (int l = 0; l < PH; ++l) {
    const double sc = -1.0 / (double)(l0 + l + 1);  // -q^l / l
    const double vx = wave_sum(acc[l].x), vy = wave_sum(acc[l].y);
    if (ln == 0) {
      out[2 * (l0 + l + 1)] = vx * sc;
      out[2 * (l0 + l + 1) + 1] = vy * sc;
    }
  }
  if (h == 0) {
    double zt = 0.0;
    const int g = isl_geo[k];
    for (int m = gisl[g] + ln; m < gisl[g + 1]; m += 64) zt += zr[m];
    a0 = wave_sum(a0);
    zf = wave_sum(zf);
    zt = wave_sum(zt);
    if (ln == 0) {
      out[0] = a0;
      out[1] = 0.0;
      out[2 * (P + 1)] = zf;
      out[2 * (P + 1) + 1] = zt;
    }
  }
}

// (E z)_i: the island's expansion at u = xi'_i / rho'_k (all P terms; the
// coefficients beyond those its far list needs are zero), plus its near
// centres directly.  One work-group per (island, right-hand side): the
// island's coefficients and near centres are the same for every lane, so
// they are read with scalar loads.
__global__ void __launch_bounds__(256)
    k_logsrc_node(int M, const int64_t *__restrict__ offs,
                  const double *__restrict__ xil,
                  const double *__restrict__ xyz,
                  const double *__restrict__ elll,
                  const double *__restrict__ rhol,
                  const double *__restrict__ cxyz,
                  const int32_t *__restrict__ near_ptr,
                  const int32_t *__restrict__ near_idx,
                  const double *__restrict__ z, int64_t ldz,
                  const double *__restrict__ Lc,
                  double *__restrict__ out, int64_t ldo, double alpha) {
  constexpr int P = kPlog, stride = log_stride<P>();
  const int k = blockIdx.x, r = blockIdx.y;
  const double *L = Lc + ((int64_t)r * M + k) * stride;
  const double ir = 1.0 / rhol[k];
  const double *zr = z + (int64_t)r * ldz;
  const int e0 = near_ptr[k], e1 = near_ptr[k + 1];
  const int64_t i1 = offs[k + 1];
  for (int64_t i = offs[k] + threadIdx.x; i < i1; i += 256) {
    const cx<double> u{xil[2 * i] * ir, xil[2 * i + 1] * ir};
    cx<double> s{L[2 * P], L[2 * P + 1]};
#pragma unroll
    for (int l = P - 1; l >= 0; --l) s = cfma(s, u, cx<double>{L[2 * l], L[2 * l + 1]});
    double tot = s.x - 0.5 * L[2 * (P + 1)] * elll[i];
    const double x0 = xyz[3 * i], x1 = xyz[3 * i + 1], x2 = xyz[3 * i + 2];
    for (int e = e0; e < e1; ++e) {
      const int m = near_idx[e];
      const double d0 = x0 - cxyz[3 * m], d1 = x1 - cxyz[3 * m + 1],
                   d2 = x2 - cxyz[3 * m + 2];
      tot += zr[m] * 0.5 * log(d0 * d0 + d1 * d1 + d2 * d2);
    }
    const double ez = -kInvPi * tot + kLog2 * 0.5 * kInvPi * L[2 * (P + 1) + 1];
    out[(int64_t)r * ldo + i] += alpha * ez;
  }
}

// The same expansion about the planar centre eta_k of the common projection
// (for the shape derivative, which needs sum_m z_m / (xi - eta_m) in that
// plane):
//   log|x - c| = log 2 + log|xi - eta| - ell(xi)/2 - ell(eta)/2,
//   ell(z) = log(1 + |z|^2),  u = (xi - eta_k)/rho_k,  q = rho_k/(eta_m - eta_k),
//   L_k[0] = sum_far z_m (log 2 + log|eta_k - eta_m| - ell(eta_m)/2),
//   L_k[l] = -sum_far z_m q^l / l,   far: |eta_m - eta_k| > 3 rho_k.
__global__ void __launch_bounds__(256)
    k_logsrc_local_plane(int M, const int32_t *__restrict__ isl_geo,
                         const int32_t *__restrict__ gisl,
                         const double *__restrict__ eta,
                         const double *__restrict__ rho,
                         const double *__restrict__ ellc,
                         const int32_t *__restrict__ near_ptr,
                         const int32_t *__restrict__ near_idx,
                         const double *__restrict__ z,
                         double *__restrict__ Lout) {
  constexpr int P = kPlog;
  constexpr int stride = log_stride<kPlog>();
  __shared__ double red[4][stride];
  const int k = blockIdx.x;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const int g = isl_geo[k];
  const int m0 = gisl[g], m1 = gisl[g + 1];
  const double ex = eta[2 * k], ey = eta[2 * k + 1], rk = rho[k];
  const int32_t *nl = near_idx + near_ptr[k];
  const int nn = near_ptr[k + 1] - near_ptr[k];
  cx<double> acc[P];
#pragma unroll
  for (int l = 0; l < P; ++l) acc[l] = cx<double>{0.0, 0.0};
  double a0 = 0.0, zf = 0.0, zt = 0.0;
  for (int m = m0 + tid; m < m1; m += 256) {
    const double zm = z[m];
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
  double *out = Lout + (int64_t)k * stride;
  for (int s = tid; s < stride; s += 256) {
    double v = red[0][s] + red[1][s] + red[2][s] + red[3][s];
    if (s >= 2 && s < 2 * (P + 1)) v *= -1.0 / (double)(s / 2);
    out[s] = v;
  }
}

// Planar-centre expansion coefficients L_k for one column z (ws.logL).
void launch_logsrc_local(const Geometry &g, Workspace &ws, const double *z,
                         hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_logsrc_local_plane, dim3(g.M), dim3(256), 0, s, g.M,
                     g.isl_geo.p, g.dgisl.p, g.deta.p, g.drho.p, g.dellc.p,
                     g.near_ptr.p, g.near_idx.p, z, ws.logL.p);
  LBS_HIP(hipGetLastError());
}

void launch_logsrc_apply(const Geometry &g, Workspace &ws, const double *z,
                         int64_t ldz, int nrhs, double *out, int64_t ldo,
                         double alpha, hipStream_t s) {
  if (g.M == 0 || g.N == 0) return;
  hipLaunchKernelGGL(k_logsrc_local, dim3(g.M, nrhs, 2), dim3(64), 0, s, g.M,
                     g.isl_geo.p, g.dgisl.p, g.far_ptr.p, g.far_cptr.p,
                     g.far_nt.p, g.far_idx.p, g.far_q.p, g.far_h.p, z, ldz,
                     ws.logL.p);
  hipLaunchKernelGGL(k_logsrc_node, dim3(g.M, nrhs), dim3(256), 0, s, g.M,
                     g.doffs.p, g.xil.p, g.xyz.p, g.elll.p, g.rhol.p,
                     g.dcenter.p, g.nearR_ptr.p, g.nearR_idx.p, z, ldz,
                     ws.logL.p, out, ldo, alpha);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------ constraint rows
// out[k] = sum over island k of y for every island that is not the first
// of its geometry; for the first island: the sum of A over the geometry's
// islands (row sum(A) = 0 of eq. eqn:sum_ak), or 0 without A.
__global__ void __launch_bounds__(256)
    k_island_sums(const int64_t *__restrict__ offs,
                  const int32_t *__restrict__ isl_geo,
                  const int32_t *__restrict__ gisl,
                  const double *__restrict__ y, int64_t ldy,
                  const double *__restrict__ arow, int64_t lda,
                  double *__restrict__ out, int64_t ldo) {
  __shared__ double red[4];
  const int k = blockIdx.x, r = blockIdx.y;
  const int g = isl_geo[k];
  const double *yr = y + (int64_t)r * ldy;
  double acc = 0.0;
  if (k == gisl[g]) {
    if (arow)
      for (int m = gisl[g] + threadIdx.x; m < gisl[g + 1]; m += 256)
        acc += arow[(int64_t)r * lda + m];
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
  hipLaunchKernelGGL(k_island_sums, dim3(g.M, nrhs), dim3(256), 0, s,
                     g.doffs.p, g.isl_geo.p, g.dgisl.p, y, ldy,
                     (const double *)nullptr, (int64_t)0, out, ldo);
  LBS_HIP(hipGetLastError());
}

void launch_constraint_rows(const Geometry &g, const double *sigma,
                            int64_t ldx, const double *A, int64_t lda,
                            int nrhs, double *out, int64_t ldo,
                            hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_island_sums, dim3(g.M, nrhs), dim3(256), 0, s,
                     g.doffs.p, g.isl_geo.p, g.dgisl.p, sigma, ldx, A, lda,
                     out, ldo);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------ Schur complement
// Per geometry (M_g islands, block at gsinv[g], row-major M_g x M_g):
// S = D - F E; local row 0 is (1, ..., 1); local row kl >= 1 is
// -sum_{i in island} 2 G(x_i, c_m).
__global__ void k_build_schur(const int32_t *__restrict__ isl_geo,
                              const int32_t *__restrict__ gisl,
                              const int64_t *__restrict__ gsinv,
                              const int64_t *__restrict__ offs,
                              const double *__restrict__ xyz,
                              const double *__restrict__ cxyz,
                              double *__restrict__ S) {
  const int k = blockIdx.y;
  const int g = isl_geo[k];
  const int Mg = gisl[g + 1] - gisl[g];
  const int ml = blockIdx.x * blockDim.x + threadIdx.x;
  if (ml >= Mg) return;
  const int kl = k - gisl[g];
  double *Sg = S + gsinv[g];
  if (kl == 0) {
    Sg[ml] = 1.0;
    return;
  }
  const int m = gisl[g] + ml;
  const double c0 = cxyz[3 * m], c1 = cxyz[3 * m + 1], c2 = cxyz[3 * m + 2];
  double acc = 0.0;
  const int64_t n = offs[k + 1] - offs[k];
  for (int64_t i = offs[k]; i < offs[k + 1]; ++i) {
    const double d0 = xyz[3 * i] - c0, d1 = xyz[3 * i + 1] - c1,
                 d2 = xyz[3 * i + 2] - c2;
    acc += log(d0 * d0 + d1 * d1 + d2 * d2);
  }
  // 2 G = -(1/2pi) log|d|^2 + log2 / 2pi
  const double sum2g = -0.5 * kInvPi * acc + 0.5 * kInvPi * kLog2 * (double)n;
  Sg[(int64_t)kl * Mg + ml] = -sum2g;
}

void launch_build_schur(const Geometry &g, double *S, hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_build_schur, dim3((g.maxM + 255) / 256, g.M),
                     dim3(256), 0, s, g.isl_geo.p, g.dgisl.p, g.dgsinv.p,
                     g.doffs.p, g.xyz.p, g.dcenter.p, S);
  LBS_HIP(hipGetLastError());
}

// Blocked Gauss-Jordan inversion with partial pivoting, in place, of every
// geometry's block S_g at once (grid z or x = geometry).  Panel J = rows and
// columns j0 .. j0 + nb - 1 of the rows not yet eliminated:
//  1. k_gjp_panel (one work-group per geometry, the panel rows j0.. held in
//     registers, RPT rows per thread): LU with partial pivoting of
//     S[j0:, J], of which the pivot rows are kept, then Binv = S_JJ^-1 of
//     the pivoted block by Gauss-Jordan elimination without further
//     interchanges (its pivots are those of the LU);
//  2. k_gjp_swap: the pivot rows exchanged over whole rows;
//  3. k_gjp_rows: R = S[J, :] (the pivot rows as they are) and W = Binv R;
//     k_gjp_cols: Cn_i = -S[i, J] Binv for the rows i outside J;
//  4. k_gjp_update: S_ij += Cn_i R_j (i, j outside J), S_iJ = Cn_i,
//     S_Jj = W_j, S_JJ = Binv.
// After the last panel, S holds (Pi S)^-1 for the row interchanges Pi, and
// the inverse is its columns permuted back (k_gjp_unpermute).  The panel
// width is 32 / RPT so that each thread keeps 32 values; RPT = 1, 2, 4 or
// 8 serves panels of up to 1024 RPT rows (at most 8192 islands).
constexpr int kGJ = 32;     // widest panel
constexpr int kGJT = 1024;  // threads of the panel kernel

// Pivot key of row r (offset ro = r - j0 < 8192) with value a = |v|: the
// bits of a with the low 13 replaced by 8191 - ro, so that the largest key
// is the largest |v| (compared to 39 bits of its mantissa), the lowest row
// among those.  Bit 13 is set so that every candidate's key exceeds the 0
// of the rows that are not candidates.
__device__ __forceinline__ unsigned long long pivot_key(double a, int ro) {
  return ((unsigned long long)__double_as_longlong(a) & ~0x1FFFull) | (1ull << 13) |
         (unsigned long long)(8191 - ro);
}

// Largest value over the 64 lanes of a wave, by the device library's wave
// reduction (DPP row and cross-row steps; the header declares it only with
// the optional 64-bit warp-sync types enabled).
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(
    unsigned long long);

// Binv (kGJ x kGJ, entries past nb 0) = S_JJ^-1 of the pivoted block whose
// rows came from rows blk_row[0:nb] of S (columns j0..), by Gauss-Jordan
// elimination without interchanges, one entry per thread (its pivots are
// those the panel LU chose).  Kept out of line so that the panel loop's
// registers are not shared with it.
template <int NB>
__device__ __noinline__ void pivot_block_inverse(const double *__restrict__ Sg, int Mg, int j0,
                                                 int nb, const int *blk_row,
                                                 double (*bl)[NB + 1],
                                                 double *__restrict__ Binv) {
  const int tid = threadIdx.x;
  const int bi = tid / NB, bj = tid % NB;  // NB <= 32: threads past NB^2 idle
  const bool live = tid < NB * NB && bi < nb && bj < nb;
  if (tid < NB * NB) bl[bi][bj] = live ? Sg[(int64_t)blk_row[bi] * Mg + j0 + bj] : 0.0;
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    double x = 0.0;
    if (live) {
      const double pinv = 1.0 / bl[k][k];
      x = bl[bi][bj];
      if (bi == k && bj == k) x = pinv;
      else if (bi == k) x = x * pinv;
      else if (bj == k) x = -x * pinv;
      else x = x - bl[bi][k] * bl[k][bj] * pinv;
    }
    __syncthreads();
    if (live) bl[bi][bj] = x;
    __syncthreads();
  }
  if (tid < kGJ * kGJ) {
    const int a = tid / kGJ, b = tid % kGJ;
    Binv[a * kGJ + b] = (a < nb && b < nb) ? bl[a][b] : 0.0;
  }
}

// LDS of the panel kernel
template <int NB>
struct PanelShared {
  unsigned long long wk[16];
  double prow[NB], crow[NB];
  int prow_id, crow_id, blk_row[NB];
  double bl[NB][NB + 1];
};

// Column K of the panel LU (every index into v a compile-time constant;
// columns below K are finished and no longer read): the pivot row p among
// the rows >= c = j0 + K, rows c and p exchanged (columns K.. only), the
// rows below c eliminated in columns K + 1 .. NB - 1.  Steps K >= nb are
// skipped (uniformly).
template <int K, int NB, int RPT>
__device__ __forceinline__ void panel_column(double (&v)[RPT][NB], int (&orig)[RPT], int j0,
                                             int nb, int Mg, int tid, PanelShared<NB> &sh,
                                             int *__restrict__ piv_g) {
  if constexpr (K < NB) {
    if (K >= nb) return;
    const int c = j0 + K;
    unsigned long long key = 0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = j0 + tid + kGJT * i;
      if (r >= c && r < Mg) {
        const unsigned long long kk = pivot_key(fabs(v[i][K]), r - j0);
        key = kk > key ? kk : key;
      }
    }
    key = __ockl_wfred_max_u64(key);
    if ((tid & 63) == 0) sh.wk[tid >> 6] = key;
    __syncthreads();
    // every wave reduces the 16 wave maxima itself
    key = __ockl_wfred_max_u64(sh.wk[tid & 15]);
    const int p = j0 + 8191 - (int)(key & 0x1FFFull);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = j0 + tid + kGJT * i;
      if (r == p) {
#pragma unroll
        for (int q = K; q < NB; ++q) sh.prow[q] = v[i][q];
        sh.prow_id = orig[i];
      }
      if (r == c) {
#pragma unroll
        for (int q = K; q < NB; ++q) sh.crow[q] = v[i][q];
        sh.crow_id = orig[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = j0 + tid + kGJT * i;
      if (r == p && r != c) {
#pragma unroll
        for (int q = K; q < NB; ++q) v[i][q] = sh.crow[q];
        orig[i] = sh.crow_id;
      } else if (r == c) {
        orig[i] = sh.prow_id;
      }
    }
    // prow, crow and wk are rewritten only after the next column's first
    // barrier
    const double inv = 1.0 / sh.prow[K];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = j0 + tid + kGJT * i;
      if (r > c && r < Mg) {
        const double l = v[i][K] * inv;
#pragma unroll
        for (int q = K + 1; q < NB; ++q) v[i][q] -= l * sh.prow[q];
      }
    }
    if (tid == 0) piv_g[c] = p;
    panel_column<K + 1, NB, RPT>(v, orig, j0, nb, Mg, tid, sh, piv_g);
  }
}

template <int RPT>
__global__ void __launch_bounds__(kGJT)
    k_gjp_panel(int j0, const int32_t *__restrict__ gisl, const int64_t *__restrict__ gsinv,
                const double *__restrict__ S, int *__restrict__ piv,
                double *__restrict__ Binv, int maxM) {
  constexpr int NB = kGJ / RPT;
  __shared__ PanelShared<NB> sh;
  const int g = blockIdx.x;
  const int Mg = gisl[g + 1] - gisl[g];
  if (j0 >= Mg) return;
  const int nb = min(NB, Mg - j0), tid = threadIdx.x;
  const double *Sg = S + gsinv[g];
  int orig[RPT];  // the row of S each register row started as
#pragma unroll
  for (int i = 0; i < RPT; ++i) orig[i] = j0 + tid + kGJT * i;
  // v[i][q]: row j0 + tid + kGJT i, column j0 + q
  double v[RPT][NB];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = j0 + tid + kGJT * i;
#pragma unroll
    for (int q = 0; q < NB; ++q)
      v[i][q] = (r < Mg && q < nb) ? Sg[(int64_t)r * Mg + j0 + q] : 0.0;
  }
  panel_column<0, NB, RPT>(v, orig, j0, nb, Mg, tid, sh, piv + (int64_t)g * maxM);
  // Binv = S_JJ^-1 of the pivoted block, read from the rows of S it came
  // from, by Gauss-Jordan elimination without interchanges (one entry per
  // thread; its pivots are those just chosen)
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = j0 + tid + kGJT * i;
    if (r < j0 + nb) sh.blk_row[r - j0] = orig[i];
  }
  __syncthreads();
  pivot_block_inverse<NB>(Sg, Mg, j0, nb, sh.blk_row, sh.bl, Binv + (int64_t)g * kGJ * kGJ);
}

// column c of S_g: the panel's row interchanges in order
__global__ void __launch_bounds__(256)
    k_gjp_swap(int j0, int NB, const int32_t *__restrict__ gisl,
               const int64_t *__restrict__ gsinv, double *__restrict__ S,
               const int *__restrict__ piv, int maxM) {
  const int g = blockIdx.z;
  const int Mg = gisl[g + 1] - gisl[g];
  if (j0 >= Mg) return;
  const int nb = min(NB, Mg - j0);
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= Mg) return;
  double *X = S + gsinv[g];
  for (int k = 0; k < nb; ++k) {
    const int p = piv[(int64_t)g * maxM + j0 + k];
    if (p == j0 + k) continue;
    const double t = X[(int64_t)(j0 + k) * Mg + c];
    X[(int64_t)(j0 + k) * Mg + c] = X[(int64_t)p * Mg + c];
    X[(int64_t)p * Mg + c] = t;
  }
}

// Work-group of 32 columns c: R[k][c] = S[j0 + k][c] (the pivot rows as
// they are) and W[k][c] = sum_q Binv[k][q] R[q][c], k < nb.
__global__ void __launch_bounds__(256)
    k_gjp_rows(int j0, int NB, const int32_t *__restrict__ gisl,
               const int64_t *__restrict__ gsinv, const double *__restrict__ S,
               const double *__restrict__ Binv, double *__restrict__ R,
               double *__restrict__ W, int maxM) {
  __shared__ double bl[kGJ][kGJ + 1];
  __shared__ double rt[kGJ][33];
  const int g = blockIdx.z;
  const int Mg = gisl[g + 1] - gisl[g];
  if (j0 >= Mg) return;
  const int nb = min(NB, Mg - j0);
  const int c0 = blockIdx.x * 32;
  if (c0 >= Mg) return;
  const double *X = S + gsinv[g];
  for (int e = threadIdx.x; e < kGJ * kGJ; e += 256) {
    const int a = e / kGJ, b = e % kGJ, c = c0 + b;
    rt[a][b] = (a < nb && c < Mg) ? X[(int64_t)(j0 + a) * Mg + c] : 0.0;
  }
  for (int e = threadIdx.x; e < kGJ * kGJ; e += 256)
    bl[e / kGJ][e % kGJ] = Binv[(int64_t)g * kGJ * kGJ + e];
  __syncthreads();
  double *Rg = R + (int64_t)g * kGJ * maxM, *Wg = W + (int64_t)g * kGJ * maxM;
  for (int e = threadIdx.x; e < nb * 32; e += 256) {
    const int k = e / 32, cl = e % 32, c = c0 + cl;
    if (c >= Mg) continue;
    double t = 0.0;
    for (int q = 0; q < nb; ++q) t += bl[k][q] * rt[q][cl];
    Rg[(int64_t)k * maxM + c] = rt[k][cl];
    Wg[(int64_t)k * maxM + c] = t;
  }
}

// Work-group of 32 rows i outside J: Cn[k][i] = -sum_q S[i][j0 + q] Binv[q][k].
__global__ void __launch_bounds__(256)
    k_gjp_cols(int j0, int NB, const int32_t *__restrict__ gisl,
               const int64_t *__restrict__ gsinv, const double *__restrict__ S,
               const double *__restrict__ Binv, double *__restrict__ Cn, int maxM) {
  __shared__ double bl[kGJ][kGJ + 1];
  __shared__ double at[32][kGJ + 1];
  const int g = blockIdx.z;
  const int Mg = gisl[g + 1] - gisl[g];
  if (j0 >= Mg) return;
  const int nb = min(NB, Mg - j0);
  const int i0 = blockIdx.x * 32;
  if (i0 >= Mg) return;
  const double *X = S + gsinv[g];
  for (int e = threadIdx.x; e < kGJ * kGJ; e += 256) {
    const int a = e / kGJ, b = e % kGJ, i = i0 + a;
    at[a][b] = (b < nb && i < Mg) ? X[(int64_t)i * Mg + j0 + b] : 0.0;
  }
  for (int e = threadIdx.x; e < kGJ * kGJ; e += 256)
    bl[e / kGJ][e % kGJ] = Binv[(int64_t)g * kGJ * kGJ + e];
  __syncthreads();
  double *Cg = Cn + (int64_t)g * kGJ * maxM;
  for (int e = threadIdx.x; e < nb * 32; e += 256) {
    const int k = e / 32, il = e % 32, i = i0 + il;
    if (i >= Mg || (i >= j0 && i < j0 + nb)) continue;
    double t = 0.0;
    for (int q = 0; q < nb; ++q) t += at[il][q] * bl[q][k];
    Cg[(int64_t)k * maxM + i] = -t;
  }
}

// Tiles of 64 x 64 entries of S_g, 4 x 4 per thread (see above for what
// each part of the tile takes).
__global__ void __launch_bounds__(256)
    k_gjp_update(int j0, int NB, const int32_t *__restrict__ gisl,
                 const int64_t *__restrict__ gsinv, double *__restrict__ S,
                 const double *__restrict__ Cn, const double *__restrict__ R,
                 const double *__restrict__ W, const double *__restrict__ Binv, int maxM) {
  __shared__ double cs[64][kGJ + 1];
  __shared__ double rs[kGJ][64 + 1];
  const int g = blockIdx.z;
  const int Mg = gisl[g + 1] - gisl[g];
  if (j0 >= Mg) return;
  const int nb = min(NB, Mg - j0);
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  if (c0 >= Mg || r0 >= Mg) return;
  const double *Cg = Cn + (int64_t)g * kGJ * maxM, *Rg = R + (int64_t)g * kGJ * maxM;
  const double *Wg = W + (int64_t)g * kGJ * maxM;
  double *Sg = S + gsinv[g];
  const int tr = (threadIdx.x >> 4) * 4, tc = (threadIdx.x & 15) * 4;
  double old[4][4];  // this thread's entries, loaded before the tile is staged
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + tr + i, c = c0 + tc + j;
      old[i][j] = (r < Mg && c < Mg) ? Sg[(int64_t)r * Mg + c] : 0.0;
    }
  for (int e = threadIdx.x; e < 64 * kGJ; e += 256) {
    const int k = e / 64, t = e % 64;
    const int r = r0 + t, c = c0 + t;
    const bool rin = r >= j0 && r < j0 + nb, cin = c >= j0 && c < j0 + nb;
    cs[t][k] = (k < nb && r < Mg && !rin) ? Cg[(int64_t)k * maxM + r] : 0.0;
    rs[k][t] = (k < nb && c < Mg && !cin) ? Rg[(int64_t)k * maxM + c] : 0.0;
  }
  __syncthreads();
  double acc[4][4] = {};
  for (int k = 0; k < nb; ++k)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += cs[tr + i][k] * rs[k][tc + j];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + tr + i;
    if (r >= Mg) continue;
    const bool rin = r >= j0 && r < j0 + nb;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tc + j;
      if (c >= Mg) continue;
      const bool cin = c >= j0 && c < j0 + nb;
      double *X = Sg + (int64_t)r * Mg + c;
      if (rin && cin) *X = Binv[((int64_t)g * kGJ + (r - j0)) * kGJ + (c - j0)];
      else if (rin) *X = Wg[(int64_t)(r - j0) * maxM + c];
      else if (cin) *X = Cg[(int64_t)(c - j0) * maxM + r];
      else *X = old[i][j] + acc[i][j];
    }
  }
}

// Sinv_g[i][j] = X_g[i][col_of[j]], one work-group per row
__global__ void __launch_bounds__(256)
    k_gjp_unpermute(const int32_t *__restrict__ isl_geo, const int32_t *__restrict__ gisl,
                    const int64_t *__restrict__ gsinv, const double *__restrict__ X,
                    const int *__restrict__ col_of, double *__restrict__ Sinv, int maxM) {
  const int row = blockIdx.x;
  const int g = isl_geo[row];
  const int Mg = gisl[g + 1] - gisl[g], rl = row - gisl[g];
  const double *xr = X + gsinv[g] + (int64_t)rl * Mg;
  double *yr = Sinv + gsinv[g] + (int64_t)rl * Mg;
  const int *cm = col_of + (int64_t)g * maxM;
  for (int j = threadIdx.x; j < Mg; j += 256) yr[j] = xr[cm[j]];
}

template <int RPT>
static void gj_panel(int j0, const Geometry &g, double *S, int *piv, double *Bi, int maxM,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_gjp_panel<RPT>, dim3(g.G), dim3(kGJT), 0, s, j0, g.dgisl.p, g.dgsinv.p, S,
                     piv, Bi, maxM);
}

void invert_blocks(const Geometry &g, double *S, double *Sinv, hipStream_t s) {
  if (g.M == 0) return;
  const int G = g.G, maxM = g.maxM;
  if (maxM > 8 * kGJT)
    throw ApiError{LBS_ERR_UNSUPPORTED, "more than 8192 islands in one geometry"};
  DBuf<int> piv, colmap;
  piv.alloc((size_t)G * maxM);
  colmap.alloc((size_t)G * maxM);
  DBuf<double> R, W, Cn, Bi;
  R.alloc((size_t)G * kGJ * maxM);
  W.alloc((size_t)G * kGJ * maxM);
  Cn.alloc((size_t)G * kGJ * maxM);
  Bi.alloc((size_t)G * kGJ * kGJ);
  const unsigned ncol = (maxM + 255) / 256, ntile = (maxM + 63) / 64, n32 = (maxM + 31) / 32;
  for (int j0 = 0; j0 < maxM;) {
    // rows still to eliminate in the largest geometry: maxM - j0
    const int h = maxM - j0;
    const int rpt = h <= kGJT ? 1 : h <= 2 * kGJT ? 2 : h <= 4 * kGJT ? 4 : 8;
    const int NB = kGJ / rpt;
    switch (rpt) {
      case 1: gj_panel<1>(j0, g, S, piv.p, Bi.p, maxM, s); break;
      case 2: gj_panel<2>(j0, g, S, piv.p, Bi.p, maxM, s); break;
      case 4: gj_panel<4>(j0, g, S, piv.p, Bi.p, maxM, s); break;
      default: gj_panel<8>(j0, g, S, piv.p, Bi.p, maxM, s); break;
    }
    hipLaunchKernelGGL(k_gjp_swap, dim3(ncol, 1, G), dim3(256), 0, s, j0, NB, g.dgisl.p,
                       g.dgsinv.p, S, piv.p, maxM);
    hipLaunchKernelGGL(k_gjp_rows, dim3(n32, 1, G), dim3(256), 0, s, j0, NB, g.dgisl.p,
                       g.dgsinv.p, S, Bi.p, R.p, W.p, maxM);
    hipLaunchKernelGGL(k_gjp_cols, dim3(n32, 1, G), dim3(256), 0, s, j0, NB, g.dgisl.p,
                       g.dgsinv.p, S, Bi.p, Cn.p, maxM);
    hipLaunchKernelGGL(k_gjp_update, dim3(ntile, ntile, G), dim3(256), 0, s, j0, NB, g.dgisl.p,
                       g.dgsinv.p, S, Cn.p, R.p, W.p, Bi.p, maxM);
    j0 += NB;
  }
  // the column map on the host: the row interchanges undone, last first
  std::vector<int> hp = piv.download(s), cm((size_t)G * maxM, 0);
  for (int q = 0; q < G; ++q) {
    const int Mg = g.gisl[q + 1] - g.gisl[q];
    int *c = cm.data() + (size_t)q * maxM;
    const int *pq = hp.data() + (size_t)q * maxM;
    for (int j = 0; j < Mg; ++j) c[j] = j;
    for (int k = Mg - 1; k >= 0; --k) std::swap(c[k], c[pq[k]]);
  }
  colmap.upload(cm, s);
  hipLaunchKernelGGL(k_gjp_unpermute, dim3(g.M), dim3(256), 0, s, g.isl_geo.p, g.dgisl.p,
                     g.dgsinv.p, S, colmap.p, Sinv, maxM);
  LBS_HIP(hipGetLastError());
  LBS_HIP(hipStreamSynchronize(s));
}

// Inversion without row interchanges.  The Schur complements of this
// problem have the constraint row of ones first and, below it, rows
// dominated by each island's own log term (the log of its radius against
// the logs of island distances), so Gauss-Jordan elimination in the natural
// order is stable for them; invert_schur checks every result and falls back
// to the pivoted elimination above when the check fails.  Panels of kNP
// columns J = j0 .. j0 + nb - 1, three launches each:
//  1. k_gjn_block: Binv = S_JJ^-1 by Gauss-Jordan elimination in the
//     natural order (one work-group per geometry);
//  2. k_gjn_rowcol: R = S[J, :], W = Binv R and Cn_i = -S[i, J] Binv for
//     the rows i outside J (one work-group per 64 columns or 64 rows);
//  3. k_gjn_update: S_ij += Cn_i R_j (i, j outside J), S_iJ = Cn_i,
//     S_Jj = W_j, S_JJ = Binv, in 64 x 64 tiles.
// After the last panel S holds S^-1 with no permutation to undo.
constexpr int kNP = 64;

// Thread t holds the entries (a0 + u, b), u < 4, of the kNP x kNP block,
// b = t mod 64, a0 = 4 (t / 64).  Step k needs the step-(k-1) values of
// row k and column k, which their owners publish in LDS (two copies, so
// that one barrier per step suffices).  The steps are bound by VALU issue
// on the one CU (about 0.6 us each; 256 threads with 16 entries each, or
// one wave with 64, take 1.5 and 4 times as long).
constexpr int kGJNT = 1024;
__global__ void __launch_bounds__(kGJNT)
    k_gjn_block(int j0, const int32_t *__restrict__ gisl, const int64_t *__restrict__ gsinv,
                const double *__restrict__ S, double *__restrict__ Binv) {
  constexpr int U = kNP * kNP / kGJNT;
  __shared__ double rowk[2][kNP], colk[2][kNP];
  const int g = blockIdx.x;
  const int Mg = gisl[g + 1] - gisl[g];
  if (j0 >= Mg) return;
  const int nb = min(kNP, Mg - j0);
  const double *Sg = S + gsinv[g];
  const int b = threadIdx.x & 63, a0 = (threadIdx.x >> 6) * U;
  double v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int a = a0 + u;
    v[u] = (a < nb && b < nb) ? Sg[(int64_t)(j0 + a) * Mg + j0 + b] : 0.0;
  }
  if (a0 == 0) rowk[0][b] = v[0];
  if (b == 0) {
#pragma unroll
    for (int u = 0; u < U; ++u) colk[0][a0 + u] = v[u];
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const int cur = k & 1, nxt = cur ^ 1;
    double ca[U];  // column k of this thread's rows (the same for the wave)
#pragma unroll
    for (int u = 0; u < U; ++u) ca[u] = colk[cur][a0 + u];
    const double pinv = 1.0 / rowk[cur][k];
    const double rkb = rowk[cur][b] * pinv;  // entry (k, b) over the pivot
    // the entries off row and column k (the padding past nb stays 0, as
    // its row and column entries are 0); row k (one wave, uniform) and
    // column k (one lane per wave) are overwritten after
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = fma(-ca[u], rkb, v[u]);
    if (b == k) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = -ca[u] * pinv;
    }
    if (k >= a0 && k < a0 + U) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (a0 + u == k) v[u] = b == k ? pinv : rowk[cur][b] * pinv;
    }
    const int kn = k + 1;
    if (kn < nb) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (a0 + u == kn) rowk[nxt][b] = v[u];
      if (b == kn) {
#pragma unroll
        for (int u = 0; u < U; ++u) colk[nxt][a0 + u] = v[u];
      }
    }
    __syncthreads();
  }
  double *Bg = Binv + (int64_t)g * kNP * kNP;
#pragma unroll
  for (int u = 0; u < U; ++u) Bg[(a0 + u) * kNP + b] = v[u];
}

// blockIdx.y = 0: columns c0 .. c0 + 15: R[k][c] = S[j0 + k][c] and
// W[k][c] = sum_q Binv[k][q] R[q][c]; blockIdx.y = 1: rows i0 .. i0 + 15
// outside J: Cn[k][i] = -sum_q S[i][j0 + q] Binv[q][k].  R, W and Cn are
// kNP x maxM per geometry; entries past nb are not written.
constexpr int kRC = 16;  // columns or rows per work-group
__global__ void __launch_bounds__(256)
    k_gjn_rowcol(int j0, const int32_t *__restrict__ gisl, const int64_t *__restrict__ gsinv,
                 const double *__restrict__ S, const double *__restrict__ Binv,
                 double *__restrict__ R, double *__restrict__ W, double *__restrict__ Cn,
                 int maxM) {
  __shared__ double bl[kNP][kNP + 1];
  __shared__ double st[kNP][kRC + 1];  // st[q][e]: S[j0 + q][e0 + e] or S[e0 + e][j0 + q]
  const int g = blockIdx.z;
  const int Mg = gisl[g + 1] - gisl[g];
  if (j0 >= Mg) return;
  const int nb = min(kNP, Mg - j0);
  const int e0 = blockIdx.x * kRC;
  if (e0 >= Mg) return;
  const bool rows = blockIdx.y == 0;
  const double *X = S + gsinv[g];
  const double *Bg = Binv + (int64_t)g * kNP * kNP;
  for (int e = threadIdx.x; e < kNP * kNP; e += 256) bl[e / kNP][e % kNP] = Bg[e];
  for (int e = threadIdx.x; e < kNP * kRC; e += 256) {
    if (rows) {
      const int q = e / kRC, c = e % kRC;
      st[q][c] = (q < nb && e0 + c < Mg) ? X[(int64_t)(j0 + q) * Mg + e0 + c] : 0.0;
    } else {
      const int i = e / kNP, q = e % kNP;
      st[q][i] = (q < nb && e0 + i < Mg) ? X[(int64_t)(e0 + i) * Mg + j0 + q] : 0.0;
    }
  }
  __syncthreads();
  const int l = threadIdx.x % kRC, e = e0 + l;
  if (e >= Mg) return;
  const int64_t base = (int64_t)g * kNP * maxM;
  if (rows) {
    for (int k = threadIdx.x / kRC; k < nb; k += 256 / kRC) {
      double t = 0.0;
      for (int q = 0; q < nb; ++q) t += bl[k][q] * st[q][l];
      R[base + (int64_t)k * maxM + e] = st[k][l];
      W[base + (int64_t)k * maxM + e] = t;
    }
  } else {
    if (e >= j0 && e < j0 + nb) return;
    for (int k = threadIdx.x / kRC; k < nb; k += 256 / kRC) {
      double t = 0.0;
      for (int q = 0; q < nb; ++q) t += st[q][l] * bl[q][k];
      Cn[base + (int64_t)k * maxM + e] = -t;
    }
  }
}

// Tiles of 64 x 64 entries, 4 x 4 per thread; the rank-nb product is
// staged through LDS in two halves of 32 terms, both operands k-major so
// that each thread reads its four rows and four columns as two 16-byte
// words each.
__global__ void __launch_bounds__(256)
    k_gjn_update(int j0, const int32_t *__restrict__ gisl, const int64_t *__restrict__ gsinv,
                 double *__restrict__ S, const double *__restrict__ Cn,
                 const double *__restrict__ R, const double *__restrict__ W,
                 const double *__restrict__ Binv, int maxM) {
  constexpr int KH = kNP / 2;
  __shared__ __align__(16) double cs[KH][64 + 4];
  __shared__ __align__(16) double rs[KH][64 + 4];
  const int g = blockIdx.z;
  const int Mg = gisl[g + 1] - gisl[g];
  if (j0 >= Mg) return;
  const int nb = min(kNP, Mg - j0);
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  if (c0 >= Mg || r0 >= Mg) return;
  const int64_t base = (int64_t)g * kNP * maxM;
  double *Sg = S + gsinv[g];
  const int tr = (threadIdx.x >> 4) * 4, tc = (threadIdx.x & 15) * 4;
  double old[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + tr + i, c = c0 + tc + j;
      old[i][j] = (r < Mg && c < Mg) ? Sg[(int64_t)r * Mg + c] : 0.0;
    }
  double acc[4][4] = {};
  for (int h = 0; h < nb; h += KH) {
    if (h > 0) __syncthreads();
    for (int e = threadIdx.x; e < 64 * KH; e += 256) {
      const int kk = e / 64, t = e % 64, k = h + kk;
      const int r = r0 + t, c = c0 + t;
      const bool rin = r >= j0 && r < j0 + nb, cin = c >= j0 && c < j0 + nb;
      cs[kk][t] = (k < nb && r < Mg && !rin) ? Cn[base + (int64_t)k * maxM + r] : 0.0;
      rs[kk][t] = (k < nb && c < Mg && !cin) ? R[base + (int64_t)k * maxM + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KH; ++kk) {
      const double2 a01 = *reinterpret_cast<const double2 *>(&cs[kk][tr]);
      const double2 a23 = *reinterpret_cast<const double2 *>(&cs[kk][tr + 2]);
      const double2 b01 = *reinterpret_cast<const double2 *>(&rs[kk][tc]);
      const double2 b23 = *reinterpret_cast<const double2 *>(&rs[kk][tc + 2]);
      const double av[4] = {a01.x, a01.y, a23.x, a23.y};
      const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + tr + i;
    if (r >= Mg) continue;
    const bool rin = r >= j0 && r < j0 + nb;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tc + j;
      if (c >= Mg) continue;
      const bool cin = c >= j0 && c < j0 + nb;
      double *X = Sg + (int64_t)r * Mg + c;
      if (rin && cin) *X = Binv[((int64_t)g * kNP + (r - j0)) * kNP + (c - j0)];
      else if (rin) *X = W[base + (int64_t)(r - j0) * maxM + c];
      else if (cin) *X = Cn[base + (int64_t)(c - j0) * maxM + r];
      else *X = old[i][j] + acc[i][j];
    }
  }
}

// om[i] = |S y - x|_i / (|S| |y| + |x|)_i for row i (the componentwise
// backward error of y as a solution of S y = x), one wave per row.
__global__ void __launch_bounds__(256)
    k_probe_backward(int M, const int32_t *__restrict__ isl_geo,
                     const int32_t *__restrict__ gisl, const int64_t *__restrict__ gsinv,
                     const double *__restrict__ S, const double *__restrict__ y,
                     const double *__restrict__ x, double *__restrict__ om) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ln = threadIdx.x & 63;
  if (row >= M) return;
  const int g = isl_geo[row];
  const int m0 = gisl[g], Mg = gisl[g + 1] - m0;
  const double *a = S + gsinv[g] + (int64_t)(row - m0) * Mg;
  const double *yr = y + m0;
  double z = 0.0, d = 0.0;
  for (int j = ln; j < Mg; j += 64) {
    z += a[j] * yr[j];
    d += fabs(a[j]) * fabs(yr[j]);
  }
  z = wave_sum(z);
  d = wave_sum(d);
  if (ln == 0) {
    const double r = fabs(z - x[row]), den = d + fabs(x[row]);
    om[row] = den > 0.0 ? r / den : r;
  }
}

static void invert_natural_order(const Geometry &g, double *X, hipStream_t s) {
  const int G = g.G, maxM = g.maxM;
  DBuf<double> R, W, Cn, Bi;
  R.alloc((size_t)G * kNP * maxM);
  W.alloc((size_t)G * kNP * maxM);
  Cn.alloc((size_t)G * kNP * maxM);
  Bi.alloc((size_t)G * kNP * kNP);
  const unsigned n64 = (maxM + 63) / 64, nrc = (maxM + kRC - 1) / kRC;
  for (int j0 = 0; j0 < maxM; j0 += kNP) {
    hipLaunchKernelGGL(k_gjn_block, dim3(G), dim3(kGJNT), 0, s, j0, g.dgisl.p, g.dgsinv.p, X,
                       Bi.p);
    hipLaunchKernelGGL(k_gjn_rowcol, dim3(nrc, 2, G), dim3(256), 0, s, j0, g.dgisl.p,
                       g.dgsinv.p, X, Bi.p, R.p, W.p, Cn.p, maxM);
    hipLaunchKernelGGL(k_gjn_update, dim3(n64, n64, G), dim3(256), 0, s, j0, g.dgisl.p,
                       g.dgsinv.p, X, Cn.p, R.p, W.p, Bi.p, maxM);
  }
  LBS_HIP(hipGetLastError());
}

// Largest componentwise backward error over the islands of y = Sinv x as a
// solution of S y = x, x a fixed probe of entries +-[0.5, 1) (NaN if any
// entry is not finite).
static double probe_backward_error(const Geometry &g, const double *S, const double *Sinv,
                                   hipStream_t s) {
  std::vector<double> hx(g.M);
  for (int i = 0; i < g.M; ++i) {
    const double m = 0.5 + (double)(((uint64_t)i * 2654435761ull) % 1000ull) / 2000.0;
    hx[i] = ((uint64_t)i * 40503ull) % 3ull == 0 ? -m : m;
  }
  DBuf<double> x, y, om;
  x.upload(hx, s);
  y.alloc(g.M);
  om.alloc(g.M);
  launch_gemv_blocks_with(g, Sinv, x.p, g.M, 1, y.p, g.M, 1.0, s);
  hipLaunchKernelGGL(k_probe_backward, dim3((g.M + 3) / 4), dim3(256), 0, s, g.M, g.isl_geo.p,
                     g.dgisl.p, g.dgsinv.p, S, y.p, x.p, om.p);
  LBS_HIP(hipGetLastError());
  const std::vector<double> ho = om.download(s);
  double w = 0.0;
  for (double v : ho)
    if (!(v <= w)) w = v;  // NaN propagates
  return w;
}

SchurInverseInfo invert_schur(const Geometry &g, double *S, double *Sinv, double tol,
                              hipStream_t s) {
  SchurInverseInfo info;
  if (g.M == 0) return info;
  if (g.maxM > 8 * kGJT)
    throw ApiError{LBS_ERR_UNSUPPORTED, "more than 8192 islands in one geometry"};
  if (tol > 0.0) {
    LBS_HIP(hipMemcpyAsync(Sinv, S, (size_t)g.gsinv[g.G] * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    invert_natural_order(g, Sinv, s);
    info.omega = probe_backward_error(g, S, Sinv, s);
    if (info.omega <= tol) return info;
  }
  invert_blocks(g, S, Sinv, s);
  info.pivoted = 1;
  return info;
}

// y[k] = alpha sum_m Sinv_g[kl][ml] x[gisl[g] + ml] (block diagonal),
// one wave per island row.
__global__ void __launch_bounds__(256)
    k_gemv_blocks(int M, const int32_t *__restrict__ isl_geo,
                  const int32_t *__restrict__ gisl,
                  const int64_t *__restrict__ gsinv,
                  const double *__restrict__ A, const double *__restrict__ x,
                  int64_t ldx, double *__restrict__ y, int64_t ldy,
                  double alpha) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ln = threadIdx.x & 63;
  const int r = blockIdx.y;
  if (row >= M) return;
  const int g = isl_geo[row];
  const int m0 = gisl[g], Mg = gisl[g + 1] - m0;
  const double *xr = x + (int64_t)r * ldx + m0;
  const double *a = A + gsinv[g] + (int64_t)(row - m0) * Mg;
  // four independent partial sums, so that four coalesced row loads per
  // lane are in flight at once (the kernel streams the whole matrix)
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  int j = ln;
  for (; j + 192 < Mg; j += 256) {
    acc0 += a[j] * xr[j];
    acc1 += a[j + 64] * xr[j + 64];
    acc2 += a[j + 128] * xr[j + 128];
    acc3 += a[j + 192] * xr[j + 192];
  }
  for (; j < Mg; j += 64) acc0 += a[j] * xr[j];
  const double acc = wave_sum((acc0 + acc1) + (acc2 + acc3));
  if (ln == 0) y[(int64_t)r * ldy + row] = alpha * acc;
}

void launch_gemv_blocks_with(const Geometry &g, const double *A,
                             const double *x, int64_t ldx, int nrhs, double *y,
                             int64_t ldy, double alpha, hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_gemv_blocks, dim3((g.M + 3) / 4, nrhs), dim3(256), 0,
                     s, g.M, g.isl_geo.p, g.dgisl.p, g.dgsinv.p, A, x, ldx, y,
                     ldy, alpha);
  LBS_HIP(hipGetLastError());
}

void launch_gemv_blocks(const Geometry &g, const double *x, int64_t ldx,
                        int nrhs, double *y, int64_t ldy, double alpha,
                        hipStream_t s) {
  launch_gemv_blocks_with(g, g.Sinv.p, x, ldx, nrhs, y, ldy, alpha, s);
}

// AT = transpose of every diagonal block of A (block per row)
__global__ void k_transpose_blocks(const int32_t *__restrict__ isl_geo,
                                   const int32_t *__restrict__ gisl,
                                   const int64_t *__restrict__ gsinv,
                                   const double *__restrict__ A,
                                   double *__restrict__ AT) {
  const int row = blockIdx.x;
  const int g = isl_geo[row];
  const int m0 = gisl[g], Mg = gisl[g + 1] - m0, rl = row - m0;
  const int64_t base = gsinv[g];
  for (int j = threadIdx.x; j < Mg; j += blockDim.x)
    AT[base + (int64_t)j * Mg + rl] = A[base + (int64_t)rl * Mg + j];
}

void launch_transpose_blocks(const Geometry &g, const double *A, double *AT,
                             hipStream_t s) {
  if (g.M == 0) return;
  hipLaunchKernelGGL(k_transpose_blocks, dim3(g.M), dim3(256), 0, s,
                     g.isl_geo.p, g.dgisl.p, g.dgsinv.p, A, AT);
  LBS_HIP(hipGetLastError());
}

// u_t += sum_m A_m G(x_t, c_m) + add[r G + geometry] over the islands of
// target t's geometry (direct, one thread per target).
__global__ void __launch_bounds__(256)
    k_eval_logsrc(int64_t T, const double *__restrict__ txyz,
                  const int32_t *__restrict__ tgeo, int G,
                  const int32_t *__restrict__ gisl,
                  const double *__restrict__ cxyz,
                  const double *__restrict__ A, int64_t lda,
                  const double *__restrict__ add, double *__restrict__ u,
                  int64_t ldu) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (t >= T) return;
  const int g = tgeo ? tgeo[t] : 0;
  const double x0 = txyz[3 * t], x1 = txyz[3 * t + 1], x2 = txyz[3 * t + 2];
  double acc = 0.0, asum = 0.0;
  const double *Ar = A + (int64_t)r * lda;
  for (int m = gisl[g]; m < gisl[g + 1]; ++m) {
    const double d0 = x0 - cxyz[3 * m], d1 = x1 - cxyz[3 * m + 1],
                 d2 = x2 - cxyz[3 * m + 2];
    acc += Ar[m] * log(d0 * d0 + d1 * d1 + d2 * d2);
    asum += Ar[m];
  }
  // G = -(1/4pi) log|d|^2 + log2/4pi
  u[(int64_t)r * ldu + t] += -0.25 * kInvPi * acc +
                             0.25 * kInvPi * kLog2 * asum + add[r * G + g];
}

// The same for one geometry, split over chunks of 256 islands (grid y) so
// that a target set of ~1e5 fills the chip: each work-group stages its
// chunk's centres and strengths in LDS, each thread sums them for one
// target into part[(r nch + chunk) T + t]; k_eval_logsrc_fin adds the
// chunks in order.
__global__ void __launch_bounds__(256)
    k_eval_logsrc_part(int64_t T, const double *__restrict__ txyz, int M,
                       const double *__restrict__ cxyz, const double *__restrict__ A,
                       int64_t lda, double *__restrict__ part) {
  __shared__ double4 sc[256];  // centre, A
  const int ch = blockIdx.y, r = blockIdx.z, tid = threadIdx.x, nch = gridDim.y;
  const int m0 = ch * 256, nm = min(256, M - m0);
  if (tid < nm) {
    const int m = m0 + tid;
    sc[tid] = make_double4(cxyz[3 * m], cxyz[3 * m + 1], cxyz[3 * m + 2],
                           A[(int64_t)r * lda + m]);
  }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * 256 + tid;
  if (t >= T) return;
  const double x0 = txyz[3 * t], x1 = txyz[3 * t + 1], x2 = txyz[3 * t + 2];
  double acc = 0.0;
  for (int j = 0; j < nm; ++j) {
    const double4 c = sc[j];
    const double d0 = x0 - c.x, d1 = x1 - c.y, d2 = x2 - c.z;
    acc += c.w * log(d0 * d0 + d1 * d1 + d2 * d2);
  }
  part[((int64_t)r * nch + ch) * T + t] = acc;
}

__global__ void __launch_bounds__(256)
    k_eval_logsrc_fin(int64_t T, int nch, const double *__restrict__ part, int M,
                      const double *__restrict__ A, int64_t lda, const double *__restrict__ add,
                      double *__restrict__ u, int64_t ldu) {
  __shared__ double red[4];
  const int r = blockIdx.y, tid = threadIdx.x;
  // sum of A (every work-group forms it; 2000 values)
  double as = 0.0;
  for (int m = tid; m < M; m += 256) as += A[(int64_t)r * lda + m];
  for (int o = 32; o > 0; o >>= 1) as += __shfl_xor(as, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = as;
  __syncthreads();
  const double asum = red[0] + red[1] + red[2] + red[3];
  const int64_t t = (int64_t)blockIdx.x * 256 + tid;
  if (t >= T) return;
  double acc = 0.0;
  for (int c = 0; c < nch; ++c) acc += part[((int64_t)r * nch + c) * T + t];
  // G = -(1/4pi) log|d|^2 + log2/4pi
  u[(int64_t)r * ldu + t] += -0.25 * kInvPi * acc + 0.25 * kInvPi * kLog2 * asum + add[r];
}

void launch_eval_logsrc(const Geometry &g, int64_t T, const double *txyz,
                        const int32_t *tgeo, const double *A, int64_t lda,
                        int nrhs, const double *add, double *u, int64_t ldu,
                        hipStream_t s, DBuf<double> *scratch) {
  if (T == 0) return;
  if (g.G == 1 && scratch) {
    const int nch = (g.M + 255) / 256;
    const size_t need = (size_t)nch * T * nrhs;
    if (scratch->n < need) scratch->alloc(need);
    const unsigned gt = (unsigned)((T + 255) / 256);
    hipLaunchKernelGGL(k_eval_logsrc_part, dim3(gt, nch, nrhs), dim3(256), 0, s, T, txyz, g.M,
                       g.dcenter.p, A, lda, scratch->p);
    hipLaunchKernelGGL(k_eval_logsrc_fin, dim3(gt, nrhs), dim3(256), 0, s, T, nch, scratch->p,
                       g.M, A, lda, add, u, ldu);
  } else
    hipLaunchKernelGGL(k_eval_logsrc, dim3((unsigned)((T + 255) / 256), nrhs),
                       dim3(256), 0, s, T, txyz, tgeo, g.G, g.dgisl.p,
                       g.dcenter.p, A, lda, add, u, ldu);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------ segmented dots
// out[(v * R + r) * nseg + s] = sum_{i in segment s} a_v[r][i] b[r][i],
// a_v[r][i] = a[v * lav + r * lac + i], b[r][i] = b[r * lbc + i].
// Segments are unions of row chunks (seg of each chunk).
constexpr int kChunkRows = 2048;

__global__ void __launch_bounds__(256)
    k_seg_partial(const int64_t *__restrict__ c0, const int64_t *__restrict__ c1,
                  int nchunk, const double *__restrict__ a, int64_t lav,
                  int64_t lac, const double *__restrict__ b, int64_t lbc,
                  double *__restrict__ part) {
  __shared__ double red[4];
  const int c = blockIdx.x, r = blockIdx.y, v = blockIdx.z;
  const int R = gridDim.y;
  const double *ar = a + (int64_t)v * lav + (int64_t)r * lac;
  const double *br = b + (int64_t)r * lbc;
  double acc = 0.0;
  for (int64_t i = c0[c] + threadIdx.x; i < c1[c]; i += 256) acc += ar[i] * br[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    part[((int64_t)v * R + r) * nchunk + c] = red[0] + red[1] + red[2] + red[3];
}

// One wave per output value: lanes stride over the segment's chunks.
__global__ void __launch_bounds__(256)
    k_seg_reduce(int nseg, int nchunk, int64_t nout,
                 const int32_t *__restrict__ sptr,
                 const int32_t *__restrict__ sidx,
                 const double *__restrict__ part, double *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ln = threadIdx.x & 63;
  if (t >= nout) return;
  const int s = (int)(t % nseg);
  const int64_t vr = t / nseg;
  double acc = 0.0;
  for (int e = sptr[s] + ln; e < sptr[s + 1]; e += 64)
    acc += part[vr * nchunk + sidx[e]];
  acc = wave_sum(acc);
  if (ln == 0) out[t] = acc;
}

void SegPlan::build(const std::vector<std::vector<std::pair<int64_t, int64_t>>> &ranges,
                    hipStream_t s) {
  std::vector<int64_t> a0, a1;
  std::vector<int32_t> ptr(1, 0), idx;
  nseg = (int)ranges.size();
  for (int g = 0; g < nseg; ++g) {
    for (auto &rg : ranges[g])
      for (int64_t x = rg.first; x < rg.second; x += kChunkRows) {
        idx.push_back((int32_t)a0.size());
        a0.push_back(x);
        a1.push_back(std::min<int64_t>(rg.second, x + kChunkRows));
      }
    ptr.push_back((int32_t)idx.size());
  }
  nchunk = (int)a0.size();
  c0.upload(a0, s);
  c1.upload(a1, s);
  sptr.upload(ptr, s);
  sidx.upload(idx, s);
}

void launch_segdots(const SegPlan &sp, int R, int nvec, const double *a,
                    int64_t lav, int64_t lac, const double *b, int64_t lbc,
                    double *out, double *scratch, hipStream_t s) {
  if (sp.nchunk > 0)
    hipLaunchKernelGGL(k_seg_partial, dim3(sp.nchunk, R, nvec), dim3(256), 0,
                       s, sp.c0.p, sp.c1.p, sp.nchunk, a, lav, lac, b, lbc,
                       scratch);
  const int64_t n = (int64_t)nvec * R * sp.nseg;
  hipLaunchKernelGGL(k_seg_reduce, dim3((unsigned)((n + 3) / 4)), dim3(256),
                     0, s, sp.nseg, sp.nchunk, n, sp.sptr.p, sp.sidx.p,
                     scratch, out);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------------ GMRES parts
// Systems s = r * G + g (right-hand side r, geometry g) run GMRES(m) in
// lockstep on one Krylov array V[j][r][row], row over the N + M unknowns of
// all geometries; row_geo gives each row's geometry.  Per-system state:
// H[s][(m+1) m] (column-major per system), cs, sn, g (m+1), y, residual,
// tolerance, active flag and the number of Arnoldi columns in use.

// w[r][i] -= sum_{j < k1} h[j S + s] V_j[r][i]
__global__ void k_maxpy_seg(int64_t n, int R, int G, int k1,
                            const int32_t *__restrict__ row_geo,
                            const double *__restrict__ V, int64_t ldv,
                            const double *__restrict__ h,
                            double *__restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n) return;
  const int S = R * G;
  const int s = r * G + row_geo[i];
  const int64_t off = (int64_t)r * n + i;
  double acc = 0.0;
  for (int j = 0; j < k1; ++j) acc += h[j * S + s] * V[(int64_t)j * ldv + off];
  w[off] -= acc;
}

void launch_maxpy_seg(int64_t n, int R, int G, int k1, const int32_t *row_geo,
                      const double *V, int64_t ldv, const double *h, double *w,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_maxpy_seg, dim3((unsigned)((n + 255) / 256), R),
                     dim3(256), 0, s, n, R, G, k1, row_geo, V, ldv, h, w);
  LBS_HIP(hipGetLastError());
}

// x[r][i] += sum_{j < k} y[s][j] V_j[r][i]   (y zero beyond each system's k)
__global__ void k_update_seg(int64_t n, int R, int G, int k, int m,
                             const int32_t *__restrict__ row_geo,
                             const double *__restrict__ V, int64_t ldv,
                             const double *__restrict__ y,
                             double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n) return;
  const int s = r * G + row_geo[i];
  const int64_t off = (int64_t)r * n + i;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc += y[(int64_t)s * m + j] * V[(int64_t)j * ldv + off];
  x[off] += acc;
}

void launch_update_seg(int64_t n, int R, int G, int k, int m,
                       const int32_t *row_geo, const double *V, int64_t ldv,
                       const double *y, double *x, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_update_seg, dim3((unsigned)((n + 255) / 256), R),
                     dim3(256), 0, s, n, R, G, k, m, row_geo, V, ldv, y, x);
  LBS_HIP(hipGetLastError());
}

// v[r][i] = active[s] ? w[r][i] / sqrt(nrm2[s]) : 0
__global__ void k_normalize_seg(int64_t n, int R, int G,
                                const int32_t *__restrict__ row_geo,
                                const double *__restrict__ nrm2,
                                const int32_t *__restrict__ active,
                                const double *__restrict__ w,
                                double *__restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n) return;
  const int s = r * G + row_geo[i];
  const double q = sqrt(fmax(nrm2[s], 0.0));
  const int64_t off = (int64_t)r * n + i;
  v[off] = (active[s] && q > 0.0) ? w[off] / q : 0.0;
}

void launch_normalize_seg(int64_t n, int R, int G, const int32_t *row_geo,
                          const double *nrm2, const int32_t *active,
                          const double *w, double *v, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize_seg, dim3((unsigned)((n + 255) / 256), R),
                     dim3(256), 0, s, n, R, G, row_geo, nrm2, active, w, v);
  LBS_HIP(hipGetLastError());
}

// Cycle start: g = (beta, 0, ...), active = beta > tol, kused = 0; counts
// active systems into *count (reset by the caller's fill).
__global__ void k_gmres_start(int S, int m, const double *__restrict__ nrm2,
                              const double *__restrict__ tol,
                              double *__restrict__ g, int32_t *__restrict__ active,
                              int32_t *__restrict__ kused,
                              int32_t *__restrict__ count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const double beta = sqrt(fmax(nrm2[s], 0.0));
  for (int j = 0; j <= m; ++j) g[(int64_t)s * (m + 1) + j] = (j == 0) ? beta : 0.0;
  const int a = beta > tol[s];
  active[s] = a;
  kused[s] = 0;
  if (a) atomicAdd(count, 1);
}

void launch_gmres_start(int S, int m, const double *nrm2, const double *tol,
                        double *g, int32_t *active, int32_t *kused,
                        int32_t *count, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_start, dim3((S + 255) / 256), dim3(256), 0, s, S,
                     m, nrm2, tol, g, active, kused, count);
  LBS_HIP(hipGetLastError());
}

// Arnoldi step k for every active system: column k of H from the two CGS
// passes (h1 + h2) and the norm, previous rotations, new rotation, g
// update, residual, convergence flag; counts systems still active.
__global__ void k_givens_seg(int S, int k, int m, const double *__restrict__ h1,
                             const double *__restrict__ h2,
                             const double *__restrict__ nrm2,
                             const double *__restrict__ tol,
                             double *__restrict__ H, double *__restrict__ cs,
                             double *__restrict__ sn, double *__restrict__ g,
                             double *__restrict__ resid,
                             int32_t *__restrict__ active,
                             int32_t *__restrict__ kused,
                             int32_t *__restrict__ count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || !active[s]) return;
  double *h = H + (int64_t)s * (m + 1) * m + (int64_t)k * (m + 1);
  double *c = cs + (int64_t)s * m, *sg = sn + (int64_t)s * m;
  double *gg = g + (int64_t)s * (m + 1);
  for (int j = 0; j <= k; ++j) h[j] = h1[j * S + s] + (h2 ? h2[j * S + s] : 0.0);
  h[k + 1] = sqrt(fmax(nrm2[s], 0.0));
  for (int j = 0; j < k; ++j) {
    const double t = c[j] * h[j] + sg[j] * h[j + 1];
    h[j + 1] = -sg[j] * h[j] + c[j] * h[j + 1];
    h[j] = t;
  }
  const double a = h[k], b = h[k + 1];
  const double den = hypot(a, b);
  double cc = 1.0, ss = 0.0;
  if (den > 0.0) {
    cc = a / den;
    ss = b / den;
  }
  c[k] = cc;
  sg[k] = ss;
  h[k] = den;
  h[k + 1] = 0.0;
  gg[k + 1] = -ss * gg[k];
  gg[k] = cc * gg[k];
  const double res = fabs(gg[k + 1]);
  resid[s] = res;
  kused[s] = k + 1;
  if (res <= tol[s] || !(res == res)) active[s] = 0;
  else atomicAdd(count, 1);
}

void launch_givens_seg(int S, int k, int m, const double *h1, const double *h2,
                       const double *nrm2, const double *tol, double *H,
                       double *cs, double *sn, double *g, double *resid,
                       int32_t *active, int32_t *kused, int32_t *count,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_givens_seg, dim3((S + 63) / 64), dim3(64), 0, s, S, k,
                     m, h1, h2, nrm2, tol, H, cs, sn, g, resid, active, kused,
                     count);
  LBS_HIP(hipGetLastError());
}

// y[s] = R_s^{-1} g_s over the first kused[s] columns (zeros beyond).
__global__ void k_backsolve_seg(int S, int m, const double *__restrict__ H,
                                const double *__restrict__ g,
                                const int32_t *__restrict__ kused,
                                double *__restrict__ y) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const double *Hs = H + (int64_t)s * (m + 1) * m;
  const double *gs = g + (int64_t)s * (m + 1);
  double *ys = y + (int64_t)s * m;
  const int k = kused[s];
  for (int i = m - 1; i >= k; --i) ys[i] = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    double acc = gs[i];
    for (int j = i + 1; j < k; ++j) acc -= Hs[(int64_t)j * (m + 1) + i] * ys[j];
    const double d = Hs[(int64_t)i * (m + 1) + i];
    ys[i] = d != 0.0 ? acc / d : 0.0;
  }
}

void launch_backsolve_seg(int S, int m, const double *H, const double *g,
                          const int32_t *kused, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_backsolve_seg, dim3((S + 63) / 64), dim3(64), 0, s, S,
                     m, H, g, kused, y);
  LBS_HIP(hipGetLastError());
}

// ------------------------------------------------------------ vectors
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

__global__ void k_fill_int(int64_t n, int32_t v, int32_t *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

void launch_fill_int(int64_t n, int32_t v, int32_t *x, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((n + 255) / 256)), dim3(256),
                     0, s, n, v, x);
  LBS_HIP(hipGetLastError());
}

// Strided copy of R columns: dst[r * ldd + i] = a * src[r * lds + i]
__global__ void k_copy_cols(int64_t n, double a, const double *__restrict__ src,
                            int64_t lds, double *__restrict__ dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i < n) dst[(int64_t)r * ldd + i] = a * src[(int64_t)r * lds + i];
}

void launch_copy_cols(int64_t n, int R, double a, const double *src, int64_t lds,
                      double *dst, int64_t ldd, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((n + 255) / 256), R),
                     dim3(256), 0, s, n, a, src, lds, dst, ldd);
  LBS_HIP(hipGetLastError());
}

// tol[s] = t * sqrt(nrm2[s])
__global__ void k_scale_sqrt(int S, double t, const double *__restrict__ nrm2,
                             double *__restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) out[s] = t * sqrt(fmax(nrm2[s], 0.0));
}

void launch_scale_sqrt(int S, double t, const double *nrm2, double *out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_scale_sqrt, dim3((S + 255) / 256), dim3(256), 0, s, S,
                     t, nrm2, out);
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
