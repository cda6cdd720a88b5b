// Evaluation of the Cauchy part of eq. eqn:u_multi at arbitrary sphere
// targets inside the handle's own quadtree (Section 5: the FMM that applies
// I + K serves the evaluation as well).  No tree is built per target set.
//
// With M_b, L_b the multipole and local expansions the node FMM forms for
// every box (levels >= 2), a target z in box B (the deepest box whose
// square holds z) receives
//     Re L_B(z) + the sources L_B leaves out,
// and L_B leaves out exactly the sources in the subtrees of B's colleagues
// (the boxes of B's level adjacent to B, B included) and in the leaves of
// coarser levels adjacent to B: by induction over the levels, L_parent
// leaves out the subtrees of the parent's colleagues and the coarser leaves
// adjacent to the parent; of the parent's colleagues' children, those not
// adjacent to B enter L_B through its V list, and of the coarser leaves
// adjacent to the parent, those not adjacent to B through its X list.  This
// holds whether B is a leaf or not, so a target in a quadrant of B that
// holds no nodes is served like one in a leaf.  The subtrees of the
// colleagues are walked from the top: a box whose 3 x 3 neighbourhood does
// not hold z is taken by its multipole (ratio sqrt(2) h / 3h = 0.47 at
// worst, the bound the V and W lists of the FMM itself have), a leaf that
// does hold it by the direct sum.  Targets outside the root square take
// the walk over the whole tree.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "cplx.h"
#include "lbs_internal.h"

namespace lbs {
namespace {

// Deepest box whose square holds (x, y), from root r (-1: outside the
// root square).  A point on a mid-line goes to the upper child, as the
// Morton keys of the tree builder put it.
__device__ int descend(double x, double y, int r, int max_level, const double *__restrict__ cxv,
                       const double *__restrict__ cyv, const double *__restrict__ rad,
                       const int32_t *__restrict__ lev, const int32_t *__restrict__ child0,
                       const int32_t *__restrict__ nchild, const uint8_t *__restrict__ leaf) {
  if (fabs(x - cxv[r]) > rad[r] || fabs(y - cyv[r]) > rad[r]) return -1;
  int b = r;
  while (!leaf[b] && lev[b] < max_level) {
    const double bx = cxv[b], by = cyv[b];
    const bool gx = x >= bx, gy = y >= by;
    const int c0 = child0[b], nc = nchild[b];
    int f = -1;
    for (int k = 0; k < nc; ++k) {
      const int ch = c0 + k;
      if ((cxv[ch] > bx) == gx && (cyv[ch] > by) == gy) f = ch;
    }
    if (f < 0) break;  // that quadrant holds no nodes
    b = f;
  }
  return b;
}

__global__ void __launch_bounds__(256)
    k_locate(int64_t n, const double *__restrict__ tx, const double *__restrict__ ty,
             const int64_t *__restrict__ idx, const int32_t *__restrict__ tgeo,
             const int32_t *__restrict__ roots, const double *__restrict__ cxv,
             const double *__restrict__ cyv, const double *__restrict__ rad,
             const int32_t *__restrict__ lev, const int32_t *__restrict__ child0,
             const int32_t *__restrict__ nchild, const uint8_t *__restrict__ leaf,
             uint64_t *__restrict__ keys, int32_t *__restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = roots[tgeo ? tgeo[idx[i]] : 0];
  const int b = descend(tx[i], ty[i], r, 1 << 30, cxv, cyv, rad, lev, child0, nchild, leaf);
  keys[i] = (uint64_t)(b + 1);
  vals[i] = (int32_t)i;
}

__global__ void __launch_bounds__(256)
    k_gather_located(int64_t n, const uint64_t *__restrict__ keys,
                     const int32_t *__restrict__ vals, const double *__restrict__ tx,
                     const double *__restrict__ ty, const int64_t *__restrict__ idx,
                     const int32_t *__restrict__ tgeo, const int32_t *__restrict__ roots,
                     double *__restrict__ ox, double *__restrict__ oy, int32_t *__restrict__ obox,
                     int32_t *__restrict__ oroot, int64_t *__restrict__ oidx) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int i = vals[j];
  ox[j] = tx[i];
  oy[j] = ty[i];
  obox[j] = (int32_t)keys[j] - 1;
  oroot[j] = roots[tgeo ? tgeo[idx[i]] : 0];
  oidx[j] = idx[i];
}

struct TreeView {
  const double *cx, *cy, *rad;
  const int32_t *lev, *parent, *child0, *nchild;
  const uint8_t *leaf;
  const int64_t *s0, *s1;
  const double *sx, *sy;
};

// Re sum_j p_j / (z - z_j) over the sources [a0, a1) (a source at z adds 0)
__device__ __forceinline__ double direct_sum(double x, double y, int64_t a0, int64_t a1,
                                             const double *__restrict__ sx,
                                             const double *__restrict__ sy,
                                             const cx<double> *__restrict__ p) {
  double f = 0.0;
  for (int64_t j = a0; j < a1; ++j) {
    const double dx = x - sx[j], dy = y - sy[j];
    const double d2 = fma(dx, dx, fma(dy, dy, 1e-300));
    const cx<double> pj = p[j];
    f += fma(pj.x, dx, pj.y * dy) / d2;
  }
  return f;
}

// Re of box b's multipole at z: sum_k a_k rho^(k+1), rho = rad_b / (z - c_b)
template <int P>
__device__ __forceinline__ double multipole_at(double x, double y, int b, const TreeView &t,
                                               const cx<double> *__restrict__ M) {
  const cx<double> rho = t.rad[b] * cinv(cx<double>{x - t.cx[b], y - t.cy[b]});
  const cx<double> *a = M + (int64_t)b * P;
  cx<double> acc = a[P - 1];
  for (int k = P - 2; k >= 0; --k) acc = cfma(acc, rho, a[k]);
  return (acc * rho).x;
}

// The sources of c's subtree at z, walked depth first without a stack
// (children are contiguous, so the next box is the next sibling or an
// ancestor's).  Levels 0 and 1 carry no multipoles and are always opened.
template <int P>
__device__ double subtree_at(double x, double y, int c, const TreeView &t,
                             const cx<double> *__restrict__ p, const cx<double> *__restrict__ M) {
  double f = 0.0;
  int b = c;
  for (;;) {
    const double h3 = 3.0 * t.rad[b];
    const bool open = t.lev[b] < 2 || (fabs(x - t.cx[b]) < h3 && fabs(y - t.cy[b]) < h3);
    if (open && !t.leaf[b]) {
      b = t.child0[b];
      continue;
    }
    f += open ? direct_sum(x, y, t.s0[b], t.s1[b], t.sx, t.sy, p) : multipole_at<P>(x, y, b, t, M);
    for (;;) {
      if (b == c) return f;
      const int pa = t.parent[b];
      if (b + 1 < t.child0[pa] + t.nchild[pa]) {
        ++b;
        break;
      }
      b = pa;
    }
  }
}

// One thread per target (targets sorted by their box), right-hand side
// blockIdx.y: out[r ldy + idx] = scale Re Psi(z).
template <int P>
__global__ void __launch_bounds__(64)
    k_eval_points(int64_t n, const double *__restrict__ tx, const double *__restrict__ ty,
                  const int32_t *__restrict__ tbox, const int32_t *__restrict__ troot,
                  const int64_t *__restrict__ tidx, TreeView t, const cx<double> *__restrict__ p,
                  int64_t ns, const cx<double> *__restrict__ M, const cx<double> *__restrict__ L,
                  int nbox, double *__restrict__ out, int64_t ldy, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = blockIdx.y;
  const cx<double> *pr = p + (int64_t)r * ns;
  const cx<double> *Mr = M + (int64_t)r * nbox * P;
  const double x = tx[i], y = ty[i];
  const int B = tbox[i], root = troot[i];
  double f = 0.0;
  if (B < 0 || t.lev[B] == 0) {
    f = subtree_at<P>(x, y, root, t, pr, Mr);
  } else {
    const int l = t.lev[B];
    const double h = t.rad[B], bx = t.cx[B], by = t.cy[B];
    if (l >= 2) {
      const double ir = 1.0 / h;
      const cx<double> w{(x - bx) * ir, (y - by) * ir};
      const cx<double> *Lb = L + ((int64_t)r * nbox + B) * P;
      cx<double> acc = Lb[P - 1];
      for (int k = P - 2; k >= 0; --k) acc = cfma(acc, w, Lb[k]);
      f = acc.x;
    }
    f += subtree_at<P>(x, y, B, t, pr, Mr);
    int coarse[8];  // at most one per neighbour square
    int nco = 0;
    for (int o = 0; o < 9; ++o) {
      if (o == 4) continue;  // B itself
      const double qx = bx + 2.0 * h * (double)(o % 3 - 1);
      const double qy = by + 2.0 * h * (double)(o / 3 - 1);
      const int c = descend(qx, qy, root, l, t.cx, t.cy, t.rad, t.lev, t.child0, t.nchild, t.leaf);
      if (c < 0) continue;
      if (t.lev[c] == l) {  // a colleague
        f += subtree_at<P>(x, y, c, t, pr, Mr);
        continue;
      }
      if (!t.leaf[c]) continue;  // no nodes in that square
      bool seen = false;         // a coarser leaf adjacent to B
      for (int k = 0; k < nco; ++k) seen = seen || coarse[k] == c;
      if (seen) continue;
      coarse[nco++] = c;
      f += direct_sum(x, y, t.s0[c], t.s1[c], t.sx, t.sy, pr);
    }
  }
  out[(int64_t)r * ldy + tidx[i]] = scale * f;
}

}  // namespace

void launch_locate_targets(int64_t n, const double *tx, const double *ty, const int64_t *idx,
                           const int32_t *tgeo, const DevPlan &pl, double *ox, double *oy,
                           int32_t *obox, int32_t *oroot, int64_t *oidx, hipStream_t s) {
  if (n <= 0) return;
  if (n >= (int64_t)INT32_MAX) throw ApiError{LBS_ERR_UNSUPPORTED, "more than 2^31 targets"};
  DBuf<uint64_t> keys;
  DBuf<int32_t> vals;
  keys.alloc((size_t)n);
  vals.alloc((size_t)n);
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_locate, dim3(g), dim3(256), 0, s, n, tx, ty, idx, tgeo, pl.roots.p,
                     pl.cx.p, pl.cy.p, pl.rad.p, pl.lev.p, pl.child0.p, pl.nchild.p, pl.leaf.p,
                     keys.p, vals.p);
  int bits = 1;
  while ((1ll << bits) <= (int64_t)pl.nbox) ++bits;
  sort_by_key(keys.p, vals.p, n, bits, s);
  hipLaunchKernelGGL(k_gather_located, dim3(g), dim3(256), 0, s, n, keys.p, vals.p, tx, ty, idx,
                     tgeo, pl.roots.p, ox, oy, obox, oroot, oidx);
  LBS_HIP(hipGetLastError());
  LBS_HIP(hipStreamSynchronize(s));  // keys, vals are released on return
}

void launch_eval_points(int P, int64_t n, const double *tx, const double *ty, const int32_t *tbox,
                        const int32_t *troot, const int64_t *tidx, const DevPlan &pl,
                        const double *pstr, const double *M, const double *L, int nrhs,
                        double *out, int64_t ldy, double scale, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  const TreeView t{pl.cx.p, pl.cy.p, pl.rad.p, pl.lev.p, pl.parent.p, pl.child0.p, pl.nchild.p,
                   pl.leaf.p, pl.s0.p, pl.s1.p, pl.sx.p, pl.sy.p};
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)nrhs);
  const auto *pc = (const cx<double> *)pstr;
  const auto *Mc = (const cx<double> *)M;
  const auto *Lc = (const cx<double> *)L;
#define LBS_EVAL_POINTS(PP)                                                                     \
  case PP:                                                                                      \
    hipLaunchKernelGGL((k_eval_points<PP>), grid, dim3(64), 0, s, n, tx, ty, tbox, troot, tidx, \
                       t, pc, pl.ns, Mc, Lc, pl.nbox, out, ldy, scale);                         \
    break;
  switch (P) {
    LBS_EVAL_POINTS(20)
    LBS_EVAL_POINTS(24)
    LBS_EVAL_POINTS(30)
    LBS_EVAL_POINTS(36)
    LBS_EVAL_POINTS(40)
    LBS_EVAL_POINTS(48)
    default:
      throw ApiError{LBS_ERR_UNSUPPORTED, "p64 must be one of 20, 24, 30, 36, 40, 48"};
  }
#undef LBS_EVAL_POINTS
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
