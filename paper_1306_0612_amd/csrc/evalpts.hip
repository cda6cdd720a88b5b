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

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

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

// 1 / d: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - d r) (each step squares the relative error)
__device__ __forceinline__ double recip_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

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
    f = fma(fma(pj.x, dx, pj.y * dy), recip_nr(d2), f);
  }
  return f;
}

// Re of box b's multipole at z: sum_k a_k rho^(k+1), rho = rad_b / (z - c_b)
template <int P>
__device__ __forceinline__ double multipole_at(double x, double y, int b, const TreeView &t,
                                               const cx<double> *__restrict__ M) {
  const double dx = x - t.cx[b], dy = y - t.cy[b];
  const double ir = t.rad[b] * recip_nr(fma(dx, dx, dy * dy));
  const cx<double> rho{dx * ir, -dy * ir};
  const cx<double> *a = M + (int64_t)b * P;
  cx<double> acc = a[P - 1];
  for (int k = P - 2; k >= 0; --k) acc = cfma(acc, rho, a[k]);
  return (acc * rho).x;
}

// c's subtree as seen from z, walked depth first without a stack (children
// are contiguous, so the next box is the next sibling or an ancestor's):
// v.far(b) for a box whose 3 x 3 neighbourhood does not hold z (taken by
// its multipole), v.direct(b) for a leaf whose neighbourhood does.  Levels
// 0 and 1 carry no multipoles and are always opened.
template <class Vis>
__device__ void walk_subtree(double x, double y, int c, const TreeView &t, Vis &v) {
  int b = c;
  for (;;) {
    const double h3 = 3.0 * t.rad[b];
    const bool open = t.lev[b] < 2 || (fabs(x - t.cx[b]) < h3 && fabs(y - t.cy[b]) < h3);
    if (open && !t.leaf[b]) {
      b = t.child0[b];
      continue;
    }
    if (open) v.direct(b);
    else v.far(b);
    for (;;) {
      if (b == c) return;
      const int pa = t.parent[b];
      if (b + 1 < t.child0[pa] + t.nchild[pa]) {
        ++b;
        break;
      }
      b = pa;
    }
  }
}

// The sources the local expansion of B leaves out, for z in B (B < 0: z
// outside the root square, or B the root: every source): the subtrees of
// B's colleagues and the coarser leaves adjacent to B.
template <class Vis>
__device__ void walk_near(double x, double y, int B, int root, const TreeView &t, Vis &v) {
  if (B < 0 || t.lev[B] == 0) {
    walk_subtree(x, y, root, t, v);
    return;
  }
  const int l = t.lev[B];
  const double h = t.rad[B], bx = t.cx[B], by = t.cy[B];
  walk_subtree(x, y, B, t, v);
  int coarse[8];  // at most one per neighbour square
  int nco = 0;
  for (int o = 0; o < 9; ++o) {
    if (o == 4) continue;  // B itself
    const double qx = bx + 2.0 * h * (double)(o % 3 - 1);
    const double qy = by + 2.0 * h * (double)(o / 3 - 1);
    const int c = descend(qx, qy, root, l, t.cx, t.cy, t.rad, t.lev, t.child0, t.nchild, t.leaf);
    if (c < 0) continue;
    if (t.lev[c] == l) {  // a colleague
      walk_subtree(x, y, c, t, v);
      continue;
    }
    if (!t.leaf[c]) continue;  // no nodes in that square
    bool seen = false;         // a coarser leaf adjacent to B
    for (int k = 0; k < nco; ++k) seen = seen || coarse[k] == c;
    if (seen) continue;
    coarse[nco++] = c;
    v.direct(c);
  }
}

template <int P>
struct SumVisitor {
  double x, y, f;
  TreeView t;
  const cx<double> *p, *M;
  __device__ void far(int b) { f += multipole_at<P>(x, y, b, t, M); }
  __device__ void direct(int b) { f += direct_sum(x, y, t.s0[b], t.s1[b], t.sx, t.sy, p); }
};

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
  const double x = tx[i], y = ty[i];
  const int B = tbox[i], root = troot[i];
  SumVisitor<P> v{x, y, 0.0, t, p + (int64_t)r * ns, M + (int64_t)r * nbox * P};
  if (B >= 0 && t.lev[B] >= 2) {
    const double ir = 1.0 / t.rad[B];
    const cx<double> w{(x - t.cx[B]) * ir, (y - t.cy[B]) * ir};
    const cx<double> *Lb = L + ((int64_t)r * nbox + B) * P;
    cx<double> acc = Lb[P - 1];
    for (int k = P - 2; k >= 0; --k) acc = cfma(acc, w, Lb[k]);
    v.f = acc.x;
  }
  walk_near(x, y, B, root, t, v);
  out[(int64_t)r * ldy + tidx[i]] = scale * v.f;
}

// ---------------------------------------------- sources at arbitrary points
// The transpose of the evaluation above: sources c_t at the located points
// t, the field at the tree's own points.  Transposing each step, a point t
// in box B enters
//   the multipole of B and of each ancestor of level >= 2 (the transpose of
//     B's local expansion at t and of the L2L steps that formed it),
//   the local expansion of every box its walk takes by multipole (the
//     transpose of that multipole's value at t),
//   the direct sums of every leaf its walk sums directly;
// then the tree's V lists (M2L), the downward pass, and at the leaves the
// local expansions, the W lists (the transpose of the X-list P2L) and the
// direct sums complete the field.  This kernel counts (FILL = false) or
// writes those (box, point) pairs: multipole, local, direct.
struct CountVisitor {
  uint32_t nl = 0, nd = 0;
  __device__ void far(int) { ++nl; }
  __device__ void direct(int) { ++nd; }
};
struct FillVisitor {
  int32_t *lb, *lt, *db, *dt;
  uint32_t lo, dof;
  int32_t ti;
  __device__ void far(int b) {
    lb[lo] = b;
    lt[lo++] = ti;
  }
  __device__ void direct(int b) {
    db[dof] = b;
    dt[dof++] = ti;
  }
};

template <bool FILL>
__global__ void __launch_bounds__(64)
    k_source_pairs(int64_t n, const double *__restrict__ tx, const double *__restrict__ ty,
                   const int32_t *__restrict__ tbox, const int32_t *__restrict__ troot,
                   TreeView t, uint32_t *__restrict__ cm, uint32_t *__restrict__ cl,
                   uint32_t *__restrict__ cd, int32_t *__restrict__ mb, int32_t *__restrict__ mt,
                   int32_t *__restrict__ lb, int32_t *__restrict__ lt, int32_t *__restrict__ db,
                   int32_t *__restrict__ dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = tx[i], y = ty[i];
  const int B = tbox[i], root = troot[i];
  uint32_t nm = 0;
  uint32_t mo = FILL ? cm[i] : 0u;
  for (int a = B; a >= 0 && t.lev[a] >= 2; a = t.parent[a]) {
    if constexpr (FILL) {
      mb[mo] = a;
      mt[mo++] = (int32_t)i;
    }
    ++nm;
  }
  if constexpr (FILL) {
    FillVisitor v{lb, lt, db, dt, cl[i], cd[i], (int32_t)i};
    walk_near(x, y, B, root, t, v);
  } else {
    CountVisitor v;
    walk_near(x, y, B, root, t, v);
    cm[i] = nm;
    cl[i] = v.nl;
    cd[i] = v.nd;
  }
}

// ptr[b] = the first position of sorted keys with key >= b (b <= nbox)
__global__ void __launch_bounds__(256)
    k_csr_ptr(int64_t n, const uint64_t *__restrict__ keys, int nbox, int64_t *__restrict__ ptr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > n) return;
  const int64_t lo = k == 0 ? -1 : (int64_t)keys[k - 1];
  const int64_t hi = k == n ? (int64_t)nbox : (int64_t)keys[k];
  for (int64_t b = lo + 1; b <= hi; ++b) ptr[b] = k;
}

// chunks of each multipole-list entry's pairs: counts, then their ranges
__global__ void __launch_bounds__(256)
    k_chunk_count(int n, const int32_t *__restrict__ list, const int64_t *__restrict__ ptr,
                  uint32_t *__restrict__ cnt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int b = list[e];
  cnt[e] = (uint32_t)((ptr[b + 1] - ptr[b] + kSrcChunk - 1) / kSrcChunk);
}

__global__ void __launch_bounds__(256)
    k_chunk_fill(int n, const int32_t *__restrict__ list, const int64_t *__restrict__ ptr,
                 const uint32_t *__restrict__ off, const double *__restrict__ cxv,
                 const double *__restrict__ cyv, const double *__restrict__ rad,
                 int64_t *__restrict__ rng, double4 *__restrict__ geo, int32_t *__restrict__ iota) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int b = list[e];
  const int64_t a0 = ptr[b], a1 = ptr[b + 1];
  const double4 gb = make_double4(cxv[b], cyv[b], 1.0 / rad[b], 0.0);
  for (uint32_t c = off[e]; c < off[e + 1]; ++c) {
    const int64_t lo = a0 + (int64_t)(c - off[e]) * kSrcChunk;
    rng[2 * (int64_t)c] = lo;
    rng[2 * (int64_t)c + 1] = lo + kSrcChunk < a1 ? lo + kSrcChunk : a1;
    geo[c] = gb;
    iota[c] = (int32_t)c;
  }
}

__global__ void __launch_bounds__(256)
    k_gather_xy(int64_t n, const int32_t *__restrict__ idx, const double *__restrict__ x,
                const double *__restrict__ y, double *__restrict__ ox, double *__restrict__ oy) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  ox[k] = x[idx[k]];
  oy[k] = y[idx[k]];
}

__global__ void __launch_bounds__(256)
    k_gather_cx(int64_t n, const int32_t *__restrict__ idx, const double2 *__restrict__ in,
                double2 *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  out[k] = in[idx[k]];
}

__global__ void __launch_bounds__(256)
    k_differ(int64_t n, const unsigned long long *__restrict__ a,
             const unsigned long long *__restrict__ b, int32_t *__restrict__ flag) {
  bool d = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d = d || a[i] != b[i];
  if (d) *flag = 1;  // every writer writes the same value
}

__global__ void __launch_bounds__(256)
    k_widen_keys(int64_t n, const int32_t *__restrict__ box, uint64_t *__restrict__ key) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  key[k] = (uint64_t)box[k];
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


bool targets_differ(int64_t n, const double *a, const double *b, int32_t *dflag,
                    int32_t *hflag, hipStream_t s) {
  if (n <= 0) return false;
  launch_fill_int(1, 0, dflag, s);
  const unsigned g = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_differ, dim3(g), dim3(256), 0, s, n, (const unsigned long long *)a,
                     (const unsigned long long *)b, dflag);
  LBS_HIP(hipGetLastError());
  LBS_HIP(hipMemcpyAsync(hflag, dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LBS_HIP(hipStreamSynchronize(s));
  return *hflag != 0;
}

void launch_gather_cx(int64_t n, const int32_t *idx, const double *in, double *out,
                      hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_cx, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, idx,
                     (const double2 *)in, (double2 *)out);
  LBS_HIP(hipGetLastError());
}

namespace {
// Wall time of the phases of a build, printed to stderr when
// LBS_HOST_TIMING is set (each mark waits for the stream first).
struct BuildClock {
  bool on = std::getenv("LBS_HOST_TIMING") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char *name, hipStream_t s) {
    if (!on) return;
    LBS_HIP(hipStreamSynchronize(s));
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[lbs host] point sources: %-14s %9.3f ms\n", name,
                 std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

// (box, point) pairs sorted by box (stable, so points keep their order
// within a box) and their CSR offsets over the plan's boxes; key is
// scratch of at least n + 1 entries.
void pairs_by_box(int64_t n, const int32_t *box, int32_t *pt, int nbox, uint64_t *key,
                  SortBufs &sc, DBuf<int64_t> &ptr, hipStream_t s) {
  ptr.alloc((size_t)nbox + 1);
  if (n > 0) {
    hipLaunchKernelGGL(k_widen_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, box,
                       key);
    int bits = 1;
    while ((1ll << bits) <= (int64_t)nbox) ++bits;
    sort_by_key(key, pt, n, bits, sc, s);
  }
  hipLaunchKernelGGL(k_csr_ptr, dim3((unsigned)((n + 256) / 256)), dim3(256), 0, s, n, key, nbox,
                     ptr.p);
  LBS_HIP(hipGetLastError());
}
}  // namespace

void build_point_sources(const DevPlan &pl, int64_t n, const double *x, const double *y,
                         const int32_t *box, const int32_t *root, PointSources &ps,
                         hipStream_t s) {
  ps.n = n;
  ps.x = x;
  ps.y = y;
  ps.n_m = 0;
  ps.nm = 0;
  if (n <= 0) return;
  if (n >= (int64_t)INT32_MAX) throw ApiError{LBS_ERR_UNSUPPORTED, "more than 2^31 points"};
  BuildClock clk;
  const TreeView t{pl.cx.p, pl.cy.p, pl.rad.p, pl.lev.p, pl.parent.p, pl.child0.p, pl.nchild.p,
                   pl.leaf.p, pl.s0.p, pl.s1.p, pl.sx.p, pl.sy.p};
  // counts of the three kinds of pairs per point, scanned into offsets
  const int64_t n1 = n + 1, nts = (n1 + 4095) / 4096;
  DBuf<uint32_t> cnt;
  cnt.alloc((size_t)(3 * n1 + 3 * nts));
  uint32_t *cm = cnt.p, *cl = cm + n1, *cd = cl + n1, *sums = cd + n1;
  LBS_HIP(hipMemsetAsync(cnt.p, 0, (size_t)(3 * n1) * sizeof(uint32_t), s));
  const unsigned g = (unsigned)((n + 63) / 64);
  hipLaunchKernelGGL(k_source_pairs<false>, dim3(g), dim3(64), 0, s, n, x, y, box, root, t, cm, cl,
                     cd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  for (uint32_t *c : {cm, cl, cd}) scan_into(c, n1, sums, s);
  uint32_t tot[3] = {0, 0, 0};
  LBS_HIP(hipMemcpyAsync(&tot[0], cm + n, 4, hipMemcpyDeviceToHost, s));
  LBS_HIP(hipMemcpyAsync(&tot[1], cl + n, 4, hipMemcpyDeviceToHost, s));
  LBS_HIP(hipMemcpyAsync(&tot[2], cd + n, 4, hipMemcpyDeviceToHost, s));
  LBS_HIP(hipStreamSynchronize(s));
  clk.mark("count", s);
  const int64_t nm = tot[0], nl = tot[1], nd = tot[2];
  const int64_t nmax = std::max<int64_t>({nm, nl, nd, 1});
  DBuf<int32_t> boxes;  // the pairs' boxes, each kind in turn
  boxes.alloc((size_t)(nm + nl + nd + 1));
  int32_t *mb = boxes.p, *lb = mb + nm, *db = lb + nl;
  ps.m_t.alloc((size_t)std::max<int64_t>(nm, 1));
  ps.l_t.alloc((size_t)std::max<int64_t>(nl, 1));
  ps.d_t.alloc((size_t)std::max<int64_t>(nd, 1));
  hipLaunchKernelGGL(k_source_pairs<true>, dim3(g), dim3(64), 0, s, n, x, y, box, root, t, cm, cl,
                     cd, mb, ps.m_t.p, lb, ps.l_t.p, db, ps.d_t.p);
  LBS_HIP(hipGetLastError());
  clk.mark("fill", s);
  DBuf<uint64_t> key;
  key.alloc((size_t)nmax + 1);
  SortBufs sc;
  DBuf<int64_t> mptr;
  pairs_by_box(nm, mb, ps.m_t.p, pl.nbox, key.p, sc, mptr, s);
  pairs_by_box(nl, lb, ps.l_t.p, pl.nbox, key.p, sc, ps.l_ptr, s);
  pairs_by_box(nd, db, ps.d_t.p, pl.nbox, key.p, sc, ps.d_ptr, s);
  ps.nm = nm;
  clk.mark("sort", s);
  // multipoles and local expansions: every box of level >= 2 (the kernels
  // pass over boxes without pairs)
  std::vector<int32_t> ml;
  ml.reserve((size_t)pl.nbox);
  for (int b = 0; b < pl.nbox; ++b)
    if (pl.host.level[b] >= 2) ml.push_back(b);
  ps.n_m = (int)ml.size();
  ps.m_list.upload(ml, s);
  // chunks of at most kSrcChunk pairs, one wave each
  {
    DBuf<uint32_t> coff;
    coff.alloc((size_t)ps.n_m + 1);
    LBS_HIP(hipMemsetAsync(coff.p, 0, ((size_t)ps.n_m + 1) * sizeof(uint32_t), s));
    const unsigned gm = (unsigned)((ps.n_m + 255) / 256);
    if (ps.n_m > 0)
      hipLaunchKernelGGL(k_chunk_count, dim3(gm), dim3(256), 0, s, ps.n_m, ps.m_list.p, mptr.p,
                         coff.p);
    DBuf<uint32_t> csum;
    csum.alloc((size_t)((ps.n_m + 1 + 4095) / 4096 + 1));
    scan_into(coff.p, (int64_t)ps.n_m + 1, csum.p, s);
    uint32_t nc = 0;
    LBS_HIP(hipMemcpyAsync(&nc, coff.p + ps.n_m, 4, hipMemcpyDeviceToHost, s));
    LBS_HIP(hipStreamSynchronize(s));
    ps.n_c = (int)nc;
    ps.c_rng.alloc((size_t)2 * std::max(ps.n_c, 1));
    ps.c_geo.alloc((size_t)std::max(ps.n_c, 1));
    ps.c_iota.alloc((size_t)std::max(ps.n_c, 1));
    ps.c_part.alloc((size_t)std::max(ps.n_c, 1) * 2 * 48);  // orders up to 48
    if (ps.n_m > 0)
      hipLaunchKernelGGL(k_chunk_fill, dim3(gm), dim3(256), 0, s, ps.n_m, ps.m_list.p, mptr.p,
                         coff.p, pl.cx.p, pl.cy.p, pl.rad.p, ps.c_rng.p, ps.c_geo.p,
                         ps.c_iota.p);
    ps.c_ptr.take(coff);
    LBS_HIP(hipStreamSynchronize(s));  // csum is released on return
  }
  ps.m_x.alloc((size_t)std::max<int64_t>(nm, 1));
  ps.m_y.alloc((size_t)std::max<int64_t>(nm, 1));
  ps.m_p.alloc((size_t)2 * std::max<int64_t>(nm, 1));
  if (nm > 0)
    hipLaunchKernelGGL(k_gather_xy, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, nm,
                       ps.m_t.p, x, y, ps.m_x.p, ps.m_y.p);
  LBS_HIP(hipGetLastError());
  LBS_HIP(hipStreamSynchronize(s));  // scratch and host lists are released on return
  clk.mark("lists", s);
}

}  // namespace lbs
