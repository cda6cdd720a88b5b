// Internal declarations shared by the host driver (api.cpp) and the HIP
// kernel files.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbs.h"
#include "tree.h"

namespace lbs {

struct HipError {
  hipError_t code;
  std::string where;
};
struct ApiError {
  lbs_status code;
  std::string msg;
};

#define LBS_HIP(call)                                                     \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess)                                                 \
      throw ::lbs::HipError{e_, std::string(#call) + " @" __FILE__ ":" +   \
                                    std::to_string(__LINE__)};            \
  } while (0)

// Device buffer with RAII release.
// A view (view()) borrows memory it does not free.
template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  bool own = true;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p && own) (void)hipFree(p);
    p = nullptr;
    n = 0;
    own = true;
  }
  void view(T *q, size_t count) {
    release();
    p = q;
    n = count;
    own = false;
  }
  void take(DBuf &o) {  // ownership of o's memory moves here
    release();
    p = o.p;
    n = o.n;
    own = o.own;
    o.p = nullptr;
    o.n = 0;
    o.own = true;
  }
  void alloc(size_t count) {
    release();
    n = count;
    if (count == 0) return;
    hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      n = 0;
      if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        throw ApiError{LBS_ERR_OUT_OF_MEMORY,
                       "device allocation of " +
                           std::to_string(count * sizeof(T)) + " bytes"};
      throw HipError{e, "hipMalloc"};
    }
  }
  void upload(const std::vector<T> &v, hipStream_t s) {
    alloc(v.size());
    if (!v.empty())
      LBS_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T),
                             hipMemcpyHostToDevice, s));
  }
  std::vector<T> download(hipStream_t s) const {
    std::vector<T> v(n);
    if (n) {
      LBS_HIP(hipMemcpyAsync(v.data(), p, n * sizeof(T),
                             hipMemcpyDeviceToHost, s));
      LBS_HIP(hipStreamSynchronize(s));
    }
    return v;
  }
};

// A pass program on the device (PassProgram in tree.h): its LDS capacity,
// the host ranges of the rounds and the component tables.
struct DevPass {
  int cap = 0;
  std::vector<int32_t> round_ptr;
  DBuf<int32_t> hdr, ext, par, stp;
};

// Quadtree and lists on the device (one FMM plan).
// A target leaf as the leaf kernels see it (one per work-group): its
// target range, the range of its flattened U-list sources, its W-list
// range, box id, level, centre and 1 / half-width.
struct LeafHdr {
  int64_t t0, nt, uf0, uf1;
  int32_t wb, we, b, lev;
  double cx, cy, ir, pad;
};

// work-groups (4 waves each) of the FP32 M2L kernel at most by default
// (option m2l_groups); its waves stride over the M2L boxes.  4096 waves are
// one resident round on 256 CUs at the kernel's occupancy of 4 per SIMD.
constexpr int kM2LGroups = 1024;

struct DevPlan {
  int nbox = 0, nlevels = 0;
  int64_t ns = 0, nt = 0;
  bool self = true;
  std::vector<int32_t> level_ptr;            // host copy
  std::vector<int32_t> leaf_t_host;          // leaves with targets
  std::vector<int32_t> leaf_s_host;          // leaves with sources
  int n_leaf_t = 0, n_leaf_s = 0, n_m2l = 0;
  int m2l_groups = kM2LGroups;               // FP32 M2L launch width
  DBuf<double> cx, cy, rad;
  DBuf<int32_t> parent, child0, nchild, quad, lev;
  DBuf<int32_t> roots;                       // root box of each geometry
  DBuf<int64_t> s0, s1, t0, t1;
  DBuf<uint8_t> leaf, has_tgt;
  DBuf<int32_t> v_ptr, v_src, w_ptr, w_src;
  // per box, the sources of its X list concatenated (as uf_* for U)
  DBuf<int64_t> xf_ptr;
  DBuf<int32_t> xf_idx;
  // per box, the sources of its U list concatenated in list order (tree
  // order indices; offsets uf_ptr[b] .. uf_ptr[b + 1])
  DBuf<int64_t> uf_ptr;
  DBuf<int32_t> uf_idx;
  DBuf<uint8_t> v_code;
  DBuf<int32_t> leaf_t, leaf_s, m2l_box;     // work lists
  // per entry of leaf_t: what the leaf kernels read about the leaf
  DBuf<LeafHdr> lt_hdr;
  // per entry of leaf_s: its source range (s0, s1) and (cx, cy, 1/rad, 0)
  DBuf<int64_t> ls_rng;
  DBuf<double4> ls_geo;
  DBuf<int32_t> m2l_wave;  // M2L boxes in the FP32 kernel's wave order
  // Upward (M2M) and downward (L2L) pass programs (PassProgram in tree.h)
  // for the FP32 ([0]) and FP64 ([1]) expansion orders of the handle.
  DevPass up[2], dn[2];
  // points in tree order
  DBuf<double> sx, sy, tx, ty;
  DBuf<int64_t> src_perm, tgt_perm;
  // handle plans: each source's position relative to its leaf (centre,
  // radius) in FP32 and src_perm as 32-bit indices, for the FP32 leaf
  // multipoles (build_p2m_inputs32; empty on evaluation plans)
  DBuf<float2> w32;
  DBuf<int32_t> perm32;
  Tree host;                                  // host tree (statistics)
};

// Translation tables for expansions of P terms (see fmm.hip).
struct Tables {
  int P = 0;
  // M2M / L2L: binomials (P x P, real) and the pre/post scale powers
  // (4 x P, complex); M2L matrix H and inverse powers (itp)
  DBuf<double> bc64, pre64, post64, h64, itp64;
  DBuf<float> bc32, pre32, post32, h32, itp32;
};
// Per-stage GPU timing with HIP events recorded on the launch stream.
enum Stage {
  ST_STRENGTHS = 0, ST_UPWARD, ST_L2L, ST_M2L, ST_P2L, ST_LEAF, ST_GAMMA,
  ST_LOGSRC, ST_CONSTRAINT, ST_NSTAGES
};
struct StageTimer {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Pending {
    int st;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  double ms[ST_NSTAGES] = {};
  int64_t cnt[ST_NSTAGES] = {};
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      LBS_HIP(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(int st, hipStream_t s) {
    hipEvent_t a = get();
    LBS_HIP(hipEventRecord(a, s));
    pending.push_back({st, a, nullptr});
  }
  void end(hipStream_t s) {
    hipEvent_t b = get();
    LBS_HIP(hipEventRecord(b, s));
    pending.back().b = b;
  }
  void collect() {
    for (auto &p : pending) {
      float f = 0;
      LBS_HIP(hipEventSynchronize(p.b));
      LBS_HIP(hipEventElapsedTime(&f, p.a, p.b));
      ms[p.st] += f;
      cnt[p.st] += 1;
    }
    pending.clear();
    used = 0;
  }
  ~StageTimer() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};
struct TimerScope {
  StageTimer *t;
  hipStream_t s;
  TimerScope(StageTimer *t_, int st, hipStream_t s_) : t(t_), s(s_) {
    if (t) t->begin(st, s);
  }
  ~TimerScope() {
    if (t) t->end(s);
  }
};


// Island geometry of a handle: G >= 1 independent geometries, nodes and
// islands numbered geometry-major (curve-major inside a geometry).
struct Geometry {
  int64_t N = 0;
  int M = 0;
  int G = 1;
  int maxM = 0;                      // largest island count of a geometry
  std::vector<int32_t> nodes;        // per island
  std::vector<int64_t> offs;         // node offset per island (M+1)
  std::vector<int64_t> gnode;        // node offset per geometry (G+1)
  std::vector<int32_t> gisl;         // island offset per geometry (G+1)
  std::vector<int64_t> gsinv;        // offset of each S^-1 block (G+1)
  std::vector<double> sign;          // orientation sign per island
  std::vector<double> cxyz;          // centres (M x 3)
  std::vector<double> eta_x, eta_y;  // projected centres
  std::vector<double> rho;           // planar island radius about eta
  // device, API order
  DBuf<double> xyz;                  // N x 3
  DBuf<double> xi, dxi, ddxi;        // complex interleaved (N x 2)
  DBuf<double> qfac;                 // (s h / pi) xi'   complex (N x 2)
  DBuf<double> tau;                  // -(s h / 2 pi) Im(xi''/xi')
  DBuf<double> gw;                   // (s h / pi) Im(conj(xi) xi' / (1+|xi|^2))
  DBuf<double> ell;                  // log(1 + |xi|^2)
  DBuf<int32_t> island;              // island of each node
  DBuf<int32_t> node_geo, isl_geo;   // geometry of each node / island
  DBuf<int32_t> row_geo;             // geometry of each unknown (N + M)
  DBuf<double> qfac_t;               // qfac in tree order
  DBuf<float2> qm32_t;               // -i qfac in tree order, FP32 (Im, -Re)
  DBuf<double> gw_t;                 // gamma weights in tree order
  DBuf<int32_t> gleaf_ptr;           // per geometry: range in leaf_s
  int gleaf_chunks = 1;              // most 2048-leaf chunks of a geometry
  DBuf<double> dcenter, deta, drho, dellc;  // centres, eta, rho, log(1+|eta|^2)
  DBuf<int64_t> doffs, dgnode, dgsinv;
  DBuf<int32_t> dgisl;
  DBuf<int32_t> near_ptr, near_idx;  // near centres per island (log sources)
  // log sources in each island's own frame (projection from the antipode of
  // its centre): node images xi', log(1 + |xi'|^2), radius max|xi'|, frame
  // vectors (e1, e2 per island), near centres (|eta'| <= 3 rho') and the
  // transposed lists (islands having a centre as near), sorted
  DBuf<double> xil, elll, rhol, frame;
  DBuf<int32_t> nearR_ptr, nearR_idx, nearRT_ptr, nearRT_idx;
  // far pairs (k, m) of the same geometry, m not near k, with the series
  // ratio q_km = 2 rho'_k (a - i b) / |c_k - c_m|^2 (interleaved complex)
  // and h_km = log|c_k - c_m|^2 / 2.  Grouped by k (far_*), each group
  // sorted by |q| (largest first, ties by m), with per chunk of kLogChunk
  // entries the number of series terms its first |q| needs (far_nt, chunk
  // offsets far_cptr).  The transposed kernel forms q_km and h_km from the
  // centres and frames instead (its m-major order would need a table of
  // every pair of a geometry).
  DBuf<int64_t> far_ptr, far_cptr;
  DBuf<int32_t> far_idx, far_nt;
  DBuf<double> far_q, far_h;
  DBuf<lbs_island> disl;             // island parameters
  DBuf<double> dsign;                // orientation sign per island
  DBuf<double> Sinv;                 // block-diagonal inverse Schur complement
  DBuf<double> SinvT;                // its transpose (adjoint; made on first use)
  // close-evaluation zone per island: cos of its angular radius (the
  // largest node distance from the centre plus ten node spacings)
  std::vector<double> zone_cos;
  bool sampled = false;              // nodes given as samples (no shape
                                     // coefficients)
};

// Targets of an evaluation that lie in the close zone of one or more
// islands (close.hip): planar position and output index per close target,
// its islands in CSR form, and the islands that occur at all.
struct ClosePlan {
  int n_tgt = 0, n_act = 0;
  DBuf<double> z;          // 2 per close target
  DBuf<int64_t> out;       // target's position in the output
  DBuf<int32_t> ptr, isl;  // islands of close target t: isl[ptr[t] .. ptr[t+1])
  DBuf<int32_t> act;       // islands with a close target
};

// Segments of rows for segmented dot products: each segment is a union of
// row chunks of at most 2048 rows.
struct SegPlan {
  int nseg = 0, nchunk = 0;
  DBuf<int64_t> c0, c1;
  DBuf<int32_t> sptr, sidx;
  void build(const std::vector<std::vector<std::pair<int64_t, int64_t>>> &ranges,
             hipStream_t s);
};

struct Workspace {
  StageTimer *timer = nullptr;
  int nrhs_cap = 0;
  DBuf<double> pstr64, mult64, loc64;
  DBuf<float> pstr32, mult32, loc32;
  DBuf<double> gam;       // per (rhs, geometry)
  DBuf<double> gpart;     // per (rhs, source leaf): partial gamma sums
  DBuf<double> gcsum;     // per (rhs, geometry, chunk): chunk sums of gpart
  DBuf<int32_t> gcnt;     // per (rhs, geometry): finished chunks (kept 0)
  DBuf<double> red;       // reduction scratch
  DBuf<double> tmpM, logL;
  void ensure(const DevPlan &pl, int P64, int P32, int nrhs, int64_t N,
              int M, int G, int Plog);
};

constexpr int kPlog = 30;  // terms of the per-island log-source expansions
constexpr int kLogChunk = 64;  // far-list entries per wave step

void set_last_error(const std::string &msg);  // message of lbs_last_error
// Device arrays of a GPU-built tree that a plan may take instead of host
// copies: the sorted position -> input index maps of sources and targets.
struct DevPerms {
  DBuf<int32_t> src, tgt;
};
// build_tree on the GPU (gtree.hip): device coordinates x[i stride],
// y[i stride]; the same Tree as the host builder.  Synchronous.  With
// keep, the maps are handed over on the device and T.src_perm /
// T.tgt_perm stay empty.
void gpu_build_tree(const double *sx, const double *sy, int64_t sstride, int64_t ns,
                    const double *tx, const double *ty, int64_t tstride, int64_t nt, bool self,
                    int leaf_max, Tree &T, hipStream_t s,
                    DevPerms *keep = nullptr);
// lbs_matvec with its scratch buffers in `bytes` of device memory at base
// (api.cpp; the entry point without allocation passes its static scratch)
lbs_status matvec_in_scratch(lbs_handle h, int32_t op, int32_t prec, int32_t nrhs,
                             const double *x, double *y, void *stream, char *base,
                             size_t bytes);

// ----- launchers (HIP files) ------------------------------------------
void build_tables(Tables &t, int P, hipStream_t s);
void launch_geometry(const lbs_island *isl_dev, int M, const int64_t *offs_dev,
                     const int32_t *island_dev, int64_t N, double *xyz,
                     double *xi, double *dxi, double *ddxi, hipStream_t s);
void launch_geometry_sampled(int64_t N, const double *x, const double *xt,
                             const double *xtt, double *xyz, double *xi,
                             double *dxi, double *ddxi, hipStream_t s);
void launch_node_coeffs(int64_t N, const int32_t *island, const double *sign,
                        const int64_t *offs, const double *xi,
                        const double *dxi, const double *ddxi, double *qfac,
                        double *tau, double *gw, double *ell, hipStream_t s);
void launch_local_frame(int64_t N, const int32_t *island,
                        const lbs_island *isl, const double *xyz, double *xil,
                        double *elll, hipStream_t s);
void launch_permute_complex(int64_t n, const int64_t *perm, const double *in,
                            double *out, hipStream_t s);

// Operator-row assembly fused into the leaf kernel:
//   out[api] = scale * field + (ident + tau[api]) sigma[api] + gamma[r G + geo[api]]
struct Assembly {
  const double *sigma = nullptr;  // API order, stride ldx (null: no terms)
  const double *tau = nullptr;    // diagonal coefficient per node
  const double *gamma = nullptr;  // per (rhs, geometry) constant
  const int32_t *geo = nullptr;   // geometry of each node (null: 0)
  int G = 1;
  double ident = 0.0;             // coefficient of sigma (1 for I + K)
  int64_t ldx = 0;
};
// The correction constants gamma[r G + g] = sum_j gw_j sigma_j over the
// nodes of geometry g, formed inside the FMM from per-leaf partial sums of
// the leaf multipole pass (gw_t in tree order; geometry g's leaves are
// positions gl_ptr[g] .. gl_ptr[g + 1] of the plan's source-leaf list,
// nchunk = the most chunks of 2048 leaves a geometry has).
struct GammaFused {
  const double *gw_t = nullptr;
  const int32_t *gl_ptr = nullptr;
  double *gamma = nullptr;
  int G = 1, nchunk = 1;
};
void fmm_apply64(const DevPlan &pl, const Tables &tb, Workspace &ws,
                 const double *qfac_t, const double *sigma, int64_t ldx,
                 int nrhs, double *out, int64_t ldy, double scale,
                 const Assembly &as, hipStream_t s,
                 const GammaFused *gf = nullptr);
// The FP64 far field alone: strengths p_j = -i q_j sigma_j (ws.pstr64),
// multipoles (ws.mult64) and local expansions (ws.loc64) of every box of
// level >= 2 that holds sources or targets.
void fmm_far64(const DevPlan &pl, const Tables &tb, Workspace &ws, const double *qfac_t,
               const double *sigma, int64_t ldx, int nrhs, hipStream_t s);
// Psi(z) = sum_j p_j / (z - z_j) and Psi'(z) (complex, FP64) at the plan's
// targets for complex strengths pin (API order of the plan's sources);
// outputs in the targets' API order, dpsi may be null.  One column.
void fmm_apply64_full(const DevPlan &pl, const Tables &tb, Workspace &ws,
                      const double *pin, double *psi, double *dpsi,
                      hipStream_t s);
// The same field only, FP32 far and near field (p32 terms).
void fmm_apply32_full(const DevPlan &pl, const Tables &tb, Workspace &ws,
                      const double *pin, double *psi, hipStream_t s);
void fmm_apply32(const DevPlan &pl, const Tables &tb, Workspace &ws,
                 const double *qfac_t, const float2 *qm32, const double *sigma, int64_t ldx,
                 int nrhs, double *out, int64_t ldy, double scale,
                 const Assembly &as, hipStream_t s,
                 const GammaFused *gf = nullptr);
// set-up of the FP32 leaf multipoles' inputs of a handle plan (w32, perm32)
void build_p2m_inputs32(DevPlan &pl, hipStream_t s);
// qm32[j] = (Im q_j, -Re q_j) in FP32 from interleaved complex qfac_t
void launch_qm32(int64_t n, const double *qfac_t, float2 *qm32, hipStream_t s);
// direct O(N^2) sums (single-geometry handles)
void direct_apply64(int64_t N, const double *xi, const double *qfac,
                    const double *sigma, int64_t ldx, int nrhs, double *out,
                    int64_t ldy, const Assembly &as, hipStream_t s);
void direct_eval64(int64_t N, const double *xi, const double *qfac,
                   const double *sigma, int64_t ldx, int64_t T,
                   const double *txi, const uint8_t *pole, int nrhs,
                   double *out, int64_t ldy, double scale, hipStream_t s);

// The islands of a handle binned for the close-pair search (close.hip).
struct CloseGridView {
  const uint64_t *keys;     // sorted cell keys
  const int32_t *ptr, *isl;  // islands of cell c: isl[ptr[c] .. ptr[c + 1])
  const double *center, *zone_cos;
  double cell;
  int nkeys;
};
// cnt[q] = number of islands whose close zone holds target idx[q]
void launch_close_count(int64_t n, const int64_t *idx, const double *txyz, const int32_t *tgeo,
                        const CloseGridView &G, int32_t *cnt, hipStream_t s);
// for the targets with pos[q] >= 0: z, out and their islands (ascending) at
// ptr[pos[q]]; used[k] = 1 for every island met
void launch_close_fill(int64_t n, const int64_t *idx, const double *txyz, const int32_t *tgeo,
                       const double *tx, const double *ty, const int32_t *pos, const int32_t *ptr,
                       const CloseGridView &G, double *z, int64_t *out, int32_t *isl,
                       uint8_t *used, hipStream_t s);
int close_list_max();  // islands per target the fill pass lists

// u += close-evaluation corrections for the targets of cp (nrhs columns;
// V: 2 N nrhs doubles of scratch for the boundary values).
void launch_close_eval(const Geometry &g, const ClosePlan &cp, int nrhs,
                       const double *sigma, int64_t ldx, double *V, double *u,
                       int64_t ldu, hipStream_t s);

// out = beta in + alpha sum_j gamma_j G(x, v_j) at n points x (vortex.hip;
// gamma: nv x nrhs; in, out: ld per column; in may be null)
void launch_vortex_field(int64_t n, const double *x, int nv, const double *v,
                         const double *gamma, int nrhs, double alpha,
                         const double *in, int64_t ldi, double beta,
                         double *out, int64_t ldo, hipStream_t s);

// dot products: out[r] = sum_i a[r*lda + i] * b[r*ldb + i], i < n
void launch_dots(int64_t n, int nrhs, const double *a, int64_t lda,
                 const double *b, int64_t ldb, double *out, double *scratch,
                 hipStream_t s);
// segmented: out[(v R + r) nseg + s] = sum_{i in s} a[v lav + r lac + i] b[r lbc + i]
void launch_segdots(const SegPlan &sp, int R, int nvec, const double *a,
                    int64_t lav, int64_t lac, const double *b, int64_t lbc,
                    double *out, double *scratch, hipStream_t s);

// log sources and constraint rows (solver.hip)
// out += alpha E z
void launch_logsrc_apply(const Geometry &g, Workspace &ws, const double *z,
                         int64_t ldz, int nrhs, double *out, int64_t ldo,
                         double alpha, hipStream_t s);
void launch_logsrc_local(const Geometry &g, Workspace &ws, const double *z,
                         hipStream_t s);
void launch_island_sums(const Geometry &g, const double *y, int64_t ldy,
                        int nrhs, double *out, int64_t ldo, hipStream_t s);
void launch_constraint_rows(const Geometry &g, const double *sigma,
                            int64_t ldx, const double *A, int64_t lda,
                            int nrhs, double *out, int64_t ldo,
                            hipStream_t s);
void launch_build_schur(const Geometry &g, double *S, hipStream_t s);
void invert_blocks(const Geometry &g, double *S, double *Sinv, hipStream_t s);
// How a handle's S^-1 was formed: pivoted = 0 by elimination in the natural
// order (accepted when the probe backward error omega <= the tolerance),
// 1 by partial pivoting; omega < 0 when the natural order was not tried.
struct SchurInverseInfo {
  int pivoted = 0;
  double omega = -1.0;
};
SchurInverseInfo invert_schur(const Geometry &g, double *S, double *Sinv, double tol,
                              hipStream_t s);
void launch_gemv_blocks(const Geometry &g, const double *x, int64_t ldx,
                        int nrhs, double *y, int64_t ldy, double alpha,
                        hipStream_t s);
void launch_gemv_blocks_with(const Geometry &g, const double *A,
                             const double *x, int64_t ldx, int nrhs, double *y,
                             int64_t ldy, double alpha, hipStream_t s);
void launch_eval_logsrc(const Geometry &g, int64_t T, const double *txyz,
                        const int32_t *tgeo, const double *A, int64_t lda,
                        int nrhs, const double *add, double *u, int64_t ldu,
                        hipStream_t s, DBuf<double> *scratch = nullptr);

// GMRES building blocks (solver.hip)
void launch_maxpy_seg(int64_t n, int R, int G, int k1, const int32_t *row_geo,
                      const double *V, int64_t ldv, const double *h, double *w,
                      hipStream_t s);
void launch_update_seg(int64_t n, int R, int G, int k, int m,
                       const int32_t *row_geo, const double *V, int64_t ldv,
                       const double *y, double *x, hipStream_t s);
void launch_normalize_seg(int64_t n, int R, int G, const int32_t *row_geo,
                          const double *nrm2, const int32_t *active,
                          const double *w, double *v, hipStream_t s);
void launch_gmres_start(int S, int m, const double *nrm2, const double *tol,
                        double *g, int32_t *active, int32_t *kused,
                        int32_t *count, hipStream_t s);
void launch_givens_seg(int S, int k, int m, const double *h1, const double *h2,
                       const double *nrm2, const double *tol, double *H,
                       double *cs, double *sn, double *g, double *resid,
                       int32_t *active, int32_t *kused, int32_t *count,
                       hipStream_t s);
void launch_backsolve_seg(int S, int m, const double *H, const double *g,
                          const int32_t *kused, double *y, hipStream_t s);
void launch_axpby(int64_t n, double a, const double *x, double b, double *y,
                  hipStream_t s);
void launch_fill(int64_t n, double v, double *x, hipStream_t s);
// ox[j] = x[perm[j] stride], oy[j] = y[perm[j] stride] (j < n)
void launch_gather_points(int64_t n, const int32_t *perm, const double *x, const double *y,
                          int64_t stride, double *ox, double *oy, hipStream_t s);
// Runs of a concatenated list-source table: for each of the ne list
// entries k, fi[eo[k] + t] = s0[box[k]] + t, t < s1[box[k]] - s0[box[k]]
void launch_flat_fill(int64_t ne, const int32_t *box, const int64_t *eo, const int64_t *s0,
                      const int64_t *s1, int32_t *fi, hipStream_t s);
// out[j] = map ? map[perm[j]] : perm[j] (j < n)
void launch_widen_perm(int64_t n, const int32_t *perm, const int64_t *map, int64_t *out,
                       hipStream_t s);
void launch_fill_int(int64_t n, int32_t v, int32_t *x, hipStream_t s);
// In-place exclusive scan of a[0 .. n) (gtree.hip); scan_into takes the
// tile sums' scratch (at least ceil(n / 4096) entries) and does not wait.
void scan_u32(uint32_t *a, int64_t n, hipStream_t s);
void scan_into(uint32_t *a, int64_t n, uint32_t *sums, hipStream_t s);
// Whether a[0 .. n) and b[0 .. n) differ bit for bit (dflag: one device
// int32, hflag: one pinned host int32; waits for the stream).  (evalpts.hip)
bool targets_differ(int64_t n, const double *a, const double *b, int32_t *dflag,
                    int32_t *hflag, hipStream_t s);
// out[k] = in[idx[k]] for complex (double2) entries (evalpts.hip)
void launch_gather_cx(int64_t n, const int32_t *idx, const double *in, double *out,
                      hipStream_t s);
// Sources at n arbitrary points (x, y) located in a plan's tree (box: the
// deepest box whose square holds the point, -1 outside the root square;
// root: its tree's root), as (box, point) pairs sorted by box: the
// multipole of every box of level >= 2 holding the point (list m_list; the
// pairs' coordinates m_x, m_y in pair order), the local
// expansions its walk takes by multipole (offsets l_ptr over the plan's
// boxes into l_t), the leaves its walk sums directly (d_ptr, d_t).
// The plan needs its tree links on the device.  (evalpts.hip)
// The multipole pairs of a box are cut into chunks of at most kSrcChunk
// (one wave each, c_rng / c_geo, chunk offsets per m_list entry c_ptr),
// whose partial multipoles (c_part) are added per box in chunk order.
constexpr int kSrcChunk = 256;
struct PointSources {
  int64_t n = 0, nm = 0;
  const double *x = nullptr, *y = nullptr;  // not owned
  int n_m = 0;  // entries of m_list (also the boxes passed for local terms)
  int n_c = 0;  // chunks of the multipole pairs
  DBuf<int32_t> m_list, m_t, l_t, d_t, c_iota;
  DBuf<int64_t> l_ptr, d_ptr, c_rng;
  DBuf<uint32_t> c_ptr;
  DBuf<double4> c_geo;
  DBuf<double> m_x, m_y, m_p, c_part;  // m_p: the pairs' strengths of a call
};
void build_point_sources(const DevPlan &pl, int64_t n, const double *x, const double *y,
                         const int32_t *box, const int32_t *root, PointSources &ps,
                         hipStream_t s);
// Psi(z) = sum_t c_t / (z - z_t) and Psi'(z) (complex, FP64) at the plan's
// targets (API order; dpsi may be null) from complex strengths pin of the
// located point sources (their order), through the plan's own expansions
// (ws.mult64, ws.loc64, one column).  (fmm.hip)
void fmm_sources64_full(const DevPlan &pl, const Tables &tb, Workspace &ws, PointSources &ps,
                        const double *pin, double *psi, double *dpsi, hipStream_t s);
// Stable sort of (keys, vals) by the low `bits` bits of the keys (gtree.hip);
// the first form waits for the stream and releases its scratch, the second
// keeps its scratch in sc for the next sort (release it only after the
// stream has finished with it).
struct SortBufs {
  DBuf<uint64_t> k2;
  DBuf<int32_t> v2;
  DBuf<uint32_t> hist, sums;
};
void sort_by_key(uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s);
void sort_by_key(uint64_t *keys, int32_t *vals, int64_t n, int bits, SortBufs &sc,
                 hipStream_t s);
// Targets located in a plan's tree (evalpts.hip): the n targets (tx, ty;
// API index idx; geometry tgeo[idx] or 0) sorted by the deepest box whose
// square holds them (-1 outside the root square), with their roots and
// API indices.  The plan needs its tree links and roots on the device.
void launch_locate_targets(int64_t n, const double *tx, const double *ty, const int64_t *idx,
                           const int32_t *tgeo, const DevPlan &pl, double *ox, double *oy,
                           int32_t *obox, int32_t *oroot, int64_t *oidx, hipStream_t s);
// out[r ldy + tidx[i]] = scale Re sum_j p_j / (z_i - z_j) for located
// targets, from the plan's FP64 expansions M, L (order P) and strengths
// pstr of its sources (far_field already run for the nrhs right-hand sides).
void launch_eval_points(int P, int64_t n, const double *tx, const double *ty, const int32_t *tbox,
                        const int32_t *troot, const int64_t *tidx, const DevPlan &pl,
                        const double *pstr, const double *M, const double *L, int nrhs,
                        double *out, int64_t ldy, double scale, hipStream_t s);
void launch_copy_cols(int64_t n, int R, double a, const double *src, int64_t lds,
                      double *dst, int64_t ldd, hipStream_t s);
void launch_scale_sqrt(int S, double t, const double *nrm2, double *out,
                       hipStream_t s);

// transposed operators and shape derivatives (adjoint.hip)
constexpr int kMomStride = 2 * kPlog + 2;  // moment slots per island
void launch_kT_assemble(const Geometry &g, const double *y, const double *F,
                        const double *ysum, double ident, double *out,
                        hipStream_t s);
void launch_real_to_complex(int64_t n, const double *y, double *out,
                            hipStream_t s);
void launch_gather_complex(int64_t n, const int64_t *idx, const double *y,
                           double *out, hipStream_t s);
void launch_dl_strengths(const Geometry &g, const double *sigma, double *out,
                         hipStream_t s);
void launch_logsrc_T(const Geometry &g, const double *y, double *mom,
                     double alpha, double *out, hipStream_t s);
void launch_FT(const Geometry &g, const double *z, double a, const double *x,
               double b, double *out, hipStream_t s);
void launch_transpose_blocks(const Geometry &g, const double *A, double *AT,
                             hipStream_t s);
void launch_evalT_logsrc(const Geometry &g, int64_t T, const double *txyz,
                         const double *w, double *out, DBuf<double> &scratch, hipStream_t s);
void launch_evalT_sigma(const Geometry &g, const double *FT,
                        const double *wsum_dev, double *out, hipStream_t s);
void launch_sum(int64_t n, const double *x, double *out, hipStream_t s);
void launch_logsrc_deriv(const Geometry &g, Workspace &ws, const double *A,
                         double *out, hipStream_t s);
void launch_shape_vjp(const Geometry &g, const double *sigma,
                      const double *lam, const double *Fl, const double *dFl,
                      const double *dFp, const double *Fw, const double *dFw,
                      const double *LSd, const double *lam_sum,
                      const double *a_sum, const double *w_sum, double *dcoef,
                      hipStream_t s);

}  // namespace lbs
