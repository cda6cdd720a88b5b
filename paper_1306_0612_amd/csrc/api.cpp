// C-ABI of liblbs (include/lbs.h): set-up, operator application, GMRES
// solve with the block preconditioner, and evaluation at sphere targets.
// A handle holds G >= 1 independent island geometries; every right-hand
// side of every geometry is its own linear system.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <tuple>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "lbs_internal.h"

// Wall-clock phases of the host-side set-up work, printed to stderr when
// the environment variable LBS_HOST_TIMING is set (a plan's phases, in ms).
namespace {
bool host_timing() {
  static const bool on = std::getenv("LBS_HOST_TIMING") != nullptr;
  return on;
}
struct HostPhase {
  const char *name;
  std::chrono::steady_clock::time_point t0;
  explicit HostPhase(const char *n) : name(n), t0(std::chrono::steady_clock::now()) {}
  ~HostPhase() {
    if (!host_timing()) return;
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[lbs host] %-28s %9.3f ms\n", name, ms);
  }
};
}  // namespace

using namespace lbs;

namespace {
thread_local std::string g_err;

template <class F>
lbs_status guard(F &&f) {
  try {
    f();
    return LBS_OK;
  } catch (const ApiError &e) {
    g_err = e.msg;
    return e.code;
  } catch (const HipError &e) {
    g_err = std::string(hipGetErrorString(e.code)) + " in " + e.where;
    return LBS_ERR_HIP;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return LBS_ERR_OUT_OF_MEMORY;
  } catch (const std::exception &e) {
    g_err = e.what();
    return LBS_ERR_INVALID_ARG;
  }
}

[[noreturn]] void fail(lbs_status c, const std::string &m) {
  throw ApiError{c, m};
}

bool p64_ok(int p) {
  return p == 20 || p == 24 || p == 30 || p == 36 || p == 40 || p == 48;
}
bool p32_ok(int p) { return p == 12 || p == 16 || p == 20 || p == 24; }

// Upload a host tree (or forest) as a device plan.  sx/sy (tx/ty) are the
// source (target) coordinates in input order; tgt_index maps a target's
// input position to the index written by the leaf kernel.
// The points of a plan whose tree was built on the GPU, on the device:
// coordinates (x[i stride], y[i stride]) of sources and targets, the maps
// the builder kept, and the target index map (device, or null).
struct DevPoints {
  const double *sx, *sy;
  int64_t sstride, ns;
  const double *tx, *ty;
  int64_t tstride, nt;
  const DevPerms *perm;
  const int64_t *tgt_index;
};

void upload_plan(Tree &T, const double *sx, const double *sy,
                 const double *tx, const double *ty,
                 const std::vector<int64_t> *tgt_index, DevPlan &pl,
                 hipStream_t s, const DevPoints *dp = nullptr) {
  HostPhase ph_plan("upload_plan");
  const int nb = T.nbox();
  pl.nbox = nb;
  pl.nlevels = T.nlevels;
  pl.self = T.self;
  pl.ns = dp ? dp->ns : (int64_t)T.src_perm.size();
  pl.nt = dp ? (T.self ? dp->ns : dp->nt) : (int64_t)T.tgt_perm.size();
  std::vector<int32_t> leaf_s, leaf_t, m2l;
  std::vector<uint8_t> has_tgt(nb);
  for (int b = 0; b < nb; ++b) {
    has_tgt[b] = T.t1[b] > T.t0[b];
    if (T.leaf[b] && T.s1[b] > T.s0[b]) leaf_s.push_back(b);
    if (T.leaf[b] && has_tgt[b]) leaf_t.push_back(b);
    if (T.level[b] >= 2 && has_tgt[b]) m2l.push_back(b);
  }
  pl.n_leaf_s = (int)leaf_s.size();
  pl.n_leaf_t = (int)leaf_t.size();
  pl.n_m2l = (int)m2l.size();
  {
    HostPhase ph("upload_plan leaf order");
    // leaf kernels: one wave per target leaf, launched heaviest octave of
    // near-field work first (box order kept within an octave), so that the
    // waves still running at the end of a launch are short ones.  Work: the
    // leaf's U-list sources times its target lanes (32-target sub-chunks
    // rounded up to powers of two, as the kernels lay them out).
    std::vector<int> oct(nb, 0);
    for (int b : leaf_t) {
      int64_t us = 0;
      for (int e = T.u_ptr[b]; e < T.u_ptr[b + 1]; ++e) us += T.s1[T.u_src[e]] - T.s0[T.u_src[e]];
      int64_t lanes = 0;
      for (int64_t c0 = 0, nt = T.t1[b] - T.t0[b]; c0 < nt; c0 += 32) {
        int64_t tp = 1;
        while (tp < std::min<int64_t>(32, nt - c0)) tp <<= 1;
        lanes += tp;
      }
      int64_t w = std::max<int64_t>(1, us * lanes);
      while (w > 1) {
        w >>= 1;
        ++oct[b];
      }
    }
    std::stable_sort(leaf_t.begin(), leaf_t.end(),
                     [&](int a, int b) { return oct[a] > oct[b]; });
  }
  {
    HostPhase ph("upload_plan M2L order");
    // M2L boxes: the FP32 kernel's waves take every W-th box (W = 4 x its
    // work-groups); with the boxes sorted by estimated work (V-list batches
    // of 8, X-list passes of 64 sources) and every other stride of W
    // reversed, each wave's share comes out even.
    const int64_t n = (int64_t)m2l.size();
    std::vector<int32_t> mw = m2l;  // the FP64 kernel keeps box order
    std::vector<int64_t> w(nb, 0);
    for (int b : mw) {
      int64_t nx = 0;
      for (int e = T.x_ptr[b]; e < T.x_ptr[b + 1]; ++e) nx += T.s1[T.x_src[e]] - T.s0[T.x_src[e]];
      const int64_t nv = T.v_ptr[b + 1] - T.v_ptr[b];
      w[b] = 4 + 2 * ((nv + 7) / 8) + (nx > 0 ? 4 + 3 * ((nx + 63) / 64) : 0);
    }
    std::stable_sort(mw.begin(), mw.end(), [&](int a, int b) { return w[a] > w[b]; });
    const int64_t W = 4 * std::min<int64_t>((n + 3) / 4, pl.m2l_groups);
    for (int64_t a = W; a < n; a += 2 * W)
      std::reverse(mw.begin() + a, mw.begin() + std::min(n, a + W));
    pl.m2l_wave.upload(mw, s);
    LBS_HIP(hipStreamSynchronize(s));  // mw is released on return
  }
  pl.leaf_t_host = leaf_t;
  pl.leaf_s_host = leaf_s;
  // the M2L kernels form the P2L sums of their boxes: every box with an
  // X list must be one of them
  for (int b = 0; b < nb; ++b)
    if (T.x_ptr[b + 1] > T.x_ptr[b] && !(T.level[b] >= 2 && has_tgt[b]))
      fail(LBS_ERR_UNSUPPORTED, "X list on a box outside the M2L boxes");
  pl.cx.upload(T.cx, s);
  pl.cy.upload(T.cy, s);
  pl.rad.upload(T.rad, s);
  pl.lev.upload(T.level, s);
  pl.s0.upload(T.s0, s);
  pl.s1.upload(T.s1, s);
  pl.t0.upload(T.t0, s);
  pl.t1.upload(T.t1, s);
  pl.v_ptr.upload(T.v_ptr, s);
  pl.v_src.upload(T.v_src, s);
  pl.v_code.upload(T.v_code, s);
  // U and X lists as per-box concatenations of their boxes' source points
  auto flat_sources = [&](const std::vector<int32_t> &ptr, const std::vector<int32_t> &idx,
                          DBuf<int64_t> &dptr, DBuf<int32_t> &didx) -> std::vector<int64_t> {
    std::vector<int64_t> fp((size_t)nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
      int64_t c = 0;
      for (int k = ptr[b]; k < ptr[b + 1]; ++k) c += T.s1[idx[k]] - T.s0[idx[k]];
      fp[b + 1] = fp[b] + c;
    }
    if (fp[nb] > INT32_MAX) fail(LBS_ERR_UNSUPPORTED, "list source table over 2^31 entries");
    // where each list entry's run starts in the table; the runs are filled
    // on the device (a wave per entry)
    const int64_t ne = ptr[nb];
    std::vector<int64_t> eo((size_t)std::max<int64_t>(ne, 1));
    for (int b = 0; b < nb; ++b) {
      int64_t e = fp[b];
      for (int k = ptr[b]; k < ptr[b + 1]; ++k) {
        eo[k] = e;
        e += T.s1[idx[k]] - T.s0[idx[k]];
      }
    }
    DBuf<int64_t> deo;
    DBuf<int32_t> dent;
    deo.upload(eo, s);
    dent.upload(idx, s);
    dptr.upload(fp, s);
    didx.alloc((size_t)std::max<int64_t>(fp[nb], 1));
    launch_flat_fill(ne, dent.p, deo.p, pl.s0.p, pl.s1.p, didx.p, s);
    LBS_HIP(hipStreamSynchronize(s));  // eo is released on return
    return fp;
  };
  {
    HostPhase ph("upload_plan U sources");
    const std::vector<int64_t> ufp = flat_sources(T.u_ptr, T.u_src, pl.uf_ptr, pl.uf_idx);
    std::vector<LeafHdr> hd(leaf_t.size());
    for (size_t i = 0; i < leaf_t.size(); ++i) {
      const int b = leaf_t[i];
      LeafHdr &h = hd[i];
      h.t0 = T.t0[b];
      h.nt = T.t1[b] - T.t0[b];
      h.uf0 = ufp[b];
      h.uf1 = ufp[b + 1];
      h.wb = T.w_ptr[b];
      h.we = T.w_ptr[b + 1];
      h.b = b;
      h.lev = T.level[b];
      h.cx = T.cx[b];
      h.cy = T.cy[b];
      h.ir = 1.0 / T.rad[b];
      h.pad = 0.0;
    }
    pl.lt_hdr.upload(hd, s);
    LBS_HIP(hipStreamSynchronize(s));  // hd is released on return
  }
  {
    HostPhase ph("upload_plan X sources");
    flat_sources(T.x_ptr, T.x_src, pl.xf_ptr, pl.xf_idx);
  }
  pl.w_ptr.upload(T.w_ptr, s);
  pl.w_src.upload(T.w_src, s);
  pl.leaf_t.upload(leaf_t, s);
  pl.leaf_s.upload(leaf_s, s);
  {
    std::vector<int64_t> rng(2 * leaf_s.size());
    std::vector<double4> geo(leaf_s.size());
    for (size_t i = 0; i < leaf_s.size(); ++i) {
      const int b = leaf_s[i];
      rng[2 * i] = T.s0[b];
      rng[2 * i + 1] = T.s1[b];
      geo[i] = make_double4(T.cx[b], T.cy[b], 1.0 / T.rad[b], 0.0);
    }
    pl.ls_rng.upload(rng, s);
    pl.ls_geo.upload(geo, s);
    LBS_HIP(hipStreamSynchronize(s));  // rng, geo are released on return
  }
  pl.m2l_box.upload(m2l, s);
  auto points = [&](const std::vector<int64_t> &perm, const double *ax,
                    const double *ay, DBuf<double> &dx, DBuf<double> &dy) {
    const int64_t n = (int64_t)perm.size();
    std::vector<double> x(n), y(n);
    for (int64_t j = 0; j < n; ++j) {
      x[j] = ax[perm[j]];
      y[j] = ay[perm[j]];
    }
    dx.upload(x, s);
    dy.upload(y, s);
    LBS_HIP(hipStreamSynchronize(s));  // x, y are released on return
  };
  HostPhase ph_pts("upload_plan points");
  if (dp) {  // gathered on the device from the builder's maps
    const int32_t *tp = T.self ? dp->perm->src.p : dp->perm->tgt.p;
    pl.sx.alloc((size_t)pl.ns);
    pl.sy.alloc((size_t)pl.ns);
    pl.tx.alloc((size_t)pl.nt);
    pl.ty.alloc((size_t)pl.nt);
    pl.src_perm.alloc((size_t)pl.ns);
    pl.tgt_perm.alloc((size_t)pl.nt);
    launch_gather_points(pl.ns, dp->perm->src.p, dp->sx, dp->sy, dp->sstride, pl.sx.p, pl.sy.p, s);
    launch_widen_perm(pl.ns, dp->perm->src.p, nullptr, pl.src_perm.p, s);
    launch_gather_points(pl.nt, tp, T.self ? dp->sx : dp->tx, T.self ? dp->sy : dp->ty,
                         T.self ? dp->sstride : dp->tstride, pl.tx.p, pl.ty.p, s);
    launch_widen_perm(pl.nt, tp, dp->tgt_index, pl.tgt_perm.p, s);
    LBS_HIP(hipStreamSynchronize(s));
    return;
  }
  points(T.src_perm, sx, sy, pl.sx, pl.sy);
  pl.src_perm.upload(T.src_perm, s);
  points(T.tgt_perm, T.self ? sx : tx, T.self ? sy : ty, pl.tx, pl.ty);
  std::vector<int64_t> perm(T.tgt_perm.size());
  for (size_t j = 0; j < perm.size(); ++j)
    perm[j] = tgt_index ? (*tgt_index)[T.tgt_perm[j]] : T.tgt_perm[j];
  pl.tgt_perm.upload(perm, s);
  LBS_HIP(hipStreamSynchronize(s));
}

// Upward / downward pass programs of the plan's tree for FP32 order p32
// and FP64 order p64 (the LDS capacity of the pass kernels depends on it);
// fp64_only: the FP64 ones alone (evaluation plans run the FP64 FMM only).
void build_passes(DevPlan &pl, int p32, int p64, hipStream_t s, bool fp64_only = false) {
  HostPhase ph("pass programs");
  for (int k = fp64_only ? 1 : 0; k < 2; ++k) {
    const int cap = k == 0 ? pass_cap(p32, 8) : pass_cap(p64, 16);
    for (int d = 0; d < 2; ++d) {
      PassProgram pp;
      build_pass_program(pl.host, d == 1, cap, pp);
      DevPass &dp = d ? pl.dn[k] : pl.up[k];
      dp.cap = cap;
      dp.round_ptr = pp.round_ptr;
      dp.hdr.upload(pp.hdr, s);
      // inputs at a fixed stride of cap slots per component (box -1 past
      // its count), so that the kernel's first loads need no header
      std::vector<int32_t> extc((size_t)2 * cap * pp.ncomp, 0);
      for (int c = 0; c < pp.ncomp; ++c) {
        const int e0 = pp.hdr[8 * (size_t)c], ne = pp.hdr[8 * (size_t)c + 1];
        if (ne > cap) fail(LBS_ERR_UNSUPPORTED, "pass component with more inputs than slots");
        for (int i = 0; i < cap; ++i) {
          int32_t *o = extc.data() + 2 * ((size_t)c * cap + i);
          if (i < ne) {
            o[0] = pp.ext[2 * (size_t)(e0 + i)];
            o[1] = pp.ext[2 * (size_t)(e0 + i) + 1];
          } else {
            o[0] = -1;
          }
        }
      }
      dp.ext.upload(extc, s);
      dp.par.upload(pp.par, s);
      dp.stp.upload(pp.stp, s);
      LBS_HIP(hipStreamSynchronize(s));  // pp is released on return
    }
  }
}

}  // namespace

namespace lbs {
void Workspace::ensure(const DevPlan &pl, int P64, int P32, int nrhs,
                       int64_t N, int M, int G, int Plog) {
  if (nrhs <= nrhs_cap) return;
  nrhs_cap = nrhs;
  pstr64.alloc((size_t)pl.ns * nrhs * 2);
  mult64.alloc((size_t)pl.nbox * P64 * nrhs * 2);
  loc64.alloc((size_t)pl.nbox * P64 * nrhs * 2);
  pstr32.alloc((size_t)pl.ns * nrhs * 2);
  mult32.alloc((size_t)pl.nbox * P32 * nrhs * 2);
  loc32.alloc((size_t)pl.nbox * P32 * nrhs * 2);
  gam.alloc((size_t)std::max(nrhs, 1) * G);
  gpart.alloc((size_t)std::max(pl.n_leaf_s, 1) * nrhs);
  {
    const int nch = (std::max(pl.n_leaf_s, 1) + 2047) / 2048;  // bound for every geometry
    gcsum.alloc((size_t)nch * G * nrhs);
    gcnt.alloc((size_t)G * nrhs);
    LBS_HIP(hipMemset(gcnt.p, 0, gcnt.n * sizeof(int32_t)));
  }
  tmpM.alloc((size_t)std::max(M, 1) * nrhs);
  logL.alloc((size_t)std::max(M, 1) * nrhs * (2 * (Plog + 1) + 2));
  // reduction scratch: plain dots (512 x nrhs) and segmented dots of up to
  // 128 vectors over the 2048-row chunks of N + M rows
  const size_t chunks = (size_t)((N + M) / 2048 + 2 * G + 4);
  red.alloc(std::max<size_t>((size_t)512 * std::max(nrhs, 128),
                             (size_t)128 * nrhs * chunks));
}
}  // namespace lbs

struct GmresState {
  int R = 0, S = 0, m = 0;
  int64_t n = 0;
  DBuf<double> V, H, cs, sn, gv, yv, h1, h2, nrm2, tol, resid;
  DBuf<int32_t> active, kused, count;
  DBuf<double> bvec, rvec, xvec, dvec, bn2;
};

// FMM plan of an evaluation at sphere targets, kept for the next call with
// the same targets.  Forward: sources = nodes, targets = the targets (one
// tree per geometry); transposed: the (non-pole) targets are the sources and
// the nodes the targets.  Targets at the north pole carry no Cauchy part and
// are left out of the trees.
struct EvalPlan {
  DBuf<double> dkey;            // device copy of the targets (T x 3)
  std::vector<int64_t> toff;    // geometry-major target offsets
  std::vector<int32_t> tgeo;    // geometry of each target
  std::vector<double> tx, ty;   // projected non-pole targets (compact)
  std::vector<int64_t> idx;     // compact position -> target index
  bool tree = false;
  DevPlan pl;
  Workspace ws;
  DBuf<double> qt;              // forward: qfac in the plan's source order
  DBuf<int64_t> didx;           // transposed: idx on the device
  DBuf<int32_t> dtgeo;
  // forward, targets located in the handle's own tree (no tree of their
  // own): sorted by the deepest box holding them, with that box (-1:
  // outside the root square), their tree's root and their API index
  bool located = false;
  DBuf<double> ltx, lty;
  DBuf<int32_t> lbox, lroot;
  DBuf<int64_t> lidx;
  // transposed, the located targets as sources of the handle's own FMM
  bool located_src = false;
  PointSources src;
  ClosePlan close;              // targets in close zones (close_eval on)
  DBuf<double> closeV;          // boundary values, 2 N per column
  DBuf<double> lpart;           // log-source partial sums per island chunk
};

// Buffers of the transposed operators (one column).
struct AdjState {
  bool ready = false;
  DBuf<double> ones;   // max(N, M) ones (segment sums)
  DBuf<double> mom;    // island moments, slot-major (kMomStride x M)
  DBuf<double> tA;     // M
  DBuf<double> lam;    // N + M
  DBuf<double> pc, Fc; // complex, N x 2
  DBuf<double> ysum;   // per geometry
  DBuf<double> lpart;  // partial sums of the transposed log-source sums
};

// HIP graphs of GMRES iterations, keyed by (operator, systems per column
// count, iteration index), and the device buffers they were captured with.
struct GraphCache {
  hipStream_t cap = nullptr;  // capture stream (non-blocking, default priority)
  std::map<std::tuple<int, int, int>, hipGraphExec_t> exec;
  std::vector<const void *> sig;
  void clear() {
    for (auto &e : exec) (void)hipGraphExecDestroy(e.second);
    exec.clear();
  }
  ~GraphCache() {
    clear();
    if (cap) (void)hipStreamDestroy(cap);
  }
};

struct lbs_ctx {
  lbs_options opt{};
  Geometry geo;
  DevPlan plan;
  Tables tab64, tab32;
  Workspace ws;
  SegPlan seg_nodes;   // one segment per geometry over the node rows
  SegPlan seg_sys;     // one segment per geometry over the N + M unknowns
  std::vector<double> xi_x, xi_y;  // node images, API order (eval trees)
  StageTimer timer;
  GmresState gm;
  AdjState adj;
  std::unique_ptr<EvalPlan> evf, evt;  // cached forward / transposed plans
  SchurInverseInfo sinv_info;          // how set-up formed S^-1
  GraphCache graphs;
  // island centres hashed by (geometry, cell of the unit cube) for the
  // close-zone search of evaluations; built on first use
  std::unordered_map<uint64_t, std::vector<int32_t>> igrid;
  double icell = 0.0;
  // the same bins on the device: sorted cell keys, islands per cell, zones
  DBuf<uint64_t> cg_keys;
  DBuf<int32_t> cg_ptr, cg_isl;
  DBuf<double> cg_zone;
  int32_t *count_host = nullptr;
  // pinned staging for target coordinates read back to the host
  double *stage_host = nullptr;
  size_t stage_n = 0;
  DBuf<int32_t> diff;  // device flag of the target comparison
  ~lbs_ctx() {
    if (count_host) (void)hipHostFree(count_host);
    if (stage_host) (void)hipHostFree(stage_host);
  }
};

namespace {

void ensure_ws(lbs_ctx &c, int nrhs) {
  c.ws.ensure(c.plan, c.opt.p64, c.opt.p32, nrhs, c.geo.N, c.geo.M, c.geo.G,
              kPlog);
}

// y = ident x + K x for the node rows (ld x / y given), with the FMM
// buffers of workspace w (sized for nrhs columns by the caller)
void apply_K_ws(lbs_ctx &c, Workspace &w, int prec, int nrhs, const double *x, int64_t ldx,
                double *y, int64_t ldy, double ident, hipStream_t s) {
  Geometry &g = c.geo;
  Assembly as;
  as.sigma = x;
  as.tau = g.tau.p;
  as.gamma = w.gam.p;
  as.geo = g.node_geo.p;
  as.G = g.G;
  as.ident = ident;
  as.ldx = ldx;
  // gamma: by a segmented dot product for the direct sum, inside the FMM
  // (partial sums of the leaf multipole pass) otherwise
  GammaFused gf;
  gf.gw_t = g.gw_t.p;
  gf.gl_ptr = g.gleaf_ptr.p;
  gf.gamma = w.gam.p;
  gf.G = g.G;
  gf.nchunk = g.gleaf_chunks;
  if (c.opt.matvec == LBS_MATVEC_DIRECT) {
    {
      TimerScope ts(w.timer, ST_GAMMA, s);
      launch_segdots(c.seg_nodes, nrhs, 1, g.gw.p, 0, 0, x, ldx, w.gam.p,
                     w.red.p, s);
    }
    TimerScope ts(w.timer, ST_LEAF, s);
    direct_apply64(g.N, g.xi.p, g.qfac.p, x, ldx, nrhs, y, ldy, as, s);
  } else if (prec == LBS_FP64) {
    fmm_apply64(c.plan, c.tab64, w, g.qfac_t.p, x, ldx, nrhs, y, ldy, 1.0,
                as, s, &gf);
  } else {
    fmm_apply32(c.plan, c.tab32, w, g.qfac_t.p, g.qm32_t.n ? g.qm32_t.p : nullptr, x, ldx,
                nrhs, y, ldy, 1.0, as, s, &gf);
  }
}

void apply_K(lbs_ctx &c, int prec, int nrhs, const double *x, int64_t ldx,
             double *y, int64_t ldy, double ident, hipStream_t s) {
  ensure_ws(c, nrhs);
  apply_K_ws(c, c.ws, prec, nrhs, x, ldx, y, ldy, ident, s);
}

// y = P^-1 A x = x + P^-1 [K x_s; 0]   (x, y: nrhs columns of length N + M)
void apply_precond_op_ws(lbs_ctx &c, Workspace &w, int prec, int nrhs, const double *x,
                         double *y, hipStream_t s) {
  Geometry &g = c.geo;
  const int64_t n = g.N + g.M;
  apply_K_ws(c, w, prec, nrhs, x, n, y, n, 0.0, s);
  {
    TimerScope ts(w.timer, ST_CONSTRAINT, s);
    launch_island_sums(g, y, n, nrhs, w.tmpM.p, g.M, s);
    launch_gemv_blocks(g, w.tmpM.p, g.M, nrhs, y + g.N, n, -1.0, s);
  }
  {
    TimerScope ts(w.timer, ST_LOGSRC, s);
    launch_logsrc_apply(g, w, y + g.N, n, nrhs, y, n, -1.0, s);
  }
  launch_axpby(n * nrhs, 1.0, x, 1.0, y, s);
}

void apply_precond_op(lbs_ctx &c, int prec, int nrhs, const double *x,
                      double *y, hipStream_t s) {
  ensure_ws(c, nrhs);
  apply_precond_op_ws(c, c.ws, prec, nrhs, x, y, s);
}

// [y_s; y_a] = [ (I+K) x_s + E x_a ; F x_s + D x_a ]
void apply_system_ws(lbs_ctx &c, Workspace &w, int prec, int nrhs, const double *x, double *y,
                     hipStream_t s) {
  Geometry &g = c.geo;
  const int64_t n = g.N + g.M;
  apply_K_ws(c, w, prec, nrhs, x, n, y, n, 1.0, s);
  {
    TimerScope ts(w.timer, ST_LOGSRC, s);
    launch_logsrc_apply(g, w, x + g.N, n, nrhs, y, n, 1.0, s);
  }
  TimerScope ts(w.timer, ST_CONSTRAINT, s);
  launch_constraint_rows(g, x, n, x + g.N, n, nrhs, y + g.N, n, s);
}

void apply_system(lbs_ctx &c, int prec, int nrhs, const double *x, double *y,
                  hipStream_t s) {
  ensure_ws(c, nrhs);
  apply_system_ws(c, c.ws, prec, nrhs, x, y, s);
}

// b = P^-1 [2 g; 0] for nrhs columns (g: ld N; b: ld N + M)
void precond_rhs(lbs_ctx &c, int nrhs, const double *gdat, double *b,
                 hipStream_t s) {
  Geometry &g = c.geo;
  const int64_t n = g.N + g.M;
  ensure_ws(c, nrhs);
  launch_copy_cols(g.N, nrhs, 2.0, gdat, g.N, b, n, s);
  launch_island_sums(g, b, n, nrhs, c.ws.tmpM.p, g.M, s);
  launch_gemv_blocks(g, c.ws.tmpM.p, g.M, nrhs, b + g.N, n, -1.0, s);
  launch_logsrc_apply(g, c.ws, b + g.N, n, nrhs, b, n, -1.0, s);
}

void ensure_gmres(lbs_ctx &c, int R) {
  GmresState &st = c.gm;
  if (st.R >= R && st.R > 0) return;
  const int m = c.opt.restart, G = c.geo.G, S = R * G;
  const int64_t n = c.geo.N + c.geo.M;
  st.R = R;
  st.S = S;
  st.m = m;
  st.n = n;
  st.V.alloc((size_t)(m + 1) * R * n);
  st.H.alloc((size_t)S * (m + 1) * m);
  st.cs.alloc((size_t)S * m);
  st.sn.alloc((size_t)S * m);
  st.gv.alloc((size_t)S * (m + 1));
  st.yv.alloc((size_t)S * m);
  st.h1.alloc((size_t)(m + 1) * S);
  st.h2.alloc((size_t)(m + 1) * S);
  st.nrm2.alloc(S);
  st.tol.alloc(S);
  st.resid.alloc(S);
  st.bn2.alloc(S);
  st.active.alloc(S);
  st.kused.alloc(S);
  st.count.alloc(1);
  st.bvec.alloc((size_t)R * n);
  st.rvec.alloc((size_t)R * n);
  st.xvec.alloc((size_t)R * n);
  st.dvec.alloc((size_t)R * n);
}

int read_count(lbs_ctx &c, hipStream_t s) {
  LBS_HIP(hipMemcpyAsync(c.count_host, c.gm.count.p, sizeof(int32_t),
                         hipMemcpyDeviceToHost, s));
  LBS_HIP(hipStreamSynchronize(s));
  return *c.count_host;
}

struct GmresOut {
  int iters = 0;
  bool conv = false;
};

using OpFn = std::function<void(const double *, double *, hipStream_t)>;

// Buffers every captured iteration reads or writes; a change of any of them
// (reallocation) invalidates the cached graphs.
std::vector<const void *> graph_signature(lbs_ctx &c) {
  const GmresState &st = c.gm;
  const Workspace &w = c.ws;
  const AdjState &a = c.adj;
  return {st.V.p, st.H.p, st.cs.p, st.sn.p, st.gv.p, st.h1.p, st.h2.p, st.nrm2.p,
          st.tol.p, st.resid.p, st.active.p, st.kused.p, st.count.p, w.pstr64.p,
          w.mult64.p, w.loc64.p, w.pstr32.p, w.mult32.p, w.loc32.p, w.gam.p,
          w.gpart.p, w.gcsum.p, w.gcnt.p, w.red.p, w.tmpM.p, w.logL.p, a.mom.p, a.tA.p, a.lam.p, a.pc.p, a.Fc.p,
          a.ysum.p, c.geo.SinvT.p};
}

// Lockstep GMRES(m) for the R * G systems op(x) = b (columns of length
// n = N + M), per-system absolute tolerances c.gm.tol.  x_zero: start from
// x = 0.  Classical Gram-Schmidt with `passes` passes (2: CGS2; 1 serves
// the inner solves of mixed-precision refinement, which stop at a loose
// tolerance and whose errors the FP64 outer residual corrects), Givens
// rotations, one 4-byte read of the number of active systems per
// iteration.  With graph_id >= 0 (and graphs enabled, stage timing off)
// the body of iteration k is captured once as a HIP graph under the key
// (graph_id, R, k) and replayed afterwards; a graph_id always comes with
// the same number of passes.
GmresOut gmres(lbs_ctx &c, const OpFn &op, int graph_id, int R, const double *b,
               double *x, bool x_zero, int max_iter, hipStream_t s, int passes) {
  GmresState &st = c.gm;
  const int64_t n = st.n;
  const int m = st.m, G = c.geo.G, S = R * G;
  double *V = st.V.p;
  const int64_t ldv = (int64_t)R * n;
  const int32_t *rg = c.geo.row_geo.p;
  GmresOut out;
  const bool use_graphs = graph_id >= 0 && c.opt.graphs && c.ws.timer == nullptr;
  if (use_graphs) {
    std::vector<const void *> sig = graph_signature(c);
    if (sig != c.graphs.sig) {
      c.graphs.clear();
      c.graphs.sig = sig;
    }
    if (!c.graphs.cap) LBS_HIP(hipStreamCreateWithFlags(&c.graphs.cap, hipStreamNonBlocking));
  }
  auto residual_into_v0 = [&]() {
    op(x, V, s);
    launch_axpby(ldv, 1.0, b, -1.0, V, s);
  };
  if (x_zero) {
    launch_fill(ldv, 0.0, x, s);
    LBS_HIP(hipMemcpyAsync(V, b, ldv * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    residual_into_v0();
  }
  while (true) {
    launch_segdots(c.seg_sys, R, 1, V, 0, n, V, n, st.nrm2.p, c.ws.red.p, s);
    launch_fill_int(1, 0, st.count.p, s);
    launch_gmres_start(S, m, st.nrm2.p, st.tol.p, st.gv.p, st.active.p,
                       st.kused.p, st.count.p, s);
    if (read_count(c, s) == 0) {
      out.conv = true;
      return out;
    }
    if (out.iters >= max_iter) return out;
    launch_normalize_seg(n, R, G, rg, st.nrm2.p, st.active.p, V, V, s);
    int alive = 1;
    int kc = 0;
    for (int k = 0; k < m; ++k) {
      double *vk = V + (int64_t)k * ldv, *w = V + (int64_t)(k + 1) * ldv;
      auto body = [&](hipStream_t q) {
        op(vk, w, q);
        launch_segdots(c.seg_sys, R, k + 1, V, ldv, n, w, n, st.h1.p, c.ws.red.p, q);
        launch_maxpy_seg(n, R, G, k + 1, rg, V, ldv, st.h1.p, w, q);
        if (passes > 1) {
          launch_segdots(c.seg_sys, R, k + 1, V, ldv, n, w, n, st.h2.p, c.ws.red.p, q);
          launch_maxpy_seg(n, R, G, k + 1, rg, V, ldv, st.h2.p, w, q);
        }
        launch_segdots(c.seg_sys, R, 1, w, 0, n, w, n, st.nrm2.p, c.ws.red.p, q);
        launch_fill_int(1, 0, st.count.p, q);
        launch_givens_seg(S, k, m, st.h1.p, passes > 1 ? st.h2.p : nullptr, st.nrm2.p,
                          st.tol.p, st.H.p,
                          st.cs.p, st.sn.p, st.gv.p, st.resid.p, st.active.p,
                          st.kused.p, st.count.p, q);
        launch_normalize_seg(n, R, G, rg, st.nrm2.p, st.active.p, w, w, q);
      };
      if (use_graphs) {
        const auto key = std::make_tuple(graph_id, R, k);
        auto it = c.graphs.exec.find(key);
        if (it == c.graphs.exec.end()) {
          hipGraph_t gr = nullptr;
          LBS_HIP(hipStreamBeginCapture(c.graphs.cap, hipStreamCaptureModeThreadLocal));
          try {
            body(c.graphs.cap);
          } catch (...) {
            (void)hipStreamEndCapture(c.graphs.cap, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            throw;
          }
          LBS_HIP(hipStreamEndCapture(c.graphs.cap, &gr));
          hipGraphExec_t ex = nullptr;
          hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          LBS_HIP(e);
          it = c.graphs.exec.emplace(key, ex).first;
        }
        LBS_HIP(hipGraphLaunch(it->second, s));
      } else {
        body(s);
      }
      alive = read_count(c, s);
      ++out.iters;
      kc = k + 1;
      if (alive == 0 || out.iters >= max_iter) break;
    }
    launch_backsolve_seg(S, m, st.H.p, st.gv.p, st.kused.p, st.yv.p, s);
    launch_update_seg(n, R, G, kc, m, rg, V, ldv, st.yv.p, x, s);
    if (alive == 0) {
      out.conv = true;
      return out;
    }
    if (out.iters >= max_iter) return out;
    residual_into_v0();
  }
}

// Operators of the forward solve: P^-1 A (left-preconditioned, eq.
// matrix_eqns_c) or A itself (eq. matrix_eqns), with the FMM of the given
// precision.  Graph ids: 0/1 preconditioned FP64/mixed, 2/3 transposed,
// 4/5 unpreconditioned.
OpFn forward_op(lbs_ctx &c, int prec, int R, bool precond) {
  lbs_ctx *pc = &c;
  if (precond)
    return [pc, prec, R](const double *in, double *out, hipStream_t q) {
      apply_precond_op(*pc, prec, R, in, out, q);
    };
  return [pc, prec, R](const double *in, double *out, hipStream_t q) {
    apply_system(*pc, prec, R, in, out, q);
  };
}

// Per-system 2-norms^2 of R columns of length N + M into out (S values).
void sys_norm2(lbs_ctx &c, int R, const double *x, double *out, hipStream_t s) {
  const int64_t n = c.geo.N + c.geo.M;
  launch_segdots(c.seg_sys, R, 1, x, 0, n, x, n, out, c.ws.red.p, s);
}

std::vector<double> download(const double *p, size_t n, hipStream_t s) {
  std::vector<double> v(n);
  LBS_HIP(hipMemcpyAsync(v.data(), p, n * sizeof(double), hipMemcpyDeviceToHost, s));
  LBS_HIP(hipStreamSynchronize(s));
  return v;
}

void check_handle(lbs_handle h) {
  if (!h) fail(LBS_ERR_INVALID_ARG, "null handle");
}

// b = [2 g; 0] for nrhs columns (g: ld N; b: ld N + M), the right-hand side
// of eq. matrix_eqns.
void system_rhs(lbs_ctx &c, int nrhs, const double *gdat, double *b, hipStream_t s) {
  Geometry &g = c.geo;
  const int64_t n = g.N + g.M;
  launch_copy_cols(g.N, nrhs, 2.0, gdat, g.N, b, n, s);
  for (int r = 0; r < nrhs; ++r) launch_fill(g.M, 0.0, b + (int64_t)r * n + g.N, s);
}

// x <- P^-1 x in place for nrhs columns of length N + M, with the block
// preconditioner P = [[I, E], [F, D]] of eq. matrix_eqns_c:
// z_a = S^-1 (x_a - F x_s), z_s = x_s - E z_a.
void apply_precond_inverse(lbs_ctx &c, int nrhs, double *x, hipStream_t s) {
  Geometry &g = c.geo;
  const int64_t n = g.N + g.M;
  ensure_ws(c, nrhs);
  double *tmp = c.ws.tmpM.p;
  launch_island_sums(g, x, n, nrhs, tmp, g.M, s);
  for (int r = 0; r < nrhs; ++r)
    launch_axpby(g.M, 1.0, x + (int64_t)r * n + g.N, -1.0, tmp + (int64_t)r * g.M, s);
  launch_gemv_blocks(g, tmp, g.M, nrhs, x + g.N, n, 1.0, s);
  launch_logsrc_apply(g, c.ws, x + g.N, n, nrhs, x, n, -1.0, s);
}

// Per-system relative residuals sqrt(rn2 / bn2) (0 where bn2 = 0) and their
// maximum; a NaN or Inf norm is an error, never a converged system.
double worst_relative(const std::vector<double> &rn2, const std::vector<double> &bn2,
                      const char *what) {
  double worst = 0;
  for (size_t q = 0; q < rn2.size(); ++q) {
    if (!std::isfinite(rn2[q]) || !std::isfinite(bn2[q]))
      fail(LBS_ERR_NOT_FINITE, std::string(what) + " is not finite (system " +
                                   std::to_string(q) + ")");
    if (bn2[q] > 0) worst = std::max(worst, std::sqrt(rn2[q] / bn2[q]));
  }
  return worst;
}

// Solve op(x) = b for the R * G systems (b in gm.bvec, x into gm.xvec) to
// the relative residual tol per system.  FP64: GMRES on op64 (two
// Gram-Schmidt passes).  Mixed: iterative refinement, the residual
// b - op64(x) in FP64 and the correction from GMRES on op32 (one pass) to
// the tolerances lbs_refine_tolerances_host describes.  Returns whether every
// system converged; throws LBS_ERR_NOT_FINITE on a non-finite residual.
bool solve_core(lbs_ctx &c, int prec, int R, const OpFn &op64, int gid64, const OpFn &op32,
                int gid32, double tol, lbs_solve_info &inf, hipStream_t s) {
  GmresState &gm = c.gm;
  const int S = R * c.geo.G;
  const int64_t n = c.geo.N + c.geo.M;
  sys_norm2(c, R, gm.bvec.p, gm.bn2.p, s);
  if (prec == LBS_FP64) {
    launch_scale_sqrt(S, tol, gm.bn2.p, gm.tol.p, s);
    GmresOut go = gmres(c, op64, gid64, R, gm.bvec.p, gm.xvec.p, true, c.opt.max_iter, s, 2);
    inf.iters = go.iters;
    inf.fp64_matvecs = go.iters;
    return go.conv;
  }
  launch_fill((int64_t)R * n, 0.0, gm.xvec.p, s);
  LBS_HIP(hipMemcpyAsync(gm.rvec.p, gm.bvec.p, (size_t)R * n * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  const std::vector<double> bn2 = download(gm.bn2.p, S, s);
  std::vector<double> rn2 = bn2, itol(S);
  int left = c.opt.max_iter;
  for (int outer = 0;; ++outer) {
    int32_t all = 0;
    const lbs_status st = lbs_refine_tolerances_host(S, rn2.data(), bn2.data(), tol,
                                                     c.opt.inner_tol, itol.data(), &all);
    if (st != LBS_OK) fail(st, "refinement residual is not finite");
    if (all) return true;
    if (outer >= c.opt.max_outer || left <= 0) return false;
    LBS_HIP(hipMemcpyAsync(gm.tol.p, itol.data(), S * sizeof(double), hipMemcpyHostToDevice, s));
    GmresOut go = gmres(c, op32, gid32, R, gm.rvec.p, gm.dvec.p, true, left, s, 1);
    inf.iters += go.iters;
    inf.fp32_matvecs += go.iters;
    left -= go.iters;
    launch_axpby((int64_t)R * n, 1.0, gm.dvec.p, 1.0, gm.xvec.p, s);
    op64(gm.xvec.p, gm.rvec.p, s);
    inf.fp64_matvecs += 1;
    launch_axpby((int64_t)R * n, 1.0, gm.bvec.p, -1.0, gm.rvec.p, s);
    sys_norm2(c, R, gm.rvec.p, gm.nrm2.p, s);
    rn2 = download(gm.nrm2.p, S, s);
    inf.outer_steps = outer + 1;
  }
}

// Terms P of the far-field log series that keep its tail
// sum_{l > P} r^l / l <= r^(P + 1) / ((P + 1)(1 - r)) below 2.5e-16 (the
// bound of the full kPlog terms at the far limit r = 1/3).
int log_terms(double r) {
  if (!(r > 0)) return 1;
  double t = r * r / (2.0 * (1.0 - r));
  int P = 1;
  while (t > 2.5e-16 && P < kPlog) {
    t *= r * (double)(P + 1) / (double)(P + 2);
    ++P;
  }
  return P;
}

// Far lists of the island-frame log-source expansions (see Geometry):
// every pair (k, m) of a geometry with m not in k's near list rp/ri.
void build_far_lists(Geometry &g, const std::vector<int32_t> &isl_geo,
                     const std::vector<double> &rl, const std::vector<double> &fr,
                     const std::vector<int32_t> &rp, const std::vector<int32_t> &ri,
                     hipStream_t s) {
  const int M = g.M;
  std::vector<int64_t> fp(M + 1, 0);
  for (int k = 0; k < M; ++k) {
    const int q = isl_geo[k];
    fp[k + 1] = fp[k] + (g.gisl[q + 1] - g.gisl[q]) - (rp[k + 1] - rp[k]);
  }
  const int64_t nf = fp[M];
  std::vector<int32_t> fidx(nf);
  std::vector<double> fq(2 * nf), fh(nf), fa(nf);  // fa = |q_km|, the sort key
  parallel_for(
      M,
      [&](int64_t k0, int64_t k1) {
        std::vector<int64_t> ord;
        std::vector<int32_t> ti;
        std::vector<double> tq, th, ta;
        for (int64_t k = k0; k < k1; ++k) {
          const int q = isl_geo[k];
          const double *ck = &g.cxyz[3 * k], *f = &fr[6 * k];
          const double rk2 = 2.0 * rl[k];
          int64_t e = fp[k];
          int32_t ne = rp[k];
          for (int m = g.gisl[q]; m < g.gisl[q + 1]; ++m) {
            if (ne < rp[k + 1] && ri[ne] == m) {  // near lists ascend in m
              ++ne;
              continue;
            }
            const double x0 = g.cxyz[3 * m], x1 = g.cxyz[3 * m + 1], x2 = g.cxyz[3 * m + 2];
            const double d0 = x0 - ck[0], d1 = x1 - ck[1], d2 = x2 - ck[2];
            const double dd = d0 * d0 + d1 * d1 + d2 * d2;
            const double a = x0 * f[0] + x1 * f[1] + x2 * f[2];
            const double b = x0 * f[3] + x1 * f[4] + x2 * f[5];
            const double ff = rk2 / dd;
            fidx[e] = m;
            fq[2 * e] = a * ff;
            fq[2 * e + 1] = -b * ff;
            fh[e] = 0.5 * std::log(dd);
            fa[e] = std::hypot(a * ff, b * ff);
            ++e;
          }
          const int64_t a0 = fp[k], n = fp[k + 1] - a0;
          ord.resize(n);
          for (int64_t i = 0; i < n; ++i) ord[i] = a0 + i;
          std::sort(ord.begin(), ord.end(), [&](int64_t u, int64_t v) {
            return fa[u] != fa[v] ? fa[u] > fa[v] : fidx[u] < fidx[v];
          });
          ti.resize(n);
          tq.resize(2 * n);
          th.resize(n);
          ta.resize(n);
          for (int64_t i = 0; i < n; ++i) {
            ti[i] = fidx[ord[i]];
            tq[2 * i] = fq[2 * ord[i]];
            tq[2 * i + 1] = fq[2 * ord[i] + 1];
            th[i] = fh[ord[i]];
            ta[i] = fa[ord[i]];
          }
          std::copy(ti.begin(), ti.end(), fidx.begin() + a0);
          std::copy(tq.begin(), tq.end(), fq.begin() + 2 * a0);
          std::copy(th.begin(), th.end(), fh.begin() + a0);
          std::copy(ta.begin(), ta.end(), fa.begin() + a0);
        }
      },
      64);
  auto chunks = [&](const std::vector<int64_t> &ptr, const std::vector<double> &mag,
                    std::vector<int64_t> &cptr, std::vector<int32_t> &nt) {
    cptr.assign(M + 1, 0);
    for (int k = 0; k < M; ++k)
      cptr[k + 1] = cptr[k] + (ptr[k + 1] - ptr[k] + kLogChunk - 1) / kLogChunk;
    nt.assign(cptr[M], 0);
    for (int k = 0; k < M; ++k)
      for (int64_t c = cptr[k]; c < cptr[k + 1]; ++c)
        nt[c] = log_terms(mag[ptr[k] + (c - cptr[k]) * kLogChunk]);
  };
  std::vector<int64_t> fc;
  std::vector<int32_t> fnt;
  chunks(fp, fa, fc, fnt);
  g.far_ptr.upload(fp, s);
  g.far_cptr.upload(fc, s);
  g.far_nt.upload(fnt, s);
  g.far_idx.upload(fidx, s);
  g.far_q.upload(fq, s);
  g.far_h.upload(fh, s);
  // the host vectors must outlive the asynchronous copies
  LBS_HIP(hipStreamSynchronize(s));
}

// Close-evaluation zones: island k's zone is the cap about its centre of
// angular radius (largest node distance from the centre) + 8 (largest
// chord between consecutive nodes); beyond it the trapezoidal rule is
// accurate to rounding (its error decays like exp(-2 pi d / spacing)).
void set_close_zones(Geometry &g, const std::vector<double> &xyz) {
  g.zone_cos.assign(g.M, 1.0);
  for (int k = 0; k < g.M; ++k) {
    const double *c = &g.cxyz[3 * k];
    double bound = 0.0, ell = 0.0;
    for (int64_t i = g.offs[k]; i < g.offs[k + 1]; ++i) {
      const double *x = &xyz[3 * i];
      const double d = std::max(-1.0, std::min(1.0, x[0] * c[0] + x[1] * c[1] + x[2] * c[2]));
      bound = std::max(bound, std::acos(d));
      const int64_t j = i + 1 < g.offs[k + 1] ? i + 1 : g.offs[k];
      const double *y = &xyz[3 * j];
      ell = std::max(ell, std::sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) +
                                    (x[2] - y[2]) * (x[2] - y[2])));
    }
    g.zone_cos[k] = std::cos(std::min(bound + 8.0 * ell, M_PI));
  }
}

// Close pairs of an evaluation: every non-pole target with the islands of
// its geometry whose close zone holds it.  On the device (close.hip) from
// the sorted cell table of the handle's islands; on the host, from the
// cached targets, when a target lies in more zones than the device pass
// lists.
void build_close_host(lbs_ctx &c, EvalPlan &ep, const std::vector<double> &hx, hipStream_t s);

void build_close(lbs_ctx &c, EvalPlan &ep, const std::vector<double> &hx, const double *txyz,
                 hipStream_t s) {
  Geometry &g = c.geo;
  if (c.cg_keys.n == 0) {  // the islands binned by the cell of their centre
    double cell = 1e-4;
    for (int k = 0; k < g.M; ++k)
      cell = std::max(cell, std::sqrt(std::max(0.0, 2.0 - 2.0 * g.zone_cos[k])));
    c.icell = cell;
    std::vector<std::pair<uint64_t, int32_t>> ki((size_t)g.M);
    for (int q = 0; q < g.G; ++q)
      for (int k = g.gisl[q]; k < g.gisl[q + 1]; ++k) {
        const double *ck = &g.cxyz[3 * k];
        uint64_t key = (uint64_t)q << 48;
        for (int a = 0; a < 3; ++a)
          key |= (uint64_t)std::floor((ck[a] + 1.0) / cell) << (32 - 16 * a);
        ki[k] = {key, k};
      }
    std::sort(ki.begin(), ki.end());
    std::vector<uint64_t> keys;
    std::vector<int32_t> ptr, isl;
    for (size_t e = 0; e < ki.size(); ++e) {
      if (e == 0 || ki[e].first != ki[e - 1].first) {
        keys.push_back(ki[e].first);
        ptr.push_back((int32_t)e);
      }
      isl.push_back(ki[e].second);
    }
    ptr.push_back((int32_t)ki.size());
    c.cg_keys.upload(keys, s);
    c.cg_ptr.upload(ptr, s);
    c.cg_isl.upload(isl, s);
    c.cg_zone.upload(g.zone_cos, s);
    LBS_HIP(hipStreamSynchronize(s));  // the host tables are released on return
  }
  const int64_t n = (int64_t)ep.idx.size();
  const CloseGridView G{c.cg_keys.p, c.cg_ptr.p, c.cg_isl.p, g.dcenter.p, c.cg_zone.p, c.icell,
                        (int)c.cg_keys.n};
  if (ep.didx.n != (size_t)n) ep.didx.upload(ep.idx, s);
  DBuf<int32_t> cnt;
  cnt.alloc((size_t)n);
  launch_close_count(n, ep.didx.p, txyz, ep.dtgeo.p, G, cnt.p, s);
  const std::vector<int32_t> hc = cnt.download(s);
  std::vector<int32_t> pos((size_t)n, -1), ptr(1, 0);
  for (int64_t q = 0; q < n; ++q) {
    if (hc[q] == 0) continue;
    if (hc[q] > close_list_max()) {
      build_close_host(c, ep, hx, s);
      return;
    }
    pos[q] = (int32_t)(ptr.size() - 1);
    ptr.push_back(ptr.back() + hc[q]);
  }
  ClosePlan &cp = ep.close;
  cp.n_tgt = (int)(ptr.size() - 1);
  if (cp.n_tgt == 0) {
    cp.n_act = 0;
    return;
  }
  DBuf<int32_t> dpos;
  DBuf<double> dtx, dty;
  DBuf<uint8_t> used;
  dpos.upload(pos, s);
  cp.ptr.upload(ptr, s);
  dtx.upload(ep.tx, s);
  dty.upload(ep.ty, s);
  cp.z.alloc((size_t)2 * cp.n_tgt);
  cp.out.alloc((size_t)cp.n_tgt);
  cp.isl.alloc((size_t)ptr.back());
  used.alloc((size_t)g.M);
  LBS_HIP(hipMemsetAsync(used.p, 0, (size_t)g.M, s));
  launch_close_fill(n, ep.didx.p, txyz, ep.dtgeo.p, dtx.p, dty.p, dpos.p, cp.ptr.p, G, cp.z.p,
                    cp.out.p, cp.isl.p, used.p, s);
  const std::vector<uint8_t> hu = used.download(s);
  std::vector<int32_t> act;
  for (int k = 0; k < g.M; ++k)
    if (hu[k]) act.push_back(k);
  cp.n_act = (int)act.size();
  cp.act.upload(act, s);
  LBS_HIP(hipStreamSynchronize(s));  // the host vectors are released on return
}

void build_close_host(lbs_ctx &c, EvalPlan &ep, const std::vector<double> &hx, hipStream_t s) {
  Geometry &g = c.geo;
  if (c.igrid.empty()) {
    double cell = 1e-4;
    for (int k = 0; k < g.M; ++k)
      cell = std::max(cell, std::sqrt(std::max(0.0, 2.0 - 2.0 * g.zone_cos[k])));
    c.icell = cell;
    std::vector<int32_t> isl_geo(g.M);
    for (int q = 0; q < g.G; ++q)
      for (int k = g.gisl[q]; k < g.gisl[q + 1]; ++k) isl_geo[k] = q;
    for (int k = 0; k < g.M; ++k) {
      const double *ck = &g.cxyz[3 * k];
      uint64_t key = (uint64_t)isl_geo[k] << 48;
      for (int a = 0; a < 3; ++a)
        key |= (uint64_t)std::floor((ck[a] + 1.0) / cell) << (32 - 16 * a);
      c.igrid[key].push_back(k);
    }
  }
  const double cell = c.icell;
  const int64_t n = (int64_t)ep.idx.size();
  std::vector<std::vector<int32_t>> near(n);
  parallel_for(n, [&](int64_t c0, int64_t c1) {
    for (int64_t q = c0; q < c1; ++q) {
      const int64_t t = ep.idx[q];
      const double *x = &hx[3 * t];
      int64_t cc[3];
      for (int a = 0; a < 3; ++a) cc[a] = (int64_t)std::floor((x[a] + 1.0) / cell);
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            const int64_t ix = cc[0] + dx, iy = cc[1] + dy, iz = cc[2] + dz;
            if (ix < 0 || iy < 0 || iz < 0) continue;
            const uint64_t key = ((uint64_t)ep.tgeo[t] << 48) | ((uint64_t)ix << 32) |
                                 ((uint64_t)iy << 16) | (uint64_t)iz;
            auto it = c.igrid.find(key);
            if (it == c.igrid.end()) continue;
            for (int32_t k : it->second) {
              const double *ck = &g.cxyz[3 * k];
              if (x[0] * ck[0] + x[1] * ck[1] + x[2] * ck[2] > g.zone_cos[k]) near[q].push_back(k);
            }
          }
      std::sort(near[q].begin(), near[q].end());
    }
  }, 2048);
  std::vector<double> z;
  std::vector<int64_t> out;
  std::vector<int32_t> ptr(1, 0), isl;
  std::vector<uint8_t> used(g.M, 0);
  for (int64_t q = 0; q < n; ++q) {
    if (near[q].empty()) continue;
    z.push_back(ep.tx[q]);
    z.push_back(ep.ty[q]);
    out.push_back(ep.idx[q]);
    for (int32_t k : near[q]) {
      isl.push_back(k);
      used[k] = 1;
    }
    ptr.push_back((int32_t)isl.size());
  }
  std::vector<int32_t> act;
  for (int k = 0; k < g.M; ++k)
    if (used[k]) act.push_back(k);
  ClosePlan &cp = ep.close;
  cp.n_tgt = (int)out.size();
  cp.n_act = (int)act.size();
  if (cp.n_tgt == 0) return;
  cp.z.upload(z, s);
  cp.out.upload(out, s);
  cp.ptr.upload(ptr, s);
  cp.isl.upload(isl, s);
  cp.act.upload(act, s);
  LBS_HIP(hipStreamSynchronize(s));  // the host vectors are released on return
}

void validate_options(const lbs_options &o) {
  if (!p64_ok(o.p64)) fail(LBS_ERR_UNSUPPORTED, "p64 must be 20/24/30/36/40/48");
  if (!p32_ok(o.p32)) fail(LBS_ERR_UNSUPPORTED, "p32 must be 12/16/20/24");
  if (o.leaf_max < 4 || o.leaf_max > 1024) fail(LBS_ERR_INVALID_ARG, "leaf_max outside [4, 1024]");
  if (o.restart < 1 || o.restart > 120) fail(LBS_ERR_INVALID_ARG, "restart outside [1, 120]");
  if (o.max_iter < 1 || o.max_outer < 1) fail(LBS_ERR_INVALID_ARG, "max_iter/max_outer < 1");
  if (!(o.inner_tol > 0 && o.inner_tol < 1)) fail(LBS_ERR_INVALID_ARG, "inner_tol outside (0, 1)");
  if (o.matvec != LBS_MATVEC_FMM && o.matvec != LBS_MATVEC_DIRECT) fail(LBS_ERR_INVALID_ARG, "bad matvec mode");
  if (o.graphs != 0 && o.graphs != 1) fail(LBS_ERR_INVALID_ARG, "graphs must be 0 or 1");
  if (o.precond != 0 && o.precond != 1) fail(LBS_ERR_INVALID_ARG, "precond must be 0 or 1");
  if (o.close_eval != 0 && o.close_eval != 1) fail(LBS_ERR_INVALID_ARG, "close_eval must be 0 or 1");
  if (o.gpu_tree != 0 && o.gpu_tree != 1) fail(LBS_ERR_INVALID_ARG, "gpu_tree must be 0 or 1");
  if (o.eval_tree != 0 && o.eval_tree != 1) fail(LBS_ERR_INVALID_ARG, "eval_tree must be 0 or 1");
  if (o.m2l_groups != 0 && (o.m2l_groups < 64 || o.m2l_groups > 8192))
    fail(LBS_ERR_INVALID_ARG, "m2l_groups must be 0 or in [64, 8192]");
  if (!(o.schur_tol <= 1e-3)) fail(LBS_ERR_INVALID_ARG, "schur_tol must be <= 1e-3 (not NaN)");
}

// Set-up of G geometries (islands and node counts concatenated
// geometry-major; isl_per_geom[g] islands each).
// Curves given as node samples (lbs_setup_sampled): x, x', x'' per node
// (N x 3 each, host) and a point inside each curve (M x 3, host).
struct Samples {
  const double *x = nullptr, *xt = nullptr, *xtt = nullptr, *centers = nullptr;
};

// Validate sampled curves and describe them as islands without shape
// coefficients (centre, a frame vector e1, r0 = 0); their bounding radii
// into `bound`.  offs: node offsets per island.
std::vector<lbs_island> sampled_islands(const Samples &sm, int M,
                                        const std::vector<int64_t> &offs,
                                        std::vector<double> &bound) {
  std::vector<lbs_island> isl(M);
  bound.assign(M, 0.0);
  for (int k = 0; k < M; ++k) {
    const std::string tag = "island " + std::to_string(k) + ": ";
    const double *c = sm.centers + 3 * k;
    if (!std::isfinite(c[0]) || !std::isfinite(c[1]) || !std::isfinite(c[2]))
      fail(LBS_ERR_GEOMETRY, tag + "non-finite centre");
    if (std::fabs(c[0] * c[0] + c[1] * c[1] + c[2] * c[2] - 1.0) > 2e-10)
      fail(LBS_ERR_GEOMETRY, tag + "centre is not a unit vector");
    lbs_island &I = isl[k];
    std::memset(&I, 0, sizeof(I));
    double e1[3] = {-c[1], c[0], 0.0};
    if (std::hypot(e1[0], e1[1]) < 1e-12) e1[0] = 1.0, e1[1] = 0.0;
    const double d = e1[0] * c[0] + e1[1] * c[1] + e1[2] * c[2];
    for (int a = 0; a < 3; ++a) e1[a] -= d * c[a];
    const double nn = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int a = 0; a < 3; ++a) {
      I.center[a] = c[a];
      I.e1[a] = e1[a] / nn;
    }
    const double e2[3] = {I.e1[1] * c[2] - I.e1[2] * c[1], I.e1[2] * c[0] - I.e1[0] * c[2],
                          I.e1[0] * c[1] - I.e1[1] * c[0]};
    // node checks, bounding radius (largest node distance plus the largest
    // chord between neighbours) and the winding number of the curve about
    // the centre in the centre's own stereographic frame
    double ang = 0.0, ell = 0.0, wind = 0.0, pa = 0.0, pb = 0.0;
    for (int64_t i = offs[k]; i < offs[k + 1]; ++i) {
      const double *x = sm.x + 3 * i, *xt = sm.xt + 3 * i, *xtt = sm.xtt + 3 * i;
      for (int a = 0; a < 3; ++a)
        if (!std::isfinite(x[a]) || !std::isfinite(xt[a]) || !std::isfinite(xtt[a]))
          fail(LBS_ERR_GEOMETRY, tag + "non-finite node sample");
      if (std::fabs(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] - 1.0) > 1e-9)
        fail(LBS_ERR_GEOMETRY, tag + "node " + std::to_string(i) + " is not on the unit sphere");
      const double h = x[0] * c[0] + x[1] * c[1] + x[2] * c[2];
      if (!(h > 0.0)) fail(LBS_ERR_GEOMETRY, tag + "curve reaches the centre's hemisphere boundary");
      ang = std::max(ang, std::acos(std::min(1.0, h)));
      const int64_t j = i + 1 < offs[k + 1] ? i + 1 : offs[k];
      const double *y = sm.x + 3 * j;
      ell = std::max(ell, std::sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) +
                                    (x[2] - y[2]) * (x[2] - y[2])));
      const double a = (x[0] * I.e1[0] + x[1] * I.e1[1] + x[2] * I.e1[2]) / (1.0 + h);
      const double b = (x[0] * e2[0] + x[1] * e2[1] + x[2] * e2[2]) / (1.0 + h);
      if (i > offs[k]) wind += std::atan2(pa * b - pb * a, pa * a + pb * b);
      pa = a;
      pb = b;
    }
    {
      const double *x = sm.x + 3 * offs[k];
      const double h = x[0] * c[0] + x[1] * c[1] + x[2] * c[2];
      const double a = (x[0] * I.e1[0] + x[1] * I.e1[1] + x[2] * I.e1[2]) / (1.0 + h);
      const double b = (x[0] * e2[0] + x[1] * e2[1] + x[2] * e2[2]) / (1.0 + h);
      wind += std::atan2(pa * b - pb * a, pa * a + pb * b);
    }
    if (std::fabs(std::fabs(wind) - 2.0 * M_PI) > 0.5)
      fail(LBS_ERR_GEOMETRY, tag + "the centre is not inside the curve");
    bound[k] = ang + ell;
  }
  return isl;
}

lbs_ctx *setup_impl(int G, const int32_t *isl_per_geom, const lbs_island *isl_in,
                    const int32_t *nodes, const lbs_options *opt,
                    hipStream_t s, const Samples *sm = nullptr) {
  HostPhase ph_all("setup (all)");
  auto ctx = std::make_unique<lbs_ctx>();
  lbs_default_options(&ctx->opt);
  if (opt) ctx->opt = *opt;
  lbs_options &o = ctx->opt;
  validate_options(o);
  if (G > 1 && o.matvec == LBS_MATVEC_DIRECT)
    fail(LBS_ERR_UNSUPPORTED, "the direct matvec serves single-geometry handles");
  Geometry &g = ctx->geo;
  g.G = G;
  g.gisl.assign(G + 1, 0);
  for (int q = 0; q < G; ++q) {
    if (isl_per_geom[q] < 1) fail(LBS_ERR_INVALID_ARG, "a geometry has no island");
    g.gisl[q + 1] = g.gisl[q] + isl_per_geom[q];
    g.maxM = std::max(g.maxM, isl_per_geom[q]);
  }
  const int M = g.gisl[G];
  if (g.maxM > 65535) fail(LBS_ERR_UNSUPPORTED, "more than 65535 islands in a geometry");
  g.M = M;
  g.nodes.assign(nodes, nodes + M);
  g.offs.assign(M + 1, 0);
  std::vector<double> bound(M);
  g.cxyz.resize(3 * M);
  for (int k = 0; k < M; ++k) {
    if (nodes[k] < 8) fail(LBS_ERR_INVALID_ARG, "island " + std::to_string(k) + ": fewer than 8 nodes");
    g.offs[k + 1] = g.offs[k] + nodes[k];
  }
  std::vector<lbs_island> smp_isl;
  if (sm) {
    smp_isl = sampled_islands(*sm, M, g.offs, bound);
    g.sampled = true;
  }
  const lbs_island *isl = sm ? smp_isl.data() : isl_in;
  for (int k = 0; k < M; ++k) {
    const lbs_island &I = isl[k];
    if (sm) {
      for (int a = 0; a < 3; ++a) g.cxyz[3 * k + a] = I.center[a];
      if (bound[k] >= 0.5 * M_PI)
        fail(LBS_ERR_GEOMETRY, "island " + std::to_string(k) + ": bounding radius >= pi/2");
      const double pole_ang = std::acos(std::max(-1.0, std::min(1.0, I.center[2])));
      if (pole_ang <= bound[k] * (1 + 1e-9) + 1e-9)
        fail(LBS_ERR_GEOMETRY, "island " + std::to_string(k) + ": north pole inside or on the bounding cap");
      continue;
    }
    double cs = 0, es = 0, dot = 0, amp = 0;
    bool fin = std::isfinite(I.r0);
    for (int a = 0; a < 3; ++a) {
      fin = fin && std::isfinite(I.center[a]) && std::isfinite(I.e1[a]);
      cs += I.center[a] * I.center[a];
      es += I.e1[a] * I.e1[a];
      dot += I.center[a] * I.e1[a];
      g.cxyz[3 * k + a] = I.center[a];
    }
    for (int a = 0; a < 16; ++a) {
      fin = fin && std::isfinite(I.coef[a]);
      amp += std::fabs(I.coef[a]);
    }
    const std::string tag = "island " + std::to_string(k) + ": ";
    if (!fin) fail(LBS_ERR_GEOMETRY, tag + "non-finite parameter");
    if (std::fabs(cs - 1) > 2e-10 || std::fabs(es - 1) > 2e-10 || std::fabs(dot) > 1e-10)
      fail(LBS_ERR_GEOMETRY, tag + "center/e1 not orthonormal");
    if (!(I.r0 > 0) || amp >= 1.0) fail(LBS_ERR_GEOMETRY, tag + "radius not positive everywhere");
    bound[k] = I.r0 * (1.0 + amp);
    if (bound[k] >= 0.5 * M_PI) fail(LBS_ERR_GEOMETRY, tag + "bounding radius >= pi/2");
    const double pole_ang = std::acos(std::max(-1.0, std::min(1.0, I.center[2])));
    if (pole_ang <= bound[k] * (1 + 1e-9) + 1e-9)
      fail(LBS_ERR_GEOMETRY, tag + "north pole inside or on the bounding cap");
  }
  g.N = g.offs[M];
  if (g.N > (int64_t)INT32_MAX) fail(LBS_ERR_INVALID_ARG, "too many nodes");
  g.gnode.assign(G + 1, 0);
  for (int q = 0; q <= G; ++q) g.gnode[q] = g.offs[g.gisl[q]];
  for (int q = 0; q < G; ++q)
    for (int a = g.gisl[q]; a < g.gisl[q + 1]; ++a)
      for (int b = a + 1; b < g.gisl[q + 1]; ++b) {
        const double d = g.cxyz[3 * a] * g.cxyz[3 * b] + g.cxyz[3 * a + 1] * g.cxyz[3 * b + 1] +
                         g.cxyz[3 * a + 2] * g.cxyz[3 * b + 2];
        const double lim = bound[a] + bound[b];
        if (lim >= M_PI || d >= std::cos(lim))
          fail(LBS_ERR_GEOMETRY, "bounding caps of islands " + std::to_string(a) + " and " +
                                     std::to_string(b) + " overlap");
      }
  const int64_t N = g.N;
  std::vector<int32_t> island(N), node_geo(N), isl_geo(M), row_geo(N + M);
  for (int q = 0; q < G; ++q)
    for (int k = g.gisl[q]; k < g.gisl[q + 1]; ++k) {
      isl_geo[k] = q;
      row_geo[N + k] = q;
      for (int64_t i = g.offs[k]; i < g.offs[k + 1]; ++i) {
        island[i] = k;
        node_geo[i] = q;
        row_geo[i] = q;
      }
    }
  g.island.upload(island, s);
  g.node_geo.upload(node_geo, s);
  g.isl_geo.upload(isl_geo, s);
  g.row_geo.upload(row_geo, s);
  g.doffs.upload(g.offs, s);
  g.dgnode.upload(g.gnode, s);
  g.dgisl.upload(g.gisl, s);
  g.dcenter.upload(g.cxyz, s);
  g.gsinv.assign(G + 1, 0);
  for (int q = 0; q < G; ++q) {
    const int64_t mq = g.gisl[q + 1] - g.gisl[q];
    g.gsinv[q + 1] = g.gsinv[q] + mq * mq;
  }
  g.dgsinv.upload(g.gsinv, s);
  g.disl.upload(std::vector<lbs_island>(isl, isl + M), s);
  g.xyz.alloc(3 * N);
  g.xi.alloc(2 * N);
  g.dxi.alloc(2 * N);
  g.ddxi.alloc(2 * N);
  if (sm) {
    DBuf<double> dx, dxt, dxtt;
    dx.upload(std::vector<double>(sm->x, sm->x + 3 * N), s);
    dxt.upload(std::vector<double>(sm->xt, sm->xt + 3 * N), s);
    dxtt.upload(std::vector<double>(sm->xtt, sm->xtt + 3 * N), s);
    launch_geometry_sampled(N, dx.p, dxt.p, dxtt.p, g.xyz.p, g.xi.p, g.dxi.p, g.ddxi.p, s);
    LBS_HIP(hipStreamSynchronize(s));  // the samples are released on return
  } else {
    launch_geometry(g.disl.p, M, g.doffs.p, g.island.p, N, g.xyz.p, g.xi.p, g.dxi.p, g.ddxi.p, s);
  }
  std::vector<double> xyz = g.xyz.download(s), xi = g.xi.download(s), dxi = g.dxi.download(s);
  for (int64_t i = 0; i < N; ++i) {
    if (!std::isfinite(xi[2 * i]) || !std::isfinite(xi[2 * i + 1]) || !std::isfinite(dxi[2 * i]) ||
        !std::isfinite(dxi[2 * i + 1]) || !(1.0 - xyz[3 * i + 2] > 1e-12))
      fail(LBS_ERR_GEOMETRY, "node " + std::to_string(i) + " is not finite or at the pole");
  }
  // orientation: +1 when the island (bounded planar interior) lies to the
  // left of the traversal, i.e. the signed area sum Im(conj(xi) xi') > 0
  g.sign.resize(M);
  for (int k = 0; k < M; ++k) {
    double area = 0;
    for (int64_t i = g.offs[k]; i < g.offs[k + 1]; ++i)
      area += xi[2 * i] * dxi[2 * i + 1] - xi[2 * i + 1] * dxi[2 * i];
    g.sign[k] = area > 0 ? 1.0 : -1.0;
  }
  g.dsign.upload(g.sign, s);
  set_close_zones(g, xyz);
  g.qfac.alloc(2 * N);
  g.tau.alloc(N);
  g.gw.alloc(N);
  g.ell.alloc(N);
  launch_node_coeffs(N, g.island.p, g.dsign.p, g.doffs.p, g.xi.p, g.dxi.p, g.ddxi.p, g.qfac.p,
                     g.tau.p, g.gw.p, g.ell.p, s);
  // log-source geometry: projected centres, planar radii, near lists
  g.eta_x.resize(M);
  g.eta_y.resize(M);
  g.rho.assign(M, 0.0);
  std::vector<double> eta(2 * M), ellc(M);
  for (int k = 0; k < M; ++k) {
    const double d = 1.0 - g.cxyz[3 * k + 2];
    g.eta_x[k] = g.cxyz[3 * k] / d;
    g.eta_y[k] = g.cxyz[3 * k + 1] / d;
    eta[2 * k] = g.eta_x[k];
    eta[2 * k + 1] = g.eta_y[k];
    ellc[k] = std::log1p(g.eta_x[k] * g.eta_x[k] + g.eta_y[k] * g.eta_y[k]);
    for (int64_t i = g.offs[k]; i < g.offs[k + 1]; ++i)
      g.rho[k] = std::max(g.rho[k], std::hypot(xi[2 * i] - g.eta_x[k], xi[2 * i + 1] - g.eta_y[k]));
  }
  std::vector<int32_t> nptr(M + 1, 0), nidx;
  for (int k = 0; k < M; ++k) {
    const int q = isl_geo[k];
    const double lim = 9.0 * g.rho[k] * g.rho[k];
    for (int m = g.gisl[q]; m < g.gisl[q + 1]; ++m) {
      const double dx = g.eta_x[m] - g.eta_x[k], dy = g.eta_y[m] - g.eta_y[k];
      if (dx * dx + dy * dy <= lim) nidx.push_back(m);
    }
    nptr[k + 1] = (int32_t)nidx.size();
  }
  g.deta.upload(eta, s);
  g.drho.upload(g.rho, s);
  g.dellc.upload(ellc, s);
  g.near_ptr.upload(nptr, s);
  g.near_idx.upload(nidx, s);
  // log sources in each island's own frame (projection from the antipode of
  // its centre): node images, radii, frames, near lists and their transpose
  {
    g.xil.alloc(2 * N);
    g.elll.alloc(N);
    launch_local_frame(N, g.island.p, g.disl.p, g.xyz.p, g.xil.p, g.elll.p, s);
    std::vector<double> xl = g.xil.download(s);
    std::vector<double> rl(M, 0.0), fr(6 * M);
    for (int k = 0; k < M; ++k) {
      for (int64_t i = g.offs[k]; i < g.offs[k + 1]; ++i)
        rl[k] = std::max(rl[k], std::hypot(xl[2 * i], xl[2 * i + 1]));
      const double *c = isl[k].center, *e1 = isl[k].e1;
      fr[6 * k] = e1[0];
      fr[6 * k + 1] = e1[1];
      fr[6 * k + 2] = e1[2];
      fr[6 * k + 3] = e1[1] * c[2] - e1[2] * c[1];
      fr[6 * k + 4] = e1[2] * c[0] - e1[0] * c[2];
      fr[6 * k + 5] = e1[0] * c[1] - e1[1] * c[0];
    }
    // centre m is near island k when |eta'| <= 3 rho'_k, i.e. with
    // h = c_m . c_k:  (1 - h) <= 9 rho'^2 (1 + h)
    std::vector<int32_t> rp(M + 1, 0), ri;
    for (int k = 0; k < M; ++k) {
      const int q = isl_geo[k];
      const double lim = 9.0 * rl[k] * rl[k];
      for (int m = g.gisl[q]; m < g.gisl[q + 1]; ++m) {
        const double h = g.cxyz[3 * m] * g.cxyz[3 * k] + g.cxyz[3 * m + 1] * g.cxyz[3 * k + 1] +
                         g.cxyz[3 * m + 2] * g.cxyz[3 * k + 2];
        if (m == k || 1.0 - h <= lim * (1.0 + h)) ri.push_back(m);
      }
      rp[k + 1] = (int32_t)ri.size();
    }
    std::vector<int32_t> tp(M + 1, 0), ti(ri.size());
    for (int32_t m : ri) ++tp[m + 1];
    for (int m = 0; m < M; ++m) tp[m + 1] += tp[m];
    std::vector<int32_t> fill(tp.begin(), tp.end() - 1);
    for (int k = 0; k < M; ++k)
      for (int e = rp[k]; e < rp[k + 1]; ++e) ti[fill[ri[e]]++] = k;
    build_far_lists(g, isl_geo, rl, fr, rp, ri, s);
    g.rhol.upload(rl, s);
    g.frame.upload(fr, s);
    g.nearR_ptr.upload(rp, s);
    g.nearR_idx.upload(ri, s);
    g.nearRT_ptr.upload(tp, s);
    g.nearRT_idx.upload(ti, s);
  }
  // quadtree forest over the node images (one tree per geometry)
  HostPhase ph_tree("setup tree + plan");
  ctx->xi_x.resize(N);
  ctx->xi_y.resize(N);
  for (int64_t i = 0; i < N; ++i) {
    ctx->xi_x[i] = xi[2 * i];
    ctx->xi_y[i] = xi[2 * i + 1];
  }
  {
    Tree &F = ctx->plan.host;
    F = Tree();
    if (G == 1 && o.gpu_tree) {
      gpu_build_tree(g.xi.p, g.xi.p + 1, 2, N, nullptr, nullptr, 0, 0, true, o.leaf_max, F, s);
    } else {
      for (int q = 0; q < G; ++q) {
        const int64_t a = g.gnode[q], n = g.gnode[q + 1] - a;
        Tree t;
        build_tree(ctx->xi_x.data() + a, ctx->xi_y.data() + a, n, nullptr, nullptr, 0, true,
                   o.leaf_max, t);
        if (G == 1) {
          F = std::move(t);
        } else {
          append_tree(F, t, a, a, a, a);
        }
      }
    }
  }
  ctx->plan.m2l_groups = o.m2l_groups > 0 ? o.m2l_groups : kM2LGroups;
  upload_plan(ctx->plan.host, ctx->xi_x.data(), ctx->xi_y.data(), nullptr, nullptr, nullptr,
              ctx->plan, s);
  build_passes(ctx->plan, o.p32, o.p64, s);
  g.qfac_t.alloc(2 * N);
  launch_permute_complex(N, ctx->plan.src_perm.p, g.qfac.p, g.qfac_t.p, s);
  g.qm32_t.alloc(N);
  launch_qm32(N, g.qfac_t.p, g.qm32_t.p, s);
  build_p2m_inputs32(ctx->plan, s);
  {
    // gamma weights in tree order, and each geometry's source leaves
    const Tree &F = ctx->plan.host;
    std::vector<double> gw = g.gw.download(s), gwt(N);
    for (int64_t j = 0; j < N; ++j) gwt[j] = gw[F.src_perm[j]];
    g.gw_t.upload(gwt, s);
    // (the forest holds each geometry's tree in turn, so its leaves are
    // contiguous in the leaf list)
    const std::vector<int32_t> &ls = ctx->plan.leaf_s_host;
    std::vector<int32_t> gp(G + 1, 0);
    int prev = 0;
    for (size_t i = 0; i < ls.size(); ++i) {
      const int q = node_geo[F.src_perm[F.s0[ls[i]]]];
      if (q < prev) fail(LBS_ERR_GEOMETRY, "source leaves not grouped by geometry");
      prev = q;
      ++gp[q + 1];
    }
    for (int q = 0; q < G; ++q) gp[q + 1] += gp[q];
    g.gleaf_chunks = 1;
    for (int q = 0; q < G; ++q)
      g.gleaf_chunks = std::max(g.gleaf_chunks, (gp[q + 1] - gp[q] + 2047) / 2048);
    g.gleaf_ptr.upload(gp, s);
    LBS_HIP(hipStreamSynchronize(s));
  }
  build_tables(ctx->tab64, o.p64, s);
  build_tables(ctx->tab32, o.p32, s);
  // segments for the per-geometry reductions
  {
    std::vector<std::vector<std::pair<int64_t, int64_t>>> rn(G), rs(G);
    for (int q = 0; q < G; ++q) {
      rn[q].push_back({g.gnode[q], g.gnode[q + 1]});
      rs[q].push_back({g.gnode[q], g.gnode[q + 1]});
      rs[q].push_back({N + g.gisl[q], N + g.gisl[q + 1]});
    }
    ctx->seg_nodes.build(rn, s);
    ctx->seg_sys.build(rs, s);
  }
  // Schur complements S = D - F E and their inverses, one block per geometry
  {
    DBuf<double> S;
    S.alloc((size_t)g.gsinv[G]);
    g.Sinv.alloc((size_t)g.gsinv[G]);
    HostPhase ph("setup Schur + inverse");
    launch_build_schur(g, S.p, s);
    ctx->sinv_info = invert_schur(g, S.p, g.Sinv.p, o.schur_tol, s);
    if (host_timing()) LBS_HIP(hipStreamSynchronize(s));
  }
  ensure_ws(*ctx, 1);
  LBS_HIP(hipHostMalloc((void **)&ctx->count_host, 2 * sizeof(int32_t), hipHostMallocDefault));
  LBS_HIP(hipStreamSynchronize(s));
  return ctx.release();
}

// The tree links (parent, children, leaf flags) and each geometry's root
// box of a plan on the device, uploaded on first use.
void ensure_links(DevPlan &pl, hipStream_t s) {
  if (pl.roots.n > 0 || pl.nbox == 0) return;
  const Tree &T = pl.host;
  pl.parent.upload(T.parent, s);
  pl.child0.upload(T.child0, s);
  pl.nchild.upload(T.nchild, s);
  pl.leaf.upload(T.leaf, s);
  std::vector<int32_t> r;  // a forest holds its geometries' trees in turn
  for (int b = 0; b < pl.nbox; ++b)
    if (T.parent[b] < 0) r.push_back(b);
  pl.roots.upload(r, s);
  LBS_HIP(hipStreamSynchronize(s));  // r is released on return
}

// The evaluation plan for these targets (cached on the handle).
EvalPlan &eval_plan(lbs_ctx &c, bool transposed, const std::vector<int64_t> &toff,
                    const double *txyz, hipStream_t s) {
  Geometry &g = c.geo;
  const int G = g.G;
  const int64_t T = toff[G];
  HostPhase ph_all("eval plan (all)");
  std::unique_ptr<EvalPlan> &slot = transposed ? c.evt : c.evf;
  if (slot && slot->toff == toff && slot->dkey.n == (size_t)(3 * T)) {
    // the same targets as the cached plan's (compared on the device)
    if (c.diff.n == 0) c.diff.alloc(1);
    if (!targets_differ(3 * T, txyz, slot->dkey.p, c.diff.p, c.count_host + 1, s)) return *slot;
  }
  slot.reset();
  if (c.stage_n < (size_t)(3 * T)) {
    if (c.stage_host) (void)hipHostFree(c.stage_host);
    c.stage_host = nullptr;
    c.stage_n = 0;
    LBS_HIP(hipHostMalloc((void **)&c.stage_host, 3 * T * sizeof(double), hipHostMallocDefault));
    c.stage_n = (size_t)(3 * T);
  }
  if (T > 0)
    LBS_HIP(hipMemcpyAsync(c.stage_host, txyz, 3 * T * sizeof(double), hipMemcpyDeviceToHost, s));
  LBS_HIP(hipStreamSynchronize(s));
  std::vector<double> hx(c.stage_host, c.stage_host + 3 * T);
  auto ep = std::make_unique<EvalPlan>();
  ep->toff = toff;
  ep->tgeo.resize(T);
  std::vector<int64_t> qoff(G + 1, 0);
  for (int q = 0; q < G; ++q) {
    for (int64_t t = toff[q]; t < toff[q + 1]; ++t) {
      ep->tgeo[t] = q;
      const double x0 = hx[3 * t], x1 = hx[3 * t + 1], x2 = hx[3 * t + 2];
      if (!std::isfinite(x0) || !std::isfinite(x1) || !std::isfinite(x2))
        fail(LBS_ERR_NOT_FINITE, "target " + std::to_string(t) + " is not finite");
      const double d = 1.0 - x2;
      if (d <= 1e-14) continue;  // the pole: Cauchy part is zero
      ep->tx.push_back(x0 / d);
      ep->ty.push_back(x1 / d);
      ep->idx.push_back(t);
    }
    qoff[q + 1] = (int64_t)ep->tx.size();
  }
  ep->dtgeo.upload(ep->tgeo, s);
  const int64_t n = (int64_t)ep->idx.size();
  // located in the handle's own tree: forward always, transposed for one
  // geometry (the adjoint entry points serve no batch)
  const bool located = c.opt.matvec != LBS_MATVEC_DIRECT && !c.opt.eval_tree &&
                       (!transposed || G == 1);
  if (n > 0 && located) {
    HostPhase ph("eval plan locate");
    if ((int)g.gnode.size() != G + 1) fail(LBS_ERR_INVALID_ARG, "geometry table");
    ensure_links(c.plan, s);
    if ((int64_t)c.plan.roots.n != G) fail(LBS_ERR_GEOMETRY, "one tree per geometry expected");
    DBuf<double> dtx, dty;
    dtx.upload(ep->tx, s);
    dty.upload(ep->ty, s);
    ep->didx.upload(ep->idx, s);
    ep->ltx.alloc((size_t)n);
    ep->lty.alloc((size_t)n);
    ep->lbox.alloc((size_t)n);
    ep->lroot.alloc((size_t)n);
    ep->lidx.alloc((size_t)n);
    launch_locate_targets(n, dtx.p, dty.p, ep->didx.p, G > 1 ? ep->dtgeo.p : nullptr, c.plan,
                          ep->ltx.p, ep->lty.p, ep->lbox.p, ep->lroot.p, ep->lidx.p, s);
    if (transposed) {
      build_point_sources(c.plan, n, ep->ltx.p, ep->lty.p, ep->lbox.p, ep->lroot.p, ep->src, s);
      ep->located_src = true;
    } else {
      ep->located = true;
    }
  } else if (n > 0 && (transposed || c.opt.matvec != LBS_MATVEC_DIRECT)) {
    Tree &F = ep->pl.host;
    const bool on_gpu = G == 1 && c.opt.gpu_tree;
    DBuf<double> dtx, dty;  // the targets' images (GPU tree), until the plan is built
    DevPerms dperm;
    DevPoints dpts{};
    if (on_gpu) {
      HostPhase ph("eval plan tree (GPU)");
      dtx.upload(ep->tx, s);
      dty.upload(ep->ty, s);
      ep->didx.upload(ep->idx, s);
      if (transposed) {
        gpu_build_tree(dtx.p, dty.p, 1, n, g.xi.p, g.xi.p + 1, 2, g.N, false, c.opt.leaf_max, F, s,
                       &dperm);
        dpts = DevPoints{dtx.p, dty.p, 1, n, g.xi.p, g.xi.p + 1, 2, g.N, &dperm, nullptr};
      } else {
        gpu_build_tree(g.xi.p, g.xi.p + 1, 2, g.N, dtx.p, dty.p, 1, n, false, c.opt.leaf_max, F, s,
                       &dperm);
        dpts = DevPoints{g.xi.p, g.xi.p + 1, 2, g.N, dtx.p, dty.p, 1, n, &dperm, ep->didx.p};
      }
    } else {
      for (int q = 0; q < G; ++q) {
        const int64_t a = g.gnode[q], nn = g.gnode[q + 1] - a;
        const int64_t ta = qoff[q], tn = qoff[q + 1] - ta;
        Tree t;
        if (transposed)
          build_tree(ep->tx.data() + ta, ep->ty.data() + ta, tn, c.xi_x.data() + a,
                     c.xi_y.data() + a, nn, false, c.opt.leaf_max, t);
        else
          build_tree(c.xi_x.data() + a, c.xi_y.data() + a, nn, ep->tx.data() + ta,
                     ep->ty.data() + ta, tn, false, c.opt.leaf_max, t);
        if (G == 1) F = std::move(t);
        else if (transposed) append_tree(F, t, ta, a, ta, a);
        else append_tree(F, t, a, ta, a, ta);
      }
    }
    HostPhase ph_up("eval plan upload");
    const DevPoints *dp = on_gpu ? &dpts : nullptr;
    if (transposed) {
      upload_plan(F, ep->tx.data(), ep->ty.data(), c.xi_x.data(), c.xi_y.data(), nullptr,
                  ep->pl, s, dp);
      build_passes(ep->pl, c.opt.p32, c.opt.p64, s, true);
      if (!on_gpu) ep->didx.upload(ep->idx, s);
    } else {
      upload_plan(F, c.xi_x.data(), c.xi_y.data(), ep->tx.data(), ep->ty.data(), &ep->idx,
                  ep->pl, s, dp);
      build_passes(ep->pl, c.opt.p32, c.opt.p64, s, true);
      ep->qt.alloc(2 * g.N);
      launch_permute_complex(g.N, ep->pl.src_perm.p, g.qfac.p, ep->qt.p, s);
    }
    ep->ws.ensure(ep->pl, c.opt.p64, c.opt.p32, 1, g.N, g.M, G, kPlog);
    ep->tree = true;
  }
  if (c.opt.close_eval && n > 0) {
    HostPhase ph("eval plan close pairs");
    build_close(c, *ep, hx, txyz, s);
  }
  ep->dkey.alloc((size_t)(3 * T));
  if (T > 0)
    LBS_HIP(hipMemcpyAsync(ep->dkey.p, txyz, 3 * T * sizeof(double), hipMemcpyDeviceToDevice, s));
  LBS_HIP(hipStreamSynchronize(s));
  slot = std::move(ep);
  return *slot;
}

// Evaluation over geometry-major targets: targets [toff[q], toff[q+1]) of
// geometry q.
void eval_impl(lbs_ctx &c, int nrhs, const double *sigma, const double *A,
               const std::vector<int64_t> &toff, const double *txyz, double *u,
               hipStream_t s) {
  Geometry &g = c.geo;
  const int G = g.G;
  const int64_t T = toff[G];
  EvalPlan &ep = eval_plan(c, false, toff, txyz, s);
  launch_fill(T * nrhs, 0.0, u, s);
  if (!ep.idx.empty()) {
    if (c.opt.matvec == LBS_MATVEC_DIRECT) {
      std::vector<double> txi(2 * T, 0.0);
      std::vector<uint8_t> pole(T, 1);
      for (size_t q = 0; q < ep.idx.size(); ++q) {
        txi[2 * ep.idx[q]] = ep.tx[q];
        txi[2 * ep.idx[q] + 1] = ep.ty[q];
        pole[ep.idx[q]] = 0;
      }
      DBuf<double> dtxi;
      dtxi.upload(txi, s);
      DBuf<uint8_t> dpole;
      dpole.upload(pole, s);
      direct_eval64(g.N, g.xi.p, g.qfac.p, sigma, g.N, T, dtxi.p, dpole.p, nrhs, u, T, 0.5, s);
      LBS_HIP(hipStreamSynchronize(s));
    } else if (ep.located) {
      // the handle's own FP64 far field, then each target from its box
      ensure_ws(c, nrhs);
      StageTimer *keep = c.ws.timer;  // not one of the operator's stages
      c.ws.timer = nullptr;
      try {
        fmm_far64(c.plan, c.tab64, c.ws, g.qfac_t.p, sigma, g.N, nrhs, s);
      } catch (...) {
        c.ws.timer = keep;
        throw;
      }
      c.ws.timer = keep;
      launch_eval_points(c.tab64.P, (int64_t)ep.idx.size(), ep.ltx.p, ep.lty.p, ep.lbox.p,
                         ep.lroot.p, ep.lidx.p, c.plan, c.ws.pstr64.p, c.ws.mult64.p,
                         c.ws.loc64.p, nrhs, u, T, 0.5, s);
    } else {
      ep.ws.ensure(ep.pl, c.opt.p64, c.opt.p32, nrhs, g.N, g.M, G, kPlog);
      fmm_apply64(ep.pl, c.tab64, ep.ws, ep.qt.p, sigma, g.N, nrhs, u, T, 0.5, Assembly{}, s);
    }
  }
  ensure_ws(c, nrhs);
  launch_segdots(c.seg_nodes, nrhs, 1, g.gw.p, 0, 0, sigma, g.N, c.ws.gam.p, c.ws.red.p, s);
  launch_axpby((int64_t)nrhs * G, 0.0, c.ws.gam.p, 0.5, c.ws.gam.p, s);
  launch_eval_logsrc(g, T, txyz, ep.dtgeo.p, A, g.M, nrhs, c.ws.gam.p, u, T, s, &ep.lpart);
  if (ep.close.n_tgt > 0) {
    if (ep.closeV.n < (size_t)2 * g.N * nrhs) ep.closeV.alloc((size_t)2 * g.N * nrhs);
    launch_close_eval(g, ep.close, nrhs, sigma, g.N, ep.closeV.p, u, T, s);
  }
  LBS_HIP(hipStreamSynchronize(s));
}

// The transposed evaluation and the shape derivative cover the trapezoidal
// rule only.
void reject_close(const EvalPlan &ep, const char *what) {
  if (ep.close.n_tgt > 0)
    fail(LBS_ERR_UNSUPPORTED, std::string(what) + ": " + std::to_string(ep.close.n_tgt) +
                                  " targets lie in the close-evaluation zone of a curve "
                                  "(set close_eval = 0 for the trapezoidal rule)");
}

// ---------------------------------------------------------------- adjoint
// Transposed system A^T lambda = r (eq. matrix_eqns transposed) by GMRES on
// A^T P^-T (right preconditioning with the transposed block preconditioner),
// whose residual is the unpreconditioned one:
//   A^T P^-T mu = mu + [K^T (P^-T mu)_s; 0],   lambda = P^-T mu,
//   P^-T [r_s; r_a] = [r_s - F^T z; z],  z = S^-T (r_a - E^T r_s).
void ensure_adj(lbs_ctx &c) {
  AdjState &a = c.adj;
  if (a.ready) return;
  const Geometry &g = c.geo;
  const int64_t n = g.N + g.M;
  a.ones.upload(std::vector<double>((size_t)std::max<int64_t>(g.N, g.M), 1.0), (hipStream_t)0);
  a.mom.alloc((size_t)g.M * kMomStride);
  a.tA.alloc((size_t)g.M);
  a.lam.alloc((size_t)n);
  a.pc.alloc((size_t)2 * g.N);
  a.Fc.alloc((size_t)2 * g.N);
  a.ysum.alloc((size_t)g.G);
  c.geo.SinvT.alloc(c.geo.Sinv.n);
  launch_transpose_blocks(g, g.Sinv.p, c.geo.SinvT.p, (hipStream_t)0);
  LBS_HIP(hipStreamSynchronize((hipStream_t)0));
  a.ready = true;
}

// lam = P^-T mu, one column of length N + M (lam and mu distinct)
void precond_T(lbs_ctx &c, const double *mu, double *lam, hipStream_t s) {
  Geometry &g = c.geo;
  AdjState &a = c.adj;
  launch_logsrc_T(g, mu, a.mom.p, -1.0, a.tA.p, s);
  launch_axpby(g.M, 1.0, mu + g.N, 1.0, a.tA.p, s);
  launch_gemv_blocks_with(g, g.SinvT.p, a.tA.p, g.M, 1, lam + g.N, g.M, 1.0, s);
  launch_FT(g, lam + g.N, 1.0, mu, -1.0, lam, s);
}

// y = ident x + K^T x over the node rows (one column); the field by the
// FP64 FMM or, for LBS_MIXED, the FP32 one
void apply_KT(lbs_ctx &c, const double *x, double *y, double ident, int prec,
              hipStream_t s) {
  Geometry &g = c.geo;
  AdjState &a = c.adj;
  launch_real_to_complex(g.N, x, a.pc.p, s);
  if (prec == LBS_MIXED) fmm_apply32_full(c.plan, c.tab32, c.ws, a.pc.p, a.Fc.p, s);
  else fmm_apply64_full(c.plan, c.tab64, c.ws, a.pc.p, a.Fc.p, nullptr, s);
  launch_segdots(c.seg_nodes, 1, 1, a.ones.p, 0, 0, x, g.N, a.ysum.p, c.ws.red.p, s);
  launch_kT_assemble(g, x, a.Fc.p, a.ysum.p, ident, y, s);
}

// y = A^T P^-T x for R columns of length N + M
void apply_op_T(lbs_ctx &c, int R, const double *x, double *y, int prec, hipStream_t s) {
  Geometry &g = c.geo;
  const int64_t n = g.N + g.M;
  for (int r = 0; r < R; ++r) {
    precond_T(c, x + r * n, c.adj.lam.p, s);
    apply_KT(c, c.adj.lam.p, y + r * n, 0.0, prec, s);
    launch_fill(g.M, 0.0, y + r * n + g.N, s);
  }
  launch_axpby((int64_t)R * n, 1.0, x, 1.0, y, s);
}

// psi (and dpsi) at the nodes of sum_t w_t / (xi - zeta_t), one column
void eval_T_field(lbs_ctx &c, EvalPlan &ep, const double *w, double *pcw, double *psi,
                  double *dpsi, hipStream_t s) {
  const int64_t N = c.geo.N;
  if (ep.located_src) {  // the targets as sources of the handle's own FMM
    launch_gather_complex(ep.src.n, ep.lidx.p, w, pcw, s);
    fmm_sources64_full(c.plan, c.tab64, c.ws, ep.src, pcw, psi, dpsi, s);
    return;
  }
  if (!ep.tree) {
    launch_fill(2 * N, 0.0, psi, s);
    if (dpsi) launch_fill(2 * N, 0.0, dpsi, s);
    return;
  }
  launch_gather_complex((int64_t)ep.idx.size(), ep.didx.p, w, pcw, s);
  fmm_apply64_full(ep.pl, c.tab64, ep.ws, pcw, psi, dpsi, s);
}

}  // namespace

namespace lbs {
void set_last_error(const std::string &msg) { g_err = msg; }

// Workspace of one operator application (op, precision, nrhs) carved from
// base in 256-byte aligned pieces (base = nullptr: sizes only); returns the
// bytes it takes.  The same buffers Workspace::ensure allocates, for the
// precision in use only.
size_t carve_workspace(const lbs_ctx &c, int op, int prec, int nrhs, char *base,
                       Workspace &w) {
  const DevPlan &pl = c.plan;
  const Geometry &g = c.geo;
  size_t off = 0;
  auto take = [&](auto &buf, size_t count) {
    using T = std::remove_pointer_t<decltype(buf.p)>;
    off = (off + 255) & ~(size_t)255;
    if (base) buf.view((T *)(base + off), count);
    off += count * sizeof(T);
  };
  const size_t R = (size_t)nrhs;
  if (c.opt.matvec != LBS_MATVEC_DIRECT) {
    if (prec == LBS_FP64) {
      take(w.pstr64, (size_t)pl.ns * R * 2);
      take(w.mult64, (size_t)pl.nbox * c.opt.p64 * R * 2);
      take(w.loc64, (size_t)pl.nbox * c.opt.p64 * R * 2);
    } else {
      take(w.pstr32, (size_t)pl.ns * R * 2);
      take(w.mult32, (size_t)pl.nbox * c.opt.p32 * R * 2);
      take(w.loc32, (size_t)pl.nbox * c.opt.p32 * R * 2);
    }
    const size_t nls = (size_t)std::max(pl.n_leaf_s, 1);
    take(w.gpart, nls * R);
    take(w.gcsum, ((nls + 2047) / 2048) * g.G * R);
    take(w.gcnt, (size_t)g.G * R);
  }
  take(w.gam, R * g.G);
  const size_t chunks = (size_t)((g.N + g.M) / 2048 + 2 * g.G + 4);
  take(w.red, std::max<size_t>((size_t)512 * std::max<size_t>(R, 128), (size_t)128 * R * chunks));
  if (op == LBS_OP_SYSTEM || op == LBS_OP_PRECOND) {
    take(w.tmpM, (size_t)std::max(g.M, 1) * R);
    take(w.logL, (size_t)std::max(g.M, 1) * R * (2 * (kPlog + 1) + 2));
  }
  return off;
}

// lbs_matvec with every buffer beyond x and y in the caller's scratch
// memory (bytes at base, device), no allocation.
lbs_status matvec_in_scratch(lbs_handle h, int32_t op, int32_t prec, int32_t nrhs,
                             const double *x, double *y, void *stream, char *base,
                             size_t bytes) {
  return guard([&] {
    check_handle(h);
    if (!x || !y) fail(LBS_ERR_INVALID_ARG, "x or y is NULL");
    if (nrhs < 1 || nrhs > 65535) fail(LBS_ERR_INVALID_ARG, "nrhs outside [1, 65535]");
    if (prec != LBS_FP64 && prec != LBS_MIXED) fail(LBS_ERR_INVALID_ARG, "bad precision");
    if (op == LBS_OP_IPLUSK_T)
      fail(LBS_ERR_UNSUPPORTED, "the transposed operator is not served without allocation");
    if (op != LBS_OP_IPLUSK && op != LBS_OP_K && op != LBS_OP_SYSTEM && op != LBS_OP_PRECOND)
      fail(LBS_ERR_INVALID_ARG, "bad op");
    lbs_ctx &c = *h;
    Workspace w;
    const size_t need = carve_workspace(c, op, prec, nrhs, nullptr, w);
    if (need > bytes)
      fail(LBS_ERR_UNSUPPORTED, "this application needs " + std::to_string(need) +
                                    " bytes of scratch; the static scratch holds " +
                                    std::to_string(bytes));
    carve_workspace(c, op, prec, nrhs, base, w);
    hipStream_t s = (hipStream_t)stream;
    // the correction sums' completion counters start at zero
    if (w.gcnt.p) launch_fill_int((int64_t)w.gcnt.n, 0, w.gcnt.p, s);
    switch (op) {
      case LBS_OP_IPLUSK:
        apply_K_ws(c, w, prec, nrhs, x, c.geo.N, y, c.geo.N, 1.0, s);
        break;
      case LBS_OP_K:
        apply_K_ws(c, w, prec, nrhs, x, c.geo.N, y, c.geo.N, 0.0, s);
        break;
      case LBS_OP_SYSTEM:
        apply_system_ws(c, w, prec, nrhs, x, y, s);
        break;
      default:
        apply_precond_op_ws(c, w, prec, nrhs, x, y, s);
        break;
    }
  });
}
}  // namespace lbs

extern "C" {

void lbs_default_options(lbs_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->p64 = 30;
  o->p32 = 16;
  o->leaf_max = 48;
  o->restart = 50;
  o->max_iter = 400;
  o->max_outer = 8;
  o->inner_tol = 1e-5;
  o->matvec = LBS_MATVEC_FMM;
  o->graphs = 1;
  o->precond = 1;
  o->close_eval = 1;
  o->gpu_tree = 1;
  o->eval_tree = 0;
  o->m2l_groups = 0;
  o->schur_tol = 1e-12;
}

lbs_status lbs_refine_tolerances_host(int32_t S, const double *rn2, const double *bn2,
                                      double tol, double inner_tol, double *itol,
                                      int32_t *all_converged) {
  if (S < 0 || (S > 0 && (!rn2 || !bn2 || !itol)) || !all_converged) {
    g_err = "null pointer or negative count";
    return LBS_ERR_INVALID_ARG;
  }
  bool all = true;
  for (int q = 0; q < S; ++q) {
    if (!std::isfinite(rn2[q]) || !std::isfinite(bn2[q]) || rn2[q] < 0 || bn2[q] < 0) {
      g_err = "residual norm of system " + std::to_string(q) + " is not finite";
      *all_converged = 0;
      return LBS_ERR_NOT_FINITE;
    }
    const double rn = std::sqrt(rn2[q]), bn = std::sqrt(bn2[q]);
    if (rn <= tol * bn) {
      itol[q] = rn;  // converged: inactive in the inner solve
    } else {
      all = false;
      itol[q] = std::max(inner_tol * rn, 0.5 * tol * bn);
    }
  }
  *all_converged = all ? 1 : 0;
  return LBS_OK;
}

const char *lbs_last_error(void) { return g_err.c_str(); }

lbs_status lbs_setup(const lbs_island *isl, int32_t M, const int32_t *nodes,
                     const lbs_options *opt, void *stream, lbs_handle *out) {
  return guard([&] {
    if (!out) fail(LBS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!isl || !nodes) fail(LBS_ERR_INVALID_ARG, "islands or nodes is NULL");
    if (M < 1) fail(LBS_ERR_INVALID_ARG, "n_islands < 1");
    *out = setup_impl(1, &M, isl, nodes, opt, (hipStream_t)stream);
  });
}

lbs_status lbs_setup_sampled(const double *x, const double *xt, const double *xtt,
                             const double *centers, int32_t M, const int32_t *nodes,
                             const lbs_options *opt, void *stream, lbs_handle *out) {
  return guard([&] {
    if (!out) fail(LBS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!x || !xt || !xtt || !centers || !nodes) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    if (M < 1) fail(LBS_ERR_INVALID_ARG, "n_islands < 1");
    Samples sm;
    sm.x = x;
    sm.xt = xt;
    sm.xtt = xtt;
    sm.centers = centers;
    *out = setup_impl(1, &M, nullptr, nodes, opt, (hipStream_t)stream, &sm);
  });
}

lbs_status lbs_setup_batch(int32_t G, const int32_t *isl_per_geom, const lbs_island *isl,
                           const int32_t *nodes, const lbs_options *opt, void *stream,
                           lbs_handle *out) {
  return guard([&] {
    if (!out) fail(LBS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!isl || !nodes || !isl_per_geom) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    if (G < 1) fail(LBS_ERR_INVALID_ARG, "n_geoms < 1");
    *out = setup_impl(G, isl_per_geom, isl, nodes, opt, (hipStream_t)stream);
  });
}

lbs_status lbs_batch_info(lbs_handle h, int32_t *G, int64_t *node_off, int32_t *isl_off) {
  return guard([&] {
    check_handle(h);
    if (G) *G = h->geo.G;
    if (node_off) std::copy(h->geo.gnode.begin(), h->geo.gnode.end(), node_off);
    if (isl_off) std::copy(h->geo.gisl.begin(), h->geo.gisl.end(), isl_off);
  });
}

lbs_status lbs_sizes(lbs_handle h, int64_t *n, int32_t *m) {
  return guard([&] {
    check_handle(h);
    if (n) *n = h->geo.N;
    if (m) *m = h->geo.M;
  });
}

lbs_status lbs_nodes(lbs_handle h, double *xyz, void *stream) {
  return guard([&] {
    check_handle(h);
    if (!xyz) fail(LBS_ERR_INVALID_ARG, "xyz is NULL");
    LBS_HIP(hipMemcpyAsync(xyz, h->geo.xyz.p, 3 * h->geo.N * sizeof(double),
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
  });
}

lbs_status lbs_matvec(lbs_handle h, int32_t op, int32_t prec, int32_t nrhs, const double *x,
                      double *y, void *stream) {
  return guard([&] {
    check_handle(h);
    if (!x || !y) fail(LBS_ERR_INVALID_ARG, "x or y is NULL");
    if (nrhs < 1 || nrhs > 65535) fail(LBS_ERR_INVALID_ARG, "nrhs outside [1, 65535]");
    if (prec != LBS_FP64 && prec != LBS_MIXED) fail(LBS_ERR_INVALID_ARG, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    lbs_ctx &c = *h;
    ensure_ws(c, nrhs);
    switch (op) {
      case LBS_OP_IPLUSK:
        apply_K(c, prec, nrhs, x, c.geo.N, y, c.geo.N, 1.0, s);
        break;
      case LBS_OP_K:
        apply_K(c, prec, nrhs, x, c.geo.N, y, c.geo.N, 0.0, s);
        break;
      case LBS_OP_SYSTEM:
        apply_system(c, prec, nrhs, x, y, s);
        break;
      case LBS_OP_PRECOND:
        apply_precond_op(c, prec, nrhs, x, y, s);
        break;
      case LBS_OP_IPLUSK_T:
        ensure_adj(c);
        for (int r = 0; r < nrhs; ++r)
          apply_KT(c, x + (int64_t)r * c.geo.N, y + (int64_t)r * c.geo.N, 1.0, prec, s);
        break;
      default:
        fail(LBS_ERR_INVALID_ARG, "bad op");
    }
  });
}

lbs_status lbs_solve(lbs_handle h, int32_t prec, int32_t nrhs, const double *gdat, double tol,
                     double *sigma, double *A, lbs_solve_info *info, void *stream) {
  bool noconv = false;
  lbs_status st = guard([&] {
    check_handle(h);
    if (!gdat || !sigma || !A) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    if (nrhs < 1 || nrhs > 65535) fail(LBS_ERR_INVALID_ARG, "nrhs outside [1, 65535]");
    if (!(tol > 0 && tol < 1)) fail(LBS_ERR_INVALID_ARG, "tol outside (0, 1)");
    if (prec != LBS_FP64 && prec != LBS_MIXED) fail(LBS_ERR_INVALID_ARG, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    lbs_ctx &c = *h;
    Geometry &g = c.geo;
    const int R = nrhs, S = R * g.G;
    const int64_t n = g.N + g.M;
    const bool pre = c.opt.precond != 0;
    auto t0 = std::chrono::steady_clock::now();
    ensure_ws(c, R);
    ensure_gmres(c, R);
    GmresState &gm = c.gm;
    lbs_solve_info inf{};
    // finite data check
    launch_dots((int64_t)g.N * R, 1, gdat, 0, gdat, 0, gm.nrm2.p, c.ws.red.p, s);
    if (!std::isfinite(download(gm.nrm2.p, 1, s)[0])) fail(LBS_ERR_NOT_FINITE, "data g is not finite");
    if (pre) precond_rhs(c, R, gdat, gm.bvec.p, s);
    else system_rhs(c, R, gdat, gm.bvec.p, s);
    const int gid = pre ? 0 : 4;
    noconv = !solve_core(c, prec, R, forward_op(c, LBS_FP64, R, pre), gid,
                         forward_op(c, LBS_MIXED, R, pre), gid + 1, tol, inf, s);
    // final residuals with the FP64 operator: r = [2 g; 0] - A x (true), and
    // P^-1 r (preconditioned) relative to P^-1 [2 g; 0]
    system_rhs(c, R, gdat, gm.dvec.p, s);
    apply_system(c, LBS_FP64, R, gm.xvec.p, gm.rvec.p, s);
    inf.fp64_matvecs += 1;
    launch_axpby((int64_t)R * n, 1.0, gm.dvec.p, -1.0, gm.rvec.p, s);
    sys_norm2(c, R, gm.rvec.p, gm.nrm2.p, s);
    sys_norm2(c, R, gm.dvec.p, gm.h2.p, s);
    inf.true_rel_resid = worst_relative(download(gm.nrm2.p, S, s), download(gm.h2.p, S, s),
                                        "true residual");
    if (pre) {
      apply_precond_inverse(c, R, gm.rvec.p, s);
      sys_norm2(c, R, gm.rvec.p, gm.nrm2.p, s);
      inf.rel_resid = worst_relative(download(gm.nrm2.p, S, s), download(gm.bn2.p, S, s),
                                     "preconditioned residual");
    } else {
      inf.rel_resid = inf.true_rel_resid;
    }
    launch_copy_cols(g.N, R, 1.0, gm.xvec.p, n, sigma, g.N, s);
    launch_copy_cols(g.M, R, 1.0, gm.xvec.p + g.N, n, A, g.M, s);
    LBS_HIP(hipStreamSynchronize(s));
    inf.ms_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
  });
  if (st == LBS_OK && noconv) {
    g_err = "GMRES reached the iteration limit before the tolerance";
    return LBS_ERR_NO_CONVERGENCE;
  }
  return st;
}

lbs_status lbs_eval(lbs_handle h, int32_t nrhs, const double *sigma, const double *A,
                    int64_t T, const double *txyz, double *u, void *stream) {
  return guard([&] {
    check_handle(h);
    if (h->geo.G != 1) fail(LBS_ERR_INVALID_ARG, "batch handle: use lbs_eval_batch");
    if (nrhs < 1 || nrhs > 65535) fail(LBS_ERR_INVALID_ARG, "nrhs outside [1, 65535]");
    if (T < 0) fail(LBS_ERR_INVALID_ARG, "n_targets < 0");
    if (T == 0) return;
    if (!sigma || !A || !txyz || !u) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    eval_impl(*h, nrhs, sigma, A, {0, T}, txyz, u, (hipStream_t)stream);
  });
}

lbs_status lbs_eval_batch(lbs_handle h, int32_t nrhs, const double *sigma, const double *A,
                          const int64_t *toff, const double *txyz, double *u, void *stream) {
  return guard([&] {
    check_handle(h);
    if (!toff) fail(LBS_ERR_INVALID_ARG, "target offsets are NULL");
    if (nrhs < 1 || nrhs > 65535) fail(LBS_ERR_INVALID_ARG, "nrhs outside [1, 65535]");
    const int G = h->geo.G;
    std::vector<int64_t> off(toff, toff + G + 1);
    if (off[0] != 0) fail(LBS_ERR_INVALID_ARG, "target offsets must start at 0");
    for (int q = 0; q < G; ++q)
      if (off[q + 1] < off[q]) fail(LBS_ERR_INVALID_ARG, "target offsets decrease");
    if (off[G] == 0) return;
    if (!sigma || !A || !txyz || !u) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    eval_impl(*h, nrhs, sigma, A, off, txyz, u, (hipStream_t)stream);
  });
}

lbs_status lbs_eval_T(lbs_handle h, int32_t nrhs, const double *w, int64_t T, const double *txyz,
                      double *gs, double *ga, void *stream) {
  return guard([&] {
    check_handle(h);
    lbs_ctx &c = *h;
    Geometry &g = c.geo;
    if (g.G != 1) fail(LBS_ERR_UNSUPPORTED, "adjoint entry points serve single-geometry handles");
    if (nrhs < 1 || nrhs > 65535) fail(LBS_ERR_INVALID_ARG, "nrhs outside [1, 65535]");
    if (T < 0) fail(LBS_ERR_INVALID_ARG, "n_targets < 0");
    if (!gs || !ga || (T > 0 && (!w || !txyz))) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    if (T == 0) {
      launch_fill((int64_t)g.N * nrhs, 0.0, gs, s);
      launch_fill((int64_t)g.M * nrhs, 0.0, ga, s);
      return;
    }
    ensure_ws(c, 1);
    ensure_adj(c);
    EvalPlan &ep = eval_plan(c, true, {0, T}, txyz, s);
    reject_close(ep, "lbs_eval_T");
    DBuf<double> pcw, wsum;
    pcw.alloc((size_t)2 * std::max<size_t>(ep.idx.size(), 1));
    wsum.alloc(1);
    for (int r = 0; r < nrhs; ++r) {
      const double *wr = w + (int64_t)r * T;
      eval_T_field(c, ep, wr, pcw.p, c.adj.Fc.p, nullptr, s);
      launch_sum(T, wr, wsum.p, s);
      launch_evalT_sigma(g, c.adj.Fc.p, wsum.p, gs + (int64_t)r * g.N, s);
      launch_evalT_logsrc(g, T, txyz, wr, ga + (int64_t)r * g.M, c.adj.lpart, s);
    }
    LBS_HIP(hipStreamSynchronize(s));
  });
}

lbs_status lbs_solve_T(lbs_handle h, int32_t prec, int32_t nrhs, const double *rs,
                       const double *ra, double tol, double *lam_s, double *lam_a,
                       lbs_solve_info *info, void *stream) {
  bool noconv = false;
  lbs_status st = guard([&] {
    check_handle(h);
    if (!rs || !lam_s || !lam_a) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    if (nrhs < 1 || nrhs > 65535) fail(LBS_ERR_INVALID_ARG, "nrhs outside [1, 65535]");
    if (!(tol > 0 && tol < 1)) fail(LBS_ERR_INVALID_ARG, "tol outside (0, 1)");
    if (prec != LBS_FP64 && prec != LBS_MIXED) fail(LBS_ERR_INVALID_ARG, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    lbs_ctx &c = *h;
    Geometry &g = c.geo;
    const int R = nrhs, S = R * g.G;
    const int64_t n = g.N + g.M;
    auto t0 = std::chrono::steady_clock::now();
    ensure_ws(c, R);
    ensure_gmres(c, R);
    ensure_adj(c);
    GmresState &gm = c.gm;
    lbs_solve_info inf{};
    launch_copy_cols(g.N, R, 1.0, rs, g.N, gm.bvec.p, n, s);
    if (ra) launch_copy_cols(g.M, R, 1.0, ra, g.M, gm.bvec.p + g.N, n, s);
    else
      for (int r = 0; r < R; ++r) launch_fill(g.M, 0.0, gm.bvec.p + r * n + g.N, s);
    launch_dots((int64_t)R * n, 1, gm.bvec.p, 0, gm.bvec.p, 0, gm.nrm2.p, c.ws.red.p, s);
    if (!std::isfinite(download(gm.nrm2.p, 1, s)[0]))
      fail(LBS_ERR_NOT_FINITE, "right-hand side is not finite");
    OpFn op64 = [&](const double *in, double *out, hipStream_t q) {
      apply_op_T(c, R, in, out, LBS_FP64, q);
    };
    OpFn op32 = [&](const double *in, double *out, hipStream_t q) {
      apply_op_T(c, R, in, out, LBS_MIXED, q);
    };
    noconv = !solve_core(c, prec, R, op64, 2, op32, 3, tol, inf, s);
    // residual of A^T lambda = b (equal to that of the right-preconditioned system)
    op64(gm.xvec.p, gm.rvec.p, s);
    inf.fp64_matvecs += 1;
    launch_axpby((int64_t)R * n, 1.0, gm.bvec.p, -1.0, gm.rvec.p, s);
    sys_norm2(c, R, gm.rvec.p, gm.nrm2.p, s);
    const double worst = worst_relative(download(gm.nrm2.p, S, s), download(gm.bn2.p, S, s),
                                        "residual");
    for (int r = 0; r < R; ++r) precond_T(c, gm.xvec.p + r * n, gm.dvec.p + r * n, s);
    launch_copy_cols(g.N, R, 1.0, gm.dvec.p, n, lam_s, g.N, s);
    launch_copy_cols(g.M, R, 1.0, gm.dvec.p + g.N, n, lam_a, g.M, s);
    LBS_HIP(hipStreamSynchronize(s));
    inf.rel_resid = worst;
    inf.true_rel_resid = worst;
    inf.ms_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
  });
  if (st == LBS_OK && noconv) {
    g_err = "GMRES reached the iteration limit before the tolerance";
    return LBS_ERR_NO_CONVERGENCE;
  }
  return st;
}

lbs_status lbs_shape_vjp(lbs_handle h, const double *sigma, const double *A, const double *lam_s,
                         int64_t T, const double *txyz, const double *w, double *dcoef,
                         void *stream) {
  return guard([&] {
    check_handle(h);
    lbs_ctx &c = *h;
    Geometry &g = c.geo;
    if (g.G != 1) fail(LBS_ERR_UNSUPPORTED, "adjoint entry points serve single-geometry handles");
    if (g.sampled) fail(LBS_ERR_UNSUPPORTED, "a sampled-curve handle has no shape coefficients");
    if (T < 0) fail(LBS_ERR_INVALID_ARG, "n_targets < 0");
    if (!sigma || !A || !lam_s || !dcoef || (T > 0 && (!w || !txyz)))
      fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    ensure_ws(c, 1);
    ensure_adj(c);
    const int64_t N = g.N;
    DBuf<double> buf;
    buf.alloc((size_t)12 * N + 8);
    double *Fl = buf.p, *dFl = Fl + 2 * N, *dFp = dFl + 2 * N, *Fw = dFp + 2 * N,
           *dFw = Fw + 2 * N, *LSd = dFw + 2 * N, *sums = LSd + 2 * N;
    AdjState &a = c.adj;
    // fields of the adjoint density and of the double-layer strengths
    launch_real_to_complex(N, lam_s, a.pc.p, s);
    fmm_apply64_full(c.plan, c.tab64, c.ws, a.pc.p, Fl, dFl, s);
    launch_dl_strengths(g, sigma, a.pc.p, s);
    fmm_apply64_full(c.plan, c.tab64, c.ws, a.pc.p, a.Fc.p, dFp, s);
    // field of the target weights at the nodes
    DBuf<double> pcw;
    if (T > 0) {
      EvalPlan &ep = eval_plan(c, true, {0, T}, txyz, s);
      reject_close(ep, "lbs_shape_vjp");
      pcw.alloc((size_t)2 * std::max<size_t>(ep.idx.size(), 1));
      eval_T_field(c, ep, w, pcw.p, Fw, dFw, s);
      launch_sum(T, w, sums + 2, s);
    } else {
      launch_fill(4 * N, 0.0, Fw, s);
      launch_fill(1, 0.0, sums + 2, s);
    }
    launch_logsrc_deriv(g, c.ws, A, LSd, s);
    launch_sum(N, lam_s, sums, s);
    launch_sum(g.M, A, sums + 1, s);
    launch_shape_vjp(g, sigma, lam_s, Fl, dFl, dFp, Fw, dFw, LSd, sums, sums + 1, sums + 2,
                     dcoef, s);
    LBS_HIP(hipStreamSynchronize(s));
  });
}

// Vortex positions: finite unit vectors (host check of a device array).
void check_vortices(int32_t nv, const double *xyz_v, const double *gamma, int nrhs,
                    hipStream_t s) {
  if (nv < 1 || nv > (1 << 24)) fail(LBS_ERR_INVALID_ARG, "n_vortices outside [1, 2^24]");
  if (!xyz_v || !gamma) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
  std::vector<double> v(3 * (size_t)nv), gm((size_t)nv * nrhs);
  LBS_HIP(hipMemcpyAsync(v.data(), xyz_v, v.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  LBS_HIP(hipMemcpyAsync(gm.data(), gamma, gm.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  LBS_HIP(hipStreamSynchronize(s));
  for (int32_t j = 0; j < nv; ++j) {
    const double *p = &v[3 * (size_t)j];
    if (!std::isfinite(p[0]) || !std::isfinite(p[1]) || !std::isfinite(p[2]) ||
        std::fabs(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] - 1.0) > 1e-9)
      fail(LBS_ERR_GEOMETRY, "vortex " + std::to_string(j) + " is not a finite unit vector");
  }
  for (double x : gm)
    if (!std::isfinite(x)) fail(LBS_ERR_NOT_FINITE, "vortex strength is not finite");
}

lbs_status lbs_set_orders(lbs_handle h, int32_t p64, int32_t p32, void *stream) {
  return guard([&] {
    check_handle(h);
    if (!p64_ok(p64)) fail(LBS_ERR_UNSUPPORTED, "p64 must be 20/24/30/36/40/48");
    if (!p32_ok(p32)) fail(LBS_ERR_UNSUPPORTED, "p32 must be 12/16/20/24");
    lbs_ctx &c = *h;
    hipStream_t s = (hipStream_t)stream;
    LBS_HIP(hipStreamSynchronize(s));
    if (p64 != c.opt.p64) build_tables(c.tab64, p64, s);
    if (p32 != c.opt.p32) build_tables(c.tab32, p32, s);
    c.opt.p64 = p64;
    c.opt.p32 = p32;
    build_passes(c.plan, p32, p64, s);
    // expansion buffers are sized by the orders: reallocate on next use
    const int cap = std::max(1, c.ws.nrhs_cap);
    c.ws.nrhs_cap = 0;
    ensure_ws(c, cap);
    c.evf.reset();
    c.evt.reset();
    // captured iterations hold the old tables and kernels
    c.graphs.clear();
    c.graphs.sig.clear();
    LBS_HIP(hipStreamSynchronize(s));
  });
}

lbs_status lbs_vortex_data(lbs_handle h, int32_t nrhs, const double *g, int32_t nv,
                           const double *xyz_v, const double *gamma, double *g_star,
                           void *stream) {
  return guard([&] {
    check_handle(h);
    if (h->geo.G != 1) fail(LBS_ERR_UNSUPPORTED, "point vortices serve single-geometry handles");
    if (nrhs < 1 || nrhs > 65535) fail(LBS_ERR_INVALID_ARG, "nrhs outside [1, 65535]");
    if (!g || !g_star) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    check_vortices(nv, xyz_v, gamma, nrhs, s);
    const Geometry &geo = h->geo;
    launch_vortex_field(geo.N, geo.xyz.p, nv, xyz_v, gamma, nrhs, -1.0, g, geo.N, 1.0, g_star,
                        geo.N, s);
  });
}

lbs_status lbs_vortex_field(lbs_handle h, int32_t nrhs, int32_t nv, const double *xyz_v,
                            const double *gamma, int64_t T, const double *txyz, double *u,
                            void *stream) {
  return guard([&] {
    check_handle(h);
    if (nrhs < 1 || nrhs > 65535) fail(LBS_ERR_INVALID_ARG, "nrhs outside [1, 65535]");
    if (T < 0) fail(LBS_ERR_INVALID_ARG, "n_targets < 0");
    if (T == 0) return;
    if (!txyz || !u) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    check_vortices(nv, xyz_v, gamma, nrhs, s);
    launch_vortex_field(T, txyz, nv, xyz_v, gamma, nrhs, 1.0, u, T, 1.0, u, T, s);
  });
}

lbs_status lbs_stage_timing(lbs_handle h, int32_t enable) {
  return guard([&] {
    check_handle(h);
    if (enable) {
      h->ws.timer = &h->timer;
    } else {
      h->timer.collect();
      h->ws.timer = nullptr;
    }
  });
}

lbs_status lbs_stage_times(lbs_handle h, double *ms, int64_t *launches, int32_t n) {
  return guard([&] {
    check_handle(h);
    if (!ms || n < ST_NSTAGES) fail(LBS_ERR_INVALID_ARG, "need LBS_NSTAGES entries");
    h->timer.collect();
    for (int i = 0; i < ST_NSTAGES; ++i) {
      ms[i] = h->timer.ms[i];
      if (launches) launches[i] = h->timer.cnt[i];
      h->timer.ms[i] = 0;
      h->timer.cnt[i] = 0;
    }
  });
}

lbs_status lbs_destroy(lbs_handle h) {
  return guard([&] { delete h; });
}

static void fill_stats(const Tree &T, lbs_tree_stats *st) {
  std::memset(st, 0, sizeof(*st));
  st->levels = T.nlevels;
  st->boxes = T.nbox();
  for (int b = 0; b < T.nbox(); ++b) st->leaves += T.leaf[b];
  st->u_pairs = (int64_t)T.u_src.size();
  st->v_pairs = (int64_t)T.v_src.size();
  st->w_pairs = (int64_t)T.w_src.size();
  st->x_pairs = (int64_t)T.x_src.size();
  st->p2p_interactions = T.p2p_pairs;
  st->m2p_evals = T.m2p_evals;
  st->p2l_evals = T.p2l_evals;
}

lbs_status lbs_tree_info(lbs_handle h, lbs_tree_stats *st) {
  return guard([&] {
    check_handle(h);
    if (!st) fail(LBS_ERR_INVALID_ARG, "stats is NULL");
    fill_stats(h->plan.host, st);
  });
}

lbs_status lbs_schur_info(lbs_handle h, int32_t *pivoted, double *omega) {
  return guard([&] {
    check_handle(h);
    if (pivoted) *pivoted = h->sinv_info.pivoted;
    if (omega) *omega = h->sinv_info.omega;
  });
}

lbs_status lbs_schur_residual(lbs_handle h, int32_t ncols, double *err, void *stream) {
  return guard([&] {
    check_handle(h);
    if (!err || ncols < 1) fail(LBS_ERR_INVALID_ARG, "err is NULL or ncols < 1");
    hipStream_t s = (hipStream_t)stream;
    const Geometry &g = h->geo;
    *err = 0.0;
    if (g.M == 0) return;
    // X: column r holds, in every geometry block, the unit vector of local
    // island (r * Mg) / ncols; Y = S (Sinv X) - X
    std::vector<double> X((size_t)g.M * ncols, 0.0);
    for (int r = 0; r < ncols; ++r)
      for (int q = 0; q < g.G; ++q) {
        const int m0 = g.gisl[q], Mg = g.gisl[q + 1] - m0;
        X[(size_t)r * g.M + m0 + (int)((int64_t)r * Mg / ncols)] = 1.0;
      }
    DBuf<double> S, dX, Y1, Y2;
    S.alloc((size_t)g.gsinv[g.G]);
    launch_build_schur(g, S.p, s);
    dX.upload(X, s);
    Y1.alloc(X.size());
    Y2.alloc(X.size());
    launch_gemv_blocks_with(g, g.Sinv.p, dX.p, g.M, ncols, Y1.p, g.M, 1.0, s);
    launch_gemv_blocks_with(g, S.p, Y1.p, g.M, ncols, Y2.p, g.M, 1.0, s);
    const std::vector<double> y = Y2.download(s);
    double e = 0.0;
    for (size_t i = 0; i < y.size(); ++i) {
      const double d = std::fabs(y[i] - X[i]);
      if (!(d <= e)) e = d;  // NaN propagates
    }
    *err = e;
  });
}

lbs_status lbs_compare_trees(const double *x, const double *y, int64_t n, const double *tx,
                             const double *ty, int64_t nt, int32_t leaf_max, int64_t *mismatch,
                             int32_t *levels, void *stream) {
  return guard([&] {
    if (!x || !y || !mismatch || (nt > 0 && (!tx || !ty)))
      fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    if (n < 1 || nt < 0 || leaf_max < 1) fail(LBS_ERR_INVALID_ARG, "n, nt or leaf_max out of range");
    hipStream_t s = (hipStream_t)stream;
    const bool self = nt == 0;
    Tree G;
    gpu_build_tree(x, y, 1, n, tx, ty, 1, nt, self, leaf_max, G, s);
    std::vector<double> hx = download(x, n, s), hy = download(y, n, s), htx, hty;
    if (!self) {
      htx = download(tx, nt, s);
      hty = download(ty, nt, s);
    }
    Tree H;
    build_tree(hx.data(), hy.data(), n, self ? nullptr : htx.data(), self ? nullptr : hty.data(),
               nt, self, leaf_max, H);
    int64_t bad = 0;
    auto cmp = [&](const auto &a, const auto &b) {
      if (a.size() != b.size()) {
        bad += 1 + (int64_t)std::max(a.size(), b.size());
        return;
      }
      for (size_t i = 0; i < a.size(); ++i) bad += a[i] != b[i];
    };
    cmp(G.cx, H.cx); cmp(G.cy, H.cy); cmp(G.rad, H.rad); cmp(G.level, H.level);
    cmp(G.parent, H.parent); cmp(G.child0, H.child0); cmp(G.nchild, H.nchild);
    cmp(G.ix, H.ix); cmp(G.iy, H.iy); cmp(G.s0, H.s0); cmp(G.s1, H.s1); cmp(G.t0, H.t0);
    cmp(G.t1, H.t1); cmp(G.leaf, H.leaf); cmp(G.level_ptr, H.level_ptr);
    cmp(G.v_ptr, H.v_ptr); cmp(G.v_src, H.v_src); cmp(G.v_code, H.v_code);
    cmp(G.x_ptr, H.x_ptr); cmp(G.x_src, H.x_src); cmp(G.u_ptr, H.u_ptr); cmp(G.u_src, H.u_src);
    cmp(G.w_ptr, H.w_ptr); cmp(G.w_src, H.w_src); cmp(G.src_perm, H.src_perm);
    cmp(G.tgt_perm, H.tgt_perm);
    bad += G.nlevels != H.nlevels;
    bad += G.x0 != H.x0 || G.y0 != H.y0 || G.R0 != H.R0;
    bad += G.p2p_pairs != H.p2p_pairs || G.m2p_evals != H.m2p_evals || G.p2l_evals != H.p2l_evals;
    *mismatch = bad;
    if (levels) *levels = G.nlevels;
  });
}

lbs_status lbs_check_tree_host(const double *x, const double *y, int64_t n, int32_t leaf_max,
                               int64_t *bad, lbs_tree_stats *st) {
  return guard([&] {
    if (!x || !y || !bad) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    if (n < 1 || leaf_max < 1) fail(LBS_ERR_INVALID_ARG, "n or leaf_max < 1");
    Tree T;
    build_tree(x, y, n, nullptr, nullptr, 0, true, leaf_max, T);
    *bad = check_coverage(T);
    if (st) fill_stats(T, st);
  });
}

lbs_status lbs_check_passes_host(const double *x, const double *y, int64_t n, int32_t leaf_max,
                                 int32_t cap, int64_t *bad, int32_t *rounds) {
  return guard([&] {
    if (!x || !y || !bad) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    if (n < 1 || leaf_max < 1) fail(LBS_ERR_INVALID_ARG, "n or leaf_max < 1");
    if (cap < 16 || cap > 1024) fail(LBS_ERR_INVALID_ARG, "cap outside 16 .. 1024");
    Tree T;
    build_tree(x, y, n, nullptr, nullptr, 0, true, leaf_max, T);
    *bad = 0;
    for (int d = 0; d < 2; ++d) {
      PassProgram pp;
      build_pass_program(T, d == 1, cap, pp);
      *bad += check_pass_program(T, pp);
      if (rounds) rounds[d] = (int32_t)pp.round_ptr.size() - 1;
    }
  });
}

}  // extern "C"
