// C-ABI of liblbs (include/lbs.h): set-up, operator application, GMRES
// solve with the block preconditioner, and evaluation at sphere targets.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "lbs_internal.h"

using namespace lbs;

namespace {
thread_local std::string g_err;

struct ErrNoConv {};

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

// Upload a host tree as a device plan.  sx/sy (tx/ty) are the source
// (target) coordinates in input order; tgt_index maps a target's input
// position to the index written by the leaf kernel.
void upload_plan(Tree &T, const double *sx, const double *sy,
                 const double *tx, const double *ty,
                 const std::vector<int64_t> *tgt_index, DevPlan &pl,
                 hipStream_t s) {
  const int nb = T.nbox();
  pl.nbox = nb;
  pl.nlevels = T.nlevels;
  pl.self = T.self;
  pl.ns = (int64_t)T.src_perm.size();
  pl.nt = (int64_t)T.tgt_perm.size();
  pl.level_ptr = T.level_ptr;
  std::vector<int32_t> quad(nb), leaf_s, leaf_t, m2l;
  std::vector<uint8_t> has_tgt(nb);
  for (int b = 0; b < nb; ++b) {
    quad[b] = (T.ix[b] & 1) | ((T.iy[b] & 1) << 1);
    has_tgt[b] = T.t1[b] > T.t0[b];
    if (T.leaf[b] && T.s1[b] > T.s0[b]) leaf_s.push_back(b);
    if (T.leaf[b] && has_tgt[b]) leaf_t.push_back(b);
    if (T.level[b] >= 2 && has_tgt[b]) m2l.push_back(b);
  }
  pl.n_leaf_s = (int)leaf_s.size();
  pl.n_leaf_t = (int)leaf_t.size();
  pl.n_m2l = (int)m2l.size();
  pl.leaf_t_host = leaf_t;
  pl.cx.upload(T.cx, s);
  pl.cy.upload(T.cy, s);
  pl.rad.upload(T.rad, s);
  pl.parent.upload(T.parent, s);
  pl.child0.upload(T.child0, s);
  pl.nchild.upload(T.nchild, s);
  pl.quad.upload(quad, s);
  pl.lev.upload(T.level, s);
  pl.s0.upload(T.s0, s);
  pl.s1.upload(T.s1, s);
  pl.t0.upload(T.t0, s);
  pl.t1.upload(T.t1, s);
  pl.leaf.upload(T.leaf, s);
  pl.has_tgt.upload(has_tgt, s);
  pl.v_ptr.upload(T.v_ptr, s);
  pl.v_src.upload(T.v_src, s);
  pl.v_code.upload(T.v_code, s);
  pl.x_ptr.upload(T.x_ptr, s);
  pl.x_src.upload(T.x_src, s);
  pl.u_ptr.upload(T.u_ptr, s);
  pl.u_src.upload(T.u_src, s);
  pl.w_ptr.upload(T.w_ptr, s);
  pl.w_src.upload(T.w_src, s);
  pl.leaf_t.upload(leaf_t, s);
  pl.leaf_s.upload(leaf_s, s);
  pl.m2l_box.upload(m2l, s);
  auto split = [](double v, float &hi, float &lo) {
    hi = (float)v;
    lo = (float)(v - (double)hi);
  };
  {
    const int64_t n = pl.ns;
    std::vector<double> x(n), y(n);
    std::vector<float> xh(n), xl(n), yh(n), yl(n);
    for (int64_t j = 0; j < n; ++j) {
      x[j] = sx[T.src_perm[j]];
      y[j] = sy[T.src_perm[j]];
      split(x[j], xh[j], xl[j]);
      split(y[j], yh[j], yl[j]);
    }
    pl.sx.upload(x, s);
    pl.sy.upload(y, s);
    pl.sxh.upload(xh, s);
    pl.sxl.upload(xl, s);
    pl.syh.upload(yh, s);
    pl.syl.upload(yl, s);
    pl.src_perm.upload(T.src_perm, s);
  }
  {
    const double *ax = T.self ? sx : tx, *ay = T.self ? sy : ty;
    const int64_t n = pl.nt;
    std::vector<double> x(n), y(n);
    std::vector<float> xh(n), xl(n), yh(n), yl(n);
    std::vector<int64_t> perm(n);
    for (int64_t j = 0; j < n; ++j) {
      const int64_t a = T.tgt_perm[j];
      x[j] = ax[a];
      y[j] = ay[a];
      split(x[j], xh[j], xl[j]);
      split(y[j], yh[j], yl[j]);
      perm[j] = tgt_index ? (*tgt_index)[a] : a;
    }
    pl.tx.upload(x, s);
    pl.ty.upload(y, s);
    pl.txh.upload(xh, s);
    pl.txl.upload(xl, s);
    pl.tyh.upload(yh, s);
    pl.tyl.upload(yl, s);
    pl.tgt_perm.upload(perm, s);
  }
  LBS_HIP(hipStreamSynchronize(s));
}

}  // namespace

namespace lbs {
void Workspace::ensure(const DevPlan &pl, int P64, int P32, int nrhs,
                       int64_t N, int M, int Plog) {
  if (nrhs <= nrhs_cap) return;
  nrhs_cap = nrhs;
  pstr64.alloc((size_t)pl.ns * nrhs * 2);
  mult64.alloc((size_t)pl.nbox * P64 * nrhs * 2);
  loc64.alloc((size_t)pl.nbox * P64 * nrhs * 2);
  pstr32.alloc((size_t)pl.ns * nrhs * 2);
  mult32.alloc((size_t)pl.nbox * P32 * nrhs * 2);
  loc32.alloc((size_t)pl.nbox * P32 * nrhs * 2);
  gam.alloc(std::max(nrhs, 1));
  red.alloc((size_t)512 * std::max(nrhs, 128));
  tmpM.alloc((size_t)std::max(M, 1) * nrhs);
  logL.alloc((size_t)std::max(M, 1) * nrhs * (2 * (Plog + 1) + 2));
  (void)N;
}
}  // namespace lbs

struct lbs_ctx {
  lbs_options opt{};
  Geometry geo;
  DevPlan plan;
  Tables tab64, tab32;
  Workspace ws;
  std::vector<double> xi_x, xi_y;  // node images, API order (eval trees)
  StageTimer timer;
  // GMRES state (vector length n = N + M)
  int64_t n = 0;
  DBuf<double> V, H, cs, sn, gv, yv, h2, nrm2, resid, bvec, rvec, xvec, dvec;
  double *resid_host = nullptr;
  ~lbs_ctx() {
    if (resid_host) (void)hipHostFree(resid_host);
  }
};

namespace {

void apply_K(lbs_ctx &c, int prec, int nrhs, const double *x, int64_t ldx,
             double *y, int64_t ldy, double ident, hipStream_t s) {
  Geometry &g = c.geo;
  c.ws.ensure(c.plan, c.opt.p64, c.opt.p32, nrhs, g.N, g.M, kPlog);
  {
    TimerScope ts(c.ws.timer, ST_GAMMA, s);
    launch_dots(g.N, nrhs, g.gw.p, 0, x, ldx, c.ws.gam.p, c.ws.red.p, s);
  }
  Assembly as;
  as.sigma = x;
  as.tau = g.tau.p;
  as.gamma = c.ws.gam.p;
  as.ident = ident;
  as.ldx = ldx;
  if (c.opt.matvec == LBS_MATVEC_DIRECT) {
    TimerScope ts(c.ws.timer, ST_LEAF, s);
    direct_apply64(g.N, g.xi.p, g.qfac.p, x, ldx, nrhs, y, ldy, as, s);
  } else if (prec == LBS_FP64) {
    fmm_apply64(c.plan, c.tab64, c.ws, g.qfac_t.p, x, ldx, nrhs, y, ldy, 1.0,
                as, s);
  } else {
    fmm_apply32(c.plan, c.tab32, c.ws, g.qfac_t.p, x, ldx, nrhs, y, ldy, 1.0,
                as, s);
  }
}

// y = P^-1 A x = x + P^-1 [K x_s; 0]   (x, y: n x nrhs with ld n = N + M)
void apply_precond_op(lbs_ctx &c, int prec, int nrhs, const double *x,
                      double *y, hipStream_t s) {
  Geometry &g = c.geo;
  const int64_t n = g.N + g.M;
  apply_K(c, prec, nrhs, x, n, y, n, 0.0, s);
  {
    TimerScope ts(c.ws.timer, ST_CONSTRAINT, s);
    launch_island_sums(g, y, n, nrhs, c.ws.tmpM.p, g.M, s);
    launch_gemv(g.M, g.Sinv.p, c.ws.tmpM.p, g.M, nrhs, y + g.N, n, -1.0, s);
  }
  {
    TimerScope ts(c.ws.timer, ST_LOGSRC, s);
    launch_logsrc_apply(g, c.ws, y + g.N, n, nrhs, y, n, -1.0, s);
  }
  launch_axpby(n * nrhs, 1.0, x, 1.0, y, s);
}

// [y_s; y_a] = [ (I+K) x_s + E x_a ; F x_s + D x_a ]
void apply_system(lbs_ctx &c, int prec, int nrhs, const double *x, double *y,
                  hipStream_t s) {
  Geometry &g = c.geo;
  const int64_t n = g.N + g.M;
  apply_K(c, prec, nrhs, x, n, y, n, 1.0, s);
  {
    TimerScope ts(c.ws.timer, ST_LOGSRC, s);
    launch_logsrc_apply(g, c.ws, x + g.N, n, nrhs, y, n, 1.0, s);
  }
  TimerScope ts(c.ws.timer, ST_CONSTRAINT, s);
  launch_constraint_rows(g, x, n, x + g.N, n, nrhs, y + g.N, n, s);
}

// b = P^-1 [2 g; 0] for one right-hand side (b has length N + M)
void precond_rhs(lbs_ctx &c, const double *gdat, double *b, hipStream_t s) {
  Geometry &g = c.geo;
  c.ws.ensure(c.plan, c.opt.p64, c.opt.p32, 1, g.N, g.M, kPlog);
  launch_fill(g.N, 0.0, b, s);
  launch_axpby(g.N, 2.0, gdat, 0.0, b, s);
  launch_island_sums(g, b, g.N, 1, c.ws.tmpM.p, g.M, s);
  launch_gemv(g.M, g.Sinv.p, c.ws.tmpM.p, g.M, 1, b + g.N, g.M, -1.0, s);
  launch_logsrc_apply(g, c.ws, b + g.N, g.M, 1, b, g.N, -1.0, s);
}

double norm2(lbs_ctx &c, const double *x, int64_t n, hipStream_t s) {
  launch_dots(n, 1, x, 0, x, 0, c.nrm2.p, c.ws.red.p, s);
  LBS_HIP(hipMemcpyAsync(c.resid_host, c.nrm2.p, sizeof(double),
                         hipMemcpyDeviceToHost, s));
  LBS_HIP(hipStreamSynchronize(s));
  return std::sqrt(std::max(0.0, *c.resid_host));
}

struct GmresOut {
  int iters = 0;
  bool conv = false;
  double est = 0;   // last residual estimate (absolute)
};

// GMRES(m) for P^-1 A x = b with x0 = x (x_zero: x = 0).  Stops when the
// Givens residual estimate is <= tol_abs.  CGS2 orthogonalisation.
GmresOut gmres(lbs_ctx &c, int prec, const double *b, double *x, bool x_zero,
               double tol_abs, int max_iter, hipStream_t s) {
  const int64_t n = c.n;
  const int m = c.opt.restart;
  double *V = c.V.p;
  double *H = c.H.p;
  GmresOut out;
  auto residual_into_v0 = [&]() {
    apply_precond_op(c, prec, 1, x, V, s);
    launch_axpby(n, 1.0, b, -1.0, V, s);
  };
  if (x_zero) {
    launch_fill(n, 0.0, x, s);
    LBS_HIP(hipMemcpyAsync(V, b, n * sizeof(double), hipMemcpyDeviceToDevice,
                           s));
  } else {
    residual_into_v0();
  }
  while (true) {
    launch_dots(n, 1, V, 0, V, 0, c.nrm2.p, c.ws.red.p, s);
    launch_init_g(m, c.nrm2.p, c.gv.p, s);
    LBS_HIP(hipMemcpyAsync(c.resid_host, c.gv.p, sizeof(double),
                           hipMemcpyDeviceToHost, s));
    LBS_HIP(hipStreamSynchronize(s));
    const double beta = *c.resid_host;
    out.est = beta;
    if (beta <= tol_abs || !(beta == beta)) {
      out.conv = beta <= tol_abs;
      return out;
    }
    if (out.iters >= max_iter) return out;
    launch_normalize(n, c.nrm2.p, V, V, nullptr, s);
    int k_used = 0;
    bool done = false;
    for (int k = 0; k < m; ++k) {
      double *vk = V + (int64_t)k * n, *w = V + (int64_t)(k + 1) * n;
      double *hc = H + (int64_t)k * (m + 1);
      apply_precond_op(c, prec, 1, vk, w, s);
      launch_dots(n, k + 1, V, n, w, 0, hc, c.ws.red.p, s);
      launch_maxpy(n, k + 1, V, n, hc, w, nullptr, s);
      launch_dots(n, k + 1, V, n, w, 0, c.h2.p, c.ws.red.p, s);
      launch_maxpy(n, k + 1, V, n, c.h2.p, w, hc, s);
      launch_dots(n, 1, w, 0, w, 0, c.nrm2.p, c.ws.red.p, s);
      launch_normalize(n, c.nrm2.p, w, w, hc + k + 1, s);
      launch_givens(k, m, H, c.cs.p, c.sn.p, c.gv.p, c.resid.p, s);
      LBS_HIP(hipMemcpyAsync(c.resid_host, c.resid.p, sizeof(double),
                             hipMemcpyDeviceToHost, s));
      LBS_HIP(hipStreamSynchronize(s));
      ++out.iters;
      k_used = k + 1;
      out.est = *c.resid_host;
      if (!(out.est == out.est)) fail(LBS_ERR_NOT_FINITE, "GMRES residual is NaN");
      if (out.est <= tol_abs) { out.conv = true; done = true; break; }
      if (out.iters >= max_iter) { done = true; break; }
    }
    launch_backsolve(k_used, m, H, c.gv.p, c.yv.p, s);
    launch_update(n, k_used, V, n, c.yv.p, x, s);
    if (done) return out;
    residual_into_v0();
  }
}

void check_handle(lbs_handle h) {
  if (!h) fail(LBS_ERR_INVALID_ARG, "null handle");
}

}  // namespace

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
}

const char *lbs_last_error(void) { return g_err.c_str(); }

lbs_status lbs_setup(const lbs_island *isl, int32_t M, const int32_t *nodes,
                     const lbs_options *opt, void *stream, lbs_handle *out) {
  return guard([&] {
    if (!out) fail(LBS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!isl || !nodes) fail(LBS_ERR_INVALID_ARG, "islands or nodes is NULL");
    if (M < 1) fail(LBS_ERR_INVALID_ARG, "n_islands < 1");
    hipStream_t s = (hipStream_t)stream;
    auto ctx = std::make_unique<lbs_ctx>();
    lbs_default_options(&ctx->opt);
    if (opt) ctx->opt = *opt;
    lbs_options &o = ctx->opt;
    if (!p64_ok(o.p64)) fail(LBS_ERR_UNSUPPORTED, "p64 must be 20/24/30/36/40/48");
    if (!p32_ok(o.p32)) fail(LBS_ERR_UNSUPPORTED, "p32 must be 12/16/20/24");
    if (o.leaf_max < 4 || o.leaf_max > 1024) fail(LBS_ERR_INVALID_ARG, "leaf_max outside [4, 1024]");
    if (o.restart < 1 || o.restart > 120) fail(LBS_ERR_INVALID_ARG, "restart outside [1, 120]");
    if (o.max_iter < 1 || o.max_outer < 1) fail(LBS_ERR_INVALID_ARG, "max_iter/max_outer < 1");
    if (!(o.inner_tol > 0 && o.inner_tol < 1)) fail(LBS_ERR_INVALID_ARG, "inner_tol outside (0, 1)");
    if (o.matvec != LBS_MATVEC_FMM && o.matvec != LBS_MATVEC_DIRECT) fail(LBS_ERR_INVALID_ARG, "bad matvec mode");

    Geometry &g = ctx->geo;
    g.M = M;
    g.nodes.assign(nodes, nodes + M);
    g.offs.assign(M + 1, 0);
    std::vector<double> bound(M);
    g.cxyz.resize(3 * M);
    for (int k = 0; k < M; ++k) {
      const lbs_island &I = isl[k];
      if (nodes[k] < 8) fail(LBS_ERR_INVALID_ARG, "island " + std::to_string(k) + ": fewer than 8 nodes");
      g.offs[k + 1] = g.offs[k] + nodes[k];
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
    for (int a = 0; a < M; ++a)
      for (int b = a + 1; b < M; ++b) {
        const double d = g.cxyz[3 * a] * g.cxyz[3 * b] + g.cxyz[3 * a + 1] * g.cxyz[3 * b + 1] +
                         g.cxyz[3 * a + 2] * g.cxyz[3 * b + 2];
        const double lim = bound[a] + bound[b];
        if (lim >= M_PI || d >= std::cos(lim))
          fail(LBS_ERR_GEOMETRY, "bounding caps of islands " + std::to_string(a) + " and " +
                                     std::to_string(b) + " overlap");
      }
    const int64_t N = g.N;
    std::vector<int32_t> island(N);
    for (int k = 0; k < M; ++k)
      for (int64_t i = g.offs[k]; i < g.offs[k + 1]; ++i) island[i] = k;
    g.island.upload(island, s);
    g.doffs.upload(g.offs, s);
    g.dcenter.upload(g.cxyz, s);
    DBuf<lbs_island> disl;
    disl.upload(std::vector<lbs_island>(isl, isl + M), s);
    g.xyz.alloc(3 * N);
    g.xi.alloc(2 * N);
    g.dxi.alloc(2 * N);
    g.ddxi.alloc(2 * N);
    launch_geometry(disl.p, M, g.doffs.p, g.island.p, N, g.xyz.p, g.xi.p, g.dxi.p, g.ddxi.p, s);
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
    DBuf<double> dsign;
    dsign.upload(g.sign, s);
    g.qfac.alloc(2 * N);
    g.tau.alloc(N);
    g.gw.alloc(N);
    g.ell.alloc(N);
    launch_node_coeffs(N, g.island.p, dsign.p, g.doffs.p, g.xi.p, g.dxi.p, g.ddxi.p, g.qfac.p,
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
      const double lim = 9.0 * g.rho[k] * g.rho[k];
      for (int m = 0; m < M; ++m) {
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
    // quadtree over the node images
    ctx->xi_x.resize(N);
    ctx->xi_y.resize(N);
    for (int64_t i = 0; i < N; ++i) {
      ctx->xi_x[i] = xi[2 * i];
      ctx->xi_y[i] = xi[2 * i + 1];
    }
    build_tree(ctx->xi_x.data(), ctx->xi_y.data(), N, nullptr, nullptr, 0, true, o.leaf_max,
               ctx->plan.host);
    upload_plan(ctx->plan.host, ctx->xi_x.data(), ctx->xi_y.data(), nullptr, nullptr, nullptr,
                ctx->plan, s);
    g.qfac_t.alloc(2 * N);
    launch_permute_complex(N, ctx->plan.src_perm.p, g.qfac.p, g.qfac_t.p, s);
    build_tables(ctx->tab64, o.p64, s);
    build_tables(ctx->tab32, o.p32, s);
    // Schur complement S = D - F E and its inverse
    {
      DBuf<double> S;
      S.alloc((size_t)M * M);
      g.Sinv.alloc((size_t)M * M);
      launch_build_schur(g, S.p, s);
      invert_dense(M, S.p, g.Sinv.p, s);
    }
    ctx->ws.ensure(ctx->plan, o.p64, o.p32, 1, N, M, kPlog);
    // GMRES storage
    ctx->n = N + M;
    const int m = o.restart;
    ctx->V.alloc((size_t)(m + 1) * ctx->n);
    ctx->H.alloc((size_t)(m + 1) * m);
    ctx->cs.alloc(m);
    ctx->sn.alloc(m);
    ctx->gv.alloc(m + 1);
    ctx->yv.alloc(m);
    ctx->h2.alloc(m + 1);
    ctx->nrm2.alloc(1);
    ctx->resid.alloc(1);
    ctx->bvec.alloc(ctx->n);
    ctx->rvec.alloc(ctx->n);
    ctx->xvec.alloc(ctx->n);
    ctx->dvec.alloc(ctx->n);
    LBS_HIP(hipHostMalloc((void **)&ctx->resid_host, 2 * sizeof(double), hipHostMallocDefault));
    LBS_HIP(hipStreamSynchronize(s));
    *out = ctx.release();
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
    if (nrhs < 1) fail(LBS_ERR_INVALID_ARG, "nrhs < 1");
    if (prec != LBS_FP64 && prec != LBS_MIXED) fail(LBS_ERR_INVALID_ARG, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    lbs_ctx &c = *h;
    c.ws.ensure(c.plan, c.opt.p64, c.opt.p32, nrhs, c.geo.N, c.geo.M, kPlog);
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
    if (nrhs < 1) fail(LBS_ERR_INVALID_ARG, "nrhs < 1");
    if (!(tol > 0 && tol < 1)) fail(LBS_ERR_INVALID_ARG, "tol outside (0, 1)");
    if (prec != LBS_FP64 && prec != LBS_MIXED) fail(LBS_ERR_INVALID_ARG, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    lbs_ctx &c = *h;
    Geometry &g = c.geo;
    const int64_t n = c.n;
    auto t0 = std::chrono::steady_clock::now();
    lbs_solve_info inf{};
    double worst = 0;
    for (int r = 0; r < nrhs; ++r) {
      const double *gr = gdat + (int64_t)r * g.N;
      // finite data check
      launch_dots(g.N, 1, gr, 0, gr, 0, c.nrm2.p, c.ws.red.p, s);
      LBS_HIP(hipMemcpyAsync(c.resid_host, c.nrm2.p, sizeof(double), hipMemcpyDeviceToHost, s));
      LBS_HIP(hipStreamSynchronize(s));
      if (!std::isfinite(*c.resid_host)) fail(LBS_ERR_NOT_FINITE, "data g is not finite");
      precond_rhs(c, gr, c.bvec.p, s);
      const double bnorm = norm2(c, c.bvec.p, n, s);
      double rel = 0;
      bool conv = true;
      if (bnorm == 0) {
        launch_fill(n, 0.0, c.xvec.p, s);
      } else if (prec == LBS_FP64) {
        GmresOut go = gmres(c, LBS_FP64, c.bvec.p, c.xvec.p, true, tol * bnorm,
                            c.opt.max_iter, s);
        inf.iters += go.iters;
        inf.fp64_matvecs += go.iters;
        conv = go.conv;
      } else {
        launch_fill(n, 0.0, c.xvec.p, s);
        LBS_HIP(hipMemcpyAsync(c.rvec.p, c.bvec.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        double rn = bnorm;
        int left = c.opt.max_iter;
        conv = false;
        for (int outer = 0; outer < c.opt.max_outer; ++outer) {
          if (rn <= tol * bnorm) { conv = true; break; }
          if (left <= 0) break;
          GmresOut go = gmres(c, LBS_MIXED, c.rvec.p, c.dvec.p, true,
                              std::max(c.opt.inner_tol * rn, 0.5 * tol * bnorm), left, s);
          inf.iters += go.iters;
          inf.fp32_matvecs += go.iters;
          left -= go.iters;
          launch_axpby(n, 1.0, c.dvec.p, 1.0, c.xvec.p, s);
          apply_precond_op(c, LBS_FP64, 1, c.xvec.p, c.rvec.p, s);
          inf.fp64_matvecs += 1;
          launch_axpby(n, 1.0, c.bvec.p, -1.0, c.rvec.p, s);
          rn = norm2(c, c.rvec.p, n, s);
          inf.outer_steps = outer + 1;
        }
        if (rn <= tol * bnorm) conv = true;
      }
      // final residual of the preconditioned system with the FP64 operator
      if (bnorm > 0) {
        apply_precond_op(c, LBS_FP64, 1, c.xvec.p, c.rvec.p, s);
        inf.fp64_matvecs += 1;
        launch_axpby(n, 1.0, c.bvec.p, -1.0, c.rvec.p, s);
        rel = norm2(c, c.rvec.p, n, s) / bnorm;
      }
      worst = std::max(worst, rel);
      if (!conv) noconv = true;
      LBS_HIP(hipMemcpyAsync(sigma + (int64_t)r * g.N, c.xvec.p, g.N * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
      LBS_HIP(hipMemcpyAsync(A + (int64_t)r * g.M, c.xvec.p + g.N, g.M * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    }
    LBS_HIP(hipStreamSynchronize(s));
    inf.rel_resid = worst;
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
    if (nrhs < 1) fail(LBS_ERR_INVALID_ARG, "nrhs < 1");
    if (T < 0) fail(LBS_ERR_INVALID_ARG, "n_targets < 0");
    if (T == 0) return;
    if (!sigma || !A || !txyz || !u) fail(LBS_ERR_INVALID_ARG, "null pointer argument");
    hipStream_t s = (hipStream_t)stream;
    lbs_ctx &c = *h;
    Geometry &g = c.geo;
    std::vector<double> hx(3 * T);
    LBS_HIP(hipMemcpyAsync(hx.data(), txyz, 3 * T * sizeof(double), hipMemcpyDeviceToHost, s));
    LBS_HIP(hipStreamSynchronize(s));
    std::vector<double> tx, ty;
    std::vector<int64_t> idx;
    for (int64_t t = 0; t < T; ++t) {
      const double x0 = hx[3 * t], x1 = hx[3 * t + 1], x2 = hx[3 * t + 2];
      if (!std::isfinite(x0) || !std::isfinite(x1) || !std::isfinite(x2))
        fail(LBS_ERR_NOT_FINITE, "target " + std::to_string(t) + " is not finite");
      const double d = 1.0 - x2;
      if (d <= 1e-14) continue;  // the pole: Cauchy part is zero
      tx.push_back(x0 / d);
      ty.push_back(x1 / d);
      idx.push_back(t);
    }
    launch_fill(T * nrhs, 0.0, u, s);
    if (!tx.empty()) {
      if (c.opt.matvec == LBS_MATVEC_DIRECT) {
        std::vector<double> txi(2 * T, 0.0);
        std::vector<uint8_t> pole(T, 1);
        for (size_t q = 0; q < idx.size(); ++q) {
          txi[2 * idx[q]] = tx[q];
          txi[2 * idx[q] + 1] = ty[q];
          pole[idx[q]] = 0;
        }
        DBuf<double> dtxi;
        dtxi.upload(txi, s);
        DBuf<uint8_t> dpole;
        dpole.upload(pole, s);
        direct_eval64(g.N, g.xi.p, g.qfac.p, sigma, g.N, T, dtxi.p, dpole.p, nrhs, u, T, 0.5, s);
        LBS_HIP(hipStreamSynchronize(s));
      } else {
        DevPlan pl;
        build_tree(c.xi_x.data(), c.xi_y.data(), g.N, tx.data(), ty.data(), (int64_t)tx.size(), false,
                   c.opt.leaf_max, pl.host);
        upload_plan(pl.host, c.xi_x.data(), c.xi_y.data(), tx.data(), ty.data(), &idx, pl, s);
        DBuf<double> qt;
        qt.alloc(2 * g.N);
        launch_permute_complex(g.N, pl.src_perm.p, g.qfac.p, qt.p, s);
        Workspace ws;
        ws.ensure(pl, c.opt.p64, c.opt.p32, nrhs, g.N, g.M, kPlog);
        fmm_apply64(pl, c.tab64, ws, qt.p, sigma, g.N, nrhs, u, T, 0.5, Assembly{}, s);
        LBS_HIP(hipStreamSynchronize(s));
      }
    }
    c.ws.ensure(c.plan, c.opt.p64, c.opt.p32, nrhs, g.N, g.M, kPlog);
    launch_dots(g.N, nrhs, g.gw.p, 0, sigma, g.N, c.ws.gam.p, c.ws.red.p, s);
    launch_axpby(nrhs, 0.0, c.ws.gam.p, 0.5, c.ws.gam.p, s);
    launch_eval_logsrc(T, txyz, g.M, g.dcenter.p, A, g.M, nrhs, c.ws.gam.p, u, T, s);
    LBS_HIP(hipStreamSynchronize(s));
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

lbs_status lbs_tree_info(lbs_handle h, lbs_tree_stats *st) {
  return guard([&] {
    check_handle(h);
    if (!st) fail(LBS_ERR_INVALID_ARG, "stats is NULL");
    const Tree &T = h->plan.host;
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
    if (st) {
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
  });
}

}  // extern "C"
