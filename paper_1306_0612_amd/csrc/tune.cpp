// Autotuner of the FMM schedule: quadtree leaf size and expansion orders.
//
// The cost balance of the adaptive FMM (Section 5) between the direct
// near field (grows with the leaf size) and the translations (grow with the
// box count and the expansion order) depends on the geometry.  For each
// candidate leaf size the tuner builds a handle, then for each candidate
// order times the operator (I + K) with HIP events and measures its
// relative error against a reference application (FP64 far field of
// order 48 on the smallest leaf size).  It returns the fastest mixed
// setting within tol_mixed and, for that leaf size, the fastest FP64 order
// within tol_fp64.  Written on the public C-ABI only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbs.h"

namespace lbs {
void set_last_error(const std::string &msg);  // api.cpp
}

namespace {

struct Dev {
  double *p = nullptr;
  explicit Dev(size_t n) {
    if (hipMalloc((void **)&p, n * sizeof(double)) != hipSuccess) p = nullptr;
  }
  ~Dev() {
    if (p) (void)hipFree(p);
  }
};

struct Handle {
  lbs_handle h = nullptr;
  ~Handle() {
    if (h) lbs_destroy(h);
  }
};

// max |a - b| / max |b| over n host values
double rel_err(const std::vector<double> &a, const std::vector<double> &b) {
  double d = 0, m = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    d = std::max(d, std::fabs(a[i] - b[i]));
    m = std::max(m, std::fabs(b[i]));
  }
  return m > 0 ? d / m : d;
}

}  // namespace

extern "C" lbs_status lbs_autotune(const lbs_island *isl, int32_t M, const int32_t *nodes,
                                   const lbs_options *base, double tol_mixed,
                                   double tol_fp64, void *stream, lbs_options *best,
                                   lbs_tune_entry *entries, int32_t max_entries,
                                   int32_t *n_entries) {
  if (!isl || !nodes || !best || M < 1 || !(tol_mixed > 0) || !(tol_fp64 > 0)) {
    lbs::set_last_error("lbs_autotune: bad argument");
    return LBS_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  lbs_options o;
  lbs_default_options(&o);
  if (base) o = *base;
  o.graphs = 0;
  int64_t N = 0;
  for (int k = 0; k < M; ++k) N += nodes[k];
  if (N < 1) return LBS_ERR_INVALID_ARG;
  const int leaves[] = {24, 32, 48, 64, 96, 128};
  const int p32s[] = {12, 16, 20, 24};
  const int p64s[] = {20, 24, 30, 36};
  Dev x(N), y(N);
  if (!x.p || !y.p) return LBS_ERR_OUT_OF_MEMORY;
  {
    // x: uniform in [-1, 1) from a 64-bit LCG (Knuth's MMIX constants)
    std::vector<double> hx(N);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    for (int64_t i = 0; i < N; ++i) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      hx[i] = (double)(st >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
    if (hipMemcpyAsync(x.p, hx.data(), N * sizeof(double), hipMemcpyHostToDevice, s) !=
        hipSuccess)
      return LBS_ERR_HIP;
  }
  std::vector<double> ref(N), out(N);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LBS_ERR_HIP;
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  auto fetch = [&](std::vector<double> &v) -> lbs_status {
    if (hipMemcpyAsync(v.data(), y.p, N * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return LBS_ERR_HIP;
    return LBS_OK;
  };
  // time `reps` applications (after one warm-up); ms per application
  auto timed = [&](lbs_handle h, int prec, double &ms) -> lbs_status {
    lbs_status st = lbs_matvec(h, LBS_OP_IPLUSK, prec, 1, x.p, y.p, stream);
    if (st != LBS_OK) return st;
    const int reps = 5;
    if (hipEventRecord(e0, s) != hipSuccess) return LBS_ERR_HIP;
    for (int r = 0; r < reps; ++r) {
      st = lbs_matvec(h, LBS_OP_IPLUSK, prec, 1, x.p, y.p, stream);
      if (st != LBS_OK) return st;
    }
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return LBS_ERR_HIP;
    float f = 0;
    if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return LBS_ERR_HIP;
    ms = f / reps;
    return fetch(out);
  };
  // reference
  {
    lbs_options r = o;
    r.leaf_max = leaves[0];
    r.p64 = 48;
    Handle h;
    lbs_status st = lbs_setup(isl, M, nodes, &r, stream, &h.h);
    if (st != LBS_OK) return st;
    st = lbs_matvec(h.h, LBS_OP_IPLUSK, LBS_FP64, 1, x.p, y.p, stream);
    if (st != LBS_OK) return st;
    if ((st = fetch(ref)) != LBS_OK) return st;
  }
  std::vector<lbs_tune_entry> all;
  for (int lm : leaves) {
    lbs_options c = o;
    c.leaf_max = lm;
    Handle h;
    lbs_status st = lbs_setup(isl, M, nodes, &c, stream, &h.h);
    if (st != LBS_OK) return st;
    for (int p : p32s) {
      if ((st = lbs_set_orders(h.h, c.p64, p, stream)) != LBS_OK) return st;
      lbs_tune_entry e{};
      e.leaf_max = lm;
      e.p32 = p;
      e.p64 = 0;
      if ((st = timed(h.h, LBS_MIXED, e.ms)) != LBS_OK) return st;
      e.err = rel_err(out, ref);
      all.push_back(e);
    }
    for (int p : p64s) {
      if ((st = lbs_set_orders(h.h, p, c.p32, stream)) != LBS_OK) return st;
      lbs_tune_entry e{};
      e.leaf_max = lm;
      e.p32 = 0;
      e.p64 = p;
      if ((st = timed(h.h, LBS_FP64, e.ms)) != LBS_OK) return st;
      e.err = rel_err(out, ref);
      all.push_back(e);
    }
  }
  // fastest mixed setting within tol_mixed, then the fastest FP64 order
  // within tol_fp64 on that leaf size
  const lbs_tune_entry *bm = nullptr, *bf = nullptr;
  for (const auto &e : all)
    if (e.p32 && e.err <= tol_mixed && (!bm || e.ms < bm->ms)) bm = &e;
  if (!bm) {
    lbs::set_last_error("lbs_autotune: no mixed setting reaches tol_mixed");
    return LBS_ERR_UNSUPPORTED;
  }
  for (const auto &e : all)
    if (e.p64 && e.leaf_max == bm->leaf_max && e.err <= tol_fp64 && (!bf || e.ms < bf->ms))
      bf = &e;
  if (!bf) {
    lbs::set_last_error("lbs_autotune: no FP64 order reaches tol_fp64");
    return LBS_ERR_UNSUPPORTED;
  }
  *best = o;
  if (base) best->graphs = base->graphs;
  else best->graphs = 1;
  best->leaf_max = bm->leaf_max;
  best->p32 = bm->p32;
  best->p64 = bf->p64;
  if (n_entries) *n_entries = (int32_t)all.size();
  if (entries)
    for (int32_t i = 0; i < std::min<int32_t>(max_entries, (int32_t)all.size()); ++i)
      entries[i] = all[i];
  return LBS_OK;
}
