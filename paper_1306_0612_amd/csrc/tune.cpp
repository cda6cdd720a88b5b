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
// within tol_fp64; then, on that leaf size and FP32 order, the fastest width
// of the persistent FP32 M2L launch.  lbs_autotune_cached keeps the results
// in a text file keyed by a hash of the problem, the device and the build.
// Written on the public C-ABI only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
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
  // the launch shape of the FP32 M2L on the chosen leaf size and order
  {
    const int widths[] = {512, 1024, 2048};
    double best_ms = 0;
    int best_w = 0;
    for (int wdt : widths) {
      lbs_options c = o;
      c.leaf_max = bm->leaf_max;
      c.p32 = bm->p32;
      c.m2l_groups = wdt;
      Handle h;
      lbs_status st = lbs_setup(isl, M, nodes, &c, stream, &h.h);
      if (st != LBS_OK) return st;
      lbs_tune_entry e{};
      e.leaf_max = c.leaf_max;
      e.p32 = c.p32;
      e.m2l_groups = wdt;
      if ((st = timed(h.h, LBS_MIXED, e.ms)) != LBS_OK) return st;
      e.err = rel_err(out, ref);
      all.push_back(e);
      if (e.err <= tol_mixed && (!best_w || e.ms < best_ms)) {
        best_ms = e.ms;
        best_w = wdt;
      }
    }
    best->m2l_groups = best_w;  // 0 (the default) if none met tol_mixed
  }
  if (n_entries) *n_entries = (int32_t)all.size();
  if (entries)
    for (int32_t i = 0; i < std::min<int32_t>(max_entries, (int32_t)all.size()); ++i)
      entries[i] = all[i];
  return LBS_OK;
}

namespace {

// 64-bit FNV-1a over a byte range, chained
uint64_t fnv1a(const void *p, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

// The cache key: the problem, the device and the compile time of the library.
uint64_t tune_key(const lbs_island *isl, int32_t M, const int32_t *nodes, const lbs_options &o,
                  double tol_mixed, double tol_fp64) {
  uint64_t h = fnv1a(isl, sizeof(lbs_island) * (size_t)M);
  h = fnv1a(nodes, sizeof(int32_t) * (size_t)M, h);
  lbs_options k = o;
  k.graphs = 0;  // not part of the schedule
  h = fnv1a(&k, sizeof(k), h);
  h = fnv1a(&tol_mixed, sizeof(double), h);
  h = fnv1a(&tol_fp64, sizeof(double), h);
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    h = fnv1a(prop.gcnArchName, std::strlen(prop.gcnArchName), h);
    h = fnv1a(&prop.multiProcessorCount, sizeof(int), h);
  }
  static const char build[] = __DATE__ " " __TIME__;
  return fnv1a(build, sizeof(build) - 1, h);
}

}  // namespace

extern "C" lbs_status lbs_autotune_cached(const lbs_island *isl, int32_t M, const int32_t *nodes,
                                          const lbs_options *base, double tol_mixed,
                                          double tol_fp64, void *stream, const char *cache_path,
                                          lbs_options *best, lbs_tune_entry *entries,
                                          int32_t max_entries, int32_t *n_entries,
                                          int32_t *hit) {
  if (hit) *hit = 0;
  if (!cache_path || !isl || !nodes || !best || M < 1) {
    lbs::set_last_error("lbs_autotune_cached: bad argument");
    return LBS_ERR_INVALID_ARG;
  }
  lbs_options o;
  lbs_default_options(&o);
  if (base) o = *base;
  char key[17];
  std::snprintf(key, sizeof(key), "%016llx",
                (unsigned long long)tune_key(isl, M, nodes, o, tol_mixed, tol_fp64));
  // line: "lbs-tune <key> <leaf> <p32> <p64> <groups> <n> then n x (leaf p32
  // p64 groups ms err)"; the last line with the key wins
  {
    std::ifstream in(cache_path);
    std::string line, found;
    while (std::getline(in, line))
      if (line.compare(0, 9, "lbs-tune ") == 0 && line.compare(9, 16, key) == 0) found = line;
    if (!found.empty()) {
      std::istringstream ls(found.substr(26));
      int lm = 0, p32 = 0, p64 = 0, grp = 0, n = 0;
      std::vector<lbs_tune_entry> all;
      bool ok = (bool)(ls >> lm >> p32 >> p64 >> grp >> n) && n >= 0;
      for (int i = 0; ok && i < n; ++i) {
        lbs_tune_entry e{};
        ok = (bool)(ls >> e.leaf_max >> e.p32 >> e.p64 >> e.m2l_groups >> e.ms >> e.err);
        all.push_back(e);
      }
      if (ok) {
        *best = o;
        best->graphs = base ? base->graphs : 1;
        best->leaf_max = lm;
        best->p32 = p32;
        best->p64 = p64;
        best->m2l_groups = grp;
        if (n_entries) *n_entries = n;
        if (entries)
          for (int32_t i = 0; i < std::min<int32_t>(max_entries, n); ++i) entries[i] = all[i];
        if (hit) *hit = 1;
        return LBS_OK;
      }
    }
  }
  std::vector<lbs_tune_entry> all(256);
  int32_t cnt = 0;
  const lbs_status st = lbs_autotune(isl, M, nodes, base, tol_mixed, tol_fp64, stream, best,
                                     all.data(), (int32_t)all.size(), &cnt);
  if (st != LBS_OK) return st;
  cnt = std::min<int32_t>(cnt, (int32_t)all.size());
  std::ostringstream os;
  os.precision(17);
  os << "lbs-tune " << key << ' ' << best->leaf_max << ' ' << best->p32 << ' ' << best->p64 << ' '
     << best->m2l_groups << ' ' << cnt;
  for (int32_t i = 0; i < cnt; ++i)
    os << ' ' << all[i].leaf_max << ' ' << all[i].p32 << ' ' << all[i].p64 << ' '
       << all[i].m2l_groups << ' ' << all[i].ms << ' ' << all[i].err;
  os << '\n';
  const std::string text = os.str();
  if (FILE *f = std::fopen(cache_path, "a")) {  // one write of the whole line
    (void)std::fwrite(text.data(), 1, text.size(), f);
    (void)std::fclose(f);
  }
  if (n_entries) *n_entries = cnt;
  if (entries)
    for (int32_t i = 0; i < std::min<int32_t>(max_entries, cnt); ++i) entries[i] = all[i];
  return LBS_OK;
}
