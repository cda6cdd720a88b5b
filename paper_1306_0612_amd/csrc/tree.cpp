// Adaptive quadtree construction and interaction lists (see tree.h).
#include "tree.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <thread>
#include <unordered_map>

namespace lbs {
namespace {

inline uint64_t spread_bits(uint64_t v) {  // 29 bits -> even positions
  v &= 0x1FFFFFFFull;
  v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
  v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
  v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  v = (v | (v << 1)) & 0x5555555555555555ull;
  return v;
}

inline uint64_t hkey(int l, int64_t ix, int64_t iy) {
  return ((uint64_t)l << 58) | ((uint64_t)ix << 29) | (uint64_t)iy;
}

// Allocator that leaves new elements uninitialised, so that the sort's
// large arrays are first touched (page-faulted) by the parallel loops that
// write them rather than zero-filled by one thread.
template <typename T>
struct NoInit : std::allocator<T> {
  template <typename U>
  struct rebind { using other = NoInit<U>; };
  NoInit() = default;
  template <typename U>
  NoInit(const NoInit<U> &) {}
  template <typename U>
  void construct(U *p) { ::new ((void *)p) U; }
  template <typename U, typename... A>
  void construct(U *p, A &&...a) { ::new ((void *)p) U(std::forward<A>(a)...); }
};
template <typename T>
using raw_vector = std::vector<T, NoInit<T>>;

struct Keyed {
  raw_vector<uint64_t> key;
  raw_vector<int64_t> perm;
};

// Points sorted by their Morton key (ties keep input order): keys formed in
// parallel, then a stable least-significant-digit radix sort of the top 44
// of the 2 kMaxLevel key bits (four passes of 11 bits, one histogram per
// chunk of points so that each pass scatters in parallel), then each run of
// points whose top bits agree (points closer than 2^-22 of the root box)
// stably sorted by the full key: the same order as a full stable sort.
void morton_sort(const double *x, const double *y, int64_t n, double lox,
                 double loy, double scale, Keyed &out) {
  const double cells = (double)(1ull << kMaxLevel);
  raw_vector<uint64_t> key((size_t)n), tk((size_t)n);
  raw_vector<int64_t> val((size_t)n), tv((size_t)n);
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nc = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(hw, 16), n / 32768));
  std::vector<int64_t> cut(nc + 1);
  for (int c = 0; c <= nc; ++c) cut[c] = n * c / nc;
  parallel_for(nc, [&](int64_t c0, int64_t c1) {
    for (int64_t i = cut[c0]; i < cut[c1]; ++i) {
      double fx = (x[i] - lox) * scale * cells;
      double fy = (y[i] - loy) * scale * cells;
      int64_t qx = (int64_t)std::floor(fx), qy = (int64_t)std::floor(fy);
      qx = std::min<int64_t>(std::max<int64_t>(qx, 0), (1ll << kMaxLevel) - 1);
      qy = std::min<int64_t>(std::max<int64_t>(qy, 0), (1ll << kMaxLevel) - 1);
      key[i] = spread_bits((uint64_t)qx) | (spread_bits((uint64_t)qy) << 1);
      val[i] = i;
    }
  }, 1);
  constexpr int D = 11, NB = 1 << D, LOW = 2 * kMaxLevel - 4 * D;
  static_assert(LOW >= 0, "four digits cover the top key bits");
  std::vector<int64_t> off((size_t)nc * NB);
  for (int sh = LOW; sh < 2 * kMaxLevel; sh += D) {
    std::fill(off.begin(), off.end(), 0);
    parallel_for(nc, [&](int64_t c0, int64_t c1) {
      for (int64_t c = c0; c < c1; ++c) {
        int64_t *h = &off[(size_t)c * NB];
        for (int64_t i = cut[c]; i < cut[c + 1]; ++i) ++h[(key[i] >> sh) & (NB - 1)];
      }
    }, 1);
    // start of (digit, chunk) in digit-major, chunk-minor order; a pass in
    // which every key has the same digit leaves the order as it is
    int64_t run = 0;
    bool trivial = false;
    for (int d = 0; d < NB && !trivial; ++d) {
      int64_t tot = 0;
      for (int c = 0; c < nc; ++c) tot += off[(size_t)c * NB + d];
      trivial = tot == n;
    }
    if (trivial) continue;
    for (int d = 0; d < NB; ++d)
      for (int c = 0; c < nc; ++c) {
        const int64_t h = off[(size_t)c * NB + d];
        off[(size_t)c * NB + d] = run;
        run += h;
      }
    parallel_for(nc, [&](int64_t c0, int64_t c1) {
      for (int64_t c = c0; c < c1; ++c) {
        int64_t *o = &off[(size_t)c * NB];
        for (int64_t i = cut[c]; i < cut[c + 1]; ++i) {
          const int64_t pos = o[(key[i] >> sh) & (NB - 1)]++;
          tk[pos] = key[i];
          tv[pos] = val[i];
        }
      }
    }, 1);
    key.swap(tk);
    val.swap(tv);
  }
  if (LOW > 0) {
    // runs of equal top bits, by the remaining low bits: insertion sort,
    // which moves an entry only past strictly larger keys (stable)
    for (int64_t a = 0; a < n;) {
      int64_t b = a + 1;
      while (b < n && (key[b] >> LOW) == (key[a] >> LOW)) ++b;
      for (int64_t i = a + 1; i < b; ++i) {
        const uint64_t kk = key[i];
        const int64_t vv = val[i];
        int64_t j = i;
        for (; j > a && key[j - 1] > kk; --j) {
          key[j] = key[j - 1];
          val[j] = val[j - 1];
        }
        key[j] = kk;
        val[j] = vv;
      }
      a = b;
    }
  }
  out.key.swap(key);
  out.perm.swap(val);
}

// Sub-range of [a, b) whose keys have quadrant q at level l + 1.
inline void child_range(const raw_vector<uint64_t> &key, int64_t a,
                        int64_t b, int l, int q, int64_t &ca, int64_t &cb) {
  if (a >= b) { ca = cb = a; return; }
  int shift = 2 * (kMaxLevel - l - 1);
  uint64_t prefix = (key[a] >> (shift + 2)) << (shift + 2);
  uint64_t lo = prefix | ((uint64_t)q << shift);
  uint64_t hi = lo + (1ull << shift);
  ca = std::lower_bound(key.begin() + a, key.begin() + b, lo) - key.begin();
  cb = std::lower_bound(key.begin() + a, key.begin() + b, hi) - key.begin();
}

// Do boxes a and b (level la <= lb) touch or overlap?
inline bool touching(const Tree &T, int a, int b) {
  int la = T.level[a], lb = T.level[b];
  if (la > lb) std::swap(a, b), std::swap(la, lb);
  int d = lb - la;
  int64_t ax0 = (int64_t)T.ix[a] << d, ax1 = ((int64_t)T.ix[a] + 1) << d;
  int64_t ay0 = (int64_t)T.iy[a] << d, ay1 = ((int64_t)T.iy[a] + 1) << d;
  int64_t bx0 = T.ix[b], bx1 = (int64_t)T.ix[b] + 1;
  int64_t by0 = T.iy[b], by1 = (int64_t)T.iy[b] + 1;
  return bx0 <= ax1 && bx1 >= ax0 && by0 <= ay1 && by1 >= ay0;
}

}  // namespace

void build_tree(const double *sx, const double *sy, int64_t ns,
                const double *tx, const double *ty, int64_t nt, bool self,
                int leaf_max, Tree &T) {
  if (leaf_max < 1) throw std::invalid_argument("leaf_max < 1");
  T = Tree();
  T.self = self;
  if (self) { tx = sx; ty = sy; nt = ns; }
  double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
  auto upd = [&](const double *x, const double *y, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
      xmin = std::min(xmin, x[i]); xmax = std::max(xmax, x[i]);
      ymin = std::min(ymin, y[i]); ymax = std::max(ymax, y[i]);
    }
  };
  upd(sx, sy, ns);
  if (!self) upd(tx, ty, nt);
  if (ns + (self ? 0 : nt) == 0) { xmin = xmax = ymin = ymax = 0; }
  T.x0 = 0.5 * (xmin + xmax);
  T.y0 = 0.5 * (ymin + ymax);
  double half = 0.5 * std::max(xmax - xmin, ymax - ymin);
  T.R0 = half * (1.0 + 1e-6) + 1e-300 + 1e-12 * std::max(
      std::fabs(T.x0), std::fabs(T.y0));
  if (!(T.R0 > 0)) T.R0 = 1.0;
  const double lox = T.x0 - T.R0, loy = T.y0 - T.R0, scale = 0.5 / T.R0;

  Keyed ks, kt;
  morton_sort(sx, sy, ns, lox, loy, scale, ks);
  if (!self) morton_sort(tx, ty, nt, lox, loy, scale, kt);
  const Keyed &kt_ref = self ? ks : kt;
  T.src_perm.assign(ks.perm.begin(), ks.perm.end());
  T.tgt_perm.assign(kt_ref.perm.begin(), kt_ref.perm.end());

  auto add_box = [&](int l, int64_t ix, int64_t iy, int par, int64_t s0,
                     int64_t s1, int64_t t0, int64_t t1) {
    double r = T.R0 / (double)(1ull << l);
    T.cx.push_back(lox + (2.0 * (double)ix + 1.0) * r);
    T.cy.push_back(loy + (2.0 * (double)iy + 1.0) * r);
    T.rad.push_back(r);
    T.level.push_back(l);
    T.parent.push_back(par);
    T.child0.push_back(-1);
    T.nchild.push_back(0);
    T.ix.push_back((int32_t)ix);
    T.iy.push_back((int32_t)iy);
    T.s0.push_back(s0); T.s1.push_back(s1);
    T.t0.push_back(t0); T.t1.push_back(t1);
    T.leaf.push_back(1);
  };
  add_box(0, 0, 0, -1, 0, ns, 0, nt);
  T.level_ptr.push_back(0);
  int lbeg = 0;
  for (int l = 0;; ++l) {
    int lend = T.nbox();
    T.level_ptr.push_back(lend);
    if (l >= kMaxLevel) break;
    for (int b = lbeg; b < lend; ++b) {
      int64_t cnt = (T.s1[b] - T.s0[b]) + (self ? 0 : (T.t1[b] - T.t0[b]));
      if (cnt <= leaf_max) continue;
      T.leaf[b] = 0;
      T.child0[b] = T.nbox();
      for (int q = 0; q < 4; ++q) {
        int64_t a0, a1, c0, c1;
        child_range(ks.key, T.s0[b], T.s1[b], l, q, a0, a1);
        if (self) { c0 = a0; c1 = a1; }
        else child_range(kt_ref.key, T.t0[b], T.t1[b], l, q, c0, c1);
        if (a1 - a0 + c1 - c0 == 0) continue;
        add_box(l + 1, 2 * (int64_t)T.ix[b] + (q & 1),
                2 * (int64_t)T.iy[b] + (q >> 1), b, a0, a1, c0, c1);
        T.nchild[b]++;
      }
    }
    lbeg = lend;
    if (T.nbox() == lend) break;
  }
  // level_ptr has one entry per level start plus the end
  while (T.level_ptr.size() >= 2 &&
         T.level_ptr[T.level_ptr.size() - 1] ==
             T.level_ptr[T.level_ptr.size() - 2])
    T.level_ptr.pop_back();
  T.nlevels = (int)T.level_ptr.size() - 1;

  const int nb = T.nbox();
  std::unordered_map<uint64_t, int32_t> where;
  where.reserve((size_t)nb * 2);
  for (int b = 0; b < nb; ++b) where[hkey(T.level[b], T.ix[b], T.iy[b])] = b;
  auto find = [&](int l, int64_t ix, int64_t iy) -> int {
    if (ix < 0 || iy < 0 || ix >= (1ll << l) || iy >= (1ll << l)) return -1;
    auto it = where.find(hkey(l, ix, iy));
    return it == where.end() ? -1 : it->second;
  };
  auto has_src = [&](int b) { return T.s1[b] > T.s0[b]; };
  auto has_tgt = [&](int b) { return T.t1[b] > T.t0[b]; };

  // V lists
  T.v_ptr.assign(nb + 1, 0);
  std::vector<std::vector<std::pair<int32_t, uint8_t>>> vl(nb);
  parallel_for(nb, [&](int64_t b0, int64_t b1) {
  for (int b = (int)b0; b < (int)b1; ++b) {
    int l = T.level[b];
    if (l < 2 || !has_tgt(b)) continue;
    int p = T.parent[b];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        int c = find(l - 1, (int64_t)T.ix[p] + dx, (int64_t)T.iy[p] + dy);
        if (c < 0) continue;
        for (int k = 0; k < T.nchild[c]; ++k) {
          int s = T.child0[c] + k;
          int ddx = T.ix[s] - T.ix[b], ddy = T.iy[s] - T.iy[b];
          if (std::abs(ddx) <= 1 && std::abs(ddy) <= 1) continue;
          if (!has_src(s)) continue;
          vl[b].push_back({s, (uint8_t)((ddx + 3) * 7 + (ddy + 3))});
        }
      }
  }
  }, 256);
  // U (descent part) and W lists, for leaves
  std::vector<std::vector<int32_t>> ud(nb), wl(nb);
  parallel_for(nb, [&](int64_t b0, int64_t b1) {
  std::vector<int> stack;
  for (int b = (int)b0; b < (int)b1; ++b) {
    if (!T.leaf[b]) continue;
    int l = T.level[b];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        int c = find(l, (int64_t)T.ix[b] + dx, (int64_t)T.iy[b] + dy);
        if (c < 0) continue;
        if (c == b || T.leaf[c]) { ud[b].push_back(c); continue; }
        stack.clear();
        for (int k = 0; k < T.nchild[c]; ++k) stack.push_back(T.child0[c] + k);
        while (!stack.empty()) {
          int d = stack.back();
          stack.pop_back();
          if (touching(T, b, d)) {
            if (T.leaf[d]) ud[b].push_back(d);
            else
              for (int k = 0; k < T.nchild[d]; ++k)
                stack.push_back(T.child0[d] + k);
          } else {
            wl[b].push_back(d);
          }
        }
      }
  }
  }, 256);
  // U = descent part + coarser adjacent leaves; X = transpose of W
  // (each list sized first, so that the appends below allocate once)
  std::vector<std::vector<int32_t>> ul(nb), xl(nb);
  {
    std::vector<int32_t> nu(nb, 0), nx(nb, 0);
    for (int b = 0; b < nb; ++b) {
      nu[b] += (int32_t)ud[b].size();
      for (int c : ud[b])
        if (T.level[c] > T.level[b]) ++nu[c];
      for (int d : wl[b]) ++nx[d];
    }
    parallel_for(nb, [&](int64_t b0, int64_t b1) {
      for (int64_t b = b0; b < b1; ++b) {
        ul[b].reserve(nu[b]);
        xl[b].reserve(nx[b]);
      }
    }, 1024);
  }
  for (int b = 0; b < nb; ++b)
    for (int c : ud[b]) {
      ul[b].push_back(c);
      if (T.level[c] > T.level[b]) ul[c].push_back(b);
    }
  for (int b = 0; b < nb; ++b)
    for (int d : wl[b]) xl[d].push_back(b);

  auto flatten = [&](std::vector<std::vector<int32_t>> &L,
                     std::vector<int32_t> &ptr, std::vector<int32_t> &idx,
                     auto keep_target, auto keep_source) {
    // sort and count per box, prefix sum, fill (all but the sum parallel)
    ptr.assign(nb + 1, 0);
    parallel_for(nb, [&](int64_t b0, int64_t b1) {
      for (int64_t b = b0; b < b1; ++b) {
        if (!keep_target((int)b)) continue;
        std::sort(L[b].begin(), L[b].end());
        int32_t n = 0;
        for (int s : L[b]) n += keep_source(s) ? 1 : 0;
        ptr[b + 1] = n;
      }
    }, 1024);
    for (int b = 0; b < nb; ++b) ptr[b + 1] += ptr[b];
    idx.resize((size_t)ptr[nb]);
    parallel_for(nb, [&](int64_t b0, int64_t b1) {
      for (int64_t b = b0; b < b1; ++b) {
        if (!keep_target((int)b)) continue;
        int32_t k = ptr[b];
        for (int s : L[b])
          if (keep_source(s)) idx[k++] = s;
      }
    }, 1024);
  };
  flatten(ul, T.u_ptr, T.u_src, has_tgt, has_src);
  flatten(wl, T.w_ptr, T.w_src, has_tgt, has_src);
  flatten(xl, T.x_ptr, T.x_src, has_tgt, has_src);
  parallel_for(nb, [&](int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; ++b) std::sort(vl[b].begin(), vl[b].end());
  }, 1024);
  for (int b = 0; b < nb; ++b) T.v_ptr[b + 1] = T.v_ptr[b] + (int32_t)vl[b].size();
  T.v_src.resize((size_t)T.v_ptr[nb]);
  T.v_code.resize((size_t)T.v_ptr[nb]);
  parallel_for(nb, [&](int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; ++b) {
      int32_t k = T.v_ptr[b];
      for (auto &e : vl[b]) {
        T.v_src[k] = e.first;
        T.v_code[k++] = e.second;
      }
    }
  }, 1024);
  tree_statistics(T);
}

void tree_statistics(Tree &T) {
  const int nb = T.nbox();
  T.p2p_pairs = T.m2p_evals = T.p2l_evals = 0;
  for (int b = 0; b < nb; ++b) {
    const int64_t ntb = T.t1[b] - T.t0[b];
    for (int k = T.u_ptr[b]; k < T.u_ptr[b + 1]; ++k) {
      int s = T.u_src[k];
      T.p2p_pairs += ntb * (T.s1[s] - T.s0[s]);
    }
    T.m2p_evals += ntb * (T.w_ptr[b + 1] - T.w_ptr[b]);
    for (int k = T.x_ptr[b]; k < T.x_ptr[b + 1]; ++k) {
      int s = T.x_src[k];
      T.p2l_evals += T.s1[s] - T.s0[s];
    }
  }
}

int64_t check_coverage(const Tree &T) {
  const int nb = T.nbox();
  std::vector<std::vector<int>> anc(nb);
  for (int b = 0; b < nb; ++b)
    for (int a = b; a >= 0; a = T.parent[a]) anc[b].push_back(a);
  auto in = [](const std::vector<int> &v, int x) {
    return std::find(v.begin(), v.end(), x) != v.end();
  };
  auto in_range = [](const std::vector<int32_t> &idx, int32_t p0, int32_t p1,
                     int x) {
    for (int k = p0; k < p1; ++k)
      if (idx[k] == x) return true;
    return false;
  };
  int64_t bad = 0;
  for (int bi = 0; bi < nb; ++bi) {
    if (!T.leaf[bi] || T.t1[bi] == T.t0[bi]) continue;
    for (int bj = 0; bj < nb; ++bj) {
      if (!T.leaf[bj] || T.s1[bj] == T.s0[bj]) continue;
      int cnt = 0;
      if (in_range(T.u_src, T.u_ptr[bi], T.u_ptr[bi + 1], bj)) ++cnt;
      for (int a : anc[bi])
        for (int k = T.v_ptr[a]; k < T.v_ptr[a + 1]; ++k)
          if (in(anc[bj], T.v_src[k])) ++cnt;
      for (int k = T.w_ptr[bi]; k < T.w_ptr[bi + 1]; ++k)
        if (in(anc[bj], T.w_src[k])) ++cnt;
      for (int a : anc[bi])
        if (in_range(T.x_src, T.x_ptr[a], T.x_ptr[a + 1], bj)) ++cnt;
      if (cnt != 1) {
        int64_t nti = T.t1[bi] - T.t0[bi], nsj = T.s1[bj] - T.s0[bj];
        int64_t pairs = nti * nsj;
        if (T.self && bi == bj) pairs -= nti;
        bad += pairs;
      }
    }
  }
  return bad;
}

}  // namespace lbs

namespace lbs {

void append_tree(Tree &F, const Tree &t, int64_t src_base, int64_t tgt_base,
                 int64_t src_index_base, int64_t tgt_index_base) {
  const int off = F.nbox();
  auto cat = [](auto &dst, const auto &src) {
    dst.insert(dst.end(), src.begin(), src.end());
  };
  cat(F.cx, t.cx);
  cat(F.cy, t.cy);
  cat(F.rad, t.rad);
  cat(F.level, t.level);
  cat(F.ix, t.ix);
  cat(F.iy, t.iy);
  cat(F.leaf, t.leaf);
  cat(F.nchild, t.nchild);
  for (int b = 0; b < t.nbox(); ++b) {
    F.parent.push_back(t.parent[b] < 0 ? -1 : t.parent[b] + off);
    F.child0.push_back(t.child0[b] < 0 ? -1 : t.child0[b] + off);
    F.s0.push_back(t.s0[b] + src_base);
    F.s1.push_back(t.s1[b] + src_base);
    F.t0.push_back(t.t0[b] + tgt_base);
    F.t1.push_back(t.t1[b] + tgt_base);
  }
  auto cat_csr = [&](std::vector<int32_t> &fp, std::vector<int32_t> &fi,
                     const std::vector<int32_t> &tp,
                     const std::vector<int32_t> &ti) {
    if (fp.empty()) fp.push_back(0);
    const int32_t base = fp.back();
    for (int b = 0; b < t.nbox(); ++b) fp.push_back(base + tp[b + 1]);
    for (int32_t v : ti) fi.push_back(v + off);
  };
  cat_csr(F.v_ptr, F.v_src, t.v_ptr, t.v_src);
  cat(F.v_code, t.v_code);
  cat_csr(F.x_ptr, F.x_src, t.x_ptr, t.x_src);
  cat_csr(F.u_ptr, F.u_src, t.u_ptr, t.u_src);
  cat_csr(F.w_ptr, F.w_src, t.w_ptr, t.w_src);
  for (int64_t v : t.src_perm) F.src_perm.push_back(v + src_index_base);
  for (int64_t v : t.tgt_perm) F.tgt_perm.push_back(v + tgt_index_base);
  F.nlevels = std::max(F.nlevels, t.nlevels);
  F.self = t.self;
  F.p2p_pairs += t.p2p_pairs;
  F.m2p_evals += t.m2p_evals;
  F.p2l_evals += t.p2l_evals;
}

}  // namespace lbs
