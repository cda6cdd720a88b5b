// Adaptive quadtree and interaction lists built on the GPU (Section 5: the
// FMM's quadtree is refined until no leaf holds more than a preset number
// of points; Section 6, Example 3 on its depth).  The output is the Tree of
// tree.h, identical to the host builder's (build_tree): the same root box,
// Morton keys, stable order, boxes in level-major order and sorted lists.
//
//  1. root box from a min/max reduction of the points;
//  2. 58-bit Morton keys (29 bits per axis) and a stable LSD radix sort of
//     (key, index) pairs, 8-bit digits: per-tile digit histograms, one
//     exclusive scan, and a stable scatter that ranks equal digits inside a
//     wave by ballots over the digit's bits;
//  3. boxes level by level: a box holding more than leaf_max points gets its
//     non-empty quadrants as children (ranges by binary search on the sorted
//     keys), appended in (parent, quadrant) order after an exclusive scan;
//  4. per leaf, its adjacent leaves (colleagues, and descendants of
//     colleagues that touch it) and the W boxes (descendants of colleagues
//     that do not touch it while their parent does) by a depth-first
//     descent in each thread; per box with targets at level >= 2, the V
//     boxes (children of the parent's colleagues that are not adjacent);
//  5. the U, W, X (transpose of W) and V pairs as 64-bit keys (box << 32 |
//     other box), sorted by the same radix sort, so each box's list comes
//     out in ascending order as the host builder's.
// Boxes at one level are in Morton order of (ix, iy), so a box is found by
// binary search of its code within its level.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include <chrono>
#include <cstdio>
#include <cstdlib>

#include "lbs_internal.h"

namespace lbs {
namespace {

// Wall time of the builder's phases, printed to stderr when
// LBS_HOST_TIMING is set (as the set-up's): mark(name) reports the time
// since the previous mark.
struct PhaseClock {
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char *name) {
    static const bool on = std::getenv("LBS_HOST_TIMING") != nullptr;
    const auto now = std::chrono::steady_clock::now();
    if (on)
      std::fprintf(stderr, "[lbs host] gpu tree: %-18s %9.3f ms\n", name,
                   std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

// ------------------------------------------------------------ radix sort
constexpr int kRsTile = 4096;  // keys per work-group (256 threads x 16)

__global__ void __launch_bounds__(256)
    k_rs_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
              int ntiles, uint32_t *__restrict__ hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int j = 0; j < kRsTile / 256; ++j) {
    const int64_t i = base + j * 256 + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// exclusive scan of h[0 .. n) in place, one work-group of 1024 threads
__global__ void __launch_bounds__(1024)
    k_scan_u32(uint32_t *__restrict__ h, int64_t n) {
  __shared__ uint32_t part[1024];
  const int64_t per = (n + 1023) / 1024;
  const int64_t a = threadIdx.x * per, b = std::min<int64_t>(n, a + per);
  uint32_t s = 0;
  for (int64_t i = a; i < b; ++i) s += h[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int64_t i = a; i < b; ++i) {
    const uint32_t v = h[i];
    h[i] = run;
    run += v;
  }
}

// Tiled exclusive scan: tiles of 4096 entries, four consecutive entries per
// thread (coalesced), thread totals scanned across the wave by shuffles and
// across the 16 waves through LDS; with offs, tile t adds offs[t] (the
// exclusive scan of the tile sums, k_tile_sums).
constexpr int kScanTile = 4096;
__device__ __forceinline__ uint32_t block_exclusive_1024(uint32_t v, uint32_t &total) {
  __shared__ uint32_t wsum[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < 16; ++w) {
    const uint32_t x = wsum[w];
    before += w < wave ? x : 0u;
    all += x;
  }
  __syncthreads();  // wsum is rewritten by the next call
  total = all;
  return before + inc - v;
}

__global__ void __launch_bounds__(1024)
    k_tile_sums(const uint32_t *__restrict__ a, int64_t n, uint32_t *__restrict__ sums) {
  const int64_t i0 = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  uint32_t v = 0;
  for (int k = 0; k < 4; ++k)
    if (i0 + k < n) v += a[i0 + k];
  uint32_t total;
  (void)block_exclusive_1024(v, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024)
    k_scan_tiles(uint32_t *__restrict__ a, int64_t n, const uint32_t *__restrict__ offs) {
  const int64_t i0 = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  uint32_t x[4], v = 0;
  for (int k = 0; k < 4; ++k) {
    x[k] = i0 + k < n ? a[i0 + k] : 0u;
    v += x[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_1024(v, total) + (offs ? offs[blockIdx.x] : 0u);
  for (int k = 0; k < 4; ++k)
    if (i0 + k < n) {
      a[i0 + k] = run;
      run += x[k];
    }
}

}  // namespace

// In-place exclusive scan of a[0 .. n) with tile sums in sums (at least
// ceil(n / 4096) entries; not needed for n <= 4096).
void scan_into(uint32_t *a, int64_t n, uint32_t *sums, hipStream_t s) {
  if (n <= 0) return;
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  if (nt == 1) {
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, a, n, nullptr);
  } else if (nt <= kScanTile) {
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nt), dim3(1024), 0, s, a, n, sums);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, sums, nt, nullptr);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(1024), 0, s, a, n, sums);
  } else {
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, s, a, n);
  }
  LBS_HIP(hipGetLastError());
}

namespace {

// Stable scatter of one tile: 16 rounds of 256 consecutive keys; a key's
// place = the digit's global offset for this tile + the digit's count in
// earlier rounds + in earlier waves of this round + earlier lanes of its
// wave (lanes with the same digit found by ballots over the 8 digit bits).
__global__ void __launch_bounds__(256)
    k_rs_scatter(const uint64_t *__restrict__ keys,
                 const int32_t *__restrict__ vals, int64_t n, int shift,
                 int ntiles, const uint32_t *__restrict__ off,
                 uint64_t *__restrict__ keys2, int32_t *__restrict__ vals2) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  run[tid] = 0;
  for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int j = 0; j < kRsTile / 256; ++j) {
    const int64_t i = base + j * 256 + tid;
    const bool valid = i < n;
    uint64_t key = 0;
    int32_t val = 0;
    int d = 0;
    if (valid) {
      key = keys[i];
      val = vals[i];
      d = (int)((key >> shift) & 255);
    }
    uint64_t match = __ballot(valid);
    for (int bit = 0; bit < 8; ++bit) {
      const bool b = (d >> bit) & 1;
      const uint64_t m = __ballot(b);
      match &= b ? m : ~m;
    }
    const int rank = __popcll(match & below);
    if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(match);
    __syncthreads();
    if (valid) {
      uint32_t pos = off[(int64_t)d * ntiles + blockIdx.x] + run[d] + (uint32_t)rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      keys2[pos] = key;
      vals2[pos] = val;
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
    __syncthreads();
  }
}

// Scratch of the radix sorts of one tree build (SortBufs), grown as needed
// and reused by every sort (fewer allocations, and no device-wide wait in a
// free between the sorts).
using SortScratch = SortBufs;
void ensure_sort(SortScratch &sc, int64_t n, int ntiles) {
  if ((int64_t)sc.k2.n < n) sc.k2.alloc((size_t)n);
  if ((int64_t)sc.v2.n < n) sc.v2.alloc((size_t)n);
  if ((int64_t)sc.hist.n < (int64_t)256 * ntiles) sc.hist.alloc((size_t)256 * ntiles);
  const int64_t nt = ((int64_t)256 * ntiles + kScanTile - 1) / kScanTile;
  if ((int64_t)sc.sums.n < nt) sc.sums.alloc((size_t)nt);
}

// Stable sort of (keys, vals) by the low `bits` bits of the keys; the
// result is back in keys / vals.
void radix_sort(uint64_t *keys, int32_t *vals, int64_t n, int bits, SortScratch &sc,
                hipStream_t s) {
  if (n <= 1) return;
  const int ntiles = (int)((n + kRsTile - 1) / kRsTile);
  ensure_sort(sc, n, ntiles);
  DBuf<uint64_t> &k2 = sc.k2;
  DBuf<int32_t> &v2 = sc.v2;
  DBuf<uint32_t> &hist = sc.hist;
  uint64_t *ka = keys, *kb = k2.p;
  int32_t *va = vals, *vb = v2.p;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8, ++passes) {
    hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(256), 0, s, ka, n, shift, ntiles, hist.p);
    scan_into(hist.p, (int64_t)256 * ntiles, sc.sums.p, s);
    hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(256), 0, s, ka, va, n, shift, ntiles,
                       hist.p, kb, vb);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (passes & 1) {
    LBS_HIP(hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    LBS_HIP(hipMemcpyAsync(vals, va, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
  LBS_HIP(hipGetLastError());
}

// ---------------------------------------------------------- points, keys
__global__ void __launch_bounds__(256)
    k_minmax(const double *__restrict__ x, const double *__restrict__ y, int64_t n,
             int64_t stride, double *__restrict__ part) {
  __shared__ double r[4][256];
  double a = INFINITY, b = -INFINITY, c = INFINITY, d = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double xv = x[i * stride], yv = y[i * stride];
    a = fmin(a, xv);
    b = fmax(b, xv);
    c = fmin(c, yv);
    d = fmax(d, yv);
  }
  r[0][threadIdx.x] = a;
  r[1][threadIdx.x] = b;
  r[2][threadIdx.x] = c;
  r[3][threadIdx.x] = d;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r[0][threadIdx.x] = fmin(r[0][threadIdx.x], r[0][threadIdx.x + o]);
      r[1][threadIdx.x] = fmax(r[1][threadIdx.x], r[1][threadIdx.x + o]);
      r[2][threadIdx.x] = fmin(r[2][threadIdx.x], r[2][threadIdx.x + o]);
      r[3][threadIdx.x] = fmax(r[3][threadIdx.x], r[3][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = r[threadIdx.x][0];
}

__device__ __forceinline__ uint64_t spread29(uint64_t v) {
  v &= 0x1FFFFFFFull;
  v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
  v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
  v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  v = (v | (v << 1)) & 0x5555555555555555ull;
  return v;
}

__global__ void __launch_bounds__(256)
    k_morton(const double *__restrict__ x, const double *__restrict__ y, int64_t n,
             int64_t stride, double lox, double loy, double scale,
             uint64_t *__restrict__ keys, int32_t *__restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double cells = (double)(1ull << kMaxLevel);
  const double fx = (x[i * stride] - lox) * scale * cells;
  const double fy = (y[i * stride] - loy) * scale * cells;
  int64_t qx = (int64_t)floor(fx), qy = (int64_t)floor(fy);
  const int64_t top = (1ll << kMaxLevel) - 1;
  qx = qx < 0 ? 0 : (qx > top ? top : qx);
  qy = qy < 0 ? 0 : (qy > top ? top : qy);
  keys[i] = spread29((uint64_t)qx) | (spread29((uint64_t)qy) << 1);
  idx[i] = (int32_t)i;
}

// ----------------------------------------------------------------- boxes
struct GBoxes {
  int64_t *s0, *s1, *t0, *t1;
  int32_t *ix, *iy, *lev, *par, *child0, *nchild;
  uint8_t *leaf;
  uint64_t *code;
};

__device__ __forceinline__ int64_t lower_key(const uint64_t *k, int64_t a, int64_t b,
                                              uint64_t v) {
  while (a < b) {
    const int64_t m = (a + b) >> 1;
    if (k[m] < v) a = m + 1;
    else b = m;
  }
  return a;
}

// child ranges of box b at level l in the sorted keys (quadrant q)
__device__ __forceinline__ void child_rng(const uint64_t *k, int64_t a, int64_t b, int l,
                                          int q, int64_t &ca, int64_t &cb) {
  if (a >= b) {
    ca = cb = a;
    return;
  }
  const int shift = 2 * (kMaxLevel - l - 1);
  const uint64_t prefix = (k[a] >> (shift + 2)) << (shift + 2);
  const uint64_t lo = prefix | ((uint64_t)q << shift), hi = lo + (1ull << shift);
  ca = lower_key(k, a, b, lo);
  cb = lower_key(k, a, b, hi);
}

// Boxes [lb, le) of level l: split those over leaf_max (below kMaxLevel);
// nc = non-empty quadrants, cr = their ranges (4 per quadrant, per box).
__global__ void __launch_bounds__(256)
    k_split_count(int l, int lb, int le, int leaf_max, int self,
                  const uint64_t *__restrict__ ks, const uint64_t *__restrict__ kt,
                  GBoxes B, int32_t *__restrict__ nc, int64_t *__restrict__ cr) {
  const int b = lb + blockIdx.x * 256 + threadIdx.x;
  if (b >= le) return;
  const int64_t cnt = (B.s1[b] - B.s0[b]) + (self ? 0 : (B.t1[b] - B.t0[b]));
  int n = 0;
  if (cnt > leaf_max && l < kMaxLevel) {
    for (int q = 0; q < 4; ++q) {
      int64_t a0, a1, c0, c1;
      child_rng(ks, B.s0[b], B.s1[b], l, q, a0, a1);
      if (self) {
        c0 = a0;
        c1 = a1;
      } else {
        child_rng(kt, B.t0[b], B.t1[b], l, q, c0, c1);
      }
      int64_t *o = cr + ((int64_t)(b - lb) * 4 + q) * 4;
      o[0] = a0;
      o[1] = a1;
      o[2] = c0;
      o[3] = c1;
      if (a1 - a0 + c1 - c0 > 0) ++n;
    }
  }
  nc[b - lb] = n;
}

__global__ void __launch_bounds__(256)
    k_split_fill(int lb, int le, GBoxes B, const int32_t *__restrict__ nc,
                 const uint32_t *__restrict__ off, const int64_t *__restrict__ cr) {
  const int b = lb + blockIdx.x * 256 + threadIdx.x;
  if (b >= le) return;
  const int n = nc[b - lb];
  if (n == 0) return;
  const int first = le + (int)off[b - lb];
  B.leaf[b] = 0;
  B.child0[b] = first;
  B.nchild[b] = n;
  int j = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t *o = cr + ((int64_t)(b - lb) * 4 + q) * 4;
    if (o[1] - o[0] + o[3] - o[2] == 0) continue;
    const int c = first + j++;
    B.s0[c] = o[0];
    B.s1[c] = o[1];
    B.t0[c] = o[2];
    B.t1[c] = o[3];
    B.ix[c] = 2 * B.ix[b] + (q & 1);
    B.iy[c] = 2 * B.iy[b] + (q >> 1);
    B.lev[c] = B.lev[b] + 1;
    B.par[c] = b;
    B.child0[c] = -1;
    B.nchild[c] = 0;
    B.leaf[c] = 1;
    B.code[c] = B.code[b] * 4 + (uint64_t)q;
  }
}

// ----------------------------------------------------------------- lists
__device__ __forceinline__ uint64_t interleave(uint64_t ix, uint64_t iy) {
  return spread29(ix) | (spread29(iy) << 1);
}

__device__ __forceinline__ int find_box(const GBoxes &B, const int32_t *lp, int l, int64_t ix,
                                        int64_t iy) {
  if (ix < 0 || iy < 0 || ix >= (1ll << l) || iy >= (1ll << l)) return -1;
  const uint64_t code = interleave((uint64_t)ix, (uint64_t)iy);
  int a = lp[l], b = lp[l + 1];
  while (a < b) {
    const int m = (a + b) >> 1;
    if (B.code[m] < code) a = m + 1;
    else b = m;
  }
  return (a < lp[l + 1] && B.code[a] == code) ? a : -1;
}

__device__ __forceinline__ bool touching(const GBoxes &B, int a, int b) {
  int la = B.lev[a], lb = B.lev[b];
  if (la > lb) {
    const int t = a;
    a = b;
    b = t;
    const int u = la;
    la = lb;
    lb = u;
  }
  const int d = lb - la;
  const int64_t ax0 = (int64_t)B.ix[a] << d, ax1 = ((int64_t)B.ix[a] + 1) << d;
  const int64_t ay0 = (int64_t)B.iy[a] << d, ay1 = ((int64_t)B.iy[a] + 1) << d;
  const int64_t bx0 = B.ix[b], bx1 = (int64_t)B.ix[b] + 1;
  const int64_t by0 = B.iy[b], by1 = (int64_t)B.iy[b] + 1;
  return bx0 <= ax1 && bx1 >= ax0 && by0 <= ay1 && by1 >= ay0;
}

// A descent pops one box and pushes at most four children, one level down,
// so the stack never holds more than 4 + 3 * kMaxLevel = 91 boxes.
constexpr int kStack = 128;

// Per leaf b: nu / nw = counts of its adjacent leaves and W boxes; with
// fill, the boxes themselves at uo[b] / wo[b].
template <bool fill>
__global__ void __launch_bounds__(64)
    k_leaf_lists(int nb, GBoxes B, const int32_t *__restrict__ lp,
                 int32_t *__restrict__ nu, int32_t *__restrict__ nw,
                 const int64_t *__restrict__ uo, const int64_t *__restrict__ wo,
                 int32_t *__restrict__ ul, int32_t *__restrict__ wl,
                 int32_t *__restrict__ overflow) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= nb || !B.leaf[b]) return;
  int stk[kStack];
  const int l = B.lev[b];
  int cu = 0, cw = 0;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy) {
      const int c = find_box(B, lp, l, (int64_t)B.ix[b] + dx, (int64_t)B.iy[b] + dy);
      if (c < 0) continue;
      if (c == b || B.leaf[c]) {
        if (fill) ul[uo[b] + cu] = c;
        ++cu;
        continue;
      }
      int sp = 0;
      for (int k = 0; k < B.nchild[c]; ++k) stk[sp++] = B.child0[c] + k;
      while (sp > 0) {
        const int d = stk[--sp];
        if (touching(B, b, d)) {
          if (B.leaf[d]) {
            if (fill) ul[uo[b] + cu] = d;
            ++cu;
          } else {
            if (sp + B.nchild[d] > kStack) {
              atomicAdd(overflow, 1);
              sp = 0;
              break;
            }
            for (int k = 0; k < B.nchild[d]; ++k) stk[sp++] = B.child0[d] + k;
          }
        } else {
          if (fill) wl[wo[b] + cw] = d;
          ++cw;
        }
      }
    }
  if (!fill) {
    nu[b] = cu;
    nw[b] = cw;
  }
}

__device__ __forceinline__ bool has_src(const GBoxes &B, int b) { return B.s1[b] > B.s0[b]; }
__device__ __forceinline__ bool has_tgt(const GBoxes &B, int b) { return B.t1[b] > B.t0[b]; }

// Pairs (target box << 32 | source box) of the U, W and X lists from the
// per-leaf lists, kept when the target box has targets and the source box
// sources (each pair once, appended at an atomic cursor; sorted later).
__global__ void __launch_bounds__(256)
    k_emit_uwx(int nb, GBoxes B, const int64_t *__restrict__ uo,
               const int64_t *__restrict__ wo, const int32_t *__restrict__ ul,
               const int32_t *__restrict__ wl, uint64_t *__restrict__ up,
               uint64_t *__restrict__ wp, uint64_t *__restrict__ xp,
               unsigned long long *__restrict__ cur) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= nb || !B.leaf[b]) return;
  for (int64_t e = uo[b]; e < uo[b + 1]; ++e) {
    const int c = ul[e];
    if (has_tgt(B, b) && has_src(B, c))
      up[atomicAdd(&cur[0], 1ull)] = ((uint64_t)b << 32) | (uint32_t)c;
    if (B.lev[c] > B.lev[b] && has_tgt(B, c) && has_src(B, b))
      up[atomicAdd(&cur[0], 1ull)] = ((uint64_t)c << 32) | (uint32_t)b;
  }
  for (int64_t e = wo[b]; e < wo[b + 1]; ++e) {
    const int d = wl[e];
    if (has_tgt(B, b) && has_src(B, d))
      wp[atomicAdd(&cur[1], 1ull)] = ((uint64_t)b << 32) | (uint32_t)d;
    if (has_tgt(B, d) && has_src(B, b))
      xp[atomicAdd(&cur[2], 1ull)] = ((uint64_t)d << 32) | (uint32_t)b;
  }
}

// V pairs of box b (level >= 2, with targets): children of the parent's
// colleagues that are not adjacent to b and hold sources; value = the
// offset code (dx + 3) * 7 + (dy + 3).  count != null: count only.
__global__ void __launch_bounds__(256)
    k_vlist(int nb, GBoxes B, const int32_t *__restrict__ lp, int32_t *__restrict__ count,
            uint64_t *__restrict__ vp, int32_t *__restrict__ vcode,
            unsigned long long *__restrict__ cur) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= nb) return;
  const int l = B.lev[b];
  int n = 0;
  if (l >= 2 && has_tgt(B, b)) {
    const int p = B.par[b];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        const int c = find_box(B, lp, l - 1, (int64_t)B.ix[p] + dx, (int64_t)B.iy[p] + dy);
        if (c < 0) continue;
        for (int k = 0; k < B.nchild[c]; ++k) {
          const int s = B.child0[c] + k;
          const int ddx = B.ix[s] - B.ix[b], ddy = B.iy[s] - B.iy[b];
          if (ddx >= -1 && ddx <= 1 && ddy >= -1 && ddy <= 1) continue;
          if (!has_src(B, s)) continue;
          if (count) {
            ++n;
          } else {
            const unsigned long long at = atomicAdd(cur, 1ull);
            vp[at] = ((uint64_t)b << 32) | (uint32_t)s;
            vcode[at] = (ddx + 3) * 7 + (ddy + 3);
          }
        }
      }
  }
  if (count) count[b] = n;
}

template <typename T>
std::vector<T> get(const T *p, size_t n, hipStream_t s) {
  std::vector<T> v(n);
  if (n) LBS_HIP(hipMemcpyAsync(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
  return v;
}

int bit_length(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

// CSR (ptr over nb boxes, idx) from pairs sorted by (box, other box)
void pairs_to_csr(const std::vector<uint64_t> &pk, int nb, std::vector<int32_t> &ptr,
                  std::vector<int32_t> &idx) {
  ptr.assign((size_t)nb + 1, 0);
  idx.resize(pk.size());
  for (size_t e = 0; e < pk.size(); ++e) {
    ++ptr[(pk[e] >> 32) + 1];
    idx[e] = (int32_t)(pk[e] & 0xFFFFFFFFull);
  }
  for (int b = 0; b < nb; ++b) ptr[b + 1] += ptr[b];
}

}  // namespace

void gpu_build_tree(const double *sx, const double *sy, int64_t sstride, int64_t ns,
                    const double *tx, const double *ty, int64_t tstride, int64_t nt, bool self,
                    int leaf_max, Tree &T, hipStream_t s, DevPerms *keep) {
  if (leaf_max < 1) throw ApiError{LBS_ERR_INVALID_ARG, "leaf_max < 1"};
  if (ns + (self ? 0 : nt) >= (int64_t)INT32_MAX)
    throw ApiError{LBS_ERR_UNSUPPORTED, "more than 2^31 points in one tree"};
  T = Tree();
  T.self = self;
  if (self) nt = ns;
  PhaseClock clk;
  // 1. root box, as the host builder (min/max are exact)
  double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
  {
    DBuf<double> part;
    part.alloc(4 * 256);
    auto reduce = [&](const double *x, const double *y, int64_t n, int64_t st) {
      if (n == 0) return;
      hipLaunchKernelGGL(k_minmax, dim3(256), dim3(256), 0, s, x, y, n, st, part.p);
      std::vector<double> h = get(part.p, 4 * 256, s);
      LBS_HIP(hipStreamSynchronize(s));
      for (int b = 0; b < 256; ++b) {
        xmin = std::min(xmin, h[4 * b]);
        xmax = std::max(xmax, h[4 * b + 1]);
        ymin = std::min(ymin, h[4 * b + 2]);
        ymax = std::max(ymax, h[4 * b + 3]);
      }
    };
    reduce(sx, sy, ns, sstride);
    if (!self) reduce(tx, ty, nt, tstride);
  }
  if (ns + (self ? 0 : nt) == 0) xmin = xmax = ymin = ymax = 0;
  T.x0 = 0.5 * (xmin + xmax);
  T.y0 = 0.5 * (ymin + ymax);
  const double half = 0.5 * std::max(xmax - xmin, ymax - ymin);
  T.R0 = half * (1.0 + 1e-6) + 1e-300 + 1e-12 * std::max(std::fabs(T.x0), std::fabs(T.y0));
  if (!(T.R0 > 0)) T.R0 = 1.0;
  const double lox = T.x0 - T.R0, loy = T.y0 - T.R0, scale = 0.5 / T.R0;
  SortScratch sorts;  // released after the last sort's work is waited for
  // 2. keys and stable sort
  DBuf<uint64_t> ks, kt;
  DBuf<int32_t> ps, pt;
  auto keys = [&](const double *x, const double *y, int64_t n, int64_t st, DBuf<uint64_t> &k,
                  DBuf<int32_t> &p) {
    k.alloc((size_t)std::max<int64_t>(n, 1));
    p.alloc((size_t)std::max<int64_t>(n, 1));
    if (n == 0) return;
    hipLaunchKernelGGL(k_morton, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n, st,
                       lox, loy, scale, k.p, p.p);
    radix_sort(k.p, p.p, n, 2 * kMaxLevel, sorts, s);
  };
  keys(sx, sy, ns, sstride, ks, ps);
  if (!self) keys(tx, ty, nt, tstride, kt, pt);
  if (!keep) {
    std::vector<int32_t> a = get(ps.p, (size_t)ns, s);
    LBS_HIP(hipStreamSynchronize(s));
    T.src_perm.assign(a.begin(), a.end());
    if (self) {
      T.tgt_perm = T.src_perm;
    } else {
      std::vector<int32_t> b = get(pt.p, (size_t)nt, s);
      LBS_HIP(hipStreamSynchronize(s));
      T.tgt_perm.assign(b.begin(), b.end());
    }
  }
  clk.mark("root, keys, sort");
  // 3. boxes, level by level (capacity grows by copying)
  struct Arr {
    DBuf<int64_t> s0, s1, t0, t1;
    DBuf<int32_t> ix, iy, lev, par, child0, nchild;
    DBuf<uint8_t> leaf;
    DBuf<uint64_t> code;
    void release() {
      s0.release(); s1.release(); t0.release(); t1.release();
      ix.release(); iy.release(); lev.release(); par.release();
      child0.release(); nchild.release(); leaf.release(); code.release();
    }
  };
  Arr arr[2];
  int cur = 0;
  int64_t cap = 0;
  auto grow = [&](int64_t need, int64_t used) {
    if (need <= cap) return;
    const int64_t nc2 = std::max<int64_t>(need, 2 * cap + 1024);
    Arr &o = arr[cur], &n = arr[1 - cur];
    auto mv = [&](auto &dst, auto &src) {
      using E = std::remove_pointer_t<decltype(dst.p)>;
      dst.alloc((size_t)nc2);
      if (used > 0) LBS_HIP(hipMemcpyAsync(dst.p, src.p, (size_t)used * sizeof(E),
                                           hipMemcpyDeviceToDevice, s));
    };
    mv(n.s0, o.s0); mv(n.s1, o.s1); mv(n.t0, o.t0); mv(n.t1, o.t1);
    mv(n.ix, o.ix); mv(n.iy, o.iy); mv(n.lev, o.lev); mv(n.par, o.par);
    mv(n.child0, o.child0); mv(n.nchild, o.nchild); mv(n.leaf, o.leaf); mv(n.code, o.code);
    LBS_HIP(hipStreamSynchronize(s));
    o.release();
    cur = 1 - cur;
    cap = nc2;
  };
  auto view = [&]() {
    Arr &a = arr[cur];
    return GBoxes{a.s0.p, a.s1.p, a.t0.p, a.t1.p, a.ix.p, a.iy.p, a.lev.p, a.par.p,
                  a.child0.p, a.nchild.p, a.leaf.p, a.code.p};
  };
  grow(std::max<int64_t>(1024, 4 * (ns + (self ? 0 : nt)) / std::max(leaf_max, 1) + 64), 0);
  {
    // root
    const int64_t r64[4] = {0, ns, 0, nt};
    const int32_t zi = 0, m1 = -1;
    const uint8_t one = 1;
    const uint64_t zc = 0;
    Arr &a = arr[cur];
    LBS_HIP(hipMemcpyAsync(a.s0.p, &r64[0], 8, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.s1.p, &r64[1], 8, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.t0.p, &r64[2], 8, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.t1.p, &r64[3], 8, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.ix.p, &zi, 4, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.iy.p, &zi, 4, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.lev.p, &zi, 4, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.par.p, &m1, 4, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.child0.p, &m1, 4, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.nchild.p, &zi, 4, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.leaf.p, &one, 1, hipMemcpyHostToDevice, s));
    LBS_HIP(hipMemcpyAsync(a.code.p, &zc, 8, hipMemcpyHostToDevice, s));
    LBS_HIP(hipStreamSynchronize(s));  // the host values are released on return
  }
  std::vector<int32_t> lp = {0};
  int nbox = 1;
  {
    DBuf<int32_t> nc;
    DBuf<uint32_t> off, sums;
    DBuf<int64_t> cr;
    int lbeg = 0;
    for (int l = 0;; ++l) {
      const int lend = nbox;
      lp.push_back(lend);
      if (l >= kMaxLevel) break;
      const int n = lend - lbeg;
      if ((int64_t)nc.n < n) {
        nc.alloc((size_t)n);
        off.alloc((size_t)n + 1);
        cr.alloc((size_t)n * 16);
        sums.alloc((size_t)(n + kScanTile) / kScanTile + 1);
      }
      hipLaunchKernelGGL(k_split_count, dim3((n + 255) / 256), dim3(256), 0, s, l, lbeg, lend,
                         leaf_max, self ? 1 : 0, ks.p, self ? ks.p : kt.p, view(), nc.p, cr.p);
      // exclusive scan of the child counts; total = off[n]
      LBS_HIP(hipMemcpyAsync(off.p, nc.p, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      uint32_t zero = 0;
      LBS_HIP(hipMemcpyAsync(off.p + n, &zero, sizeof(uint32_t), hipMemcpyHostToDevice, s));
      scan_into(off.p, (int64_t)n + 1, sums.p, s);
      uint32_t total = 0;
      LBS_HIP(hipMemcpyAsync(&total, off.p + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      LBS_HIP(hipStreamSynchronize(s));
      if (total == 0) break;
      grow((int64_t)nbox + total, nbox);
      hipLaunchKernelGGL(k_split_fill, dim3((n + 255) / 256), dim3(256), 0, s, lbeg, lend,
                         view(), nc.p, off.p, cr.p);
      nbox += (int)total;
      lbeg = lend;
    }
    LBS_HIP(hipGetLastError());
  }
  clk.mark("levels");
  while (lp.size() >= 2 && lp[lp.size() - 1] == lp[lp.size() - 2]) lp.pop_back();
  T.level_ptr = lp;
  T.nlevels = (int)lp.size() - 1;
  const GBoxes B = view();
  // 4. per-leaf adjacent leaves and W boxes (count, scan, fill)
  DBuf<int32_t> dlp, nu, nw, ul, wl, ovf;
  DBuf<int64_t> uo, wo;
  const std::vector<int32_t> zero1(1, 0);  // host sources of async copies live
  const std::vector<unsigned long long> zero4(4, 0ull);  // until the syncs below
  {
    std::vector<int32_t> lpx = lp;
    while ((int)lpx.size() < kMaxLevel + 2) lpx.push_back(lpx.back());
    dlp.upload(lpx, s);
    nu.alloc((size_t)nbox);
    nw.alloc((size_t)nbox);
    ovf.upload(zero1, s);
    LBS_HIP(hipMemsetAsync(nu.p, 0, (size_t)nbox * sizeof(int32_t), s));
    LBS_HIP(hipMemsetAsync(nw.p, 0, (size_t)nbox * sizeof(int32_t), s));
    LBS_HIP(hipStreamSynchronize(s));
    hipLaunchKernelGGL(k_leaf_lists<false>, dim3((nbox + 63) / 64), dim3(64), 0, s, nbox, B,
                       dlp.p, nu.p, nw.p, (const int64_t *)nullptr, (const int64_t *)nullptr,
                       (int32_t *)nullptr, (int32_t *)nullptr, ovf.p);
    std::vector<int32_t> hnu = get(nu.p, (size_t)nbox, s), hnw = get(nw.p, (size_t)nbox, s);
    LBS_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> huo((size_t)nbox + 1, 0), hwo((size_t)nbox + 1, 0);
    for (int b = 0; b < nbox; ++b) {
      huo[b + 1] = huo[b] + hnu[b];
      hwo[b + 1] = hwo[b] + hnw[b];
    }
    uo.upload(huo, s);
    wo.upload(hwo, s);
    ul.alloc((size_t)std::max<int64_t>(huo[nbox], 1));
    wl.alloc((size_t)std::max<int64_t>(hwo[nbox], 1));
    hipLaunchKernelGGL(k_leaf_lists<true>, dim3((nbox + 63) / 64), dim3(64), 0, s, nbox, B,
                       dlp.p, nu.p, nw.p, uo.p, wo.p, ul.p, wl.p, ovf.p);
    const std::vector<int32_t> o = get(ovf.p, 1, s);
    LBS_HIP(hipStreamSynchronize(s));  // host arrays stay alive until here
    if (o[0] != 0) throw ApiError{LBS_ERR_UNSUPPORTED, "quadtree descent deeper than its stack"};
    clk.mark("leaf lists");
    // 5. pairs
    const int64_t nu_tot = huo[nbox], nw_tot = hwo[nbox];
    DBuf<uint64_t> up, wp, xp, vp;
    DBuf<int32_t> uv, wv, xv, vcode, vcnt;
    DBuf<unsigned long long> cursor;
    up.alloc((size_t)std::max<int64_t>(2 * nu_tot, 1));
    wp.alloc((size_t)std::max<int64_t>(nw_tot, 1));
    xp.alloc((size_t)std::max<int64_t>(nw_tot, 1));
    cursor.upload(zero4, s);
    hipLaunchKernelGGL(k_emit_uwx, dim3((nbox + 255) / 256), dim3(256), 0, s, nbox, B, uo.p, wo.p,
                       ul.p, wl.p, up.p, wp.p, xp.p, cursor.p);
    vcnt.alloc((size_t)nbox);
    hipLaunchKernelGGL(k_vlist, dim3((nbox + 255) / 256), dim3(256), 0, s, nbox, B, dlp.p, vcnt.p,
                       (uint64_t *)nullptr, (int32_t *)nullptr, (unsigned long long *)nullptr);
    std::vector<int32_t> hv = get(vcnt.p, (size_t)nbox, s);
    LBS_HIP(hipStreamSynchronize(s));
    int64_t nv_tot = 0;
    for (int32_t c : hv) nv_tot += c;
    vp.alloc((size_t)std::max<int64_t>(nv_tot, 1));
    vcode.alloc((size_t)std::max<int64_t>(nv_tot, 1));
    hipLaunchKernelGGL(k_vlist, dim3((nbox + 255) / 256), dim3(256), 0, s, nbox, B, dlp.p,
                       (int32_t *)nullptr, vp.p, vcode.p, cursor.p + 3);
    std::vector<unsigned long long> cnt = get(cursor.p, 4, s);
    LBS_HIP(hipStreamSynchronize(s));
    const int bits = 32 + bit_length((uint64_t)nbox);
    auto sort_pairs = [&](DBuf<uint64_t> &k, DBuf<int32_t> &v, int64_t n, const int32_t *payload) {
      v.alloc((size_t)std::max<int64_t>(n, 1));
      if (n == 0) return;
      if (payload) {
        LBS_HIP(hipMemcpyAsync(v.p, payload, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      } else {
        LBS_HIP(hipMemsetAsync(v.p, 0, (size_t)n * sizeof(int32_t), s));
      }
      radix_sort(k.p, v.p, n, bits, sorts, s);
    };
    sort_pairs(up, uv, (int64_t)cnt[0], nullptr);
    sort_pairs(wp, wv, (int64_t)cnt[1], nullptr);
    sort_pairs(xp, xv, (int64_t)cnt[2], nullptr);
    DBuf<int32_t> vv;
    sort_pairs(vp, vv, (int64_t)cnt[3], vcode.p);
    std::vector<uint64_t> hu = get(up.p, (size_t)cnt[0], s), hw = get(wp.p, (size_t)cnt[1], s),
                          hx = get(xp.p, (size_t)cnt[2], s), hvk = get(vp.p, (size_t)cnt[3], s);
    std::vector<int32_t> hvc = get(vv.p, (size_t)cnt[3], s);
    LBS_HIP(hipStreamSynchronize(s));
    clk.mark("pairs + sorts");
    pairs_to_csr(hu, nbox, T.u_ptr, T.u_src);
    pairs_to_csr(hw, nbox, T.w_ptr, T.w_src);
    pairs_to_csr(hx, nbox, T.x_ptr, T.x_src);
    pairs_to_csr(hvk, nbox, T.v_ptr, T.v_src);
    T.v_code.assign(hvc.begin(), hvc.end());
  }
  // 6. box arrays to the host; centres and radii as the host builder
  {
    std::vector<int64_t> s0 = get(B.s0, nbox, s), s1 = get(B.s1, nbox, s), t0 = get(B.t0, nbox, s),
                         t1 = get(B.t1, nbox, s);
    std::vector<int32_t> ix = get(B.ix, nbox, s), iy = get(B.iy, nbox, s),
                         lev = get(B.lev, nbox, s), par = get(B.par, nbox, s),
                         c0 = get(B.child0, nbox, s), nch = get(B.nchild, nbox, s);
    std::vector<uint8_t> lf = get(B.leaf, nbox, s);
    LBS_HIP(hipStreamSynchronize(s));
    T.s0 = s0;
    T.s1 = s1;
    T.t0 = t0;
    T.t1 = t1;
    T.ix = ix;
    T.iy = iy;
    T.level = lev;
    T.parent = par;
    T.child0 = c0;
    T.nchild = nch;
    T.leaf = lf;
    T.cx.resize(nbox);
    T.cy.resize(nbox);
    T.rad.resize(nbox);
    for (int b = 0; b < nbox; ++b) {
      const double r = T.R0 / (double)(1ull << lev[b]);
      T.cx[b] = lox + (2.0 * (double)ix[b] + 1.0) * r;
      T.cy[b] = loy + (2.0 * (double)iy[b] + 1.0) * r;
      T.rad[b] = r;
    }
  }
  tree_statistics(T);
  if (keep) {  // the maps stay on the device (a self tree has one)
    keep->src.take(ps);
    if (!self) keep->tgt.take(pt);
  }
  clk.mark("boxes to host");
}

namespace {
__global__ void __launch_bounds__(256)
    k_gather_points(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ x,
                    const double *__restrict__ y, int64_t stride, double *__restrict__ ox,
                    double *__restrict__ oy) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const int64_t i = (int64_t)perm[j] * stride;
  ox[j] = x[i];
  oy[j] = y[i];
}

// one wave per list entry
__global__ void __launch_bounds__(256)
    k_flat_fill(int64_t ne, const int32_t *__restrict__ box, const int64_t *__restrict__ eo,
                const int64_t *__restrict__ s0, const int64_t *__restrict__ s1,
                int32_t *__restrict__ fi) {
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= ne) return;
  const int c = box[k];
  const int64_t a = s0[c], len = s1[c] - a, o = eo[k];
  for (int64_t t = threadIdx.x & 63; t < len; t += 64) fi[o + t] = (int32_t)(a + t);
}

__global__ void __launch_bounds__(256)
    k_widen_perm(int64_t n, const int32_t *__restrict__ perm, const int64_t *__restrict__ map,
                 int64_t *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  out[j] = map ? map[perm[j]] : (int64_t)perm[j];
}
}  // namespace

void launch_gather_points(int64_t n, const int32_t *perm, const double *x, const double *y,
                          int64_t stride, double *ox, double *oy, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, perm,
                     x, y, stride, ox, oy);
  LBS_HIP(hipGetLastError());
}

void launch_flat_fill(int64_t ne, const int32_t *box, const int64_t *eo, const int64_t *s0,
                      const int64_t *s1, int32_t *fi, hipStream_t s) {
  if (ne <= 0) return;
  hipLaunchKernelGGL(k_flat_fill, dim3((unsigned)((ne + 3) / 4)), dim3(256), 0, s, ne, box, eo, s0,
                     s1, fi);
  LBS_HIP(hipGetLastError());
}

void scan_u32(uint32_t *a, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  DBuf<uint32_t> sums;
  if (n > kScanTile) sums.alloc((size_t)((n + kScanTile - 1) / kScanTile));
  scan_into(a, n, sums.p, s);
  if (sums.p) LBS_HIP(hipStreamSynchronize(s));  // sums is released on return
}

void sort_by_key(uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s) {
  SortScratch sc;
  radix_sort(keys, vals, n, bits, sc, s);
  LBS_HIP(hipStreamSynchronize(s));  // the scratch is released on return
}

void sort_by_key(uint64_t *keys, int32_t *vals, int64_t n, int bits, SortBufs &sc,
                 hipStream_t s) {
  radix_sort(keys, vals, n, bits, sc, s);
}

void launch_widen_perm(int64_t n, const int32_t *perm, const int64_t *map, int64_t *out,
                       hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_widen_perm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, perm,
                     map, out);
  LBS_HIP(hipGetLastError());
}

}  // namespace lbs
