// Adaptive quadtree and the four interaction lists of the adaptive 2D FMM
// (host side, plain C++; no GPU needed).
//
// The paper evaluates every product with I + K by the 2D Coulomb FMM on an
// adaptive quadtree that is refined until no leaf holds more than a preset
// number of points (Section 5; Section 6, Example 3).  Lists (for a box b):
//   U(b)  leaf b: leaves adjacent to b, b included          -> direct sum
//   V(b)  children of the parent's colleagues not adjacent to b -> M2L
//   W(b)  leaf b: descendants of b's colleagues that are not adjacent to b
//         while their parent is                               -> M2P
//   X(b)  leaves c with b in W(c)                              -> P2L
#pragma once
#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

namespace lbs {

// fn(begin, end) over [0, n) split into contiguous ranges, one per host
// thread (at most 16; small n runs inline).
template <typename F>
void parallel_for(int64_t n, F fn, int64_t grain = 4096) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = (int)std::min<int64_t>(std::min(hw, 16), (n + grain - 1) / grain);
  if (nt <= 1) {
    fn((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int t = 0; t < nt; ++t) {
    const int64_t a = n * t / nt, b = n * (t + 1) / nt;
    th.emplace_back([=, &fn] { fn(a, b); });
  }
  for (auto &x : th) x.join();
}

constexpr int kMaxLevel = 29;   // Morton keys of 29 bits per axis

struct Tree {
  double x0 = 0, y0 = 0, R0 = 1;  // root centre and half-width
  int nlevels = 0;                // number of levels present (root = 0)
  bool self = true;               // targets are the sources
  // boxes in level-major order; children of a box are contiguous
  std::vector<double> cx, cy, rad;
  std::vector<int32_t> level, parent, child0, nchild, ix, iy;
  std::vector<int64_t> s0, s1, t0, t1;  // source / target ranges (sorted)
  std::vector<uint8_t> leaf;
  std::vector<int32_t> level_ptr;       // boxes of level l: [lp[l], lp[l+1])
  // CSR lists over boxes
  std::vector<int32_t> v_ptr, v_src;
  std::vector<uint8_t> v_code;          // (dx + 3) * 7 + (dy + 3)
  std::vector<int32_t> x_ptr, x_src;
  std::vector<int32_t> u_ptr, u_src;
  std::vector<int32_t> w_ptr, w_src;
  std::vector<int64_t> src_perm, tgt_perm;  // sorted position -> input index
  int64_t p2p_pairs = 0, m2p_evals = 0, p2l_evals = 0;

  int nbox() const { return (int)cx.size(); }
};

// Build the tree over ns source points and nt target points.  With
// self == true the targets are the sources (tx, ty, nt ignored).  A box is
// split while it holds more than leaf_max points (sources + targets, or
// sources when self) and its level is below kMaxLevel.  Lists keep only
// pairs that move information from a box holding sources to one holding
// targets.
void build_tree(const double *sx, const double *sy, int64_t ns,
                const double *tx, const double *ty, int64_t nt, bool self,
                int leaf_max, Tree &T);

// Pair and evaluation counts of the lists (p2p_pairs, m2p_evals, p2l_evals).
void tree_statistics(Tree &T);

// Append tree t to the forest F: box indices shift by F's box count, point
// ranges by src_base / tgt_base, permutation entries by the index bases.
void append_tree(Tree &F, const Tree &t, int64_t src_base, int64_t tgt_base,
                 int64_t src_index_base, int64_t tgt_index_base);

// Count ordered point pairs (i in targets, j in sources, i != j when self)
// covered zero or several times by U, V, W and X.  O(leaves^2 depth).
int64_t check_coverage(const Tree &T);

// Program of the upward (M2M) or downward (L2L) pass (passes.cpp): the
// work boxes cut into components of at most `cap` LDS expansion slots, one
// work-group each, launched round by round.
//   hdr  8 per component: ext offset, #ext, par offset, #par, stp offset,
//        #steps, root box, round
//   ext  2 per input slot (slots 0, 1, ...): box, mode | q << 2; the input
//        is the box's expansion, times pre[q] (mode 1), post[q] (mode 2)
//        or as it is (mode 0)
//   par  4 per work box, in step order: box | quadrant << 30, then
//        upward:   0, and the slots of its children by quadrant (16 bits
//                  each, kPassNone absent); its own result goes to slot
//                  #ext + its index
//        downward: own-part slot | parent-version slot << 16, and the
//                  slots its children's parent versions go to, by quadrant
//   stp  per component, #steps + 1 offsets into its par entries (one step
//        per level: deepest first upward, shallowest first downward)
constexpr int kPassNone = 0xFFFF;
constexpr int kPassMaxSteps = 31;
struct PassProgram {
  int cap = 0, ncomp = 0;
  bool down = false;
  std::vector<int32_t> round_ptr;  // components of round k: [rp[k], rp[k+1])
  std::vector<int32_t> hdr, ext, par, stp;
};
void build_pass_program(const Tree &T, bool down, int cap, PassProgram &pp);

// Errors found by running the program on the host with scalar stand-ins
// for the expansions (0: every work box computed once, from inputs that
// were final or written by then, with the right result).
int64_t check_pass_program(const Tree &T, const PassProgram &pp);

// LDS expansion slots per work-group of the pass kernels for expansions of
// P coefficients of cbytes bytes each (8: FP32, 16: FP64), within 60 KB with
// the binomial and scale tables and the step descriptors.
constexpr int pass_cap(int P, int cbytes) {
  const int fixed = P * P * (cbytes / 2) + 9 * P * cbytes + 128;  // + a slot of zeros
  const int c = (61440 - fixed) / (P * cbytes + 16);
  return (c > 1024 ? 1024 : c) & ~7;
}

}  // namespace lbs
