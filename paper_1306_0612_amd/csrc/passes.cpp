// Programs of the upward (M2M) and downward (L2L) passes of the FMM
// (Section 5): the translations between levels, laid out so that one
// work-group carries a connected piece of the tree through many levels with
// every intermediate expansion kept in LDS.
//
// Work boxes.  Upward: boxes at level >= 2 with a child holding sources
// (their multipole comes from the children's).  Downward: boxes at level
// >= 3 holding targets (local = own part + the parent's local translated),
// and level-2 boxes with a child holding targets (local = own part).
//
// Components.  The work boxes are cut into connected subtrees whose LDS
// needs fit `cap` expansion slots: upward, one slot per box computed plus
// one per input (a child that is a leaf or the root of another component);
// downward, two per box (its own part and the parent's translated local).
// Each component is one work-group of one round (one launch); upward a
// component runs after the components whose roots it reads, downward after
// the component that finishes its root's parent.

#include <algorithm>
#include <stdexcept>

#include "tree.h"

namespace lbs {
namespace {

inline int quad_of(const Tree &T, int b) { return (T.ix[b] & 1) | ((T.iy[b] & 1) << 1); }

}  // namespace

void build_pass_program(const Tree &T, bool down, int cap, PassProgram &pp) {
  if (cap < 16 || cap >= kPassNone) throw std::invalid_argument("pass capacity out of range");
  const int nb = T.nbox();
  if (nb >= (1 << 30)) throw std::length_error("more than 2^30 boxes in one plan");
  pp = PassProgram();
  pp.cap = cap;
  pp.down = down;
  auto holds = [&](int b) { return down ? T.t1[b] > T.t0[b] : T.s1[b] > T.s0[b]; };
  auto kids = [&](int b, int out[4]) {  // children that hold points, quadrant order
    int n = 0;
    if (!T.leaf[b])
      for (int c = T.child0[b]; c < T.child0[b] + T.nchild[b]; ++c)
        if (holds(c)) out[n++] = c;
    return n;
  };
  std::vector<uint8_t> work(nb, 0);
  for (int b = 0; b < nb; ++b) {
    if (T.level[b] < 2 || !holds(b)) continue;
    int k[4];
    const int nk = kids(b, k);
    work[b] = down ? (T.level[b] >= 3 || nk > 0) : nk > 0;
  }
  // Rounds by dynamic programming from the deepest level up.  h(b) is the
  // round of b's component counted from the side the pass starts at
  // (upward from the bottom; downward the same count, launched in reverse),
  // cost(b) the slots b's component needs below and at b.  With R the
  // largest h of b's work children (1 without any), b joins the components
  // of all its children with h = R when the slots add up to at most cap;
  // otherwise b starts a component of round R + 1 whose children are all
  // separate (upward: inputs).  A child is either merged or in an earlier
  // launch, never in the same one; fewer rounds at a child never cost its
  // parent a round, so the count of rounds is as small as this merging
  // rule allows.
  // boxes by level (a batch forest appends whole trees, so its boxes are
  // not in level order)
  std::vector<std::vector<int32_t>> by_level(std::max(T.nlevels, 1));
  for (int b = 0; b < nb; ++b) {
    if (T.level[b] < 0 || T.level[b] >= T.nlevels) throw std::logic_error("box level out of range");
    by_level[T.level[b]].push_back(b);
  }
  const int unit = down ? 2 : 1;
  std::vector<int32_t> cost(nb, 0), h(nb, 0);
  std::vector<uint8_t> root(nb, 0), merged(nb, 0);
  for (int l = T.nlevels - 1; l >= 2; --l)
    for (int b : by_level[l]) {
      if (!work[b]) continue;
      int k[4];
      const int nk = kids(b, k);
      int R = 1;
      for (int i = 0; i < nk; ++i)
        if (work[k[i]]) R = std::max(R, (int)h[k[i]]);
      int c = unit;
      for (int i = 0; i < nk; ++i) {
        if (work[k[i]] && h[k[i]] == R) c += cost[k[i]];
        else if (!down) c += 1;  // an input slot
      }
      if (c <= cap) {
        h[b] = R;
        cost[b] = c;
        for (int i = 0; i < nk; ++i) {
          if (!work[k[i]]) continue;
          if (h[k[i]] == R) merged[k[i]] = 1;
          else root[k[i]] = 1;
        }
      } else {
        h[b] = R + 1;
        cost[b] = unit + (down ? 0 : nk);
        for (int i = 0; i < nk; ++i)
          if (work[k[i]]) root[k[i]] = 1;
      }
      if (l == 2) root[b] = 1;
    }
  int nrounds = 0;
  for (int b = 0; b < nb; ++b)
    if (work[b] && root[b]) nrounds = std::max(nrounds, (int)h[b]);
  // components: roots, each with the children merged into it, recursively
  std::vector<int32_t> comp(nb, -1);
  std::vector<int> roots;
  std::vector<int32_t> round;
  for (int b = 0; b < nb; ++b)
    if (work[b] && root[b]) {
      roots.push_back(b);
      round.push_back(down ? nrounds + 1 - h[b] : h[b]);
    }
  std::vector<std::vector<int32_t>> members(roots.size());
  for (size_t ci = 0; ci < roots.size(); ++ci) {
    std::vector<int32_t> &m = members[ci];
    m.push_back(roots[ci]);
    comp[roots[ci]] = (int32_t)ci;
    for (size_t i = 0; i < m.size(); ++i) {
      int k[4];
      const int nk = kids(m[i], k);
      for (int j = 0; j < nk; ++j) {
        if (!work[k[j]] || !merged[k[j]]) continue;
        comp[k[j]] = (int32_t)ci;
        m.push_back(k[j]);
      }
    }
  }
  // emit, round by round, larger components first within a round
  std::vector<int32_t> order(roots.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (round[a] != round[b]) return round[a] < round[b];
    return members[a].size() > members[b].size();
  });
  pp.round_ptr.assign(1, 0);
  std::vector<int32_t> slot_of(nb, -1);  // a box's slot in the component being emitted
  int cur = 1;
  for (size_t oi = 0; oi < order.size(); ++oi) {
    const int ci = order[oi];
    while (round[ci] > cur) {
      pp.round_ptr.push_back((int32_t)oi);
      ++cur;
    }
    std::vector<int32_t> m = members[ci];
    std::stable_sort(m.begin(), m.end(), [&](int a, int b) {
      if (T.level[a] != T.level[b]) return down ? T.level[a] < T.level[b] : T.level[a] > T.level[b];
      return a < b;
    });
    const int nm = (int)m.size();
    const int32_t e0 = (int32_t)(pp.ext.size() / 2), p0 = (int32_t)(pp.par.size() / 4),
                  s0 = (int32_t)pp.stp.size();
    auto pack2 = [](int a, int b) { return (int32_t)((uint32_t)a | ((uint32_t)b << 16)); };
    if (!down) {
      // inputs: children that are leaves or other components' roots
      std::vector<int32_t> ks;
      for (int b : m) {
        int k[4];
        const int nk = kids(b, k);
        for (int j = 0; j < nk; ++j)
          if (!work[k[j]] || root[k[j]]) ks.push_back(k[j]);
      }
      const int ne = (int)ks.size();
      for (int j = 0; j < ne; ++j) {
        pp.ext.push_back(ks[j]);
        pp.ext.push_back(1 | (quad_of(T, ks[j]) << 2));  // times pre[q]
      }
      for (int j = 0; j < ne; ++j) slot_of[ks[j]] = j;
      for (int j = 0; j < nm; ++j) slot_of[m[j]] = ne + j;
      auto slot = [&](int c) -> int { return slot_of[c]; };
      for (int j = 0; j < nm; ++j) {
        const int b = m[j];
        int sq[4] = {kPassNone, kPassNone, kPassNone, kPassNone}, k[4];
        const int nk = kids(b, k);
        for (int i = 0; i < nk; ++i) sq[quad_of(T, k[i])] = slot(k[i]);
        pp.par.push_back((int32_t)((uint32_t)b | ((uint32_t)quad_of(T, b) << 30)));
        pp.par.push_back(0);
        pp.par.push_back(pack2(sq[0], sq[1]));
        pp.par.push_back(pack2(sq[2], sq[3]));
      }
      if (ne + nm > cap) throw std::logic_error("upward component over capacity");
    } else {
      // inputs: own parts of the members (slot = member index), then the
      // local of the root's parent times post[q_root] (slot nm)
      const int r = m[0];
      const bool staged = T.level[r] >= 3;
      for (int b : m) {
        pp.ext.push_back(b);
        pp.ext.push_back(0);
      }
      if (staged) {
        pp.ext.push_back(T.parent[r]);
        pp.ext.push_back(2 | (quad_of(T, r) << 2));  // times post[q]
      }
      auto ver = [&](int i) -> int {
        if (i == 0) return staged ? nm : kPassNone;
        return nm + (staged ? 1 : 0) + i - 1;
      };
      for (int i = 0; i < nm; ++i) slot_of[m[i]] = i;
      for (int i = 0; i < nm; ++i) {
        const int b = m[i];
        int cv[4] = {kPassNone, kPassNone, kPassNone, kPassNone}, k[4];
        const int nk = kids(b, k);
        for (int j = 0; j < nk; ++j) {
          if (comp[k[j]] != ci || root[k[j]]) continue;
          cv[quad_of(T, k[j])] = ver(slot_of[k[j]]);
        }
        pp.par.push_back((int32_t)((uint32_t)b | ((uint32_t)quad_of(T, b) << 30)));
        pp.par.push_back(pack2(i, ver(i)));
        pp.par.push_back(pack2(cv[0], cv[1]));
        pp.par.push_back(pack2(cv[2], cv[3]));
      }
      if (2 * nm > cap) throw std::logic_error("downward component over capacity");
    }
    // steps: one per level, in member order
    pp.stp.push_back(0);
    for (int j = 1; j <= nm; ++j)
      if (j == nm || T.level[m[j]] != T.level[m[j - 1]]) pp.stp.push_back(j);
    const int32_t ne = (int32_t)(pp.ext.size() / 2) - e0;
    const int32_t ns = (int32_t)pp.stp.size() - s0 - 1;
    if (ns > kPassMaxSteps) throw std::logic_error("component spans too many levels");
    const int32_t h[8] = {e0, ne, p0, nm, s0, ns, roots[ci], round[ci]};
    pp.hdr.insert(pp.hdr.end(), h, h + 8);
  }
  pp.round_ptr.push_back((int32_t)order.size());
  pp.ncomp = (int)order.size();
}

int64_t check_pass_program(const Tree &T, const PassProgram &pp) {
  // Runs the program on the host with scalar stand-ins for expansions:
  // upward, a box's value is its number of sources (leaves: given; a parent:
  // the sum over its children); downward, every own part is 1 and a local
  // is its own part plus the parent's local, so that a level-l box ends at
  // l - 1.  Also checks every read against what is final or written by then.
  const bool down = pp.down;
  const int nb = T.nbox();
  int64_t err = 0;
  auto holds = [&](int b) { return down ? T.t1[b] > T.t0[b] : T.s1[b] > T.s0[b]; };
  std::vector<int64_t> val(nb, 0);
  std::vector<uint8_t> final(nb, 0), done(nb, 0);
  if (!down)
    for (int b = 0; b < nb; ++b)
      if (T.leaf[b] && holds(b)) {
        val[b] = T.s1[b] - T.s0[b];
        final[b] = 1;
      }
  const int ncomp = (int)pp.hdr.size() / 8;
  for (size_t rr = 0; rr + 1 < pp.round_ptr.size(); ++rr) {
    std::vector<int> fin;
    for (int c = pp.round_ptr[rr]; c < pp.round_ptr[rr + 1]; ++c) {
      if (c < 0 || c >= ncomp) return err + 1;
      const int32_t *h = &pp.hdr[8 * (size_t)c];
      const int e0 = h[0], ne = h[1], p0 = h[2], np = h[3], s0 = h[4], ns = h[5];
      const int nslot = down ? 2 * np : ne + np;
      if (nslot > pp.cap || ns > kPassMaxSteps) ++err;
      std::vector<int64_t> sl(std::max(nslot, ne) + 1, 0);
      std::vector<uint8_t> wr(sl.size(), 0);
      for (int e = 0; e < ne; ++e) {
        const int box = pp.ext[2 * (size_t)(e0 + e)], md = pp.ext[2 * (size_t)(e0 + e) + 1];
        if (box < 0 || box >= nb) return err + 1;
        const int mode = md & 3, q = md >> 2;
        const int want = down ? (e < np ? 0 : 2) : 1;
        if (mode != want) ++err;
        if (mode == 1 && q != ((T.ix[box] & 1) | ((T.iy[box] & 1) << 1))) ++err;
        if (mode == 0) {
          sl[e] = 1;
        } else {
          if (!final[box]) ++err;
          sl[e] = val[box];
        }
        wr[e] = 1;
      }
      if (pp.stp[s0] != 0 || pp.stp[s0 + ns] != np) ++err;
      for (int st = 0; st < ns; ++st) {
        std::vector<std::pair<int, int64_t>> writes;
        for (int j = pp.stp[s0 + st]; j < pp.stp[s0 + st + 1]; ++j) {
          const int32_t *d = &pp.par[4 * (size_t)(p0 + j)];
          const int box = (int)((uint32_t)d[0] & 0x3FFFFFFFu), q = (int)((uint32_t)d[0] >> 30);
          if (box < 0 || box >= nb) return err + 1;
          if (q != ((T.ix[box] & 1) | ((T.iy[box] & 1) << 1))) ++err;
          if (done[box]) ++err;
          done[box] = 1;
          int sq[4] = {d[2] & 0xFFFF, (int)((uint32_t)d[2] >> 16), d[3] & 0xFFFF,
                       (int)((uint32_t)d[3] >> 16)};
          auto rd = [&](int s) -> int64_t {
            if (s < 0 || s >= (int)sl.size() || !wr[s]) {
              ++err;
              return 0;
            }
            return sl[s];
          };
          int64_t v = 0;
          if (!down) {
            for (int k = 0; k < 4; ++k)
              if (sq[k] != kPassNone) v += rd(sq[k]);
            writes.push_back({ne + j, v});
          } else {
            const int own = d[1] & 0xFFFF, ver = (int)((uint32_t)d[1] >> 16);
            v = rd(own) + (ver != kPassNone ? rd(ver) : 0);
            for (int k = 0; k < 4; ++k)
              if (sq[k] != kPassNone) writes.push_back({sq[k], v});
          }
          val[box] = v;
          fin.push_back(box);
        }
        for (auto &w : writes) {  // visible from the next step on
          if (w.first < 0 || w.first >= (int)sl.size()) return err + 1;
          sl[w.first] = w.second;
          wr[w.first] = 1;
        }
      }
    }
    for (int b : fin) final[b] = 1;
  }
  for (int b = 0; b < nb; ++b) {
    bool kid = false;
    if (!T.leaf[b])
      for (int c = T.child0[b]; c < T.child0[b] + T.nchild[b]; ++c) kid |= holds(c);
    const bool work = T.level[b] >= 2 && holds(b) && (down ? (T.level[b] >= 3 || kid) : kid);
    if (work != (bool)done[b]) ++err;
    if (!work) continue;
    const int64_t want = down ? T.level[b] - 1 : T.s1[b] - T.s0[b];
    if (val[b] != want) ++err;
  }
  return err;
}

}  // namespace lbs
