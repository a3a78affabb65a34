// Host-side forest topology: leaf table in key order, refinement with 2:1
// balance across faces, edges and corners, coarsening, and the remap lists
// (Sec. 2.2).  The paper delegates this to p4est on the CPU; here it is a
// small single-process implementation over a hash set of leaves.
#include <algorithm>
#include <unordered_set>

#include "foap4_internal.h"
#include "morton.h"

namespace f4 {

using Key4 = std::array<int32_t, 4>;
using LeafSet = std::unordered_set<Key4, LeafHash>;

static inline Key4 k4(int32_t l, const int32_t g[3]) { return Key4{l, g[0], g[1], g[2]}; }

void Topology::init_uniform(int ndim_, const int32_t nt_[3], int level) {
  ndim = ndim_;
  for (int d = 0; d < 3; d++) nt[d] = (d < ndim) ? nt_[d] : 1;
  leaves.clear();
  const int32_t ex = nt[0] << level, ey = nt[1] << level, ez = (ndim == 3) ? (nt[2] << level) : 1;
  leaves.reserve((size_t)ex * ey * ez);
  for (int32_t z = 0; z < ez; z++)
    for (int32_t y = 0; y < ey; y++)
      for (int32_t x = 0; x < ex; x++) leaves.push_back(Leaf{level, {x, y, z}});
  sort_and_index();
}

uint64_t Topology::key(const Leaf &l) const { return leaf_key(ndim, nt, l.level, l.g); }

int32_t Topology::tree_id(const Leaf &l) const {
  int32_t t[3] = {0, 0, 0};
  for (int d = 0; d < ndim; d++) t[d] = l.g[d] >> l.level;
  return t[0] + nt[0] * (t[1] + nt[1] * t[2]);
}

void Topology::sort_and_index() {
  std::vector<std::pair<uint64_t, Leaf>> tmp;
  tmp.reserve(leaves.size());
  for (const Leaf &l : leaves) tmp.push_back({key(l), l});
  std::sort(tmp.begin(), tmp.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
  for (size_t i = 0; i < tmp.size(); i++) leaves[i] = tmp[i].second;
  index_.clear();
  index_.reserve(leaves.size() * 2);
  for (size_t i = 0; i < leaves.size(); i++) index_[k4(leaves[i].level, leaves[i].g)] = (int64_t)i;
}

int64_t Topology::find(int32_t level, const int32_t g[3]) const {
  auto it = index_.find(k4(level, g));
  return it == index_.end() ? -1 : it->second;
}

namespace {

struct Ctx {
  int ndim;
  int32_t nt[3];
  int per[3];
  std::vector<std::array<int, 3>> offs;  // the 3^d - 1 neighbour directions
  Ctx(int nd, const int32_t *n, const int *p) : ndim(nd) {
    for (int d = 0; d < 3; d++) {
      nt[d] = n[d];
      per[d] = p[d];
    }
    for (int dz = (nd == 3 ? -1 : 0); dz <= (nd == 3 ? 1 : 0); dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++)
          if (dx || dy || dz) offs.push_back({dx, dy, dz});
  }
  // periodic wrap of region g at level l; false if g lies beyond the end of
  // a bounded axis (there is no region there)
  bool wrap(int32_t l, int32_t g[3]) const {
    for (int d = 0; d < ndim; d++) {
      const int32_t E = nt[d] << l;
      if ((g[d] < 0 || g[d] >= E) && !per[d]) return false;
      g[d] = ((g[d] % E) + E) % E;
    }
    return true;
  }
  // leaf of s covering region (l, g) at a level <= l, as its level (-1: none)
  int32_t covering(const LeafSet &s, int32_t l, const int32_t g[3], Key4 *hit) const {
    for (int32_t lc = l; lc >= 0; lc--) {
      const int sh = l - lc;
      const Key4 k{lc, g[0] >> sh, g[1] >> sh, ndim == 3 ? (g[2] >> sh) : 0};
      if (s.count(k)) {
        if (hit) *hit = k;
        return lc;
      }
    }
    return -1;
  }
  void children(const Key4 &p, Key4 out[8]) const {
    for (int c = 0; c < (1 << ndim); c++)
      out[c] = Key4{p[0] + 1, 2 * p[1] + (c & 1), 2 * p[2] + ((c >> 1) & 1), ndim == 3 ? 2 * p[3] + ((c >> 2) & 1) : 0};
  }
};

}  // namespace

bool Topology::regrid(const int8_t *flags, int lmin, int lmax, std::vector<Leaf> &out, std::vector<int32_t> &op,
                      std::vector<int32_t> &src, std::vector<int32_t> &arg) const {
  Ctx C(ndim, nt, periodic);
  const int nch = 1 << ndim;
  // 1. refine flagged leaves
  LeafSet cur;
  cur.reserve(leaves.size() * 2);
  for (size_t n = 0; n < leaves.size(); n++) {
    const Leaf &L = leaves[n];
    const Key4 k = k4(L.level, L.g);
    if (flags[n] > 0 && L.level < lmax) {
      Key4 ch[8];
      C.children(k, ch);
      for (int c = 0; c < nch; c++) cur.insert(ch[c]);
    } else {
      cur.insert(k);
    }
  }
  // 2. 2:1 balance with corner connectivity: refine the coarser leaf of any
  //    touching pair whose levels differ by more than one, to a fixpoint
  for (;;) {
    std::vector<Key4> refine;
    for (const Key4 &k : cur) {
      if (k[0] < 2) continue;
      for (const auto &o : C.offs) {
        int32_t h[3] = {k[1] + o[0], k[2] + o[1], ndim == 3 ? k[3] + o[2] : 0};
        if (!C.wrap(k[0], h)) continue;
        Key4 hit;
        const int32_t lc = C.covering(cur, k[0], h, &hit);
        if (lc >= 0 && lc < k[0] - 1) refine.push_back(hit);
      }
    }
    if (refine.empty()) break;
    std::sort(refine.begin(), refine.end());
    refine.erase(std::unique(refine.begin(), refine.end()), refine.end());
    for (const Key4 &k : refine) {
      cur.erase(k);
      Key4 ch[8];
      C.children(k, ch);
      for (int c = 0; c < nch; c++) cur.insert(ch[c]);
    }
  }
  // 3. coarsen complete families of old leaves flagged -1 above lmin whose
  //    parent touches only leaves of level <= parent level + 1
  std::unordered_map<Key4, int, LeafHash> fam;
  for (size_t n = 0; n < leaves.size(); n++) {
    const Leaf &L = leaves[n];
    if (flags[n] < 0 && L.level > lmin && cur.count(k4(L.level, L.g))) {
      const Key4 p{L.level - 1, L.g[0] >> 1, L.g[1] >> 1, ndim == 3 ? (L.g[2] >> 1) : 0};
      fam[p]++;
    }
  }
  std::vector<Key4> merge;
  for (const auto &kv : fam) {
    if (kv.second != nch) continue;
    const Key4 &p = kv.first;
    bool ok = true;
    for (const auto &o : C.offs) {
      if (!ok) break;
      int32_t r[3] = {p[1] + o[0], p[2] + o[1], ndim == 3 ? p[3] + o[2] : 0};
      if (!C.wrap(p[0], r)) continue;
      // cells of level lp + 2 in region r along the contact with the parent
      int lo[3], hi[3];
      for (int d = 0; d < 3; d++) {
        if (d >= ndim) { lo[d] = hi[d] = 0; continue; }
        if (o[d] == 1) { lo[d] = hi[d] = 0; }
        else if (o[d] == -1) { lo[d] = hi[d] = 3; }
        else { lo[d] = 0; hi[d] = 3; }
      }
      for (int sz = lo[2]; sz <= hi[2] && ok; sz++)
        for (int sy = lo[1]; sy <= hi[1] && ok; sy++)
          for (int sx = lo[0]; sx <= hi[0] && ok; sx++) {
            const int32_t c[3] = {4 * r[0] + sx, 4 * r[1] + sy, ndim == 3 ? 4 * r[2] + sz : 0};
            const int32_t lc = C.covering(cur, p[0] + 2, c, nullptr);
            if (lc < 0 || lc > p[0] + 1) ok = false;
          }
    }
    if (ok) merge.push_back(p);
  }
  for (const Key4 &p : merge) {
    Key4 ch[8];
    C.children(p, ch);
    for (int c = 0; c < nch; c++) cur.erase(ch[c]);
    cur.insert(p);
  }
  // new leaf table in key order
  Topology nt_;
  nt_.ndim = ndim;
  for (int d = 0; d < 3; d++) {
    nt_.nt[d] = nt[d];
    nt_.periodic[d] = periodic[d];
  }
  nt_.leaves.reserve(cur.size());
  for (const Key4 &k : cur) nt_.leaves.push_back(Leaf{k[0], {k[1], k[2], k[3]}});
  nt_.sort_and_index();
  bool same = nt_.leaves.size() == leaves.size();
  for (size_t i = 0; same && i < leaves.size(); i++) {
    const Leaf &a = nt_.leaves[i], &b = leaves[i];
    same = a.level == b.level && a.g[0] == b.g[0] && a.g[1] == b.g[1] && a.g[2] == b.g[2];
  }
  if (same) return false;
  op.clear();
  src.clear();
  arg.clear();
  for (const Leaf &L : nt_.leaves) {
    const int64_t same_i = find(L.level, L.g);
    if (same_i >= 0) {
      op.push_back(0); src.push_back((int32_t)same_i); arg.push_back(0);
      continue;
    }
    if (L.level > 0) {
      const int32_t pg[3] = {L.g[0] >> 1, L.g[1] >> 1, ndim == 3 ? (L.g[2] >> 1) : 0};
      const int64_t pi = find(L.level - 1, pg);
      if (pi >= 0) {
        int cid = 0;
        for (int d = 0; d < ndim; d++) cid |= (L.g[d] & 1) << d;
        op.push_back(1); src.push_back((int32_t)pi); arg.push_back(cid);
        continue;
      }
    }
    const int32_t c0[3] = {2 * L.g[0], 2 * L.g[1], ndim == 3 ? 2 * L.g[2] : 0};
    const int64_t ci = find(L.level + 1, c0);
    op.push_back(2); src.push_back((int32_t)ci); arg.push_back(0);
  }
  out.swap(nt_.leaves);
  return true;
}

}  // namespace f4
