// Hierarchical partition of the points and the box schedule, host C++.
//
// Follows Sec. 3 (opening paragraphs): the root box holds all points, a box
// with more than m points is split into its 2^d children, adaptive trees are
// 2:1 balanced, and boxes are adjacent when their closed boxes meet (share a
// face, edge or corner).  The readings fixed here (quantization, Morton ids,
// tree order of the points, neighbours of coarser leaves, colour order) are
// stated in include/rsrs.h next to rsrs_build_tree and rsrs_tree_schedule.
#include "tree.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <unordered_map>
#include <utility>

namespace rsrs {
namespace {

struct Node {
  int32_t c[3] = {0, 0, 0};
  std::vector<int64_t> pts;  // user indices, ascending
  bool split = false;
};

using Key = std::pair<int, uint64_t>;  // (level, Morton code at that level)

uint64_t morton(const int32_t* c, int d, int nbits) {
  uint64_t code = 0;
  for (int bit = 0; bit < nbits; ++bit)
    for (int a = 0; a < d; ++a)
      code |= (uint64_t)((c[a] >> bit) & 1) << (bit * d + a);
  return code;
}

struct Builder {
  int d, Q, m;
  int64_t n;
  std::vector<int64_t> q;  // n x d quantized coordinates
  std::map<Key, Node> nodes;

  Key key_of(int lev, const int32_t* c) const { return Key(lev, morton(c, d, Q)); }

  // Creates the non-empty children of the box `k`; returns their keys.
  std::vector<Key> split(const Key& k) {
    Node& nd = nodes[k];
    nd.split = true;
    const int lev = k.first;
    const int sh = Q - lev - 1;
    std::vector<int64_t> lists[8];
    for (int64_t p : nd.pts) {
      int ci = 0;
      for (int a = 0; a < d; ++a) ci |= (int)((q[p * d + a] >> sh) & 1) << a;
      lists[ci].push_back(p);
    }
    int32_t pc[3] = {nd.c[0], nd.c[1], nd.c[2]};
    std::vector<Key> out;
    for (int ci = 0; ci < (1 << d); ++ci) {
      if (lists[ci].empty()) continue;
      Node ch;
      for (int a = 0; a < d; ++a) ch.c[a] = 2 * pc[a] + ((ci >> a) & 1);
      ch.pts = std::move(lists[ci]);
      Key ck = key_of(lev + 1, ch.c);
      out.push_back(ck);
      nodes.emplace(ck, std::move(ch));
    }
    return out;
  }

  void extent(const Key& k, const Node& nd, int64_t* lo, int64_t* hi) const {
    const int64_t w = (int64_t)1 << (Q - k.first);
    for (int a = 0; a < d; ++a) {
      lo[a] = (int64_t)nd.c[a] * w;
      hi[a] = lo[a] + w;
    }
  }
};

bool touches(const int64_t* lo1, const int64_t* hi1, const int64_t* lo2, const int64_t* hi2,
             int d) {
  for (int a = 0; a < d; ++a)
    if (!(lo1[a] <= hi2[a] && lo2[a] <= hi1[a])) return false;
  return true;
}

}  // namespace

std::string build_tree(const double* pts, int64_t n, int dim, int leaf_size, int qbits,
                       const double* lo, double side, Tree& t) {
  if (dim != 2 && dim != 3) return "dim must be 2 or 3";
  if (n < 1) return "n must be >= 1";
  if (leaf_size < 1) return "leaf_size must be >= 1";
  if (qbits <= 0) qbits = 20;
  if (qbits > 20) return "qbits must be <= 20";
  if (!(side > 0.0) || !std::isfinite(side)) return "root_side must be finite and > 0";
  Builder B;
  B.d = dim;
  B.Q = qbits;
  B.m = leaf_size;
  B.n = n;
  B.q.resize((size_t)n * dim);
  const double scale = std::ldexp(1.0, qbits);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < dim; ++a) {
      const double x = pts[i * dim + a];
      if (!std::isfinite(x)) return "non-finite point coordinate";
      double v = (x - lo[a]) / side;
      v = v * scale;
      v = std::floor(v);
      if (v < 0.0) v = 0.0;
      if (v > scale - 1.0) v = scale - 1.0;
      B.q[i * dim + a] = (int64_t)v;
    }

  Node root;
  root.pts.resize(n);
  for (int64_t i = 0; i < n; ++i) root.pts[i] = i;
  const Key rk(0, 0);
  B.nodes.emplace(rk, std::move(root));
  std::vector<Key> frontier{rk};
  while (!frontier.empty()) {
    std::vector<Key> nxt;
    for (const Key& k : frontier) {
      const Node& nd = B.nodes[k];
      if ((int64_t)nd.pts.size() > leaf_size && k.first < qbits) {
        auto ch = B.split(k);
        nxt.insert(nxt.end(), ch.begin(), ch.end());
      }
    }
    frontier.swap(nxt);
  }

  // 2:1 balance: split every leaf whose closed box meets a leaf >= 2 levels finer.
  for (;;) {
    std::vector<Key> leaves;
    for (auto& kv : B.nodes)
      if (!kv.second.split) leaves.push_back(kv.first);
    const size_t nl = leaves.size();
    std::vector<int64_t> lo(nl * 3), hi(nl * 3);
    int maxlev = 0;
    for (size_t i = 0; i < nl; ++i) {
      B.extent(leaves[i], B.nodes[leaves[i]], &lo[i * 3], &hi[i * 3]);
      maxlev = std::max(maxlev, leaves[i].first);
    }
    // leaves grouped by level for the "two or more levels finer" scan
    std::vector<std::vector<size_t>> bylev(maxlev + 1);
    for (size_t i = 0; i < nl; ++i) bylev[leaves[i].first].push_back(i);
    std::vector<Key> marked;
    for (size_t i = 0; i < nl; ++i) {
      const int l0 = leaves[i].first;
      bool hit = false;
      for (int l1 = l0 + 2; l1 <= maxlev && !hit; ++l1)
        for (size_t j : bylev[l1])
          if (touches(&lo[i * 3], &hi[i * 3], &lo[j * 3], &hi[j * 3], dim)) {
            hit = true;
            break;
          }
      if (hit && l0 < qbits) marked.push_back(leaves[i]);
    }
    if (marked.empty()) break;
    for (const Key& k : marked) B.split(k);
  }

  // ids: map order is (level, Morton code)
  const int64_t nbox = (int64_t)B.nodes.size();
  std::map<Key, int64_t> id;
  t = Tree();
  t.dim = dim;
  t.qbits = qbits;
  t.leaf_size = leaf_size;
  t.n = n;
  t.level.resize(nbox);
  t.coords.resize(nbox * dim);
  t.parent.assign(nbox, -1);
  t.is_leaf.resize(nbox);
  t.pt_begin.assign(nbox, 0);
  t.pt_end.assign(nbox, 0);
  {
    int64_t i = 0;
    for (auto& kv : B.nodes) {
      id[kv.first] = i;
      t.level[i] = kv.first.first;
      for (int a = 0; a < dim; ++a) t.coords[i * dim + a] = kv.second.c[a];
      t.is_leaf[i] = kv.second.split ? 0 : 1;
      t.nlevels = std::max(t.nlevels, (int)kv.first.first);
      ++i;
    }
  }
  std::vector<std::vector<int64_t>> children(nbox);
  for (auto& kv : B.nodes) {
    if (kv.first.first == 0) continue;
    int32_t pc[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) pc[a] = kv.second.c[a] >> 1;
    const int64_t p = id.at(B.key_of(kv.first.first - 1, pc));
    const int64_t me = id.at(kv.first);
    t.parent[me] = p;
    children[p].push_back(me);
  }
  t.child_off.assign(nbox + 1, 0);
  for (int64_t b = 0; b < nbox; ++b) {
    std::sort(children[b].begin(), children[b].end());
    t.child_off[b + 1] = t.child_off[b] + (int64_t)children[b].size();
  }
  t.child_ids.reserve(t.child_off[nbox]);
  for (int64_t b = 0; b < nbox; ++b)
    t.child_ids.insert(t.child_ids.end(), children[b].begin(), children[b].end());

  // tree order of points: leaves by Morton code of their first finest cell
  std::vector<std::pair<uint64_t, int64_t>> lk;
  for (auto& kv : B.nodes)
    if (!kv.second.split)
      lk.emplace_back(kv.first.second << (dim * (qbits - kv.first.first)), id.at(kv.first));
  std::stable_sort(lk.begin(), lk.end(),
                   [](const auto& x, const auto& y) { return x.first < y.first; });
  t.perm.resize(n);
  {
    std::vector<const Node*> byid(nbox);
    for (auto& kv : B.nodes) byid[id.at(kv.first)] = &kv.second;
    int64_t pos = 0;
    for (auto& e : lk) {
      const int64_t b = e.second;
      t.pt_begin[b] = pos;
      for (int64_t p : byid[b]->pts) t.perm[pos++] = p;
      t.pt_end[b] = pos;
    }
  }
  for (int64_t b = nbox - 1; b >= 0; --b) {
    if (t.is_leaf[b]) continue;
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    for (int64_t j = t.child_off[b]; j < t.child_off[b + 1]; ++j) {
      mn = std::min(mn, t.pt_begin[t.child_ids[j]]);
      mx = std::max(mx, t.pt_end[t.child_ids[j]]);
    }
    t.pt_begin[b] = mn;
    t.pt_end[b] = mx;
  }

  // level lists and neighbour CSR (representatives: level-l boxes and coarser leaves)
  t.level_boxes.assign(t.nlevels + 1, {});
  for (int64_t b = 0; b < nbox; ++b) t.level_boxes[t.level[b]].push_back(b);
  t.nb_off.assign(t.nlevels + 1, {});
  t.nb_ids.assign(t.nlevels + 1, {});
  for (int lev = 1; lev <= t.nlevels; ++lev) {
    auto& off = t.nb_off[lev];
    auto& ids = t.nb_ids[lev];
    off.push_back(0);
    for (int64_t b : t.level_boxes[lev]) {
      const int64_t w = (int64_t)1 << (qbits - lev);
      int64_t blo[3], bhi[3];
      for (int a = 0; a < dim; ++a) {
        blo[a] = (int64_t)t.coords[b * dim + a] * w;
        bhi[a] = blo[a] + w;
      }
      std::vector<int64_t> found;
      for (int l1 = 0; l1 <= lev; ++l1) {
        const int64_t W = (int64_t)1 << (qbits - l1);
        const int64_t ncell = (int64_t)1 << l1;
        int64_t jlo[3] = {0, 0, 0}, jhi[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) {
          jlo[a] = std::max<int64_t>(0, (blo[a] + W - 1) / W - 1);
          jhi[a] = std::min<int64_t>(ncell - 1, bhi[a] / W);
        }
        int32_t c[3];
        for (int64_t z = (dim == 3 ? jlo[2] : 0); z <= (dim == 3 ? jhi[2] : 0); ++z)
          for (int64_t y = jlo[1]; y <= jhi[1]; ++y)
            for (int64_t x = jlo[0]; x <= jhi[0]; ++x) {
              c[0] = (int32_t)x;
              c[1] = (int32_t)y;
              c[2] = (int32_t)z;
              auto it = id.find(B.key_of(l1, c));
              if (it == id.end()) continue;
              const int64_t o = it->second;
              if (o == b) continue;
              if (l1 < lev && !t.is_leaf[o]) continue;
              found.push_back(o);
            }
      }
      std::sort(found.begin(), found.end());
      ids.insert(ids.end(), found.begin(), found.end());
      off.push_back((int64_t)ids.size());
    }
  }
  return "";
}

void make_schedule(const Tree& t, int k, Schedule& s) {
  const int64_t nbox = t.nbox();
  s = Schedule();
  s.k = k;
  s.colour.assign(nbox, -1);
  s.b_count.assign(nbox, 0);
  s.l_count.assign(nbox, 0);
  std::vector<int64_t> remaining(nbox, 0);
  std::vector<int64_t> act(nbox, 0);
  for (int lev = t.nlevels; lev >= 1; --lev) {
    const auto& boxes = t.level_boxes[lev];
    const auto& off = t.nb_off[lev];
    const auto& ids = t.nb_ids[lev];
    for (int64_t b : boxes) {
      if (t.is_leaf[b]) {
        s.b_count[b] = t.npts(b);
      } else {
        int64_t c = 0;
        for (int64_t j = t.child_off[b]; j < t.child_off[b + 1]; ++j) c += remaining[t.child_ids[j]];
        s.b_count[b] = c;
      }
    }
    // processed boxes and their closed neighbourhoods
    std::vector<size_t> proc;  // positions in `boxes`
    for (size_t i = 0; i < boxes.size(); ++i)
      if (s.b_count[boxes[i]] > k) proc.push_back(i);
    std::vector<std::pair<int64_t, int64_t>> visit;  // (pattern, id)
    for (size_t i : proc) {
      const int64_t b = boxes[i];
      int64_t pat = 0, pw = 1;
      for (int a = 0; a < t.dim; ++a) {
        pat += (int64_t)(t.coords[b * t.dim + a] % 3) * pw;
        pw *= 3;
      }
      visit.emplace_back(pat, (int64_t)i);
    }
    std::sort(visit.begin(), visit.end(), [&](const auto& x, const auto& y) {
      if (x.first != y.first) return x.first < y.first;
      return boxes[x.second] < boxes[y.second];
    });
    std::unordered_map<int64_t, std::vector<int64_t>> owners;  // member -> coloured boxes
    int ncol = 0;
    for (auto& v : visit) {
      const size_t i = (size_t)v.second;
      const int64_t b = boxes[i];
      std::vector<int64_t> closed(ids.begin() + off[i], ids.begin() + off[i + 1]);
      closed.push_back(b);
      std::vector<char> used(ncol + 1, 0);
      for (int64_t x : closed) {
        auto it = owners.find(x);
        if (it == owners.end()) continue;
        for (int64_t b2 : it->second) used[s.colour[b2]] = 1;
      }
      int c = 0;
      while (c < (int)used.size() && used[c]) ++c;
      s.colour[b] = c;
      ncol = std::max(ncol, c + 1);
      for (int64_t x : closed) owners[x].push_back(b);
    }
    std::vector<std::vector<int64_t>> classes(ncol);
    for (size_t i : proc) classes[s.colour[boxes[i]]].push_back(boxes[i]);
    for (auto& cl : classes) std::sort(cl.begin(), cl.end());
    // active counts of the representatives while this level runs
    for (int64_t b : boxes) act[b] = s.b_count[b];
    for (int64_t b = 0; b < nbox; ++b)
      if (t.is_leaf[b] && t.level[b] < lev) act[b] = t.npts(b);
    std::unordered_map<int64_t, size_t> pos;
    for (size_t i = 0; i < boxes.size(); ++i) pos[boxes[i]] = i;
    for (auto& cl : classes) {
      for (int64_t b : cl) {
        const size_t i = pos[b];
        int64_t l = s.b_count[b];
        for (int64_t j = off[i]; j < off[i + 1]; ++j) l += act[ids[j]];
        s.l_count[b] = l;
      }
      for (int64_t b : cl) act[b] = k;
    }
    for (int64_t b : boxes) remaining[b] = s.b_count[b] > k ? k : s.b_count[b];
    s.levels.push_back(lev);
    s.classes.push_back(std::move(classes));
  }
  if (t.nlevels == 0) {
    s.root_count = t.n;
  } else {
    int64_t c = 0;
    for (int64_t b : t.level_boxes[1]) c += remaining[b];
    s.root_count = c;
  }
}

int64_t samples_required(const Tree& t, const Schedule& s, int k, int p) {
  int64_t lmax = -1;
  for (int64_t b = 0; b < t.nbox(); ++b)
    if (s.colour[b] >= 0) lmax = std::max(lmax, s.l_count[b]);
  int64_t need = lmax >= 0 ? lmax + k + p : 0;
  return std::max(need, s.root_count);
}

}  // namespace rsrs

namespace rsrs {

// Algorithmic work of a fixed-rank factorization (cost terms of Sec. 4.5 for
// the steps of Algorithm 1), per processed box with b active points, n active
// neighbour points, l = b + n, k_B = min(k, b), r = b - k_B:
//   2(4 s l^2 - 4/3 l^3)   thin QR with Q of the two s x l test-matrix panels
//   8 b s l                two projections;  4 s b k_B  pivoted QR, k_B steps
//   8 r k_B s              sparsification;   4 r s l    two extractions
//   2/3 r^3                LU of X_RR;       4 r^2 (k_B + n)  K_U, K_L
//   8 r (k_B + n) s        elimination
// bytes: e s (2l + 2b + 2n) read, e s (4b + 2n) written, e (stored entries)
// with stored entries r k_B + r^2 + 2 r (k_B + n).  The symmetric variant
// halves every two-sided term (not the pivoted QR or the LU) and stores one
// multiplier.  The root adds a thin QR with Q of the s x |B_t| panel, the
// product with Y, a triangular solve and an LU; it stores |B_t|^2 entries.
void work_model(const Tree& t, const Schedule& sc, int k, int64_t s, bool sym, int esize,
                int subset_p, double* flops, double* bytes, int64_t* stored) {
  const double h = sym ? 0.5 : 1.0, ds = (double)s, e = (double)esize;
  double f = 0.0, by = 0.0;
  int64_t st = 0;
  for (const auto& lev : sc.classes)
    for (const auto& cl : lev)
      for (int64_t bx : cl) {
        const int64_t b = sc.b_count[bx], n = sc.l_count[bx] - b;
        const int64_t kb = std::min<int64_t>(k, b), r = b - kb, l = b + n;
        // columns of the nullification, ID and extraction
        const double dc = subset_p >= 0 ? (double)std::min<int64_t>(s, l + k + subset_p) : ds;
        const double db = (double)b, dn = (double)n, dk = (double)kb, dr = (double)r, dl = (double)l;
        f += h * 2.0 * (4.0 * dc * dl * dl - (4.0 / 3.0) * dl * dl * dl) + h * 8.0 * db * dc * dl +
             4.0 * dc * db * dk + h * 8.0 * dr * dk * ds + h * 4.0 * dr * dc * dl +
             (2.0 / 3.0) * dr * dr * dr + h * 4.0 * dr * dr * (dk + dn) + h * 8.0 * dr * (dk + dn) * ds;
        const int64_t sb = r * kb + r * r + (sym ? 1 : 2) * r * (kb + n);
        st += sb;
        by += h * e * (dc * (double)(2 * l + 2 * b) + ds * (double)(2 * n)) + h * e * ds * (double)(4 * b + 2 * n) +
              e * (double)sb;
      }
  const double nt = (double)sc.root_count;
  f += (4.0 * ds * nt * nt - (4.0 / 3.0) * nt * nt * nt) + 2.0 * ds * nt * nt + nt * nt * nt +
       (2.0 / 3.0) * nt * nt * nt;
  st += sc.root_count * sc.root_count;
  by += e * (2.0 * nt * ds + nt * nt);
  if (flops) *flops = f;
  if (bytes) *bytes = by;
  if (stored) *stored = st;
}

}  // namespace rsrs
