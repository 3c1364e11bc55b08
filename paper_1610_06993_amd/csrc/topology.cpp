// Host topology of libcgp: mesh validation, nested 1:4 subdivision (Section 2.2),
// node numbering that makes injection a prefix and interpolation a two-parent
// average (Remark 2.2, Eqs. 29-30), CSR patterns with slot maps, and element
// colouring for race-free colour-by-colour assembly on the GPU.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "internal.h"

namespace cgp {
namespace topo {

static inline uint64_t ekey(int a, int b) {
  if (a > b) std::swap(a, b);
  return (uint64_t(uint32_t(a)) << 32) | uint32_t(b);
}

cgp_status validate(int n, const double *xy, int t, const int *tri, int nb, const int *bedge, const int *bkind) {
  if (n <= 0 || t <= 0 || nb < 0 || !xy || !tri || (nb > 0 && (!bedge || !bkind))) {
    set_error("mesh: empty mesh or null array");
    return CGP_E_ARG;
  }
  std::vector<uint64_t> keys;
  keys.reserve(size_t(3) * t);
  for (int e = 0; e < t; e++) {
    const int *v = tri + 3 * size_t(e);
    for (int k = 0; k < 3; k++)
      if (v[k] < 0 || v[k] >= n) {
        set_error("mesh: triangle " + std::to_string(e) + " has a node index out of range");
        return CGP_E_MESH;
      }
    double ax = xy[2 * v[1]] - xy[2 * v[0]], ay = xy[2 * v[1] + 1] - xy[2 * v[0] + 1];
    double bx = xy[2 * v[2]] - xy[2 * v[0]], by = xy[2 * v[2] + 1] - xy[2 * v[0] + 1];
    double a2 = ax * by - bx * ay;
    if (!(a2 > 0.0)) {
      set_error("mesh: triangle " + std::to_string(e) + " is clockwise, degenerate or non-finite");
      return CGP_E_MESH;
    }
    for (int k = 0; k < 3; k++) keys.push_back(ekey(v[k], v[(k + 1) % 3]));
  }
  std::sort(keys.begin(), keys.end());
  // edge multiplicities
  std::unordered_map<uint64_t, int> boundary;  // edges used once -> tag count
  for (size_t i = 0; i < keys.size();) {
    size_t j = i;
    while (j < keys.size() && keys[j] == keys[i]) j++;
    if (j - i > 2) {
      set_error("mesh: an edge is shared by more than two triangles");
      return CGP_E_MESH;
    }
    if (j - i == 1) boundary.emplace(keys[i], 0);
    i = j;
  }
  for (int k = 0; k < nb; k++) {
    auto it = boundary.find(ekey(bedge[2 * k], bedge[2 * k + 1]));
    if (it == boundary.end() || it->second != 0 || (bkind[k] != CGP_EDGE_VEL_DIRICHLET && bkind[k] != CGP_EDGE_OUTFLOW)) {
      set_error("mesh: boundary edge " + std::to_string(k) + " is not a free edge, is repeated, or has a bad kind");
      return CGP_E_MESH;
    }
    it->second = 1;
  }
  for (auto &kv : boundary)
    if (kv.second == 0) {
      set_error("mesh: a boundary edge has no kind tag");
      return CGP_E_MESH;
    }
  return CGP_OK;
}

void edges(const HostLevel &L, std::vector<int> &edge) {
  std::vector<uint64_t> keys;
  keys.reserve(size_t(3) * L.t);
  for (int e = 0; e < L.t; e++)
    for (int k = 0; k < 3; k++) keys.push_back(ekey(L.tri[3 * size_t(e) + k], L.tri[3 * size_t(e) + (k + 1) % 3]));
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  edge.resize(2 * keys.size());
  for (size_t r = 0; r < keys.size(); r++) {
    edge[2 * r] = int(keys[r] >> 32);
    edge[2 * r + 1] = int(keys[r] & 0xffffffffu);
  }
}

void refine(const HostLevel &c, HostLevel &f) {
  const int nc = c.n, ne = c.ne;
  // midpoint numbers through a hash of the coarse edges (rank in sorted order)
  std::unordered_map<uint64_t, int> rank;
  rank.reserve(size_t(ne) * 2);
  for (int r = 0; r < ne; r++) rank.emplace(ekey(c.edge[2 * r], c.edge[2 * r + 1]), r);
  auto mid = [&](int a, int b) { return nc + rank.at(ekey(a, b)); };
  f.n = nc + ne;
  f.t = 4 * c.t;
  f.nb = 2 * c.nb;
  f.xy.resize(2 * size_t(f.n));
  std::copy(c.xy.begin(), c.xy.end(), f.xy.begin());
  f.parent.resize(2 * size_t(ne));
  for (int r = 0; r < ne; r++) {
    int a = c.edge[2 * r], b = c.edge[2 * r + 1];
    f.xy[2 * size_t(nc + r)] = (c.xy[2 * size_t(a)] + c.xy[2 * size_t(b)]) * 0.5;
    f.xy[2 * size_t(nc + r) + 1] = (c.xy[2 * size_t(a) + 1] + c.xy[2 * size_t(b) + 1]) * 0.5;
    f.parent[2 * r] = a;
    f.parent[2 * r + 1] = b;
  }
  f.tri.resize(3 * size_t(f.t));
  for (int e = 0; e < c.t; e++) {
    int v0 = c.tri[3 * size_t(e)], v1 = c.tri[3 * size_t(e) + 1], v2 = c.tri[3 * size_t(e) + 2];
    int m01 = mid(v0, v1), m12 = mid(v1, v2), m20 = mid(v2, v0);
    const int ch[12] = {v0, m01, m20, m01, v1, m12, m20, m12, v2, m01, m12, m20};
    std::memcpy(&f.tri[12 * size_t(e)], ch, sizeof ch);
  }
  f.bedge.resize(2 * size_t(f.nb));
  f.bkind.resize(size_t(f.nb));
  for (int k = 0; k < c.nb; k++) {
    int a = c.bedge[2 * k], b = c.bedge[2 * k + 1], m = mid(a, b);
    f.bedge[4 * k] = a;
    f.bedge[4 * k + 1] = m;
    f.bedge[4 * k + 2] = m;
    f.bedge[4 * k + 3] = b;
    f.bkind[2 * k] = f.bkind[2 * k + 1] = c.bkind[k];
  }
  edges(f, f.edge);
  f.ne = int(f.edge.size() / 2);
}

void csr(int n, const std::vector<int> &tri, HostCSR &A) {
  // node -> incident elements, then per row the sorted union of their nodes
  const int t = int(tri.size() / 3);
  std::vector<int> cnt(n + 1, 0), adj(tri.size());
  for (int v : tri) cnt[v + 1]++;
  std::partial_sum(cnt.begin(), cnt.end(), cnt.begin());
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  for (int e = 0; e < t; e++)
    for (int k = 0; k < 3; k++) adj[fill[tri[3 * size_t(e) + k]]++] = e;
  A.n = n;
  A.rp.assign(n + 1, 0);
  A.col.clear();
  A.col.reserve(size_t(n) * 8);
  std::vector<int> row;
  for (int i = 0; i < n; i++) {
    row.clear();
    row.push_back(i);
    for (int q = cnt[i]; q < cnt[i + 1]; q++)
      for (int k = 0; k < 3; k++) row.push_back(tri[3 * size_t(adj[q]) + k]);
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    A.col.insert(A.col.end(), row.begin(), row.end());
    A.rp[i + 1] = int(A.col.size());
  }
  A.nnz = int(A.col.size());
}

void slots(const std::vector<int> &tri, const HostCSR &A, std::vector<int> &slot) {
  const size_t t = tri.size() / 3;
  slot.resize(9 * t);
  for (size_t e = 0; e < t; e++)
    for (int a = 0; a < 3; a++) {
      int r = tri[3 * e + a];
      const int *b0 = A.col.data() + A.rp[r], *b1 = A.col.data() + A.rp[r + 1];
      for (int b = 0; b < 3; b++) slot[9 * e + 3 * a + b] = int(std::lower_bound(b0, b1, tri[3 * e + b]) - A.col.data());
    }
}

// SplitMix64 output mixing function (Steele, Lea & Flood 2014); a bijection, so no ties.
uint64_t priority(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Jones-Plassmann rounds: an uncoloured element all of whose uncoloured
// node-sharing neighbours have lower priority takes the smallest colour unused
// by its coloured neighbours.  Those are exactly its higher-priority
// neighbours, so the result equals greedy first-fit in decreasing priority.
void colour(int n, const std::vector<int> &tri, HostColouring &C) {
  const int t = int(tri.size() / 3);
  std::vector<int> cnt(n + 1, 0), adj(tri.size());
  for (int v : tri) cnt[v + 1]++;
  std::partial_sum(cnt.begin(), cnt.end(), cnt.begin());
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  for (int e = 0; e < t; e++)
    for (int k = 0; k < 3; k++) adj[fill[tri[3 * size_t(e) + k]]++] = e;
  std::vector<uint64_t> pri(t);
  for (int e = 0; e < t; e++) pri[e] = priority(uint64_t(e));
  C.colour.assign(t, -1);
  std::vector<int> todo(t), next, chosen;
  std::iota(todo.begin(), todo.end(), 0);
  C.ncol = 0;
  while (!todo.empty()) {
    next.clear();
    chosen.clear();
    for (int e : todo) {
      bool local_max = true;
      for (int k = 0; k < 3 && local_max; k++) {
        int v = tri[3 * size_t(e) + k];
        for (int q = cnt[v]; q < cnt[v + 1]; q++) {
          int o = adj[q];
          if (o != e && C.colour[o] < 0 && pri[o] > pri[e]) { local_max = false; break; }
        }
      }
      (local_max ? chosen : next).push_back(e);
    }
    for (int e : chosen) {
      uint64_t used[4] = {0, 0, 0, 0};
      for (int k = 0; k < 3; k++) {
        int v = tri[3 * size_t(e) + k];
        for (int q = cnt[v]; q < cnt[v + 1]; q++) {
          int c = C.colour[adj[q]];
          if (c >= 0) used[c >> 6] |= 1ull << (c & 63);
        }
      }
      int c = 0;
      while (used[c >> 6] >> (c & 63) & 1) c++;
      C.colour[e] = c;
      C.ncol = std::max(C.ncol, c + 1);
    }
    todo.swap(next);
  }
  C.cptr.assign(C.ncol + 1, 0);
  for (int e = 0; e < t; e++) C.cptr[C.colour[e] + 1]++;
  std::partial_sum(C.cptr.begin(), C.cptr.end(), C.cptr.begin());
  std::vector<int> pos(C.cptr.begin(), C.cptr.end() - 1);
  C.perm.resize(t);
  for (int e = 0; e < t; e++) C.perm[pos[C.colour[e]]++] = e;  // stable: ids ascending within a colour
}

}  // namespace topo
}  // namespace cgp
