// Mesh graph construction on the host: adjacency (Eq. 2), degrees, and the
// normal matrix of the anchored system (Eq. 12).  One-off per mesh.
#include "mesh_host.h"

#include <algorithm>
#include <numeric>

namespace dmc {

bool build_adjacency(int32_t n, int32_t n_tris, const int32_t* tris, HostCsr& C,
                     std::string& msg) {
  std::vector<uint64_t> pairs;
  pairs.reserve(static_cast<size_t>(n_tris) * 6);
  for (int32_t t = 0; t < n_tris; ++t) {
    const int32_t v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    for (int e = 0; e < 3; ++e) {
      const int32_t a = v[e], b = v[(e + 1) % 3];
      if (a < 0 || a >= n || b < 0 || b >= n) {
        msg = "triangle " + std::to_string(t) + " has a vertex index out of range";
        return false;
      }
      if (a == b) continue;
      pairs.push_back((static_cast<uint64_t>(a) << 32) | static_cast<uint32_t>(b));
      pairs.push_back((static_cast<uint64_t>(b) << 32) | static_cast<uint32_t>(a));
    }
  }
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  C.n = n;
  C.rowptr.assign(n + 1, 0);
  C.col.resize(pairs.size());
  for (size_t e = 0; e < pairs.size(); ++e) {
    const int32_t a = static_cast<int32_t>(pairs[e] >> 32);
    C.col[e] = static_cast<int32_t>(pairs[e] & 0xffffffffu);
    C.rowptr[a + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) C.rowptr[i + 1] += C.rowptr[i];
  C.val.assign(pairs.size(), 1.0);
  return true;
}

void build_normal_matrix(const HostCsr& C, int32_t laplacian, const int32_t* anchors,
                         int32_t n_anchors, HostCsr& M) {
  const int32_t n = C.n;
  // Row k of L: diagonal a_k and off-diagonal b_k on each neighbour j of k.
  std::vector<double> diag(n), off(n);
  for (int32_t k = 0; k < n; ++k) {
    const double d = C.rowptr[k + 1] - C.rowptr[k];
    if (laplacian == DMC_LAP_COMBINATORIAL) {
      diag[k] = d;
      off[k] = -1.0;
    } else {
      diag[k] = 1.0;
      off[k] = -1.0 / d;
    }
  }
  std::vector<char> is_anchor(n, 0);
  for (int32_t a = 0; a < n_anchors; ++a) is_anchor[anchors[a]] = 1;
  // (L^T L)_{ab} = sum_k L_ka L_kb; L_ka != 0 iff k == a or k in ring(a).
  // Gustavson accumulation per row a over k in {a} u ring(a).
  M.n = n;
  M.rowptr.assign(n + 1, 0);
  M.col.clear();
  M.val.clear();
  std::vector<double> acc(n, 0.0);
  std::vector<int32_t> mark(n, -1), list;
  list.reserve(64);
  int32_t a = 0;
  auto add = [&](int32_t b, double v) {
    if (mark[b] != a) {
      mark[b] = a;
      list.push_back(b);
      acc[b] = 0.0;
    }
    acc[b] += v;
  };
  for (a = 0; a < n; ++a) {
    list.clear();
    // k = a: L_aa = diag[a]; row a of L has diag[a] at a and off[a] at ring(a)
    {
      const double la = diag[a];
      add(a, la * diag[a]);
      for (int32_t e = C.rowptr[a]; e < C.rowptr[a + 1]; ++e) add(C.col[e], la * off[a]);
    }
    for (int32_t e = C.rowptr[a]; e < C.rowptr[a + 1]; ++e) {
      const int32_t k = C.col[e];
      const double lka = off[k];  // a is a neighbour of k
      add(k, lka * diag[k]);
      for (int32_t f = C.rowptr[k]; f < C.rowptr[k + 1]; ++f) add(C.col[f], lka * off[k]);
    }
    if (is_anchor[a]) add(a, 1.0);
    std::sort(list.begin(), list.end());
    for (int32_t b : list) {
      M.col.push_back(b);
      M.val.push_back(acc[b]);
    }
    M.rowptr[a + 1] = static_cast<int32_t>(M.col.size());
  }
}

int32_t unanchored_components(const HostCsr& C, const int32_t* anchors, int32_t n_anchors) {
  const int32_t n = C.n;
  std::vector<int32_t> comp(n, -1), stack;
  int32_t nc = 0;
  for (int32_t s = 0; s < n; ++s) {
    if (comp[s] >= 0) continue;
    comp[s] = nc;
    stack.push_back(s);
    while (!stack.empty()) {
      const int32_t v = stack.back();
      stack.pop_back();
      for (int32_t e = C.rowptr[v]; e < C.rowptr[v + 1]; ++e) {
        const int32_t u = C.col[e];
        if (comp[u] < 0) {
          comp[u] = nc;
          stack.push_back(u);
        }
      }
    }
    ++nc;
  }
  std::vector<char> has(nc, 0);
  for (int32_t a = 0; a < n_anchors; ++a) has[comp[anchors[a]]] = 1;
  int32_t missing = 0;
  for (int32_t c = 0; c < nc; ++c) missing += has[c] ? 0 : 1;
  return missing;
}

}  // namespace dmc
