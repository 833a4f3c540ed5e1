// Mesh graph construction on the host: adjacency (Eq. 2), degrees, and the
// normal matrix of the anchored system (Eq. 12).  One-off per mesh.
#include "mesh_host.h"

#include <algorithm>
#include <numeric>

namespace dmc {

bool build_adjacency(int32_t n, int32_t n_tris, const int32_t* tris, HostCsr& C,
                     std::string& msg) {
  // half-edges bucketed by their first vertex (counting sort), then each
  // vertex's short list sorted and deduplicated
  std::vector<int32_t> cnt(static_cast<size_t>(n) + 1, 0);
  for (int32_t t = 0; t < n_tris; ++t) {
    const int32_t v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    for (int e = 0; e < 3; ++e) {
      const int32_t a = v[e], b = v[(e + 1) % 3];
      if (a < 0 || a >= n || b < 0 || b >= n) {
        msg = "triangle " + std::to_string(t) + " has a vertex index out of range";
        return false;
      }
      if (a == b) continue;
      cnt[a + 1]++;
      cnt[b + 1]++;
    }
  }
  for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> nb(cnt[n]), fill(cnt.begin(), cnt.end() - 1);
  for (int32_t t = 0; t < n_tris; ++t) {
    const int32_t v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    for (int e = 0; e < 3; ++e) {
      const int32_t a = v[e], b = v[(e + 1) % 3];
      if (a == b) continue;
      nb[fill[a]++] = b;
      nb[fill[b]++] = a;
    }
  }
  C.n = n;
  C.rowptr.assign(n + 1, 0);
  C.col.clear();
  C.col.reserve(nb.size() / 2 + 1);
  for (int32_t i = 0; i < n; ++i) {
    const auto b0 = nb.begin() + cnt[i], b1 = nb.begin() + cnt[i + 1];
    std::sort(b0, b1);
    const auto u1 = std::unique(b0, b1);
    C.col.insert(C.col.end(), b0, u1);
    C.rowptr[i + 1] = static_cast<int32_t>(C.col.size());
  }
  C.val.assign(C.col.size(), 1.0);
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
  // Gustavson accumulation per row a over k in {a} u ring(a), rows in
  // parallel, twice: the first pass counts each row's entries, the second
  // writes them at the row's place.
  M.n = n;
  M.rowptr.assign(n + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int32_t r = 0; r < n; ++r) M.rowptr[r + 1] += M.rowptr[r];
      M.col.resize(M.rowptr[n]);
      M.val.resize(M.rowptr[n]);
    }
#pragma omp parallel
    {
      std::vector<double> acc(n);
      std::vector<int32_t> mark(n, -1), list;
      list.reserve(64);
#pragma omp for schedule(static, 1024)
      for (int32_t a = 0; a < n; ++a) {
        list.clear();
        auto add = [&](int32_t b, double v) {
          if (mark[b] != a) {
            mark[b] = a;
            list.push_back(b);
            acc[b] = 0.0;
          }
          acc[b] += v;
        };
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
        if (pass == 0) {
          M.rowptr[a + 1] = static_cast<int32_t>(list.size());
          continue;
        }
        std::sort(list.begin(), list.end());
        int32_t o = M.rowptr[a];
        for (int32_t b : list) {
          M.col[o] = b;
          M.val[o++] = acc[b];
        }
      }
    }
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
