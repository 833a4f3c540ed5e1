// Host-side sparse Cholesky of the normal matrix of the anchored system
// (Eq. 12): nested-dissection ordering, symbolic analysis, level-parallel
// numeric factorisation, explicit inverses of the diagonal blocks.
#include "chol_host.h"

#include <omp.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <memory>
#include <numeric>

namespace dmc {
namespace {

// Recursive bisection of a graph by breadth-first level sets: the `thick`
// consecutive levels around the one that splits the vertices in half
// (counted from a pseudo-peripheral vertex) are the separator; it is
// numbered after both halves.  On the graph of M itself one level separates;
// on the mesh adjacency C, whose square is M's pattern, two do (vertices
// three or more levels apart are not coupled in M).  The two halves of the
// top kTaskDepth levels are ordered by parallel tasks, each into its own
// segment of the ordering (left half, right half, separator, as in the serial
// order); a task touches the marks of its own vertices only, and reads the
// tags of other vertices, which never carry its own tag.
struct NdOut {
  std::vector<int32_t> order;                      // this subtree's vertices in order
  std::vector<std::pair<int32_t, int32_t>> nodes;  // its dissection nodes, ranges in `order`
};

class Dissector {
 public:
  static constexpr int kTaskDepth = 6;

  Dissector(const HostCsr& G, int32_t leaf, int32_t thick)
      : G_(G), leaf_(std::max(leaf, 2)), thick_(thick), tag_(new std::atomic<int32_t>[G.n]),
        seen_(G.n, 0), lev_(G.n, 0) {
    for (int32_t v = 0; v < G.n; ++v) tag_[v].store(0, std::memory_order_relaxed);
  }

  // the ordering and the (begin, end) ranges of the dissection nodes in it
  void run(std::vector<int32_t>& order, std::vector<std::pair<int32_t, int32_t>>& nodes) {
    std::vector<int32_t> all(G_.n);
    std::iota(all.begin(), all.end(), 0);
    NdOut out;
#pragma omp parallel
#pragma omp single
    rec(all, out, 0);
    order.swap(out.order);
    nodes.swap(out.nodes);
  }

 private:
  int32_t tag(int32_t v) const { return tag_[v].load(std::memory_order_relaxed); }

  void bfs(int32_t s, int32_t member, std::vector<int32_t>& vis, int32_t& id) {
    id = bfs_id_.fetch_add(1, std::memory_order_relaxed) + 1;
    vis.clear();
    vis.push_back(s);
    seen_[s] = id;
    lev_[s] = 0;
    for (size_t h = 0; h < vis.size(); ++h) {
      const int32_t u = vis[h];
      for (int32_t e = G_.rowptr[u]; e < G_.rowptr[u + 1]; ++e) {
        const int32_t v = G_.col[e];
        if (v == u || tag(v) != member || seen_[v] == id) continue;
        seen_[v] = id;
        lev_[v] = lev_[u] + 1;
        vis.push_back(v);
      }
    }
  }

  static void leaf_of(const std::vector<int32_t>& S, NdOut& out) {
    out.nodes.emplace_back((int32_t)out.order.size(), (int32_t)(out.order.size() + S.size()));
    out.order.insert(out.order.end(), S.begin(), S.end());
  }

  // the orderings of two independent vertex sets, X's before Y's, appended
  void pair(std::vector<int32_t>& X, std::vector<int32_t>& Y, NdOut& out, int depth) {
    NdOut ox, oy;
    if (depth < kTaskDepth) {
#pragma omp task shared(X, ox)
      rec(X, ox, depth + 1);
      rec(Y, oy, depth + 1);
#pragma omp taskwait
    } else {
      rec(X, ox, depth + 1);
      rec(Y, oy, depth + 1);
    }
    for (NdOut* o : {&ox, &oy}) {
      const int32_t base = (int32_t)out.order.size();
      for (const auto& nd : o->nodes) out.nodes.emplace_back(base + nd.first, base + nd.second);
      out.order.insert(out.order.end(), o->order.begin(), o->order.end());
    }
  }

  void rec(std::vector<int32_t>& S, NdOut& out, int depth) {
    if ((int32_t)S.size() <= leaf_) {
      leaf_of(S, out);
      return;
    }
    const int32_t member = stamp_.fetch_add(1, std::memory_order_relaxed) + 1;
    for (int32_t v : S) tag_[v].store(member, std::memory_order_relaxed);
    std::vector<int32_t> vis;
    int32_t id = 0;
    bfs(S[0], member, vis, id);
    if (vis.size() < S.size()) {  // not connected: recurse per component
      std::vector<int32_t> rest;
      rest.reserve(S.size() - vis.size());
      for (int32_t v : S)
        if (seen_[v] != id) rest.push_back(v);
      std::vector<int32_t> comp(vis);
      S.clear();
      S.shrink_to_fit();
      pair(comp, rest, out, depth);
      return;
    }
    int32_t u = vis.back();
    for (int it = 0; it < 2; ++it) {
      bfs(u, member, vis, id);
      if (vis.back() == u) break;
      u = vis.back();
    }
    bfs(u, member, vis, id);
    const int32_t maxl = lev_[vis.back()];
    if (maxl < thick_ + 1) {
      leaf_of(S, out);
      return;
    }
    std::vector<int32_t> cnt(maxl + 1, 0);
    for (int32_t v : vis) cnt[lev_[v]]++;
    const int32_t half = (int32_t)S.size() / 2;
    int32_t l = 0, acc = 0;
    for (l = 0; l <= maxl; ++l) {
      acc += cnt[l];
      if (acc >= half) break;
    }
    l = std::min(std::max(l, 1), maxl - thick_);
    std::vector<int32_t> A, B, Sep;
    for (int32_t v : vis) {
      if (lev_[v] < l)
        A.push_back(v);
      else if (lev_[v] >= l + thick_)
        B.push_back(v);
      else
        Sep.push_back(v);
    }
    S.clear();
    S.shrink_to_fit();
    pair(A, B, out, depth);
    out.nodes.emplace_back((int32_t)out.order.size(), (int32_t)(out.order.size() + Sep.size()));
    out.order.insert(out.order.end(), Sep.begin(), Sep.end());
  }

  const HostCsr& G_;
  int32_t leaf_, thick_;
  std::unique_ptr<std::atomic<int32_t>[]> tag_;
  std::vector<int32_t> seen_, lev_;
  std::atomic<int32_t> stamp_{0}, bfs_id_{0};
};

struct Segment {
  int32_t d, p1, p2;  // rows [p1, p2) of supernode d fall in the target's columns
};

}  // namespace

bool build_cholesky_symbolic(const HostCsr& M, int32_t leaf, CholFactor& f, std::string& msg,
                             const HostCsr* adjacency) {
  const int32_t n = M.n;
  f = CholFactor();
  f.n = n;
  std::vector<std::pair<int32_t, int32_t>> nodes;  // (begin, end) in the ordering
  {
    Dissector dis(adjacency ? *adjacency : M, leaf, adjacency ? 2 : 1);
    dis.run(f.perm, nodes);
  }
  std::vector<int32_t> iperm(n);
  for (int32_t p = 0; p < n; ++p) iperm[f.perm[p]] = p;
  std::sort(nodes.begin(), nodes.end());

  // lower triangle of P M P^T: by column (rows >= j, with values) and by row.
  // M's pattern is symmetric, so column j's rows are the neighbours u of
  // vertex perm[j] with iperm[u] >= j, taken in increasing u (the order a
  // scan of M's rows gives), each with its value from row u; row i's columns
  // are the entries of vertex perm[i]'s row with iperm <= i, in row order.
  // Counts, then entries, both by rows and columns in parallel.
  std::vector<int32_t>& acol_ptr = f.acol_ptr;
  acol_ptr.assign(n + 1, 0);
  std::vector<int32_t> arow_ptr(n + 1, 0);
#pragma omp parallel for schedule(static, 1024)
  for (int32_t j = 0; j < n; ++j) {
    const int32_t v = f.perm[j];
    int32_t nc = 0, nr = 0;
    for (int32_t e = M.rowptr[v]; e < M.rowptr[v + 1]; ++e) {
      const int32_t q = iperm[M.col[e]];
      nc += q >= j;
      nr += q <= j;
    }
    acol_ptr[j + 1] = nc;
    arow_ptr[j + 1] = nr;
  }
  for (int32_t j = 0; j < n; ++j) {
    acol_ptr[j + 1] += acol_ptr[j];
    arow_ptr[j + 1] += arow_ptr[j];
  }
  std::vector<int32_t>& acol_row = f.acol_row;
  std::vector<double>& acol_val = f.acol_val;
  acol_row.resize(acol_ptr[n]);
  acol_val.resize(acol_ptr[n]);
  std::vector<int32_t> arow_col(arow_ptr[n]);
#pragma omp parallel for schedule(static, 1024)
  for (int32_t j = 0; j < n; ++j) {
    const int32_t v = f.perm[j];
    int32_t oc = acol_ptr[j], orr = arow_ptr[j];
    for (int32_t e = M.rowptr[v]; e < M.rowptr[v + 1]; ++e) {
      const int32_t u = M.col[e], q = iperm[u];
      if (q <= j) arow_col[orr++] = q;
      if (q >= j) {
        // M[u][v] from row u (sorted columns)
        const int32_t* c0 = M.col.data() + M.rowptr[u];
        const int32_t* c1 = M.col.data() + M.rowptr[u + 1];
        const int32_t* at = std::lower_bound(c0, c1, v);
        acol_row[oc] = q;
        acol_val[oc++] = M.val[at - M.col.data()];
      }
    }
  }
  // elimination tree (Liu, with path compression)
  std::vector<int32_t> parent(n, -1), anc(n, -1);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = arow_ptr[i]; e < arow_ptr[i + 1]; ++e) {
      int32_t r = arow_col[e];
      if (r >= i) continue;
      while (anc[r] != -1 && anc[r] != i) {
        const int32_t nx = anc[r];
        anc[r] = i;
        r = nx;
      }
      if (anc[r] == -1) {
        anc[r] = i;
        parent[r] = i;
      }
    }
  // nonzeros of the exact factor: column counts by row subtrees (each row i
  // of L is the union of the etree paths from the columns of row i of A)
  // (rows in parallel, each thread with its own marks)
  int64_t below = 0;
#pragma omp parallel reduction(+ : below)
  {
    std::vector<int32_t> mk(n, -1);
#pragma omp for schedule(static, 1024)
    for (int32_t i = 0; i < n; ++i) {
      mk[i] = i;
      for (int32_t e = arow_ptr[i]; e < arow_ptr[i + 1]; ++e)
        for (int32_t r = arow_col[e]; mk[r] != i; r = parent[r]) {
          ++below;
          mk[r] = i;
        }
    }
  }
  f.nnz_exact = (int64_t)n + below;
  std::vector<int32_t> mark(n, -1);

  // supernodes = dissection nodes; their row structures, bottom up: the rows
  // of s below its columns are those of A in its columns and those of its
  // children in the supernodal tree below their own columns (the structure of
  // a supernode is the union of its columns' structures in L)
  const int32_t ns = (int32_t)nodes.size();
  f.nsuper = ns;
  f.sn_start.resize(ns + 1);
  for (int32_t s = 0; s < ns; ++s) f.sn_start[s] = nodes[s].first;
  f.sn_start[ns] = n;
  std::vector<int32_t> sn_of(n);
  for (int32_t s = 0; s < ns; ++s)
    for (int32_t j = f.sn_start[s]; j < f.sn_start[s + 1]; ++j) sn_of[j] = s;
  f.sn_rowptr.assign(ns + 1, 0);
  std::fill(mark.begin(), mark.end(), -1);
  std::vector<std::vector<int32_t>> kids(ns);
  std::vector<int32_t> extra;
  for (int32_t s = 0; s < ns; ++s) {
    const int32_t a = f.sn_start[s], b = f.sn_start[s + 1];
    extra.clear();
    for (int32_t j = a; j < b; ++j)
      for (int32_t e = acol_ptr[j]; e < acol_ptr[j + 1]; ++e) {
        const int32_t r = acol_row[e];
        if (r >= b && mark[r] != s) {
          mark[r] = s;
          extra.push_back(r);
        }
      }
    for (int32_t c : kids[s]) {
      const int32_t wc = f.sn_start[c + 1] - f.sn_start[c];
      for (int32_t t = f.sn_rowptr[c] + wc; t < f.sn_rowptr[c + 1]; ++t) {
        const int32_t r = f.rowidx[t];
        if (r >= b && mark[r] != s) {
          mark[r] = s;
          extra.push_back(r);
        }
      }
    }
    std::sort(extra.begin(), extra.end());
    for (int32_t j = a; j < b; ++j) f.rowidx.push_back(j);
    f.rowidx.insert(f.rowidx.end(), extra.begin(), extra.end());
    f.sn_rowptr[s + 1] = (int32_t)f.rowidx.size();
    if (!extra.empty()) kids[sn_of[extra[0]]].push_back(s);
  }
  // supernodal tree and levels
  f.sn_parent.assign(ns, -1);
  f.sn_level.assign(ns, 0);
  for (int32_t s = 0; s < ns; ++s) {
    const int32_t w = f.sn_start[s + 1] - f.sn_start[s];
    const int32_t m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
    if (m > w) f.sn_parent[s] = sn_of[f.rowidx[f.sn_rowptr[s] + w]];
  }
  for (int32_t s = 0; s < ns; ++s)
    if (f.sn_parent[s] >= 0)
      f.sn_level[f.sn_parent[s]] = std::max(f.sn_level[f.sn_parent[s]], f.sn_level[s] + 1);
  f.nlevels = 0;
  for (int32_t s = 0; s < ns; ++s) f.nlevels = std::max(f.nlevels, f.sn_level[s] + 1);

  // contributions by row, and update segments by target supernode
  f.contrib_ptr.assign(n + 1, 0);
  std::vector<std::vector<Segment>> updates(ns);
  for (int32_t s = 0; s < ns; ++s) {
    const int32_t w = f.sn_start[s + 1] - f.sn_start[s];
    const int32_t r0 = f.sn_rowptr[s], r1 = f.sn_rowptr[s + 1];
    for (int32_t i = r0 + w; i < r1; ++i) f.contrib_ptr[f.rowidx[i] + 1]++;
    int32_t i = w;
    while (i < r1 - r0) {
      const int32_t t = sn_of[f.rowidx[r0 + i]];
      int32_t j = i;
      while (j < r1 - r0 && sn_of[f.rowidx[r0 + j]] == t) ++j;
      updates[t].push_back(Segment{s, i, j});
      i = j;
    }
  }
  for (int32_t j = 0; j < n; ++j) f.contrib_ptr[j + 1] += f.contrib_ptr[j];
  f.contrib_sn.resize(f.contrib_ptr[n]);
  f.contrib_pos.resize(f.contrib_ptr[n]);
  {
    std::vector<int32_t> fill(f.contrib_ptr.begin(), f.contrib_ptr.end() - 1);
    for (int32_t s = 0; s < ns; ++s) {
      const int32_t w = f.sn_start[s + 1] - f.sn_start[s];
      const int32_t r0 = f.sn_rowptr[s], r1 = f.sn_rowptr[s + 1];
      for (int32_t i = r0 + w; i < r1; ++i) {
        const int32_t r = f.rowidx[i];
        f.contrib_sn[fill[r]] = s;
        f.contrib_pos[fill[r]++] = i - r0;
      }
    }
  }

  // update segments by target, flattened (targets in order, segments in
  // increasing source supernode)
  f.seg_ptr.assign(ns + 1, 0);
  for (int32_t t = 0; t < ns; ++t) f.seg_ptr[t + 1] = f.seg_ptr[t] + (int32_t)updates[t].size();
  f.seg_d.resize(f.seg_ptr[ns]);
  f.seg_p1.resize(f.seg_ptr[ns]);
  f.seg_p2.resize(f.seg_ptr[ns]);
  for (int32_t t = 0; t < ns; ++t)
    for (size_t g = 0; g < updates[t].size(); ++g) {
      f.seg_d[f.seg_ptr[t] + g] = updates[t][g].d;
      f.seg_p1[f.seg_ptr[t] + g] = updates[t][g].p1;
      f.seg_p2[f.seg_ptr[t] + g] = updates[t][g].p2;
    }
  // block offsets, update slots, and the flops of the numeric factorisation
  f.sn_valptr.assign(ns + 1, 0);
  f.sn_invptr.assign(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s) {
    const int64_t w = f.sn_start[s + 1] - f.sn_start[s];
    const int64_t m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
    f.sn_valptr[s + 1] = f.sn_valptr[s] + m * w;
    f.sn_invptr[s + 1] = f.sn_invptr[s] + w * w;
  }
  f.slot_base.assign(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s) {
    const int64_t w = f.sn_start[s + 1] - f.sn_start[s];
    const int64_t m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
    f.slot_base[s + 1] = f.slot_base[s] + (m - w);
  }
  f.contrib_slot.resize(f.contrib_sn.size());
  for (size_t e = 0; e < f.contrib_sn.size(); ++e) {
    const int32_t d = f.contrib_sn[e];
    const int32_t wd = f.sn_start[d + 1] - f.sn_start[d];
    f.contrib_slot[e] = (int32_t)(f.slot_base[d] + f.contrib_pos[e] - wd);
  }
  double flops = 0.0;
  for (int32_t t = 0; t < ns; ++t) {
    for (int32_t g = f.seg_ptr[t]; g < f.seg_ptr[t + 1]; ++g) {
      const int32_t d = f.seg_d[g];
      const double wd = f.sn_start[d + 1] - f.sn_start[d];
      const double md = f.sn_rowptr[d + 1] - f.sn_rowptr[d];
      for (int32_t qi = f.seg_p1[g]; qi < f.seg_p2[g]; ++qi) flops += 2.0 * (md - qi) * wd;
    }
    const double w = f.sn_start[t + 1] - f.sn_start[t];
    const double m = f.sn_rowptr[t + 1] - f.sn_rowptr[t];
    flops += m * w * (w - 1) - 2.0 * w * (w - 1) * (2 * w - 1) / 6.0 + w * w * w / 3.0;
  }
  f.flops = flops;
  return true;
}

bool factor_numeric_host(CholFactor& f, std::string& msg) {
  const int32_t n = f.n, ns = f.nsuper;
  const std::vector<int32_t>& acol_ptr = f.acol_ptr;
  const std::vector<int32_t>& acol_row = f.acol_row;
  const std::vector<double>& acol_val = f.acol_val;
  f.val.assign(f.sn_valptr[ns], 0.0);
  f.inv.assign(f.sn_invptr[ns], 0.0);
  std::vector<std::vector<int32_t>> by_level(f.nlevels);
  for (int32_t s = 0; s < ns; ++s) by_level[f.sn_level[s]].push_back(s);
  int failed = -1;
  double flops = 0.0;  // counted as the loops run (f.flops holds the symbolic count)
  for (int32_t lv = 0; lv < f.nlevels && failed < 0; ++lv) {
    const std::vector<int32_t>& list = by_level[lv];
#pragma omp parallel reduction(+ : flops)
    {
      std::vector<int32_t> pos(n, -1);
#pragma omp for schedule(dynamic, 1)
      for (size_t li = 0; li < list.size(); ++li) {
        const int32_t s = list[li];
        const int32_t a = f.sn_start[s], b = f.sn_start[s + 1], w = b - a;
        const int32_t r0 = f.sn_rowptr[s], m = f.sn_rowptr[s + 1] - r0;
        const int32_t* R = f.rowidx.data() + r0;
        for (int32_t t = 0; t < m; ++t) pos[R[t]] = t;
        double* Ls = f.val.data() + f.sn_valptr[s];
        for (int32_t j = a; j < b; ++j)
          for (int32_t e = acol_ptr[j]; e < acol_ptr[j + 1]; ++e)
            Ls[(size_t)pos[acol_row[e]] * w + (j - a)] = acol_val[e];
        for (int32_t g = f.seg_ptr[s]; g < f.seg_ptr[s + 1]; ++g) {
          const Segment sg{f.seg_d[g], f.seg_p1[g], f.seg_p2[g]};
          const int32_t d = sg.d;
          const int32_t wd = f.sn_start[d + 1] - f.sn_start[d];
          const int32_t rd0 = f.sn_rowptr[d], md = f.sn_rowptr[d + 1] - rd0;
          const int32_t* Rd = f.rowidx.data() + rd0;
          const double* Ld = f.val.data() + f.sn_valptr[d];
          for (int32_t qi = sg.p1; qi < sg.p2; ++qi) {
            const int32_t colx = Rd[qi] - a;
            const double* lq = Ld + (size_t)qi * wd;
            for (int32_t ri = qi; ri < md; ++ri) {
              const double* lr = Ld + (size_t)ri * wd;
              double acc = 0.0;
              for (int32_t q = 0; q < wd; ++q) acc += lr[q] * lq[q];
              Ls[(size_t)pos[Rd[ri]] * w + colx] -= acc;
            }
            flops += 2.0 * (double)(md - qi) * wd;
          }
        }
        // dense left-looking Cholesky of the diagonal block fused with the
        // triangular solve of the rows below it
        bool ok = true;
        for (int32_t j = 0; j < w && ok; ++j) {
          const double* lj = Ls + (size_t)j * w;
          for (int32_t i = j; i < m; ++i) {
            double* li = Ls + (size_t)i * w;
            double sum = li[j];
            for (int32_t q = 0; q < j; ++q) sum -= li[q] * lj[q];
            if (i == j) {
              if (!(sum > 0.0)) {
                ok = false;
                break;
              }
              li[j] = std::sqrt(sum);
            } else {
              li[j] = sum / lj[j];
            }
          }
          flops += 2.0 * (double)(m - j) * j;
        }
        if (!ok) {
#pragma omp critical
          failed = s;
        } else {
          // inverse of the lower-triangular diagonal block, row by row
          double* Vs = f.inv.data() + f.sn_invptr[s];
          for (int32_t i = 0; i < w; ++i) {
            double* vi = Vs + (size_t)i * w;
            const double* li = Ls + (size_t)i * w;
            for (int32_t q = 0; q < i; ++q) {
              const double lq = li[q];
              const double* vq = Vs + (size_t)q * w;
              for (int32_t c = 0; c <= q; ++c) vi[c] -= lq * vq[c];
            }
            vi[i] += 1.0;
            const double inv_d = 1.0 / li[i];
            for (int32_t c = 0; c <= i; ++c) vi[c] *= inv_d;
          }
          flops += (double)w * w * w / 3.0;
        }
        for (int32_t t = 0; t < m; ++t) pos[R[t]] = -1;
      }
    }
  }
  (void)flops;
  if (failed >= 0) {
    msg = "normal matrix is not numerically positive definite (supernode " +
          std::to_string(failed) + ")";
    return false;
  }
  // solve operators B_s = [inv(L_ss); L_os inv(L_ss)] and update slots
  f.bcol.assign(f.sn_valptr[ns], 0.0);
  f.brow.assign(f.sn_valptr[ns], 0.0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t s = 0; s < ns; ++s) {
    const int32_t w = f.sn_start[s + 1] - f.sn_start[s];
    const int32_t m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
    const double* Ls = f.val.data() + f.sn_valptr[s];
    const double* Vs = f.inv.data() + f.sn_invptr[s];
    double* Br = f.brow.data() + f.sn_valptr[s];
    double* Bc = f.bcol.data() + f.sn_valptr[s];
    for (int32_t i = 0; i < w; ++i)
      for (int32_t q = 0; q <= i; ++q) Br[(size_t)i * w + q] = Vs[(size_t)i * w + q];
    for (int32_t i = w; i < m; ++i) {
      const double* li = Ls + (size_t)i * w;
      double* bi = Br + (size_t)i * w;
      for (int32_t p = 0; p < w; ++p) {
        const double lp = li[p];
        const double* vp = Vs + (size_t)p * w;
        for (int32_t q = 0; q <= p; ++q) bi[q] += lp * vp[q];
      }
    }
    for (int32_t i = 0; i < m; ++i)
      for (int32_t q = 0; q < w; ++q) Bc[(size_t)q * m + i] = Br[(size_t)i * w + q];
  }
  return true;
}

bool build_cholesky(const HostCsr& M, int32_t leaf, CholFactor& f, std::string& msg,
                    const HostCsr* adjacency) {
  return build_cholesky_symbolic(M, leaf, f, msg, adjacency) && factor_numeric_host(f, msg);
}

void chol_solve_host(const CholFactor& f, int32_t ncols, const double* r, double* z) {
  const int32_t n = f.n;
  std::vector<double> W((size_t)n * ncols), Y((size_t)n * ncols), X((size_t)n * ncols);
  std::vector<double> U((size_t)f.slot_base[f.nsuper] * ncols);
  std::vector<std::vector<int32_t>> by_level(f.nlevels);
  for (int32_t s = 0; s < f.nsuper; ++s) by_level[f.sn_level[s]].push_back(s);
  // forward: W_s = r_s - (updates from descendants); [Y_s; U_s] = B_s W_s
  for (int32_t lv = 0; lv < f.nlevels; ++lv)
    for (int32_t s : by_level[lv]) {
      const int32_t a = f.sn_start[s], w = f.sn_start[s + 1] - a;
      const int32_t m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
      for (int32_t j = a; j < a + w; ++j)
        for (int32_t c = 0; c < ncols; ++c) {
          double acc = r[(size_t)f.perm[j] * ncols + c];
          for (int32_t e = f.contrib_ptr[j]; e < f.contrib_ptr[j + 1]; ++e)
            acc -= U[(size_t)f.contrib_slot[e] * ncols + c];
          W[(size_t)j * ncols + c] = acc;
        }
      const double* Bc = f.bcol.data() + f.sn_valptr[s];
      for (int32_t i = 0; i < m; ++i)
        for (int32_t c = 0; c < ncols; ++c) {
          double acc = 0.0;
          for (int32_t q = 0; q < w; ++q) acc += Bc[(size_t)q * m + i] * W[(size_t)(a + q) * ncols + c];
          if (i < w)
            Y[(size_t)(a + i) * ncols + c] = acc;
          else
            U[(size_t)(f.slot_base[s] + i - w) * ncols + c] = acc;
        }
    }
  // backward: X_s = B_s^T [Y_s; -X_(rows of s below its diagonal block)]
  for (int32_t lv = f.nlevels - 1; lv >= 0; --lv)
    for (int32_t s : by_level[lv]) {
      const int32_t a = f.sn_start[s], w = f.sn_start[s + 1] - a;
      const int32_t rb = f.sn_rowptr[s], m = f.sn_rowptr[s + 1] - rb;
      const double* Br = f.brow.data() + f.sn_valptr[s];
      for (int32_t t = 0; t < w; ++t)
        for (int32_t c = 0; c < ncols; ++c) {
          double acc = 0.0;
          for (int32_t i = 0; i < m; ++i) {
            const double v = i < w ? Y[(size_t)(a + i) * ncols + c]
                                   : -X[(size_t)f.rowidx[rb + i] * ncols + c];
            acc += Br[(size_t)i * w + t] * v;
          }
          X[(size_t)(a + t) * ncols + c] = acc;
        }
    }
  for (int32_t j = 0; j < n; ++j)
    for (int32_t c = 0; c < ncols; ++c) z[(size_t)f.perm[j] * ncols + c] = X[(size_t)j * ncols + c];
}

}  // namespace dmc
