// Sparse Cholesky factorisation of the normal matrix L^T L + I_N^T I_N of the
// anchored system (Eq. 12), computed once per mesh on the host and used by
// the decoder as the preconditioner of its conjugate gradients.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mesh_host.h"

namespace dmc {

struct CholFactor {
  int32_t n = 0;
  std::vector<int32_t> perm;       // elimination position -> vertex
  int32_t nsuper = 0;
  std::vector<int32_t> sn_start;   // [nsuper+1] first column of each supernode
  std::vector<int32_t> sn_rowptr;  // [nsuper+1] into rowidx
  std::vector<int32_t> rowidx;     // rows of each supernode: its own columns, then the rest
  std::vector<int64_t> sn_valptr;  // [nsuper+1] into val: m_s x w_s row-major block
  std::vector<double> val;
  std::vector<int64_t> sn_invptr;  // [nsuper+1] into inv: w_s x w_s inverse of the diagonal block
  std::vector<double> inv;
  // Solve operator per supernode, B_s = [inv(L_ss); L_os inv(L_ss)] (m_s x w_s),
  // stored column-major (bcol, for the forward solve) and row-major (brow, for
  // the backward solve); offsets are sn_valptr.
  std::vector<double> bcol, brow;
  // update slots: rows w_s..m_s-1 of supernode s own slots
  // slot_base[s] .. slot_base[s] + m_s - w_s - 1
  std::vector<int64_t> slot_base;  // [nsuper+1]
  std::vector<int32_t> contrib_slot;  // per contribution (same order as contrib_sn)
  std::vector<int32_t> sn_parent;
  std::vector<int32_t> sn_level;   // 0 for leaves, 1 + max over children otherwise
  int32_t nlevels = 0;
  // for every column j: the (supernode d, row position i in d) pairs with
  // rowidx[d][i] == j and i >= width(d): the entries of row j left of the
  // diagonal block, in increasing d
  std::vector<int32_t> contrib_ptr;  // [n+1]
  std::vector<int32_t> contrib_sn;
  std::vector<int32_t> contrib_pos;
  // lower triangle of P M P^T by column (rows >= the column, with values):
  // the entries the numeric factorisation starts from
  std::vector<int32_t> acol_ptr, acol_row;
  std::vector<double> acol_val;
  // updates of each target supernode t: segments seg_ptr[t] .. seg_ptr[t+1]-1,
  // each the rows [p1, p2) of a descendant d whose row indices are columns of t
  // (so rows p1 .. m_d - 1 of d update t), in increasing d
  std::vector<int32_t> seg_ptr, seg_d, seg_p1, seg_p2;
  int64_t nnz_exact = 0;             // nonzeros of the exact factor
  double flops = 0.0;                // numeric factorisation flops (updates, Cholesky, inverses)
};

// Nested-dissection ordering (recursive bisection by breadth-first level
// sets of the graph of M; parts of at most `leaf` vertices end the recursion)
// followed by symbolic and numeric supernodal factorisation, one supernode per
// dissection node.  Returns false with a message if M is not numerically
// positive definite.
// With `adjacency` (the mesh's C, whose square has M's pattern) the
// dissection runs on C with two-level separators (a third of the edges to
// visit); the factor is of M either way.
bool build_cholesky(const HostCsr& M, int32_t leaf, CholFactor& f, std::string& msg,
                    const HostCsr* adjacency = nullptr);

// The ordering and symbolic part alone (everything but val, inv, bcol and
// brow): what the device factorisation starts from.
bool build_cholesky_symbolic(const HostCsr& M, int32_t leaf, CholFactor& f, std::string& msg,
                             const HostCsr* adjacency = nullptr);

// The numeric part on the host (val, inv, bcol, brow) after the symbolic one.
bool factor_numeric_host(CholFactor& f, std::string& msg);

// z = (L L^T)^{-1} r on the host, by the same blocked algorithm as the device
// solve (gather of updates, multiplication by the inverse diagonal blocks).
// r and z are [n][ncols] row-major in vertex order; they may alias.
void chol_solve_host(const CholFactor& f, int32_t ncols, const double* r, double* z);

}  // namespace dmc
