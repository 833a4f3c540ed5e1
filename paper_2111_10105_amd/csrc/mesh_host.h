// Host-side mesh graph construction (run once per mesh, before any launch).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmc.h"

namespace dmc {

struct HostCsr {
  int32_t n = 0;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
};

// Binary adjacency C of Eq. (2) from a triangle list: edge (a, b) for every
// triangle side, both directions, duplicates merged, self loops dropped; column
// indices sorted within each row.  Returns false (with msg) on an index out of
// range.
bool build_adjacency(int32_t n, int32_t n_tris, const int32_t* tris, HostCsr& C,
                     std::string& msg);

// L^T L + I_N^T I_N for the Laplacian of Eq. (3) (uniform, L = I - D^-1 C) or
// Eq. (1) (combinatorial, L = D - C), with sorted column indices.
void build_normal_matrix(const HostCsr& C, int32_t laplacian, const int32_t* anchors,
                         int32_t n_anchors, HostCsr& M);

// Connected components of C; returns the number of components without an
// anchor.
int32_t unanchored_components(const HostCsr& C, const int32_t* anchors, int32_t n_anchors);

}  // namespace dmc
