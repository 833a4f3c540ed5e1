// Driver of the host-side mesh and sparse-Cholesky code (mesh_host.cpp,
// chol_host.cpp) for a build with the address and undefined-behaviour
// sanitizers: it reads one mesh, builds the adjacency of Eq. (2), checks the
// anchored components, forms the normal matrix of Eq. (12), factorises it
// (dissection on the mesh graph, as the library does) with the given leaf
// size and solves three right-hand sides on the host,
// then prints the relative residual.
// Input file: int32 n, n_tris, n_anchors, laplacian, leaf, then the
// triangles [3 n_tris] and the anchors [n_anchors].
// Exit status: 0 solved, 2 rejected mesh, 3 unanchored component, 4 not
// positive definite, 1 bad input file.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_2111_10105_amd/csrc/chol_host.h"
#include "../../paper_2111_10105_amd/csrc/mesh_host.h"

static bool read_all(FILE* f, int32_t* p, size_t count) {
  return std::fread(p, sizeof(int32_t), count, f) == count;
}

int main(int argc, char** argv) {
  if (argc < 2) return 1;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 1;
  int32_t hdr[5];
  if (!read_all(f, hdr, 5)) return 1;
  const int32_t n = hdr[0], nt = hdr[1], nc = hdr[2], lap = hdr[3], leaf = hdr[4];
  if (n < 1 || nt < 1 || nc < 0) return 1;
  std::vector<int32_t> tris(3 * (size_t)nt), anchors(nc);
  if (!read_all(f, tris.data(), tris.size()) || !read_all(f, anchors.data(), anchors.size()))
    return 1;
  std::fclose(f);

  dmc::HostCsr C, M;
  std::string msg;
  if (!dmc::build_adjacency(n, nt, tris.data(), C, msg)) {
    std::printf("rejected: %s\n", msg.c_str());
    return 2;
  }
  const int32_t missing = dmc::unanchored_components(C, anchors.data(), nc);
  if (missing > 0) {
    std::printf("unanchored components: %d\n", missing);
    return 3;
  }
  dmc::build_normal_matrix(C, lap, anchors.data(), nc, M);
  dmc::CholFactor F;
  if (!dmc::build_cholesky(M, leaf, F, msg, &C)) {
    std::printf("not factorised: %s\n", msg.c_str());
    return 4;
  }
  const int32_t ncols = 3;
  std::vector<double> B((size_t)n * ncols), X((size_t)n * ncols);
  uint32_t state = 12345u;
  for (double& b : B) {
    state = state * 1664525u + 1013904223u;
    b = (double)(state >> 8) / 16777216.0 - 0.5;
  }
  dmc::chol_solve_host(F, ncols, B.data(), X.data());
  double rmax = 0.0, bmax = 0.0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t c = 0; c < ncols; ++c) {
      double acc = 0.0;
      for (int32_t e = M.rowptr[i]; e < M.rowptr[i + 1]; ++e)
        acc += M.val[e] * X[(size_t)M.col[e] * ncols + c];
      rmax = std::fmax(rmax, std::fabs(acc - B[(size_t)i * ncols + c]));
      bmax = std::fmax(bmax, std::fabs(B[(size_t)i * ncols + c]));
    }
  std::printf("supernodes %d levels %d resid %.3e\n", F.nsuper, F.nlevels, rmax / bmax);
  return 0;
}
