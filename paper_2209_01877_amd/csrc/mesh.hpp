// Host-side mesh processing: face adjacency, boundary tags, FP64 geometry and
// element renumbering (the grid renumbering of arXiv 2209.01877, Sec. III.B).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace tetdg {

struct HostMesh {
  int64_t n = 0;                  // elements
  std::vector<int64_t> vid;       // [n][4] sorted ascending per element
  std::vector<double> xyz;        // [n][4][3] in the same (sorted) order
  std::vector<int64_t> nbr;       // [n][4] neighbour across local face f, or -tag (<= -1) on a boundary
  std::vector<uint8_t> nface;     // [n][4] neighbour's local face index (0 on boundary)
  int64_t n_interior = 0, n_boundary = 0;
};

// Sort vertices, match faces, tag boundaries.  Returns "" or an error message.
std::string build_topology(int64_t n, const int64_t* elem_vid, const double* elem_xyz, int64_t n_bface,
                           const int64_t* bface_vid, const int32_t* bface_tag, HostMesh& out);

// Per-element geometry in the mesh's order: M = |det J| J^-1 (row-major 3x3),
// inverse volume 1/|K| = 6/|det J|, and X0 with J (row-major) for point evaluation.
std::string build_geometry(const HostMesh& m, std::vector<double>& M, std::vector<double>& inv_vol,
                           std::vector<double>& x0j);

// Permutation new -> old.  mode: 0 identity, 1 RCM, 2 Morton, 3 Hilbert.  With
// group_codes the RCM/curve order is refined by grouping equal neighbour face codes
// inside windows of 256 elements.
std::vector<int64_t> renumber(const HostMesh& m, int mode, bool group_codes);

}  // namespace tetdg
