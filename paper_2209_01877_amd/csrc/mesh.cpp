// Face matching, geometry and renumbering (see mesh.hpp).
#include "mesh.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

namespace tetdg {

namespace {
struct FaceSlot {
  int64_t k0, k1, k2;
  int64_t e;
  int32_t f;
};
bool key_less(const FaceSlot& a, const FaceSlot& b) {
  if (a.k0 != b.k0) return a.k0 < b.k0;
  if (a.k1 != b.k1) return a.k1 < b.k1;
  if (a.k2 != b.k2) return a.k2 < b.k2;
  if (a.e != b.e) return a.e < b.e;
  return a.f < b.f;
}
bool key_eq(const FaceSlot& a, const FaceSlot& b) { return a.k0 == b.k0 && a.k1 == b.k1 && a.k2 == b.k2; }
}  // namespace

std::string build_topology(int64_t n, const int64_t* elem_vid, const double* elem_xyz, int64_t n_bface,
                           const int64_t* bface_vid, const int32_t* bface_tag, HostMesh& m) {
  m.n = n;
  m.vid.resize(4 * n);
  m.xyz.resize(12 * n);
  for (int64_t e = 0; e < n; ++e) {
    std::array<int, 4> ord = {0, 1, 2, 3};
    const int64_t* v = elem_vid + 4 * e;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return v[a] < v[b]; });
    for (int i = 0; i < 4; ++i) {
      m.vid[4 * e + i] = v[ord[i]];
      for (int d = 0; d < 3; ++d) m.xyz[12 * e + 3 * i + d] = elem_xyz[12 * e + 3 * ord[i] + d];
    }
    for (int i = 1; i < 4; ++i)
      if (m.vid[4 * e + i] == m.vid[4 * e + i - 1])
        return "element " + std::to_string(e) + " repeats a vertex id";
  }
  std::vector<FaceSlot> slots(4 * n);
  for (int64_t e = 0; e < n; ++e)
    for (int f = 0; f < 4; ++f) {
      int64_t k[3];
      int c = 0;
      for (int i = 0; i < 4; ++i)
        if (i != f) k[c++] = m.vid[4 * e + i];
      slots[4 * e + f] = {k[0], k[1], k[2], e, f};
    }
  std::sort(slots.begin(), slots.end(), key_less);
  std::vector<FaceSlot> bkeys(n_bface);
  for (int64_t b = 0; b < n_bface; ++b) {
    int64_t k[3] = {bface_vid[3 * b], bface_vid[3 * b + 1], bface_vid[3 * b + 2]};
    std::sort(k, k + 3);
    if (bface_tag[b] < 1 || bface_tag[b] > 2) return "boundary face " + std::to_string(b) + " has an unknown tag";
    bkeys[b] = {k[0], k[1], k[2], bface_tag[b], 0};
  }
  std::sort(bkeys.begin(), bkeys.end(), [](const FaceSlot& a, const FaceSlot& b) {
    if (a.k0 != b.k0) return a.k0 < b.k0;
    if (a.k1 != b.k1) return a.k1 < b.k1;
    return a.k2 < b.k2;
  });
  m.nbr.assign(4 * n, 0);
  m.nface.assign(4 * n, 0);
  m.n_interior = m.n_boundary = 0;
  size_t i = 0;
  while (i < slots.size()) {
    size_t j = i + 1;
    while (j < slots.size() && key_eq(slots[i], slots[j])) ++j;
    const size_t cnt = j - i;
    if (cnt > 2) return "a face is shared by more than two elements (vertex ids " + std::to_string(slots[i].k0) + ")";
    if (cnt == 2) {
      const FaceSlot &a = slots[i], &b = slots[i + 1];
      if (a.e == b.e) return "element " + std::to_string(a.e) + " meets itself across a face";
      m.nbr[4 * a.e + a.f] = b.e;
      m.nface[4 * a.e + a.f] = (uint8_t)b.f;
      m.nbr[4 * b.e + b.f] = a.e;
      m.nface[4 * b.e + b.f] = (uint8_t)a.f;
      ++m.n_interior;
    } else {
      const FaceSlot& a = slots[i];
      auto it = std::lower_bound(bkeys.begin(), bkeys.end(), a, [](const FaceSlot& x, const FaceSlot& y) {
        if (x.k0 != y.k0) return x.k0 < y.k0;
        if (x.k1 != y.k1) return x.k1 < y.k1;
        return x.k2 < y.k2;
      });
      if (it == bkeys.end() || !key_eq(*it, a))
        return "face (" + std::to_string(a.k0) + "," + std::to_string(a.k1) + "," + std::to_string(a.k2) +
               ") of element " + std::to_string(a.e) + " is unmatched and not a boundary face";
      m.nbr[4 * a.e + a.f] = -it->e;  // -tag
      ++m.n_boundary;
    }
    i = j;
  }
  return "";
}

std::string build_geometry(const HostMesh& m, std::vector<double>& M, std::vector<double>& inv_vol,
                           std::vector<double>& x0j) {
  M.resize(9 * m.n);
  inv_vol.resize(m.n);
  x0j.resize(12 * m.n);
  for (int64_t e = 0; e < m.n; ++e) {
    const double* X = &m.xyz[12 * e];
    double J[3][3];  // J[d][c] = (X_{c+1} - X0)_d
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) J[d][c] = X[3 * (c + 1) + d] - X[d];
    // cofactor matrix: inverse = adj / det
    double C[3][3];
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    double scale = 0.0;
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) scale = std::max(scale, std::fabs(J[d][c]));
    if (!(std::fabs(det) > 1e-13 * scale * scale * scale))
      return "element " + std::to_string(e) + " has (near) zero volume";
    // J^-1[r][c] = C[c][r] / det ; M = |det| J^-1 = sign(det) C^T
    const double sg = det > 0 ? 1.0 : -1.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) M[9 * e + 3 * r + c] = sg * C[c][r];
    inv_vol[e] = 6.0 / std::fabs(det);
    for (int d = 0; d < 3; ++d) {
      x0j[12 * e + d] = X[d];
      for (int c = 0; c < 3; ++c) x0j[12 * e + 3 + 3 * d + c] = J[d][c];
    }
  }
  return "";
}

namespace {

std::vector<int64_t> rcm(const HostMesh& m) {
  const int64_t n = m.n;
  auto deg = [&](int64_t e) {
    int d = 0;
    for (int f = 0; f < 4; ++f) d += m.nbr[4 * e + f] >= 0;
    return d;
  };
  std::vector<int64_t> order;
  order.reserve(n);
  std::vector<char> seen(n, 0);
  std::vector<int64_t> level(n, -1);
  // breadth-first search from `root`; returns the visit order and the last level
  auto bfs = [&](int64_t root, std::vector<int64_t>& visit) {
    visit.clear();
    std::vector<int64_t> lev;
    visit.push_back(root);
    level[root] = 0;
    size_t head = 0;
    while (head < visit.size()) {
      const int64_t e = visit[head++];
      int64_t nb[4];
      int c = 0;
      for (int f = 0; f < 4; ++f) {
        const int64_t o = m.nbr[4 * e + f];
        if (o >= 0 && level[o] < 0) {
          level[o] = level[e] + 1;
          nb[c++] = o;
        }
      }
      std::sort(nb, nb + c, [&](int64_t a, int64_t b) { return deg(a) != deg(b) ? deg(a) < deg(b) : a < b; });
      for (int i = 0; i < c; ++i) visit.push_back(nb[i]);
    }
  };
  std::vector<int64_t> visit;
  for (int64_t s = 0; s < n; ++s) {
    if (seen[s]) continue;
    // George-Liu pseudo-peripheral node: repeat BFS from a node of the last level
    int64_t root = s;
    int64_t ecc = -1;
    for (int it = 0; it < 8; ++it) {
      bfs(root, visit);
      const int64_t last = level[visit.back()];
      int64_t best = visit.back();
      for (auto it2 = visit.rbegin(); it2 != visit.rend() && level[*it2] == last; ++it2)
        if (deg(*it2) < deg(best)) best = *it2;
      for (int64_t v : visit) level[v] = -1;
      if (last <= ecc) break;
      ecc = last;
      root = best;
    }
    bfs(root, visit);
    for (int64_t v : visit) seen[v] = 1;
    order.insert(order.end(), visit.begin(), visit.end());
  }
  std::reverse(order.begin(), order.end());
  return order;
}

uint64_t spread3(uint64_t x) {
  // insert two zero bits between each of the low 21 bits
  x &= 0x1fffffULL;
  x = (x | (x << 32)) & 0x1f00000000ffffULL;
  x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
  x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
  x = (x | (x << 2)) & 0x1249249249249249ULL;
  return x;
}

// Hilbert index of a point with `bits` bits per axis (Skilling's transform of the
// coordinates into the transposed Hilbert index, then bit interleaving).
uint64_t hilbert3(uint32_t X[3], int bits) {
  const uint32_t Mbit = 1u << (bits - 1);
  for (uint32_t Q = Mbit; Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
  uint32_t t = 0;
  for (uint32_t Q = Mbit; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  for (int i = 0; i < 3; ++i) X[i] ^= t;
  uint64_t h = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> b) & 1u);
  return h;
}

std::vector<int64_t> curve(const HostMesh& m, bool hilbert) {
  const int64_t n = m.n;
  std::vector<double> c(3 * n);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t e = 0; e < n; ++e)
    for (int d = 0; d < 3; ++d) {
      double s = 0;
      for (int v = 0; v < 4; ++v) s += m.xyz[12 * e + 3 * v + d];
      c[3 * e + d] = 0.25 * s;
      lo[d] = std::min(lo[d], c[3 * e + d]);
      hi[d] = std::max(hi[d], c[3 * e + d]);
    }
  double span = 0;
  for (int d = 0; d < 3; ++d) span = std::max(span, hi[d] - lo[d]);
  if (span <= 0) span = 1;
  const int bits = 21;
  const double scale = (double)((1u << bits) - 1) / span;
  std::vector<std::pair<uint64_t, int64_t>> key(n);
  for (int64_t e = 0; e < n; ++e) {
    uint32_t X[3];
    for (int d = 0; d < 3; ++d) X[d] = (uint32_t)std::llround((c[3 * e + d] - lo[d]) * scale);
    const uint64_t k = hilbert ? hilbert3(X, bits) : (spread3(X[0]) << 2) | (spread3(X[1]) << 1) | spread3(X[2]);
    key[e] = {k, e};
  }
  std::sort(key.begin(), key.end());
  std::vector<int64_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = key[i].second;
  return order;
}

}  // namespace

// Within consecutive windows of W elements of a locality-preserving order, stable-sort
// the elements by the 8-bit code of their neighbours' local faces.  The stage kernel runs
// one MFMA chain per distinct neighbour face table present in a 16-element tile, so tiles
// with uniform codes cost less.  After a space-filling curve, W = 4096 leaves about 16
// elements per code, so most tiles are uniform, and its elements still lie in a compact
// region (about the set a device-wide sweep works on at once; much larger windows lose
// that locality).  After RCM, whose point is a small bandwidth, W = 256 keeps it small.
void group_by_face_code(const HostMesh& m, std::vector<int64_t>& order, size_t W) {
  std::vector<std::pair<int, int64_t>> key;
  for (size_t s = 0; s < order.size(); s += W) {
    const size_t t = std::min(order.size(), s + W);
    key.clear();
    for (size_t i = s; i < t; ++i) {
      const int64_t e = order[i];
      int code = 0;
      for (int f = 0; f < 4; ++f) code = (code << 2) | (m.nbr[4 * e + f] >= 0 ? m.nface[4 * e + f] : 0);
      key.push_back({code, e});
    }
    std::stable_sort(key.begin(), key.end(), [](const std::pair<int, int64_t>& a, const std::pair<int, int64_t>& b) {
      return a.first < b.first;
    });
    for (size_t i = s; i < t; ++i) order[i] = key[i - s].second;
  }
}

std::vector<int64_t> renumber(const HostMesh& m, int mode, bool group_codes) {
  std::vector<int64_t> order;
  if (mode == 1) {
    order = rcm(m);
  } else if (mode == 2) {
    order = curve(m, false);
  } else if (mode == 3) {
    order = curve(m, true);
  } else {
    order.resize(m.n);
    std::iota(order.begin(), order.end(), 0);
    return order;
  }
  if (group_codes) group_by_face_code(m, order, mode == 1 ? 256 : 4096);
  return order;
}

}  // namespace tetdg
