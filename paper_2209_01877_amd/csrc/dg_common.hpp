// Shared compile-time description of the DG kernels: order-dependent sizes,
// the MFMA precision traits and the packed operand-table layout.  Included by
// the HIP kernels and by the host code that packs the tables.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tetdg {

template <int P>
struct Ord {
  static constexpr int NP = (P + 1) * (P + 2) * (P + 3) / 6;  // modes
  static constexpr int NQ = (P + 1) * (P + 1) * (P + 1);      // volume points
  static constexpr int NF = (P + 1) * (P + 1);                // points per face
  static constexpr int MT = (NP + 15) / 16;                   // 16-row tiles of modes
  static constexpr int QT = (NQ + 15) / 16;                   // 16-row tiles of volume points
  static constexpr int FT = (NF + 15) / 16;                   // 16-row tiles per face
};

// Operand tables: one "slot" = the A operand of one MFMA for all 64 lanes.  With
// KW == 1 (16x16x4 f64/f32) lane l holds A[l % 16][l / 16]; with KW == 8
// (16x16x32 bf16/f16) lane l holds A[l % 16][8 (l / 16) + m], m = 0..7.
//
// D-row map: lane group g = l / 16, accumulator element j holds output row
// drow(g, j): g + 4 j for the f64 instruction, 4 g + j for the f32-accumulating ones.
inline constexpr int drow(bool f64, int g, int j) { return f64 ? g + 4 * j : 4 * g + j; }

template <int P, int KW>
struct Layout {
  using O = Ord<P>;
  static constexpr int KS = KW == 1 ? (O::NP + 3) / 4 : (O::NP + 31) / 32;  // k-steps over modes
  static constexpr int PK = KW == 1 ? 12 : 2;   // projection k-steps per (mode tile, point tile)
  static constexpr int LK = KW == 1 ? 4 : 1;    // lift k-steps per (mode tile, face, face tile)
  static constexpr int n_interp = O::QT * KS;
  static constexpr int n_trace = 4 * O::FT * KS;
  static constexpr int n_proj = O::MT * O::QT * PK;
  static constexpr int n_lift = O::MT * 4 * O::FT * LK;
  static constexpr int off_interp = 0;
  static constexpr int off_trace = off_interp + n_interp;
  static constexpr int off_proj = off_trace + n_trace;
  static constexpr int off_lift = off_proj + n_proj;
  static constexpr int n_slots = off_lift + n_lift;
  __host__ __device__ static constexpr int interp(int qt, int s) { return off_interp + qt * KS + s; }
  __host__ __device__ static constexpr int trace(int f, int ft, int s) { return off_trace + (f * O::FT + ft) * KS + s; }
  __host__ __device__ static constexpr int proj(int mt, int qt, int pk) { return off_proj + (mt * O::QT + qt) * PK + pk; }
  __host__ __device__ static constexpr int lift(int mt, int f, int ft, int lk) {
    return off_lift + ((mt * 4 + f) * O::FT + ft) * LK + lk;
  }
};

// Adjoint (VJP) tables (f64 or f32, 16x16x4 operand layout).
//   interp(qt, s)    : A[point][mode] = phi_m(xi_q)              (as the forward tables)
//   trace(f, ft, s)  : A[point][mode] = phi_m(xi_f(q))
//   tinterp(qt, d, s): A[point][mode] = w_q dphi_m/dxi_d(xi_q)
//   ttrace(f, ft, s) : A[point][mode] = w^f_q phi_m(xi_f(q))
//   tproj(mt, qt, j) : A[mode][point] = phi_m(xi_q)   (point values -> modes, accumulator order)
//   tlift(mt,f,ft,j) : A[mode][point] = phi_m(xi_f(q))
template <int P>
struct VjpLayout {
  using O = Ord<P>;
  static constexpr int KS = (O::NP + 3) / 4;
  static constexpr int n_interp = O::QT * KS;
  static constexpr int n_trace = 4 * O::FT * KS;
  static constexpr int n_tinterp = O::QT * 3 * KS;
  static constexpr int n_ttrace = 4 * O::FT * KS;
  static constexpr int n_tproj = O::MT * O::QT * 4;
  static constexpr int n_tlift = O::MT * 4 * O::FT * 4;
  static constexpr int off_interp = 0;
  static constexpr int off_trace = off_interp + n_interp;
  static constexpr int off_tinterp = off_trace + n_trace;
  static constexpr int off_ttrace = off_tinterp + n_tinterp;
  static constexpr int off_tproj = off_ttrace + n_ttrace;
  static constexpr int off_tlift = off_tproj + n_tproj;
  static constexpr int n_slots = off_tlift + n_tlift;
  __host__ __device__ static constexpr int interp(int qt, int s) { return off_interp + qt * KS + s; }
  __host__ __device__ static constexpr int trace(int f, int ft, int s) { return off_trace + (f * O::FT + ft) * KS + s; }
  __host__ __device__ static constexpr int tinterp(int qt, int d, int s) { return off_tinterp + (qt * 3 + d) * KS + s; }
  __host__ __device__ static constexpr int ttrace(int f, int ft, int s) { return off_ttrace + (f * O::FT + ft) * KS + s; }
  __host__ __device__ static constexpr int tproj(int mt, int qt, int j) { return off_tproj + (mt * O::QT + qt) * 4 + j; }
  __host__ __device__ static constexpr int tlift(int mt, int f, int ft, int j) {
    return off_tlift + ((mt * 4 + f) * O::FT + ft) * 4 + j;
  }
};

// Internal state layout: [5 variables][ceil(N_p / 4) mode quads][epad elements][4 modes].
// Four consecutive modes of one element are contiguous, so the four lane groups of an
// MFMA column (which hold modes 4s .. 4s+3 of one element) read one 32-byte run, and a
// neighbour's coefficients touch a quarter of the cache lines of a plain plane layout.
inline constexpr int npq_of(int np) { return (np + 3) / 4; }
__host__ __device__ inline int64_t sidx(int v, int mode, int64_t e, int64_t epad, int npq) {
  return (((int64_t)v * npq + (mode >> 2)) * epad + e) * 4 + (mode & 3);
}

// Device mesh view (structure of arrays, element index fastest, padded length epad).
struct MeshView {
  const double* M;       // [9][epad]  |det J| J^-1, row-major 3x3
  const double* inv_vol; // [epad]     1/|K|
  const int32_t* nbr;    // [4][epad]  neighbour internal index, or -1 farfield / -2 slip wall
  const int32_t* fcode;  // [epad]     bits 2f..2f+1: neighbour's local face across face f
  const int32_t* perm;   // [epad]     internal -> caller index (padding -> 0)
  const double* x0j;     // [12][epad] X0 (3) and J (row-major 9)
  int64_t n_elem, epad;
};

}  // namespace tetdg
