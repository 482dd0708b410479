// MFMA column-tile helpers shared by the stage kernel and the viscous kernels: where a
// lane finds its coefficient operands, and the short-last-tile contraction of the FP32
// and FP64 paths.  Header-only, included by the .hip files.
#pragma once
#include <hip/hip_runtime.h>

#include "dg_kernels.hpp"

namespace tetdg {

// Per-lane offsets (bytes, relative to the state base) of the coefficient planes a
// lane reads for its MFMA B operands: with KW = 1 lane group g holds mode 4 s + g of
// k-step s; with KW = 8 it holds modes 32 s + 8 g + m.  Modes past N_p (and mode 0 in
// the mixed modes, whose mean is added separately) are clamped to a valid plane and
// zeroed after the load, so every load is unconditional.
template <class Pr, int NP, int KS>
struct OperandMap {
  static constexpr int NV = Pr::KW == 1 ? KS : 8 * KS;  // loads per variable
  uint32_t off[NV];                                     // mode offset within a variable, bytes
  bool keep[NV];
  __device__ void init(int g, uint32_t quad_bytes) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int mode = Pr::KW == 1 ? 4 * i + g : 32 * (i / 8) + 8 * g + (i % 8);
      const int mc = mode < NP ? mode : NP - 1;
      keep[i] = mode < NP && !(Pr::mixed && mode == 0);
      off[i] = (uint32_t)(mc >> 2) * quad_bytes + (uint32_t)(mc & 3) * sizeof(typename Pr::S);
    }
  }
};

template <class Pr, int NP, int KS, int NV = 5>
__device__ __forceinline__ void load_operands(const char* __restrict__ base, uint32_t var_bytes, uint32_t elem_off,
                                              const OperandMap<Pr, NP, KS>& om, typename Pr::Op (&b)[NV][KS]) {
  using S = typename Pr::S;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const char* vb = base + (size_t)v * var_bytes;
    if constexpr (Pr::KW == 1) {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const S x = *reinterpret_cast<const S*>(vb + om.off[s] + elem_off);
        b[v][s] = om.keep[s] ? typename Pr::Op(x) : typename Pr::Op(0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int i = 8 * s + m;
          const double x = double(*reinterpret_cast<const S*>(vb + om.off[i] + elem_off));
          b[v][s][m] = (typename Pr::E1)(om.keep[i] ? float(x) : 0.0f);
        }
    }
  }
}

// Projection / lift MFMA for one mode tile: the 4x4x1 block form for the short last
// tile of the fp32 path (see kTail4; fp64 handles that tile with tail_fma), else the
// precision's 16x16 instruction.
template <class Pr, bool kTail4>
__device__ __forceinline__ typename Pr::Acc mfma_tile(bool last, typename Pr::Op a, typename Pr::Op b,
                                                      typename Pr::Acc c) {
  if constexpr (kTail4 && !Pr::f64) {
    if (last) return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
  }
  return Pr::mfma(a, b, c);
}

// FP64 short last tile: acc[v][r] += A[r] y[v] for the tile's modes r = 0..3, with the
// four table values of this lane group's point read once (a broadcast within the group).
template <class Pr>
__device__ __forceinline__ void tail_fma(const typename Pr::Op* __restrict__ t, const typename Pr::T (&y)[5],
                                         typename Pr::Acc (&acc)[5]) {
  const double a0 = t[0], a1 = t[1], a2 = t[2], a3 = t[3];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    acc[v][0] = __builtin_fma(a0, y[v], acc[v][0]);
    acc[v][1] = __builtin_fma(a1, y[v], acc[v][1]);
    acc[v][2] = __builtin_fma(a2, y[v], acc[v][2]);
    acc[v][3] = __builtin_fma(a3, y[v], acc[v][3]);
  }
}

}  // namespace tetdg
