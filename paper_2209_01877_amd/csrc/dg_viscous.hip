// Viscous (Navier-Stokes) terms of eq. 11 in BR1 form for gfx950, FP64 and FP32.
//
// The paper rewrites the viscous equations with the auxiliary variable Z = grad U and
// takes the viscous interface flux in the form of Bassi and Rebay (BR1): both the
// lifting of Z and the viscous flux use central interface values.  Per element K,
// variable v, mode i, direction k:
//   |K| Z_k,i = -sum_q w_q |det J| dphi_i/dx_k U(q) + sum_f sum_q w^f_q (U- + U+)/2 N_k phi_i
//   Rv_i      = -(Vv_i - Sv_i) / |K|,   Vv_i = int_K F_v(U, Z) . grad phi_i,
//               Sv_i = sum_f int_f (F_v(U-, Z-) + F_v(U+, Z+))/2 . n phi_i
// with the inviscid ghost state as U+ on boundary faces and Z+ = Z- there.  Three kernels,
// each in the column-tile structure of the stage kernel (16 elements per wavefront, the
// same MFMA operand tables):
//   grad_kernel     : Z for the three directions (stored as 15 state-layout variables 5 k + v)
//   visc_kernel     : the volume term and the element's own half of every face term of Rv;
//                     the own half F_v(U-, Z-) . N / 2 at the face points is also stored
//   visc_nbr_kernel : adds the neighbours' halves, read from that store, to Rv
// Rv is read by the stage kernel's epilogue as an added residual.  Since the BR1 interface
// flux is an average, the face term splits into two halves; the neighbour's half at our
// face points is minus its own half at its face points (opposite normal, and two elements
// sharing a face parametrise it identically), so it is computed once, by its owner.  Each
// kernel writes only its own elements' outputs: no atomics.
#include <hip/hip_runtime.h>

#include "dg_kernels.hpp"
#include "dg_launch.hpp"
#include "dg_tile.hpp"

namespace tetdg {

namespace {

// Viscous flux F_v,j (j = 0..2, rows of Fv) at one point from U and Z[k][w] = d_k U_w,
// constant mu, Fourier heat flux with kappa = mu gamma / ((gamma - 1) Pr), T = p / rho.
template <class T>
__device__ __forceinline__ void visc_flux(const T U[5], const T Z[3][5], T gm1, T mu, T kappa, T Fv[3][5]) {
  const T ir = T(1) / U[0];
  const T u[3] = {U[1] * ir, U[2] * ir, U[3] * ir};
  const T q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T p = gm1 * (U[4] - T(0.5) * U[0] * q2);
  const T tt = p * ir;
  T gu[3][3], gT[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T ug = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      gu[k][i] = (Z[k][1 + i] - u[i] * Z[k][0]) * ir;
      ug += u[i] * gu[k][i];
    }
    const T gp = gm1 * (Z[k][4] - T(0.5) * q2 * Z[k][0] - U[0] * ug);
    gT[k] = (gp - tt * Z[k][0]) * ir;
  }
  const T div = gu[0][0] + gu[1][1] + gu[2][2];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T e = kappa * gT[j];
    Fv[j][0] = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T tij = mu * (gu[j][i] + gu[i][j]);
      if (i == j) tij -= T(2.0 / 3.0) * mu * div;
      Fv[j][1 + i] = tij;
      e += u[i] * tij;
    }
    Fv[j][4] = e;
  }
}

// FP32 up to P3 fits two waves per SIMD without spilling; FP64 and P4 take one.
template <int P, class Pr>
constexpr int visc_min_blocks() {
  return (!Pr::f64 && P <= 3) ? 2 : 1;
}

template <int P, class Pr>
constexpr bool visc_lds() {
  // at most 96 KB, and within the LDS share of each resident workgroup (160 KB per CU)
  constexpr size_t share = 160 * 1024 / visc_min_blocks<P, Pr>();
  return sizeof(typename Pr::Op) * Layout<P, 1>::n_slots * 64 <= (share < 96 * 1024 ? share : 96 * 1024);
}

// Shared prologue: tables (LDS when they fit), lane coordinates, the XCD-local sweep.
#define TDG_VISC_PROLOGUE                                                                          \
  using O = Ord<P>;                                                                                \
  using L = Layout<P, 1>;                                                                          \
  using S = typename Pr::S;                                                                        \
  using T = typename Pr::T;                                                                        \
  using Op = typename Pr::Op;                                                                      \
  using Acc = typename Pr::Acc;                                                                    \
  constexpr int NP = O::NP, NQ = O::NQ, NF = O::NF, MT = O::MT, QT = O::QT, FT = O::FT, KS = L::KS; \
  constexpr int NPQ = npq_of(NP);                                                                  \
  constexpr bool kTail4 = NP - 16 * (MT - 1) <= 4;                                                 \
  constexpr bool kLds = visc_lds<P, Pr>();                                                         \
  __shared__ Op lds_tab[kLds ? L::n_slots * 64 : 1];                                               \
  const Op* __restrict__ tab;                                                                      \
  if constexpr (kLds) {                                                                            \
    const Op* src = reinterpret_cast<const Op*>(a.tab);                                            \
    for (int i = threadIdx.x; i < L::n_slots * 64; i += blockDim.x) lds_tab[i] = src[i];           \
    __syncthreads();                                                                               \
    tab = lds_tab;                                                                                 \
  } else {                                                                                         \
    tab = reinterpret_cast<const Op*>(a.tab);                                                      \
  }                                                                                                \
  const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;                               \
  const MeshView& mv = a.mesh;                                                                     \
  const int64_t epad = mv.epad;                                                                    \
  const uint32_t quad_bytes = (uint32_t)(epad * 4 * sizeof(S));                                    \
  const uint32_t var_bytes = quad_bytes * NPQ;                                                     \
  const char* __restrict__ ubase = reinterpret_cast<const char*>(a.u);                             \
  const T gamma = T(a.gamma), gm1 = T(a.gamma - 1.0);                                              \
  T far[5];                                                                                        \
  for (int v = 0; v < 5; ++v) far[v] = T(a.far[v]);                                                \
  OperandMap<Pr, NP, KS> om;                                                                       \
  om.init(g, quad_bytes);                                                                          \
  const int nblk = gridDim.x;                                                                      \
  const int nwb = blockDim.x >> 6;                                                                 \
  const int nx = (nblk % 8 == 0) ? 8 : 1;                                                          \
  const int xcd = blockIdx.x % nx;                                                                 \
  const int64_t waves_x = (int64_t)(nblk / nx) * nwb;                                              \
  const int64_t wave_x = (int64_t)(blockIdx.x / nx) * nwb + (threadIdx.x >> 6);                    \
  const int64_t ngroups = epad / 16;                                                               \
  const int64_t chunk = (ngroups + nx - 1) / nx;                                                   \
  const int64_t g_begin = xcd * chunk;                                                             \
  const int64_t g_end = g_begin + chunk < ngroups ? g_begin + chunk : ngroups;

// Accumulate the projection of one 16-point tile: acc[mt][v] += P(mt, qt, 4 dd + j) y[dd][v].
template <class Pr, int MT, bool kTail4, class L>
__device__ __forceinline__ void project_point(const typename Pr::Op* __restrict__ tab, int qt, int j, int lane, int g,
                                              typename Pr::T (&y)[3][5], typename Pr::Acc (&acc)[MT][5]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
      if constexpr (kTail4 && Pr::f64) {
        if (mt == MT - 1) {
          tail_fma<Pr>(tab + L::proj(mt, qt, 4 * dd + j) * 64 + 16 * g, y[dd], acc[mt]);
          continue;
        }
      }
      const typename Pr::Op av = tab[L::proj(mt, qt, 4 * dd + j) * 64 + lane];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[mt][v] = mfma_tile<Pr, kTail4>(mt == MT - 1, av, y[dd][v], acc[mt][v]);
    }
}

// One direction dd of one point j of the projection: acc[mt][v] += P(mt, qt, 4 dd + j) y[v].
template <class Pr, int MT, bool kTail4, class L>
__device__ __forceinline__ void project_dir(const typename Pr::Op* __restrict__ tab, int qt, int j, int dd, int lane,
                                            int g, typename Pr::T (&y)[5], typename Pr::Acc (&acc)[MT][5]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    if constexpr (kTail4 && Pr::f64) {
      if (mt == MT - 1) {
        tail_fma<Pr>(tab + L::proj(mt, qt, 4 * dd + j) * 64 + 16 * g, y, acc[mt]);
        continue;
      }
    }
    const typename Pr::Op av = tab[L::proj(mt, qt, 4 * dd + j) * 64 + lane];
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[mt][v] = mfma_tile<Pr, kTail4>(mt == MT - 1, av, y[v], acc[mt][v]);
  }
}

// One point lk of the lift of a face tile: acc[mt][v] += L(mt, f, ft, lk) h[v].
template <class Pr, int MT, bool kTail4, class L>
__device__ __forceinline__ void lift_point(const typename Pr::Op* __restrict__ tab, int f, int ft, int lk, int lane,
                                           int g, typename Pr::T (&h)[5], typename Pr::Acc (&acc)[MT][5]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    if constexpr (kTail4 && Pr::f64) {
      if (mt == MT - 1) {
        tail_fma<Pr>(tab + L::lift(mt, f, ft, lk) * 64 + 16 * g, h, acc[mt]);
        continue;
      }
    }
    const typename Pr::Op av = tab[L::lift(mt, f, ft, lk) * 64 + lane];
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[mt][v] = mfma_tile<Pr, kTail4>(mt == MT - 1, av, h[v], acc[mt][v]);
  }
}

// Accumulate the lift of one face tile: acc[mt][v] += L(mt, f, ft, lk) fh[v][lk].
template <class Pr, int MT, bool kTail4, class L>
__device__ __forceinline__ void lift_face(const typename Pr::Op* __restrict__ tab, int f, int ft, int lane, int g,
                                          typename Pr::T (&fh)[5][4], typename Pr::Acc (&acc)[MT][5]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int lk = 0; lk < 4; ++lk) {
      if constexpr (kTail4 && Pr::f64) {
        if (mt == MT - 1) {
          typename Pr::T fl[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) fl[v] = fh[v][lk];
          tail_fma<Pr>(tab + L::lift(mt, f, ft, lk) * 64 + 16 * g, fl, acc[mt]);
          continue;
        }
      }
      const typename Pr::Op av = tab[L::lift(mt, f, ft, lk) * 64 + lane];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[mt][v] = mfma_tile<Pr, kTail4>(mt == MT - 1, av, fh[v][lk], acc[mt][v]);
    }
}

// Sum the lane groups' shares of the short last tile and place them in the accumulator
// rows of the precision (as in the stage kernel).
template <class Pr, int MT, bool kTail4>
__device__ __forceinline__ void finish_tail(int g, typename Pr::Acc (&acc)[MT][5]) {
  if constexpr (kTail4) {
    using T = typename Pr::T;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        x[j] = acc[MT - 1][v][j];
        x[j] += __shfl_xor(x[j], 16);
        x[j] += __shfl_xor(x[j], 32);
      }
      if constexpr (Pr::f64) {
        acc[MT - 1][v] = typename Pr::Acc{g == 0 ? x[0] : g == 1 ? x[1] : g == 2 ? x[2] : x[3], 0.0, 0.0, 0.0};
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[MT - 1][v][j] = x[j];
      }
    }
  }
}

// out(variable base + v) = scale * acc (all modes of the element's valid quads; padding 0).
template <class Pr, int NP, int MT>
__device__ __forceinline__ void store_tile(char* __restrict__ obase, uint32_t var_bytes, uint32_t quad_bytes, int e,
                                           int g, double scale, const typename Pr::Acc (&acc)[MT][5]) {
  using S = typename Pr::S;
  constexpr int NPQ = npq_of(NP);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int mode = 16 * mt + drow(Pr::f64, g, j);
        if ((mode >> 2) < NPQ) {
          const double x = mode < NP ? scale * double(acc[mt][v][j]) : 0.0;
          *reinterpret_cast<S*>(obase + (size_t)v * var_bytes + (uint32_t)(mode >> 2) * quad_bytes +
                                ((size_t)e * 4 + (mode & 3)) * sizeof(S)) = S(x);
        }
      }
}

// BR1 lifting: Z_k = (-int U d_k phi + sum_f int (U- + U+)/2 N_k phi) / |K|.
// Both terms are linear in the rows of M = |det J| J^-1: the volume integrand's contravariant
// components are M[d][k] U, and the face normal is N_f,k = sum_d M[d][k] n_f,d with the
// reference face normals n_0 = (1, 1, 1), n_1 = -e_0, n_2 = -e_1, n_3 = -e_2.  So one
// interpolation, one set of traces and three reference-direction sums
//   D_d = sum_q w_q dphi/dxi_d U(q) - sum_f n_f,d int_f Uhat phi
// serve all three directions: Z_k = -(sum_d M[d][k] D_d) / |K|.
template <int P, class Pr>
__global__ __launch_bounds__(256, (visc_min_blocks<P, Pr>())) void grad_kernel(ViscArgs a) {
  TDG_VISC_PROLOGUE
  char* __restrict__ zout = reinterpret_cast<char*>(a.out);
  for (int64_t grp = g_begin + wave_x; grp < g_end; grp += waves_x) {
    const int e = (int)(grp * 16 + col);
    double Md[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Md[i] = mv.M[i * epad + e];
    const int fcode = mv.fcode[e];
    int nbr[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) nbr[f] = mv.nbr[f * epad + e];
    Op bc[5][KS];
    load_operands<Pr, NP, KS>(ubase, var_bytes, (uint32_t)e * 4 * sizeof(S), om, bc);
    Acc acc[3][MT][5];  // D_d, d = reference direction
#pragma unroll
    for (int dd = 0; dd < 3; ++dd)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[dd][mt][v] = Acc{0, 0, 0, 0};
    // volume: U at the points, projected on the three reference gradients
#pragma unroll 1
    for (int qt = 0; qt < QT; ++qt) {
      Acc d[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) d[v] = Acc{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const Op av = tab[L::interp(qt, s) * 64 + lane];
#pragma unroll
        for (int v = 0; v < 5; ++v) d[v] = Pr::mfma(av, bc[v][s], d[v]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = 16 * qt + drow(Pr::f64, g, j);
        T y[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) y[v] = q < NQ ? T(d[v][j]) : T(0);
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) project_dir<Pr, MT, kTail4, L>(tab, qt, j, dd, lane, g, y, acc[dd]);
      }
    }
    // faces: Uhat = (U- + U+)/2 lifted once per face, into the directions where n_f,d != 0
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      T N[3];
      face_normal<T>(f, Md, N);
      const int nbf = f == 0 ? nbr[0] : f == 1 ? nbr[1] : f == 2 ? nbr[2] : nbr[3];
      const int fpl = (fcode >> (2 * f)) & 3;
      const int en = nbf >= 0 ? nbf : e;
      Op bn[5][KS];
      load_operands<Pr, NP, KS>(ubase, var_bytes, (uint32_t)en * 4 * sizeof(S), om, bn);
#pragma unroll 1
      for (int ft = 0; ft < FT; ++ft) {
        Acc dm[5], dp[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) dm[v] = dp[v] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const Op av = tab[L::trace(f, ft, s) * 64 + lane];
#pragma unroll
          for (int v = 0; v < 5; ++v) dm[v] = Pr::mfma(av, bc[v][s], dm[v]);
        }
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
          const bool mine = nbf >= 0 && fpl == c;
          if (__any(mine)) {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
              const Op av = tab[L::trace(c, ft, s) * 64 + lane];
#pragma unroll
              for (int v = 0; v < 5; ++v) dp[v] = Pr::mfma(av, mine ? bn[v][s] : Op(0), dp[v]);
            }
          }
        }
        // n_f,d Uhat: +Uhat for face 0 (all d), -Uhat for face f > 0 (d = f - 1)
        const T sgn = f == 0 ? T(0.5) : T(-0.5);
        T fh[5][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int q = 16 * ft + drow(Pr::f64, g, j);
          T um[5], up[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            um[v] = T(dm[v][j]);
            up[v] = T(dp[v][j]);
          }
          if (nbf < 0) ghost_state<T>(-nbf, um, N, far, up);
#pragma unroll
          for (int v = 0; v < 5; ++v) fh[v][j] = q < NF ? sgn * (um[v] + up[v]) : T(0);
        }
#pragma unroll
        for (int dd = 0; dd < 3; ++dd)
          if (f == 0 || f == dd + 1) lift_face<Pr, MT, kTail4, L>(tab, f, ft, lane, g, fh, acc[dd]);
      }
    }
    // Z_k = -(sum_d M[d][k] D_d) / |K|
    const double ivol = mv.inv_vol[e];
    T Mt[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Mt[i] = T(Md[i]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Acc z[MT][5];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            z[mt][v][j] = Mt[k] * T(acc[0][mt][v][j]) + Mt[3 + k] * T(acc[1][mt][v][j]) + Mt[6 + k] * T(acc[2][mt][v][j]);
      finish_tail<Pr, MT, kTail4>(g, z);
      if (e < mv.n_elem) store_tile<Pr, NP, MT>(zout + (size_t)(5 * k) * var_bytes, var_bytes, quad_bytes, e, g, -ivol, z);
    }
  }
}

// Viscous residual Rv = -(Vv - Sv) / |K| from U and Z.
template <int P, class Pr>
__global__ __launch_bounds__(256, (visc_min_blocks<P, Pr>())) void visc_kernel(ViscArgs a) {
  TDG_VISC_PROLOGUE
  const char* __restrict__ zbase = reinterpret_cast<const char*>(a.z);
  char* __restrict__ obase = reinterpret_cast<char*>(a.out);
  S* __restrict__ hb = reinterpret_cast<S*>(a.hbuf);
  const T mu = T(a.mu), kappa = T(a.mu * a.gamma / ((a.gamma - 1.0) * a.prandtl));
  for (int64_t grp = g_begin + wave_x; grp < g_end; grp += waves_x) {
    const int e = (int)(grp * 16 + col);
    const uint32_t eoff = (uint32_t)e * 4 * sizeof(S);
    double Md[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Md[i] = mv.M[i * epad + e];
    T Mt[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Mt[i] = T(Md[i]);
    const int fcode = mv.fcode[e];
    int nbr[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) nbr[f] = mv.nbr[f * epad + e];
    Acc acc[MT][5];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[mt][v] = Acc{0, 0, 0, 0};

    // values of U (w = 0) and Z_k (w = 1 + k) of the element at the points of a tile, by
    // table t(s), accumulated into out[w][v] (interpolation / trace contractions)
    auto gather = [&](uint32_t el_off, auto&& table, Acc (&out)[4][5]) {
      // the element's own operands are the same in every tile: an opaque offset keeps their
      // loads inside the loop (hoisted out, 20 variables x KS operands stay live and spill)
      asm volatile("" : "+v"(el_off));
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const char* src = w == 0 ? ubase : zbase + (size_t)(5 * (w - 1)) * var_bytes;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          Op b[1][KS];
          load_operands<Pr, NP, KS, 1>(src + (size_t)v * var_bytes, var_bytes, el_off, om, b);
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            const Op av = tab[table(s) * 64 + lane];
            out[w][v] = Pr::mfma(av, b[0][s], out[w][v]);
          }
        }
      }
    };
    auto zero = [&](Acc (&out)[4][5]) {
#pragma unroll
      for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int v = 0; v < 5; ++v) out[w][v] = Acc{0, 0, 0, 0};
    };
    auto point = [&](const Acc (&vals)[4][5], int j, T (&U)[5], T (&Z)[3][5]) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        U[v] = T(vals[0][v][j]);
#pragma unroll
        for (int k = 0; k < 3; ++k) Z[k][v] = T(vals[1 + k][v][j]);
      }
    };

    // ---------------- volume: Vv = int F_v(U, Z) . grad phi
#pragma unroll 1
    for (int qt = 0; qt < QT; ++qt) {
      Acc vals[4][5];
      zero(vals);
      gather(eoff, [&](int s) { return L::interp(qt, s); }, vals);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = 16 * qt + drow(Pr::f64, g, j);
        T U[5], Z[3][5], Fv[3][5];
        point(vals, j, U, Z);
        visc_flux<T>(U, Z, gm1, mu, kappa, Fv);
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
          T y[5];
#pragma unroll
          for (int v = 0; v < 5; ++v)
            y[v] = q < NQ ? Mt[3 * dd] * Fv[0][v] + Mt[3 * dd + 1] * Fv[1][v] + Mt[3 * dd + 2] * Fv[2][v] : T(0);
          project_dir<Pr, MT, kTail4, L>(tab, qt, j, dd, lane, g, y, acc);
        }
      }
    }

    // ---------------- faces: Sv = sum_f int (F_v- + F_v+)/2 . N phi, the own half here
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      T N[3];
      face_normal<T>(f, Md, N);
      const int nbf = f == 0 ? nbr[0] : f == 1 ? nbr[1] : f == 2 ? nbr[2] : nbr[3];
      const int fpl = (fcode >> (2 * f)) & 3;
#pragma unroll 1
      for (int ft = 0; ft < FT; ++ft) {
        // own half (and, on a boundary face, the ghost half with Z+ = Z-)
        {
          Acc vals[4][5];
          zero(vals);
          gather(eoff, [&](int s) { return L::trace(f, ft, s); }, vals);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int q = 16 * ft + drow(Pr::f64, g, j);
            T U[5], Z[3][5], Fv[3][5], h[5];
            point(vals, j, U, Z);
            visc_flux<T>(U, Z, gm1, mu, kappa, Fv);
#pragma unroll
            for (int v = 0; v < 5; ++v) h[v] = Fv[0][v] * N[0] + Fv[1][v] * N[1] + Fv[2][v] * N[2];
            if (nbf < 0) {
              T Ub[5];
              ghost_state<T>(-nbf, U, N, far, Ub);
              visc_flux<T>(Ub, Z, gm1, mu, kappa, Fv);
#pragma unroll
              for (int v = 0; v < 5; ++v) h[v] += Fv[0][v] * N[0] + Fv[1][v] * N[1] + Fv[2][v] * N[2];
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) h[v] = q < NF ? T(0.5) * h[v] : T(0);
            lift_point<Pr, MT, kTail4, L>(tab, f, ft, j, lane, g, h, acc);
            // the own half of an interior face, for the neighbour's side of this face: per
            // (element, face, variable) 16 FT values, the point held in register j of lane
            // group g at 16 ft + 4 g + j, so that a reader's lane gets its four points at once
            if (nbf >= 0 && e < mv.n_elem) {
#pragma unroll
              for (int v = 0; v < 5; ++v) hb[((((size_t)e * 4 + f) * 5 + v) * FT + ft) * 16 + 4 * g + j] = S(h[v]);
            }
          }
        }
      }
    }
    finish_tail<Pr, MT, kTail4>(g, acc);
    // acc = Vv - Sv (the lift tables carry the face integral's minus sign): Rv = -acc / |K|
    if (e < mv.n_elem) store_tile<Pr, NP, MT>(obase, var_bytes, quad_bytes, e, g, -mv.inv_vol[e], acc);
  }
}

// Neighbour halves of the viscous face term: Rv += -(sum_f int_f (F_v+ . N / 2) phi) / |K|
// (with the lift tables' sign), where F_v+ . N / 2 at our face point q is minus the
// neighbour's stored own half at point q of its face f+.
// Light kernel: the lift tables are read through the caches (no LDS staging), so several
// workgroups share a CU.
template <int P, class Pr>
__global__ __launch_bounds__(256) void visc_nbr_kernel(ViscArgs a) {
  using O = Ord<P>;
  using L = Layout<P, 1>;
  using S = typename Pr::S;
  using T = typename Pr::T;
  using Op = typename Pr::Op;
  using Acc = typename Pr::Acc;
  constexpr int NP = O::NP, NF = O::NF, MT = O::MT, FT = O::FT;
  constexpr int NPQ = npq_of(NP);
  constexpr bool kTail4 = NP - 16 * (MT - 1) <= 4;
  const Op* __restrict__ tab = reinterpret_cast<const Op*>(a.tab);
  const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
  const MeshView& mv = a.mesh;
  const int64_t epad = mv.epad;
  const uint32_t quad_bytes = (uint32_t)(epad * 4 * sizeof(S));
  const uint32_t var_bytes = quad_bytes * NPQ;
  const int nblk = gridDim.x;
  const int nwb = blockDim.x >> 6;
  const int nx = (nblk % 8 == 0) ? 8 : 1;
  const int xcd = blockIdx.x % nx;
  const int64_t waves_x = (int64_t)(nblk / nx) * nwb;
  const int64_t wave_x = (int64_t)(blockIdx.x / nx) * nwb + (threadIdx.x >> 6);
  const int64_t ngroups = epad / 16;
  const int64_t chunk = (ngroups + nx - 1) / nx;
  const int64_t g_begin = xcd * chunk;
  const int64_t g_end = g_begin + chunk < ngroups ? g_begin + chunk : ngroups;
  const S* __restrict__ hb = reinterpret_cast<const S*>(a.hbuf);
  char* __restrict__ obase = reinterpret_cast<char*>(a.out);
  for (int64_t grp = g_begin + wave_x; grp < g_end; grp += waves_x) {
    const int e = (int)(grp * 16 + col);
    const int fcode = mv.fcode[e];
    int nbr[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) nbr[f] = mv.nbr[f * epad + e];
    Acc acc[MT][5];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[mt][v] = Acc{0, 0, 0, 0};
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      const int nbf = f == 0 ? nbr[0] : f == 1 ? nbr[1] : f == 2 ? nbr[2] : nbr[3];
      if (!__any(nbf >= 0)) continue;
      const int fpl = (fcode >> (2 * f)) & 3;
      const size_t rec = nbf >= 0 ? ((size_t)nbf * 4 + fpl) * 5 * FT * 16 : 0;
      typedef S s4_t __attribute__((ext_vector_type(4)));
#pragma unroll 1
      for (int ft = 0; ft < FT; ++ft) {
        T h[4][5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          // the neighbour's values at points 16 ft + drow(g, j), j = 0..3 (zero past N_f)
          const s4_t x = *reinterpret_cast<const s4_t*>(hb + rec + ((size_t)v * FT + ft) * 16 + 4 * g);
#pragma unroll
          for (int j = 0; j < 4; ++j) h[j][v] = nbf >= 0 ? -T(x[j]) : T(0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) lift_point<Pr, MT, kTail4, L>(tab, f, ft, j, lane, g, h[j], acc);
      }
    }
    finish_tail<Pr, MT, kTail4>(g, acc);
    if (e < mv.n_elem) {
      const double scale = -mv.inv_vol[e];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int mode = 16 * mt + drow(Pr::f64, g, j);
            if (mode < NP) {
              S* o = reinterpret_cast<S*>(obase + (size_t)v * var_bytes + (uint32_t)(mode >> 2) * quad_bytes +
                                          ((size_t)e * 4 + (mode & 3)) * sizeof(S));
              *o = S(double(*o) + scale * double(acc[mt][v][j]));
            }
          }
    }
  }
}

template <class K>
hipError_t launch_visc_grid(K kern, const ViscArgs& a, hipStream_t stream) {
  int per_cu = 0;
  hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
  if (err != hipSuccess) return err;
  if (per_cu < 1) per_cu = 1;
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t ngroups = a.mesh.epad / 16;
  int64_t want = (ngroups + 3) / 4;
  int64_t fill = (int64_t)ncu * per_cu;
  int64_t nblk = want < fill ? want : fill;
  if (a.max_blocks > 0 && nblk > a.max_blocks) nblk = a.max_blocks;
  if (nblk >= 8) nblk -= nblk % 8;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(256), 0, stream, a);
  return hipGetLastError();
}

#undef TDG_VISC_PROLOGUE

}  // namespace

hipError_t launch_grad(int p, int prec, const ViscArgs& a, hipStream_t stream) {
#define TDG_CASE(PP)                                                                            \
  if (p == PP)                                                                                  \
    return prec == 1 ? launch_visc_grid(grad_kernel<PP, PrecF32>, a, stream)                   \
                     : launch_visc_grid(grad_kernel<PP, PrecF64>, a, stream);
  TDG_CASE(1) TDG_CASE(2) TDG_CASE(3) TDG_CASE(4)
#undef TDG_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_visc(int p, int prec, const ViscArgs& a, hipStream_t stream) {
#define TDG_CASE(PP)                                                                            \
  if (p == PP)                                                                                  \
    return prec == 1 ? launch_visc_grid(visc_kernel<PP, PrecF32>, a, stream)                   \
                     : launch_visc_grid(visc_kernel<PP, PrecF64>, a, stream);
  TDG_CASE(1) TDG_CASE(2) TDG_CASE(3) TDG_CASE(4)
#undef TDG_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_visc_nbr(int p, int prec, const ViscArgs& a, hipStream_t stream) {
#define TDG_CASE(PP)                                                                            \
  if (p == PP)                                                                                  \
    return prec == 1 ? launch_visc_grid(visc_nbr_kernel<PP, PrecF32>, a, stream)               \
                     : launch_visc_grid(visc_nbr_kernel<PP, PrecF64>, a, stream);
  TDG_CASE(1) TDG_CASE(2) TDG_CASE(3) TDG_CASE(4)
#undef TDG_CASE
  return hipErrorInvalidValue;
}

}  // namespace tetdg
