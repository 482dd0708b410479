// Fused element-centric DG residual + SSP-RK3 stage kernel for gfx950.
//
// One wavefront owns 16 elements at a time (the 16 columns of a 16x16 MFMA tile).
// Every contraction of the residual is a small dense matrix (reference table)
// times the 16 elements' coefficient or point-value columns, one MFMA per k-step
// and conserved variable:
//   volume values   U_q      = B  c       (points x modes)          -> pointwise flux
//   volume integral V_i     += sum_q,d w_q dphi_i/dxi_d (M F(U_q))_d  (modes x points)
//   own traces      U-_fq    = B_f c
//   neighbour trace U+_fq    = B_{f+} c+  (f+ = neighbour's local face; the four
//                                          possible tables are applied and selected per lane)
//   face integral   V_i     -= sum_q w_q phi_i(xi_f(q)) Fhat_N(U-, U+)
// and the MFMA accumulator layout of one contraction is fed directly as the B
// operand of the next (the table k-order is permuted on the host to match), so
// point values never leave registers.  Each element computes its four faces from
// its own and its neighbours' coefficients: the face integral reaches both
// neighbours without atomics or a face buffer (the cell-based gather of the
// paper's Sec. III.A, with the face flux recomputed on both sides).
//
// Epilogue: R = (V - S) / |K| (orthonormal basis, affine map: M_K = |K| I), then either
// R is stored (residual) or U_out = a U0 + (1 - a)(U_in + dt R) (SSP-RK3 stage).
//
// Mixed precisions (bf16 / fp16 operands, fp32 accumulation and fluxes) split
// every quantity into its cell-mean part and a deviation: phi_0 = 1, so the
// mean coefficient c_0 is added in fp32 after the low-precision contraction of
// c_1..; the pointwise fluxes enter the projections as deviations from the flux
// of the cell means, whose own projection uses fp64 moments in the epilogue.
// A uniform state therefore gives exactly zero deviation terms.
#include <hip/hip_runtime.h>

#include "dg_kernels.hpp"
#include "dg_launch.hpp"

namespace tetdg {

// Per-lane offsets (bytes, relative to the state base) of the coefficient planes a
// lane reads for its MFMA B operands: with KW = 1 lane group g holds mode 4 s + g of
// k-step s; with KW = 8 it holds modes 32 s + 8 g + m.  Modes past N_p (and mode 0 in
// the mixed modes, whose mean is added separately) are clamped to a valid plane and
// zeroed after the load, so every load is unconditional.
template <class Pr, int NP, int KS>
struct OperandMap {
  static constexpr int NV = Pr::KW == 1 ? KS : 8 * KS;  // loads per variable
  uint32_t off[NV];                                     // plane offset, bytes
  bool keep[NV];
  __device__ void init(int g, uint32_t plane_bytes) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int mode = Pr::KW == 1 ? 4 * i + g : 32 * (i / 8) + 8 * g + (i % 8);
      keep[i] = mode < NP && !(Pr::mixed && mode == 0);
      off[i] = (uint32_t)(mode < NP ? mode : NP - 1) * plane_bytes;
    }
  }
};

template <class Pr, int NP, int KS>
__device__ __forceinline__ void load_operands(const char* __restrict__ base, uint32_t var_bytes, uint32_t elem_off,
                                              const OperandMap<Pr, NP, KS>& om, typename Pr::Op (&b)[5][KS]) {
  using S = typename Pr::S;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
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

// Two workgroups per CU (two waves per SIMD, at most 256 registers per lane) where the
// live state fits; fp64 and P4 keep one (their tables and operands need the registers).
template <int P, class Pr>
constexpr int stage_min_blocks() {
  return (P <= 3 && !Pr::f64) ? 2 : 1;
}

template <int P, class Pr, bool kLds>
__global__ __launch_bounds__(256, (stage_min_blocks<P, Pr>())) void stage_kernel(StageArgs a) {
  using O = Ord<P>;
  using L = Layout<P, Pr::KW>;
  using S = typename Pr::S;
  using T = typename Pr::T;
  using Op = typename Pr::Op;
  using Acc = typename Pr::Acc;
  constexpr int NP = O::NP, NQ = O::NQ, NF = O::NF, MT = O::MT, QT = O::QT, FT = O::FT, KS = L::KS;

  __shared__ Op lds_tab[kLds ? L::n_slots * 64 : 1];
  const Op* __restrict__ tab;
  if constexpr (kLds) {
    const Op* src = reinterpret_cast<const Op*>(a.tab);
    for (int i = threadIdx.x; i < L::n_slots * 64; i += blockDim.x) lds_tab[i] = src[i];
    __syncthreads();
    tab = lds_tab;
  } else {
    tab = reinterpret_cast<const Op*>(a.tab);
  }

  const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
  const char* __restrict__ ubase = reinterpret_cast<const char*>(a.u_in);
  const MeshView& mv = a.mesh;
  const int64_t epad = mv.epad;
  const uint32_t plane = (uint32_t)(epad * sizeof(S));  // bytes of one (variable, mode) plane
  const uint32_t var_bytes = plane * NP;
  const T gamma = T(a.gamma), gm1 = T(a.gamma - 1.0);
  T far[5];
  double far64[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    far64[v] = a.far[v];
    far[v] = T(a.far[v]);
  }
  OperandMap<Pr, NP, KS> om;
  om.init(g, plane);

  // Work distribution: workgroups are dispatched round-robin over the 8 XCDs, so block b
  // runs on XCD b % 8.  Each XCD owns one contiguous eighth of the 16-element groups and
  // its wavefronts sweep that range together (group = start + k * waves + wave), so at any
  // time an XCD's waves work on a narrow window of consecutive elements whose own and
  // neighbour coefficients fit in that XCD's L2.
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

  for (int64_t grp = g_begin + wave_x; grp < g_end; grp += waves_x) {
    const int e = (int)(grp * 16 + col);
    const uint32_t eoff = (uint32_t)e * sizeof(S);
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

    Op bc[5][KS];
    T c0t[5], ybar[3][5];
    if constexpr (Pr::mixed) {
      const Op* q = reinterpret_cast<const Op*>(a.q_in);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
#pragma unroll
        for (int s = 0; s < KS; ++s) bc[v][s] = q[(((int64_t)e * 5 + v) * KS + s) * 4 + g];
        c0t[v] = a.c0_in[v * epad + e];
      }
      contra_flux<T>(c0t, Mt, gm1, ybar);
    } else {
      load_operands<Pr, NP, KS>(ubase, var_bytes, eoff, om, bc);
    }

    Acc acc[MT][5];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[mt][v] = Acc{0, 0, 0, 0};

    // ------------------------------------------------------------ volume integral
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
      // contravariant flux (minus the cell-mean flux in the mixed modes) at point j of this tile
      auto point_flux = [&](int j, T yy[3][5]) {
        const int q = 16 * qt + drow_of<Pr>(g, j);
        T u[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) u[v] = T(d[v][j]) + (Pr::mixed ? c0t[v] : T(0));
        if (q < NQ) {
          contra_flux<T>(u, Mt, gm1, yy);
        } else {
#pragma unroll
          for (int dd = 0; dd < 3; ++dd)
#pragma unroll
            for (int v = 0; v < 5; ++v) yy[dd][v] = Pr::mixed ? ybar[dd][v] : T(0);
        }
        if constexpr (Pr::mixed) {
          // a point carrying exactly the cell mean has zero deviation (independent of how
          // the compiler schedules the two flux evaluations)
          bool mean = true;
#pragma unroll
          for (int v = 0; v < 5; ++v) mean = mean && (u[v] == c0t[v]);
#pragma unroll
          for (int dd = 0; dd < 3; ++dd)
#pragma unroll
            for (int v = 0; v < 5; ++v) yy[dd][v] = mean ? T(0) : yy[dd][v] - ybar[dd][v];
        }
      };
      if constexpr (Pr::KW == 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          T yy[3][5];
          point_flux(j, yy);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
              const Op av = tab[L::proj(mt, qt, 4 * dd + j) * 64 + lane];
#pragma unroll
              for (int v = 0; v < 5; ++v) acc[mt][v] = Pr::mfma(av, Pr::op1(yy[dd][v]), acc[mt][v]);
            }
        }
      } else {
#pragma unroll
        for (int jp = 0; jp < 2; ++jp) {
          T ya[3][5], yb[3][5];
          point_flux(2 * jp, ya);
          point_flux(2 * jp + 1, yb);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            Op b;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
              const int dd = m & 3;
              b[m] = (typename Pr::E1)(dd == 3 ? T(0) : (m < 4 ? ya[dd][v] : yb[dd][v]));
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
              acc[mt][v] = Pr::mfma(tab[L::proj(mt, qt, jp) * 64 + lane], b, acc[mt][v]);
          }
        }
      }
    }

    // ------------------------------------------------------------ face integrals
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      T N[3];
      if constexpr (Pr::mixed) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
          N[c] = f == 0 ? (Mt[c] + Mt[3 + c] + Mt[6 + c]) : f == 1 ? -Mt[c] : f == 2 ? -Mt[3 + c] : -Mt[6 + c];
      } else {
        face_normal<T>(f, Md, N);
      }
      const T nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
      const int nbf = f == 0 ? nbr[0] : f == 1 ? nbr[1] : f == 2 ? nbr[2] : nbr[3];
      const int fpl = (fcode >> (2 * f)) & 3;
      const int en = nbf >= 0 ? nbf : e;
      const uint32_t enoff = (uint32_t)en * sizeof(S);
      Op bn[5][KS];
      T c0n[5], fhbar[5];
      if constexpr (Pr::mixed) {
        const Op* q = reinterpret_cast<const Op*>(a.q_in);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
#pragma unroll
          for (int s = 0; s < KS; ++s) bn[v][s] = q[(((int64_t)en * 5 + v) * KS + s) * 4 + g];
          c0n[v] = a.c0_in[v * epad + en];
        }
        if (nbf < 0) ghost_state<T>(-nbf, c0t, N, far, c0n);
        num_flux<T>(a.flux, c0t, c0n, N, nn, gamma, fhbar);
      } else {
        load_operands<Pr, NP, KS>(ubase, var_bytes, enoff, om, bn);
      }
#pragma unroll 1
      for (int ft = 0; ft < FT; ++ft) {
        Acc dm[5], dp[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) dm[v] = dp[v] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const Op av = tab[L::trace(f, ft, s) * 64 + lane];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            Op own = bc[v][s];
            if constexpr (Pr::mixed)
              own = reinterpret_cast<const Op*>(a.q_in)[(((int64_t)e * 5 + v) * KS + s) * 4 + g];
            dm[v] = Pr::mfma(av, own, dm[v]);
          }
        }
        // neighbour trace B_{f+} c+: the table depends on the neighbour's local face f+, which
        // varies by column; for every f+ present in the 16 columns the B operand is masked to
        // the columns having that f+, so all candidates accumulate into one result
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
          const bool mine = nbf >= 0 && fpl == c;
          if (__any(mine)) {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
              const Op av = tab[L::trace(c, ft, s) * 64 + lane];
#pragma unroll
              for (int v = 0; v < 5; ++v) dp[v] = Pr::mfma(av, mine ? bn[v][s] : Op{}, dp[v]);
            }
          }
        }
        T fh[5][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int q = 16 * ft + drow_of<Pr>(g, j);
          T um[5], up[5], fl[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            um[v] = T(dm[v][j]) + (Pr::mixed ? c0t[v] : T(0));
            up[v] = T(dp[v][j]) + (Pr::mixed ? c0n[v] : T(0));
          }
          if (nbf < 0) ghost_state<T>(-nbf, um, N, far, up);
          if (q < NF) {
            num_flux<T>(a.flux, um, up, N, nn, gamma, fl);
          } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) fl[v] = Pr::mixed ? fhbar[v] : T(0);
          }
          bool mean = Pr::mixed;
#pragma unroll
          for (int v = 0; v < 5; ++v) mean = mean && (um[v] == c0t[v]) && (up[v] == c0n[v]);
#pragma unroll
          for (int v = 0; v < 5; ++v) fh[v][j] = Pr::mixed ? (mean ? T(0) : fl[v] - fhbar[v]) : fl[v];
        }
        if constexpr (Pr::KW == 1) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int lk = 0; lk < 4; ++lk) {
              const Op av = tab[L::lift(mt, f, ft, lk) * 64 + lane];
#pragma unroll
              for (int v = 0; v < 5; ++v) acc[mt][v] = Pr::mfma(av, Pr::op1(fh[v][lk]), acc[mt][v]);
            }
        } else {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            Op b;
#pragma unroll
            for (int m = 0; m < 8; ++m) b[m] = (typename Pr::E1)(m < 4 ? fh[v][m] : T(0));
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
              acc[mt][v] = Pr::mfma(tab[L::lift(mt, f, ft, 0) * 64 + lane], b, acc[mt][v]);
          }
        }
      }
    }

    // ------------------------------------------------------------ epilogue
    // mixed: fp64 projection of the cell-mean fluxes, sum_k mom_k[i] Fbar_k with the three
    // volume directions and the four faces (k = 0..6), as two fp64 MFMA k-steps per mode
    // tile.  Lane group g supplies k = g (volume direction g, or face 0 for g = 3) and
    // k = 4 + g (face g + 1, or zero); the table rows are permuted so that the fp64
    // accumulator rows line up with the fp32 accumulator rows of the same lane.
    d4_t mean_acc[Pr::mixed ? MT : 1][5];
    if constexpr (Pr::mixed) {
#pragma unroll
      for (int i = 0; i < 9; ++i) Md[i] = mv.M[i * epad + e];
      double c0[5], x0[5], x1[5], yg[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) c0[v] = double(*reinterpret_cast<const S*>(ubase + (size_t)v * var_bytes + eoff));
      {
        // contravariant mean flux in direction min(g, 2) only: blend the row of M arithmetically
        // (a select chain would be turned into an indexed, stack-resident array)
        const double w0 = g == 0 ? 1.0 : 0.0, w1 = g == 1 ? 1.0 : 0.0, w2 = g >= 2 ? 1.0 : 0.0;
        double Mrow[9];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          Mrow[c] = w0 * Md[c] + w1 * Md[3 + c] + w2 * Md[6 + c];
          Mrow[3 + c] = 0.0;
          Mrow[6 + c] = 0.0;
        }
        double y3[3][5];
        contra_flux<double>(c0, Mrow, a.gamma - 1.0, y3);
#pragma unroll
        for (int v = 0; v < 5; ++v) yg[v] = y3[0][v];
      }
      {
        const int f = g == 3 ? 0 : g + 1;
        double N[3], cn[5], fb[5];
        face_normal<double>(f, Md, N);
        const double nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        const int nbf = f == 0 ? nbr[0] : f == 1 ? nbr[1] : f == 2 ? nbr[2] : nbr[3];
        if (nbf >= 0) {
#pragma unroll
          for (int v = 0; v < 5; ++v)
            cn[v] = double(*reinterpret_cast<const S*>(ubase + (size_t)v * var_bytes + (uint32_t)nbf * sizeof(S)));
        } else {
          ghost_state<double>(-nbf, c0, N, far64, cn);
        }
        num_flux<double>(a.flux, c0, cn, N, nn, a.gamma, fb);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          x0[v] = g == 3 ? fb[v] : yg[v];
          x1[v] = g == 3 ? 0.0 : fb[v];
        }
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const double a0 = a.mean_tab[(2 * mt) * 64 + lane], a1 = a.mean_tab[(2 * mt + 1) * 64 + lane];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          d4_t m = {0, 0, 0, 0};
          m = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x0[v], m, 0, 0, 0);
          m = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x1[v], m, 0, 0, 0);
          mean_acc[mt][v] = m;
        }
      }
    }
    const double ivol = mv.inv_vol[e];
    if (e < mv.n_elem) {
      const char* u0base = reinterpret_cast<const char*>(a.u0);
      char* obase = reinterpret_cast<char*>(a.u_out);
      const bool comp = Pr::mixed && a.q_out != nullptr;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        double o[5][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int mode = 16 * mt + drow_of<Pr>(g, j);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            double r = double(acc[mt][v][j]);
            if constexpr (Pr::mixed) r += mean_acc[mt][v][j];
            r *= ivol;
            o[v][j] = 0.0;
            if (mode < NP) {
              const size_t off = (size_t)v * var_bytes + (size_t)mode * plane + eoff;
              double out;
              if (a.rk) {
                const double uin = double(*reinterpret_cast<const S*>(ubase + off));
                const double u0 = a.alpha == 0.0 ? 0.0 : double(*reinterpret_cast<const S*>(u0base + off));
                out = a.alpha * u0 + (1.0 - a.alpha) * (uin + a.dt * r);
              } else {
                out = r;
              }
              *reinterpret_cast<S*>(obase + off) = S(out);
              o[v][j] = out;
            }
          }
        }
        if constexpr (Pr::mixed) {
          if (comp) {
            // operand companion of the result: modes 1.. in the operand precision, mean in fp32
            using E1 = typename Pr::E1;
            typedef E1 e4_t __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int v = 0; v < 5; ++v) {
              e4_t h;
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const int mode = 16 * mt + 4 * g + j;
                h[j] = (E1)((mode > 0 && mode < NP) ? float(o[v][j]) : 0.0f);
              }
              *reinterpret_cast<e4_t*>(reinterpret_cast<E1*>(a.q_out) + ((int64_t)e * 5 + v) * (32 * KS) + 16 * mt +
                                       4 * g) = h;
              if (mt == 0 && g == 0) a.c0_out[v * epad + e] = float(o[v][0]);
            }
          }
        }
      }
      if constexpr (Pr::mixed) {
        // zero the companion slots past the last mode tile
        if (comp) {
#pragma unroll
          for (int mt = MT; mt < 2 * KS; ++mt)
#pragma unroll
            for (int v = 0; v < 5; ++v)
              *reinterpret_cast<uint2*>(reinterpret_cast<typename Pr::E1*>(a.q_out) + ((int64_t)e * 5 + v) * (32 * KS) +
                                        16 * mt + 4 * g) = uint2{0, 0};
        }
      }
    }
  }
}

// Operand companion of an fp64 state (mixed modes): one thread per (element, variable).
template <int P, class Pr>
__global__ void pack_kernel(MeshView m, const double* __restrict__ u, typename Pr::E1* __restrict__ q,
                            float* __restrict__ c0) {
  using O = Ord<P>;
  constexpr int NP = O::NP, KS = Layout<P, 8>::KS;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m.epad * 5) return;
  const int64_t e = t / 5;
  const int v = (int)(t % 5);
  typename Pr::E1* dst = q + (e * 5 + v) * (32 * KS);
#pragma unroll
  for (int mode = 0; mode < 32 * KS; ++mode) {
    const float x = (mode > 0 && mode < NP) ? float(u[(int64_t)(v * NP + mode) * m.epad + e]) : 0.0f;
    dst[mode] = (typename Pr::E1)x;
  }
  c0[v * m.epad + e] = float(u[(int64_t)(v * NP) * m.epad + e]);
}

size_t companion_bytes(int p, int64_t epad) {
  const int np = (p + 1) * (p + 2) * (p + 3) / 6;
  const int ks = (np + 31) / 32;
  const size_t q = (size_t)epad * 5 * 32 * ks * 2;
  return ((q + 255) & ~(size_t)255) + (size_t)epad * 5 * sizeof(float);
}

hipError_t launch_pack(int p, int prec, const MeshView& m, const void* u, void* q, float* c0, hipStream_t s) {
  const unsigned nb = (unsigned)((m.epad * 5 + 255) / 256);
#define TDG_PACK(PP)                                                                                          \
  if (p == PP) {                                                                                             \
    if (prec == 2)                                                                                           \
      hipLaunchKernelGGL((pack_kernel<PP, PrecBF16>), dim3(nb), dim3(256), 0, s, m, (const double*)u,        \
                         (__bf16*)q, c0);                                                                    \
    else                                                                                                     \
      hipLaunchKernelGGL((pack_kernel<PP, PrecF16>), dim3(nb), dim3(256), 0, s, m, (const double*)u,         \
                         (_Float16*)q, c0);                                                                  \
    return hipGetLastError();                                                                                \
  }
  TDG_PACK(1) TDG_PACK(2) TDG_PACK(3) TDG_PACK(4)
#undef TDG_PACK
  return hipErrorInvalidValue;
}

template <int P, class Pr>
static hipError_t launch_stage_impl(const StageArgs& a, hipStream_t stream) {
  using L = Layout<P, Pr::KW>;
  constexpr size_t tab_bytes = sizeof(typename Pr::Op) * L::n_slots * 64;
  constexpr bool lds = tab_bytes <= 96 * 1024;
  auto kern = stage_kernel<P, Pr, lds>;
  int per_cu = 0;
  hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
  if (err != hipSuccess) return err;
  if (per_cu < 1) per_cu = 1;
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t ngroups = a.mesh.epad / 16;
  int64_t want = (ngroups + 3) / 4;  // one group per wavefront at least
  int64_t fill = (int64_t)ncu * per_cu;
  int64_t nblk = want < fill ? want : fill;
  if (a.max_blocks > 0 && nblk > a.max_blocks) nblk = a.max_blocks;
  if (nblk >= 8) nblk -= nblk % 8;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_stage(int p, int prec, const StageArgs& a, hipStream_t stream) {
#define TDG_CASE(PP, PR)                                                     \
  if (p == PP) return launch_stage_impl<PP, PR>(a, stream);
  switch (prec) {
    case 0:
      TDG_CASE(1, PrecF64) TDG_CASE(2, PrecF64) TDG_CASE(3, PrecF64) TDG_CASE(4, PrecF64) break;
    case 1:
      TDG_CASE(1, PrecF32) TDG_CASE(2, PrecF32) TDG_CASE(3, PrecF32) TDG_CASE(4, PrecF32) break;
    case 2:
      TDG_CASE(1, PrecBF16) TDG_CASE(2, PrecBF16) TDG_CASE(3, PrecBF16) TDG_CASE(4, PrecBF16) break;
    case 3:
      TDG_CASE(1, PrecF16) TDG_CASE(2, PrecF16) TDG_CASE(3, PrecF16) TDG_CASE(4, PrecF16) break;
    default:
      break;
  }
#undef TDG_CASE
  return hipErrorInvalidValue;
}

}  // namespace tetdg
