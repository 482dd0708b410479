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
// of the cell means, whose own projection uses fp64 moments in the epilogue.  The
// pointwise fluxes round identically at every call site (explicit fused multiply-adds
// only), so a point whose state equals the cell mean gives exactly zero deviation: a
// uniform state keeps its residual at fp64 round-off.
//
// Latency: the neighbour operands of face 0 are requested before the volume integral
// and those of face f + 1 as soon as face f's neighbour trace has consumed its own, so
// the face phase waits on no memory; the epilogue issues all reads of a mode tile at once.
#include <hip/hip_runtime.h>

#include "dg_kernels.hpp"
#include "dg_launch.hpp"
#include "dg_tile.hpp"

namespace tetdg {

// Packed pair of operand-precision values (KW = 8 modes); a placeholder otherwise.
template <class Pr, bool = (Pr::KW == 8)>
struct LiftPair {
  using E1 = float;
  typedef float type __attribute__((ext_vector_type(2)));
};
template <class Pr>
struct LiftPair<Pr, true> {
  using E1 = typename Pr::E1;
  typedef E1 type __attribute__((ext_vector_type(2)));
};

// Workgroups per CU the stage kernel is compiled for: two (two waves per SIMD, at most
// 256 registers per lane) for FP32 and the mixed modes up to P3 and for FP64 up to P2;
// FP64 at P3 (~400 registers) and every P4 kernel run one wave per SIMD.
template <int P, class Pr>
constexpr int stage_min_blocks() {
  return (P <= 3 && !Pr::f64) || (P <= 2 && Pr::f64) ? 2 : 1;
}

// FP64 at P1, P2 (two waves per SIMD) and P4 (tables in global memory): the current face's
// neighbour operands wait in LDS instead of registers.
template <int P, class Pr>
constexpr bool stage_nbr_lds() {
  return Pr::f64 && P != 3;
}

// kLds: reference tables staged in LDS; kRoe: Roe's interface flux instead of Rusanov's
// (a compile-time choice keeps the other flux's code and registers out of the kernel).
// kEpi, the epilogue's form (a compile-time choice, so that the epilogue's state reads sit
// in no branch; mixed modes and FP32 / FP64 up to P3, the other kernels take kEpiRK and
// branch): the RK stage update, the residual without it, the update of a stage with
// alpha = 0 (SSP-RK3's first, and the mixed modes' regrouped third), which does not read
// U0, or (mixed modes) the update that
// stores alpha_w U0 + (1 - alpha_w) times the stage result and writes the result's fp64
// cell means beside its companion.
enum : int { kEpiRK = 0, kEpiResid = 1, kEpiRK0 = 2, kEpiRKW = 3 };
template <int P, class Pr, bool kLds, bool kRoe, int kEpi>
__global__ __launch_bounds__(256, (stage_min_blocks<P, Pr>())) void stage_kernel(StageArgs a) {
  using O = Ord<P>;
  using L = Layout<P, Pr::KW>;
  using S = typename Pr::S;
  using T = typename Pr::T;
  using Op = typename Pr::Op;
  using Acc = typename Pr::Acc;
  constexpr int NP = O::NP, NQ = O::NQ, NF = O::NF, MT = O::MT, QT = O::QT, FT = O::FT, KS = L::KS;

  __shared__ Op lds_tab[kLds ? L::n_slots * 64 : 1];
  // mixed modes: per-wave staging of the operand companion written by the epilogue, so
  // that each element's record leaves as whole 16-byte slots.  An element's record (5 x
  // 32 KS operand values) is followed by 8 padding values, so that the 16 columns' records
  // start in different LDS banks (a 320-byte stride put four columns on each bank group).
  constexpr int CES = 5 * 32 * KS + 8;  // record stride, operand values
  __shared__ Op lds_comp[Pr::mixed ? 4 * 16 * CES / 8 : 1];
  // mixed modes: per-wave exchange of the cell-mean face data.  The four lane groups of a
  // column hold the same element, so lane group g evaluates face g's mean flux, neighbour
  // mean and normal once, and every lane reads face f's record here: 7 float pairs
  // (neighbour / ghost mean 5, mean flux 5, N 3, |N| 1), pair-major so that the lanes of a
  // wave access consecutive 8-byte words
  typedef float f2v_t __attribute__((ext_vector_type(2)));
  __shared__ f2v_t lds_face[Pr::mixed ? 7 * 4 * 64 : 1];
  // the current face's neighbour operands in LDS (FP64 at P1, P2 and P4), one slot per
  // lane (each lane reads back only what it wrote): this keeps the kernel within its
  // registers (two waves per SIMD at P1 and P2; fewer spills at P4)
  constexpr bool kNbrLds = stage_nbr_lds<P, Pr>();
  __shared__ Op lds_nbr[kNbrLds ? 4 * 5 * KS * 64 : 1];
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
  const int wslot = threadIdx.x >> 6;  // wavefront within the workgroup
  if constexpr (Pr::mixed) {
    // the staging records' padding (modes past the last, the slots past the last mode
    // tile) is never written by the epilogue: zero it once
    uint32_t* z = reinterpret_cast<uint32_t*>(lds_comp) + wslot * 8 * CES;
    for (int i = lane; i < 8 * CES; i += 64) z[i] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const char* __restrict__ ubase = reinterpret_cast<const char*>(a.u_in);
  const MeshView& mv = a.mesh;
  const int64_t epad = mv.epad;
  constexpr int NPQ = npq_of(NP);
  // FP32 / FP64: when the last mode tile holds at most 4 modes (P1, P3, P4), a 16-row MFMA
  // would waste 12 of its rows.  Its projection and lift instead let lane group g
  // accumulate its own points' share of those modes for its 16 elements — as 4x4x1 MFMA
  // blocks in fp32 (a quarter of the 16x16x4 cost), as fp64 FMAs with the four table
  // values read once per lane group — and the four shares are summed across lane groups
  // before the epilogue.
  constexpr bool kTail4 = Pr::KW == 1 && NP - 16 * (MT - 1) <= 4;
  // Mixed modes, P3 and P4: the last mode tile holds at most 4 modes.  Its table rows put
  // mode 16 (MT - 1) + g in register 0 of lane group g (fp32 accumulator row 4 g, fp64
  // accumulator row g) and zeros elsewhere, so that the epilogue handles that tile as one
  // value per lane, all lanes busy.
  constexpr bool kSpread = Pr::mixed && MT >= 2 && NP - 16 * (MT - 1) <= 4;
  const uint32_t quad_bytes = (uint32_t)(epad * 4 * sizeof(S));  // one (variable, mode quad) plane
  const uint32_t var_bytes = quad_bytes * NPQ;
  const T gamma = T(a.gamma), gm1 = T(a.gamma - 1.0);
  // step size (device-computed when adaptive), times the stage's factor
  const double dt = (a.dt_dev ? *a.dt_dev : a.dt) * a.dt_scale;
  T far[5];
  double far64[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    far64[v] = a.far[v];
    far[v] = T(a.far[v]);
  }
  OperandMap<Pr, NP, KS> om;
  om.init(g, quad_bytes);

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
    const uint32_t eoff = (uint32_t)e * 4 * sizeof(S);
    double Md[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Md[i] = mv.M[i * epad + e];
    // Mixed modes: the pointwise deviation fluxes (volume and face) are linear in M and in
    // the face normals built from it, and M = |det J| J^-1 scales as h^2, so on small
    // elements they would fall below the normal range of fp16 operands.  They are computed
    // with M scaled by a power of two (largest entry in [0.5, 1)), which changes no fp32
    // rounding, and the contractions' fp32 results are scaled back exactly in the epilogue.
    double unscale = 1.0;
    T Mt[9];
    if constexpr (Pr::mixed) {
      double mx = 0.0;
#pragma unroll
      for (int i = 0; i < 9; ++i) mx = fmax(mx, fabs(Md[i]));
      int ex = 0;
      (void)frexp(mx, &ex);
      unscale = ldexp(1.0, ex);
      const double sc = ldexp(1.0, -ex);
#pragma unroll
      for (int i = 0; i < 9; ++i) Mt[i] = T(Md[i] * sc);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) Mt[i] = T(Md[i]);
    }
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
    } else {
      load_operands<Pr, NP, KS>(ubase, var_bytes, eoff, om, bc);
    }
    // operands of the neighbour across face f (the element itself on a boundary face)
    auto load_nbr = [&](int f, Op (&bx)[5][KS], T (&cx)[5]) {
      const int nbf = f == 0 ? nbr[0] : f == 1 ? nbr[1] : f == 2 ? nbr[2] : nbr[3];
      const int en = nbf >= 0 ? nbf : e;
      if constexpr (Pr::mixed) {
        const Op* q = reinterpret_cast<const Op*>(a.q_in);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
#pragma unroll
          for (int s = 0; s < KS; ++s) bx[v][s] = q[(((int64_t)en * 5 + v) * KS + s) * 4 + g];
        }
        (void)cx;
      } else {
        load_operands<Pr, NP, KS>(ubase, var_bytes, (uint32_t)en * 4 * sizeof(S), om, bx);
      }
    };
    Op bn[5][KS];
    T c0n[5];
    if constexpr (!kNbrLds) load_nbr(0, bn, c0n);
    // mixed: lane group g's face (face g): the neighbour's cell mean (its load is issued here
    // and consumed after the volume integral)
    const int nbg = g == 0 ? nbr[0] : g == 1 ? nbr[1] : g == 2 ? nbr[2] : nbr[3];
    T cmg[5];
    if constexpr (Pr::mixed) {
#pragma unroll
      for (int v = 0; v < 5; ++v) cmg[v] = a.c0_in[v * epad + (nbg >= 0 ? nbg : e)];
      contra_flux<T>(c0t, Mt, gm1, ybar);
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
#pragma unroll
          for (int dd = 0; dd < 3; ++dd)
#pragma unroll
            for (int v = 0; v < 5; ++v) yy[dd][v] -= ybar[dd][v];
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
              if constexpr (kTail4 && Pr::f64) {
                if (mt == MT - 1) {
                  tail_fma<Pr>(tab + L::proj(mt, qt, 4 * dd + j) * 64 + 16 * g, yy[dd], acc[mt]);
                  continue;
                }
              }
              const Op av = tab[L::proj(mt, qt, 4 * dd + j) * 64 + lane];
#pragma unroll
              for (int v = 0; v < 5; ++v) acc[mt][v] = mfma_tile<Pr, kTail4>(mt == MT - 1, av, Pr::op1(yy[dd][v]), acc[mt][v]);
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
    if constexpr (Pr::mixed) {
      // face g of this lane's element: normal, neighbour (or ghost) mean and the mean flux,
      // staged for the whole wave (the fence orders these writes after the previous group's
      // reads of the same slots)
      T Ng[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        Ng[c] = g == 0 ? (Mt[c] + Mt[3 + c] + Mt[6 + c]) : g == 1 ? -Mt[c] : g == 2 ? -Mt[3 + c] : -Mt[6 + c];
      const T nng = sqrt(Ng[0] * Ng[0] + Ng[1] * Ng[1] + Ng[2] * Ng[2]);
      if (nbg < 0) ghost_state<T>(-nbg, c0t, Ng, far, cmg);
      T fhg[5];
      num_flux<kRoe, T>(c0t, cmg, Ng, nng, gamma, fhg);
      f2v_t* slot = lds_face + wslot * 64 + lane;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      slot[0 * 256] = f2v_t{cmg[0], cmg[1]};
      slot[1 * 256] = f2v_t{cmg[2], cmg[3]};
      slot[2 * 256] = f2v_t{cmg[4], fhg[0]};
      slot[3 * 256] = f2v_t{fhg[1], fhg[2]};
      slot[4 * 256] = f2v_t{fhg[3], fhg[4]};
      slot[5 * 256] = f2v_t{Ng[0], Ng[1]};
      slot[6 * 256] = f2v_t{Ng[2], nng};
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      T c0nn[5];
      T N[3];
      T nn;
      const int nbf = f == 0 ? nbr[0] : f == 1 ? nbr[1] : f == 2 ? nbr[2] : nbr[3];
      const int fpl = (fcode >> (2 * f)) & 3;
      T fhbar[5];
      Op* const nslot = lds_nbr + wslot * (5 * KS * 64) + lane;
      if constexpr (kNbrLds) {
        load_nbr(f, bn, c0nn);
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int s = 0; s < KS; ++s) nslot[(v * KS + s) * 64] = bn[v][s];
        // the reads below must come from LDS (not be forwarded from the registers)
        asm volatile("" ::: "memory");
      }
      if constexpr (Pr::mixed) {
        // face f's record, written by lane group f of this column
        const f2v_t* slot = lds_face + wslot * 64 + 16 * f + col;
        const f2v_t r0 = slot[0 * 256], r1 = slot[1 * 256], r2 = slot[2 * 256], r3 = slot[3 * 256],
                    r4 = slot[4 * 256], r5 = slot[5 * 256], r6 = slot[6 * 256];
        c0n[0] = r0[0], c0n[1] = r0[1], c0n[2] = r1[0], c0n[3] = r1[1], c0n[4] = r2[0];
        fhbar[0] = r2[1], fhbar[1] = r3[0], fhbar[2] = r3[1], fhbar[3] = r4[0], fhbar[4] = r4[1];
        N[0] = r5[0], N[1] = r5[1], N[2] = r6[0];
        nn = r6[1];
      } else {
        face_normal<T>(f, Md, N);
        nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
      }
#pragma unroll 1
      for (int ft = 0; ft < FT; ++ft) {
        Acc dm[5], dp[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) dm[v] = dp[v] = Acc{0, 0, 0, 0};
        // own trace B_f c, from the operands kept in registers since the group's start
        Op own[5][KS];
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int s = 0; s < KS; ++s) own[v][s] = bc[v][s];
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
              for (int v = 0; v < 5; ++v) {
                const Op bv = kNbrLds ? nslot[(v * KS + s) * 64] : bn[v][s];
                dp[v] = Pr::mfma(av, mine ? bv : Op{}, dp[v]);
              }
            }
          }
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const Op av = tab[L::trace(f, ft, s) * 64 + lane];
#pragma unroll
          for (int v = 0; v < 5; ++v) dm[v] = Pr::mfma(av, own[v][s], dm[v]);
        }
        // the neighbour operands are consumed: request the next face's while this face's
        // own trace, fluxes and lifting are computed
        if (!kNbrLds && f < 3 && ft == FT - 1) load_nbr(f + 1, bn, c0nn);
        // face flux (deviation) at the tile's points: fp32 values for KW = 1, packed operand
        // pairs for KW = 8 (the lift's B operand holds the four points in k = 8 g + 0..3)
        T fh[5][Pr::KW == 1 ? 4 : 1];
        typedef typename LiftPair<Pr>::type e2_t;
        e2_t fhp[5][2];
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
            num_flux<kRoe, T>(um, up, N, nn, gamma, fl);
          } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) fl[v] = Pr::mixed ? fhbar[v] : T(0);
          }
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const T x = Pr::mixed ? fl[v] - fhbar[v] : fl[v];
            if constexpr (Pr::KW == 1)
              fh[v][j] = x;
            else
              fhp[v][j >> 1][j & 1] = (typename LiftPair<Pr>::E1)x;
          }
        }
        if constexpr (Pr::KW == 1) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int lk = 0; lk < 4; ++lk) {
              if constexpr (kTail4 && Pr::f64) {
                if (mt == MT - 1) {
                  T fl[5];
#pragma unroll
                  for (int v = 0; v < 5; ++v) fl[v] = fh[v][lk];
                  tail_fma<Pr>(tab + L::lift(mt, f, ft, lk) * 64 + 16 * g, fl, acc[mt]);
                  continue;
                }
              }
              const Op av = tab[L::lift(mt, f, ft, lk) * 64 + lane];
#pragma unroll
              for (int v = 0; v < 5; ++v) acc[mt][v] = mfma_tile<Pr, kTail4>(mt == MT - 1, av, Pr::op1(fh[v][lk]), acc[mt][v]);
            }
        } else {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            Op b;
#pragma unroll
            for (int m = 0; m < 8; ++m) b[m] = m < 4 ? fhp[v][m >> 1][m & 1] : (typename Pr::E1)0.0f;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
              acc[mt][v] = Pr::mfma(tab[L::lift(mt, f, ft, 0) * 64 + lane], b, acc[mt][v]);
          }
        }
      }
      (void)c0nn;
    }

    // ------------------------------------------------------------ epilogue
    // mixed: fp64 projection of the cell-mean fluxes, sum_k mom_k[i] Fbar_k with the three
    // volume directions and the four faces (k = 0..6), as two fp64 MFMA k-steps per mode
    // tile.  Lane group g supplies k = g (volume direction g, or face 0 for g = 3) and
    // k = 4 + g (face g + 1, or zero); the table rows are permuted so that the fp64
    // accumulator rows line up with the fp32 accumulator rows of the same lane.
    if constexpr (kTail4) {
      // sum the lane groups' shares of the last tile (register r: mode 16 (MT - 1) + r) and
      // move them to the accumulator rows of the precision: fp32 row 4 g + j (lane group 0
      // holds the tile's modes in its registers), fp64 row g + 4 j (mode r in register 0
      // of lane group r)
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
          acc[MT - 1][v] = Acc{g == 0 ? x[0] : g == 1 ? x[1] : g == 2 ? x[2] : x[3], 0.0, 0.0, 0.0};
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[MT - 1][v][j] = x[j];
        }
      }
    }
    // Every lane takes part in the epilogue's MFMAs (the A operand rows are spread over
    // all lanes); only the stores are limited to the mesh's elements.
    const bool live = e < mv.n_elem;
    const char* u0base = reinterpret_cast<const char*>(a.u0);
    char* obase = reinterpret_cast<char*>(a.u_out);
    const bool comp = Pr::mixed && a.q_out != nullptr;
    typedef S s4_t __attribute__((ext_vector_type(4)));
    // fp64 data of the cell-mean fluxes (mixed modes)
    double Me[Pr::mixed ? 9 : 1], c0e[Pr::mixed ? 5 : 1], c0g[Pr::mixed ? 5 : 1];
    const int fg = g == 3 ? 0 : g + 1;
    const int ng = fg == 0 ? nbr[0] : fg == 1 ? nbr[1] : fg == 2 ? nbr[2] : nbr[3];
    // mixed: the mean-flux projection's A operands of every tile, requested before the
    // state values (loads complete in order, so waiting for them then leaves the state
    // reads in flight)
    double mtab[Pr::mixed ? MT : 1][2];
    // fp64 cell means of the stage's state: mode 0 of u_in, or mean_in when u_in holds
    // another combination (a uniform choice of base and strides)
    const char* const mbase = a.mean_in ? reinterpret_cast<const char*>(a.mean_in) : ubase;
    const uint32_t mvs = a.mean_in ? (uint32_t)(epad * sizeof(double)) : var_bytes;
    const uint32_t mes = a.mean_in ? (uint32_t)sizeof(double) : (uint32_t)(4 * sizeof(S));
    if constexpr (Pr::mixed) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        mtab[mt][0] = a.mean_tab[(uint32_t)((2 * mt) * 64 + lane)];
        mtab[mt][1] = a.mean_tab[(uint32_t)((2 * mt + 1) * 64 + lane)];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) Me[i] = mv.M[i * epad + e];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        c0e[v] = *reinterpret_cast<const double*>(mbase + (size_t)v * mvs + (uint32_t)e * mes);
        c0g[v] = *reinterpret_cast<const double*>(mbase + (size_t)v * mvs + (uint32_t)(ng >= 0 ? ng : e) * mes);
      }
    }
    // State values of mode tile mt (mode = 16 mt + drow(g, j)): with the fp32 accumulator
    // layout they form one mode quad per lane (one vector access); with the fp64 layout
    // they sit at position g of four quads.  Padding modes of the last quad are written 0.
    double uin[5][4], u0v[5][4], radd[5][4];
    // kSpread: the last tile's values, one per lane (mode 16 (MT - 1) + g at position g of
    // quad 4 (MT - 1)), requested together with those of the tile before it
    double tin[kSpread ? 5 : 1], t0v[kSpread ? 5 : 1];
    // a per-lane 32-bit byte offset, kept opaque so that the compiler adds it to the uniform
    // base at the access (one register) instead of keeping 64-bit per-lane addresses
    // across the group loop
    auto lane_off = [](uint32_t x) {
      asm("" : "+v"(x));
      return x;
    };
    // Mixed modes, and FP32 / FP64 up to P3 (kFlat): the state reads and the stores of the
    // result are unconditional.  (At P4 the FP32 / FP64 kernels keep the branches: without
    // them they spill more.)
    // Loads inside lane-dependent or uniform branches keep the compiler from counting the
    // outstanding loads across the branch, so that every later wait also waits for them.
    // Padding elements (e >= n_elem, inside the padded arrays) read valid memory and store
    // zeros; a stage with alpha = 0 leaves U0 unread (kEpiRK0).
    constexpr bool kFlat = Pr::mixed || P <= 3;
    constexpr bool kU0 = kEpi == kEpiRK || kEpi == kEpiRKW;
    const bool rk = kFlat ? kEpi != kEpiResid : a.rk != 0;
    auto load_tail = [&]() {
#pragma unroll
      for (int v = 0; v < (kSpread ? 5 : 1); ++v) tin[v] = t0v[v] = 0.0;
      if (!rk) return;
#pragma unroll
      for (int v = 0; v < (kSpread ? 5 : 1); ++v) {
        const uint32_t o = lane_off(eoff + (uint32_t)(4 * (MT - 1)) * quad_bytes + (uint32_t)g * sizeof(S));
        tin[v] = double(*reinterpret_cast<const S*>(ubase + (size_t)v * var_bytes + o));
        if constexpr (kU0) t0v[v] = double(*reinterpret_cast<const S*>(u0base + (size_t)v * var_bytes + o));
      }
    };
    auto load_tile = [&](int mt) {
#pragma unroll
      for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int j = 0; j < 4; ++j) uin[v][j] = u0v[v][j] = radd[v][j] = 0.0;
      if (!kFlat && !live) return;
      if constexpr (!Pr::mixed) {
        // an added residual part (the viscous terms) in the state's layout and precision
        if (a.r_add) {
          const char* rb = reinterpret_cast<const char*>(a.r_add);
#pragma unroll
          for (int v = 0; v < 5; ++v)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int mode = 16 * mt + drow_of<Pr>(g, j);
              if ((mode >> 2) < NPQ)
                radd[v][j] = double(*reinterpret_cast<const S*>(rb + (size_t)v * var_bytes + (uint32_t)(mode >> 2) * quad_bytes +
                                                                 ((size_t)e * 4 + (mode & 3)) * sizeof(S)));
            }
        }
      }
      if (!rk) return;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        // uniform base of the variable + a 32-bit per-lane offset (one register, and the
        // loads' scalar-base addressing form)
        const size_t vb = (size_t)v * var_bytes;
        if constexpr (kFlat && Pr::f64) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int qd = 4 * mt + j;
            if (qd < NPQ) {
              const uint32_t o = lane_off(eoff + (uint32_t)qd * quad_bytes + (uint32_t)g * sizeof(S));
              uin[v][j] = double(*reinterpret_cast<const S*>(ubase + vb + o));
              if constexpr (kU0) u0v[v][j] = double(*reinterpret_cast<const S*>(u0base + vb + o));
            }
          }
        } else if constexpr (kFlat) {
          // quads past the last read the last one and count as zero
          const int qd = 4 * mt + g;
          const uint32_t o = lane_off(eoff + (uint32_t)(qd < NPQ ? qd : NPQ - 1) * quad_bytes);
          const s4_t x = *reinterpret_cast<const s4_t*>(ubase + vb + o);
#pragma unroll
          for (int j = 0; j < 4; ++j) uin[v][j] = qd < NPQ ? double(x[j]) : 0.0;
          if constexpr (kU0) {
            const s4_t y = *reinterpret_cast<const s4_t*>(u0base + vb + o);
#pragma unroll
            for (int j = 0; j < 4; ++j) u0v[v][j] = qd < NPQ ? double(y[j]) : 0.0;
          }
        } else if constexpr (!Pr::f64) {
          const int qd = 4 * mt + g;
          if (qd < NPQ) {
            const size_t o = vb + eoff + (size_t)qd * quad_bytes;
            const s4_t x = *reinterpret_cast<const s4_t*>(ubase + o);
#pragma unroll
            for (int j = 0; j < 4; ++j) uin[v][j] = double(x[j]);
            if (a.alpha != 0.0) {
              const s4_t y = *reinterpret_cast<const s4_t*>(u0base + o);
#pragma unroll
              for (int j = 0; j < 4; ++j) u0v[v][j] = double(y[j]);
            }
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int qd = 4 * mt + j;
            if (qd < NPQ) {
              const size_t o = vb + eoff + (size_t)qd * quad_bytes + (size_t)g * sizeof(S);
              uin[v][j] = double(*reinterpret_cast<const S*>(ubase + o));
              if (a.alpha != 0.0) u0v[v][j] = double(*reinterpret_cast<const S*>(u0base + o));
            }
          }
        }
      }
    };

    // mixed: fp64 projection of the cell-mean fluxes, sum_k mom_k[i] Fbar_k with the three
    // volume directions and the four faces (k = 0..6), as two fp64 MFMA k-steps per mode
    // tile.  Lane group g supplies k = g (volume direction g, or face 0 for g = 3) and
    // k = 4 + g (face g + 1, or zero); the table rows are permuted so that the fp64
    // accumulator rows line up with the fp32 accumulator rows of the same lane.
    double x0[Pr::mixed ? 5 : 1], x1[Pr::mixed ? 5 : 1];
    if constexpr (Pr::mixed) {
      double yg[5];
      {
        // contravariant mean flux in direction min(g, 2) only: blend the row of M
        // arithmetically (a select chain would become an indexed, stack-resident array)
        const double w0 = g == 0 ? 1.0 : 0.0, w1 = g == 1 ? 1.0 : 0.0, w2 = g >= 2 ? 1.0 : 0.0;
        double Mrow[9];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          Mrow[c] = w0 * Me[c] + w1 * Me[3 + c] + w2 * Me[6 + c];
          Mrow[3 + c] = 0.0;
          Mrow[6 + c] = 0.0;
        }
        double y3[3][5];
        contra_flux<double>(c0e, Mrow, a.gamma - 1.0, y3);
#pragma unroll
        for (int v = 0; v < 5; ++v) yg[v] = y3[0][v];
      }
      double N[3], fb[5];
      face_normal<double>(fg, Me, N);
      const double nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
      if (ng < 0) ghost_state<double>(-ng, c0e, N, far64, c0g);
      num_flux<kRoe, double>(c0e, c0g, N, nn, a.gamma, fb);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        x0[v] = g == 3 ? fb[v] : yg[v];
        x1[v] = g == 3 ? 0.0 : fb[v];
      }
    }
    const double ivol = mv.inv_vol[e];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      if (!(kSpread && mt == MT - 1)) load_tile(mt);
      if (kSpread && mt == (MT >= 2 ? MT - 2 : 0)) load_tail();
      double a0 = 0.0, a1 = 0.0;
      if constexpr (Pr::mixed) {
        a0 = mtab[mt][0];
        a1 = mtab[mt][1];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        d4_t mean = {0, 0, 0, 0};
        if constexpr (Pr::mixed) {
          mean = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x0[v], mean, 0, 0, 0);
          mean = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x1[v], mean, 0, 0, 0);
        }
        const bool spread = kSpread && mt == MT - 1;
        double o[4], oc[4];  // stored values; values of the companion (the stage result)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int mode = spread ? (j == 0 ? 16 * mt + g : NP) : 16 * mt + drow_of<Pr>(g, j);
          double r = double(acc[mt][v][j]) * unscale;
          if constexpr (Pr::mixed) r += mean[j];
          r *= ivol;
          r += radd[v][j];
          const double ui = spread ? tin[kSpread ? v : 0] : uin[v][j];
          const double u0 = spread ? t0v[kSpread ? v : 0] : u0v[v][j];
          const double out = rk ? a.alpha * u0 + (1.0 - a.alpha) * (ui + dt * r) : r;
          double st = out;
          if constexpr (kEpi == kEpiRKW) st = a.alpha_w * u0 + (1.0 - a.alpha_w) * out;
          o[j] = mode < NP && (!kFlat || live) ? st : 0.0;
          oc[j] = mode < NP && (!kFlat || live) ? out : 0.0;
        }
        if (!kFlat && !live) continue;
        char* const ob = obase + (size_t)v * var_bytes;
        if (spread) {
          *reinterpret_cast<S*>(ob + lane_off(eoff + (uint32_t)(4 * mt) * quad_bytes + (uint32_t)g * sizeof(S))) = S(o[0]);
        } else if constexpr (!Pr::f64) {
          const int qd = 4 * mt + g;
          if (qd < NPQ) {
            s4_t x;
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = S(o[j]);
            // streamed out: not read again within this launch
            s4_t* dst = kFlat ? reinterpret_cast<s4_t*>(ob + lane_off(eoff + (uint32_t)qd * quad_bytes))
                              : reinterpret_cast<s4_t*>(ob + eoff + (size_t)qd * quad_bytes);
            __builtin_nontemporal_store(x, dst);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int qd = 4 * mt + j;
            if (qd < NPQ) *reinterpret_cast<S*>(ob + eoff + (size_t)qd * quad_bytes + (size_t)g * sizeof(S)) = o[j];
          }
        }
        if constexpr (Pr::mixed) {
          if (comp) {
            // operand companion of the result: modes 1.. in the operand precision, mean in fp32
            using E1 = typename Pr::E1;
            typedef E1 e4_t __attribute__((ext_vector_type(4)));
            E1* rec = reinterpret_cast<E1*>(lds_comp) + (wslot * 16 + col) * CES + v * (32 * KS) + 16 * mt;
            if (spread) {
              // mode 16 mt + g from every lane group (modes 16 mt + 4 .. 15 are padding, zero
              // since the kernel's start)
              rec[g] = to_operand<E1>(oc[0]);
            } else {
              e4_t h;
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const int mode = 16 * mt + 4 * g + j;
                h[j] = mode > 0 ? to_operand<E1>(oc[j]) : (E1)0.0f;
              }
              // modes 16 mt + 4 g .. + 3 of (col, v) into this wave's staging record
              *reinterpret_cast<e4_t*>(rec + 4 * g) = h;
            }
            if (mt == 0 && g == 0) {
              a.c0_out[v * epad + e] = float(oc[0]);
              if constexpr (kEpi == kEpiRKW) a.mean_out[v * epad + e] = oc[0];
            }
          }
        }
      }
    }
    if constexpr (Pr::mixed) {
      if (comp) {
        // every lane sends the 16-byte slot it reads as an MFMA operand (modes 32 s + 8 g ..
        // + 7), so the 4 lanes of a column write their element's whole record (its padding
        // slots zero since the kernel's start).  The slots were written by other lanes of
        // this wave: order the LDS writes before the reads (and, after them, the reads
        // before the next group's writes)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (live) {
          // the element's record, then the lane's 16-byte slot within it
          Op* qrec = reinterpret_cast<Op*>(a.q_out) + (size_t)e * (5 * KS * 4);
          asm("" : "+v"(qrec));
#pragma unroll
          for (int v = 0; v < 5; ++v)
#pragma unroll
            for (int s = 0; s < KS; ++s)
              qrec[(v * KS + s) * 4 + g] = lds_comp[(wslot * 16 + col) * (CES / 8) + (v * KS + s) * 4 + g];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
}

// Operand companion of an fp64 state (mixed modes).  A workgroup packs 64 consecutive
// elements (E_pad is a multiple of 64): the fp64 mode quads are read with the element
// index fastest (contiguous 32-byte quads), converted into the records in LDS, and the
// 64 records, contiguous in q, leave as 16-byte slots.
template <int P, class Pr>
__global__ __launch_bounds__(256) void pack_kernel(MeshView m, const double* __restrict__ u,
                                                   typename Pr::E1* __restrict__ q, float* __restrict__ c0) {
  using E1 = typename Pr::E1;
  using O = Ord<P>;
  constexpr int NP = O::NP, REC = 32 * Layout<P, 8>::KS, NPQ = npq_of(NP), RQ = REC / 4;
  __shared__ E1 rec[64 * 5 * REC];
  const int64_t e0 = (int64_t)blockIdx.x * 64;
  typedef double d4v_t __attribute__((ext_vector_type(4)));
  typedef E1 e4v_t __attribute__((ext_vector_type(4)));
  // all of a thread's state reads are issued before the first conversion
  constexpr int NL = 5 * NPQ * 64, NIT = (NL + 255) / 256;
  d4v_t x[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = (int)threadIdx.x + 256 * it;
    if (i < NL) {
      const int el = i % 64, vk = i / 64;  // vk = v * NPQ + k
      x[it] = *reinterpret_cast<const d4v_t*>(u + ((int64_t)vk * m.epad + e0 + el) * 4);
    }
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = (int)threadIdx.x + 256 * it;
    if (i < NL) {
      const int el = i % 64, vk = i / 64, v = vk / NPQ, k = vk % NPQ;
      e4v_t h;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int mode = 4 * k + j;
        h[j] = (mode > 0 && mode < NP) ? to_operand<E1>(x[it][j]) : (E1)0.0f;
      }
      *reinterpret_cast<e4v_t*>(rec + (el * 5 + v) * REC + 4 * k) = h;
      if (k == 0) c0[v * m.epad + e0 + el] = float(x[it][0]);
    }
  }
  // the record slots past the last mode quad
  for (int i = threadIdx.x; i < 5 * (RQ - NPQ) * 64; i += 256) {
    const int el = i % 64, r = i / 64, v = r / (RQ - NPQ), k = NPQ + r % (RQ - NPQ);
    *reinterpret_cast<e4v_t*>(rec + (el * 5 + v) * REC + 4 * k) = e4v_t{(E1)0.0f, (E1)0.0f, (E1)0.0f, (E1)0.0f};
  }
  __syncthreads();
  const uint4* src = reinterpret_cast<const uint4*>(rec);
  uint4* dst = reinterpret_cast<uint4*>(q + e0 * 5 * REC);
  for (int i = threadIdx.x; i < 64 * 5 * REC * (int)sizeof(E1) / 16; i += 256) dst[i] = src[i];
}

size_t companion_bytes(int p, int64_t epad) {
  const int np = (p + 1) * (p + 2) * (p + 3) / 6;
  const int ks = (np + 31) / 32;
  const size_t q = (size_t)epad * 5 * 32 * ks * 2;
  return ((q + 255) & ~(size_t)255) + (size_t)epad * 5 * sizeof(float);
}

hipError_t launch_pack(int p, int prec, const MeshView& m, const void* u, void* q, float* c0, hipStream_t s) {
  if (m.epad % 64 != 0) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)(m.epad / 64);
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
  // stage the tables in LDS when they fit beside the companion staging and face-record
  // areas in the LDS share of one workgroup (160 KB per CU over the workgroups resident per CU)
  constexpr size_t comp_bytes =
      Pr::mixed ? sizeof(typename Pr::Op) / 8 * 4 * 16 * (5 * 32 * L::KS + 8) + 2 * sizeof(float) * 7 * 4 * 64 : 0;
  constexpr size_t nbr_bytes = stage_nbr_lds<P, Pr>() ? sizeof(typename Pr::Op) * 4 * 5 * L::KS * 64 : 0;
  constexpr bool lds = tab_bytes + comp_bytes + nbr_bytes <= 160 * 1024 / stage_min_blocks<P, Pr>();
  auto kern = a.flux == 1 ? stage_kernel<P, Pr, lds, true, kEpiRK> : stage_kernel<P, Pr, lds, false, kEpiRK>;
  if constexpr (Pr::mixed || P <= 3) {  // the kernel's kFlat
    if (!a.rk)
      kern = a.flux == 1 ? stage_kernel<P, Pr, lds, true, kEpiResid> : stage_kernel<P, Pr, lds, false, kEpiResid>;
    else if (a.alpha == 0.0)
      kern = a.flux == 1 ? stage_kernel<P, Pr, lds, true, kEpiRK0> : stage_kernel<P, Pr, lds, false, kEpiRK0>;
  }
  if constexpr (Pr::mixed) {
    if (a.rk && a.alpha != 0.0 && a.alpha_w != 0.0)
      kern = a.flux == 1 ? stage_kernel<P, Pr, lds, true, kEpiRKW> : stage_kernel<P, Pr, lds, false, kEpiRKW>;
  }
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
