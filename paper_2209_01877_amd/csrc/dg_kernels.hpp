// Device-side building blocks of the DG kernels: MFMA precision traits, the
// Euler flux at a point, the Rusanov face flux with an area-weighted normal,
// and boundary ghost states.  Header-only, included by the .hip files.
#pragma once
#include <hip/hip_runtime.h>

#include "dg_common.hpp"

namespace tetdg {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- precision traits
// S  : storage type of the state (global memory)
// T  : arithmetic type of the pointwise fluxes
// Op : MFMA operand type per lane, KW values per lane per slot
struct PrecF64 {
  using S = double;
  using T = double;
  using Op = double;
  using Acc = d4_t;
  static constexpr int KW = 1;
  static constexpr bool f64 = true;
  static constexpr bool mixed = false;
  __device__ static Acc mfma(Op a, Op b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static Op op1(T x) { return x; }
};
struct PrecF32 {
  using S = float;
  using T = float;
  using Op = float;
  using Acc = f4_t;
  static constexpr int KW = 1;
  static constexpr bool f64 = false;
  static constexpr bool mixed = false;
  __device__ static Acc mfma(Op a, Op b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static Op op1(T x) { return x; }
};
struct PrecBF16 {
  using S = double;
  using T = float;
  using Op = bf8_t;
  using E1 = __bf16;
  using Acc = f4_t;
  static constexpr int KW = 8;
  static constexpr bool f64 = false;
  static constexpr bool mixed = true;
  __device__ static Acc mfma(Op a, Op b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
struct PrecF16 {
  using S = double;
  using T = float;
  using Op = h8_t;
  using E1 = _Float16;
  using Acc = f4_t;
  static constexpr int KW = 8;
  static constexpr bool f64 = false;
  static constexpr bool mixed = true;
  __device__ static Acc mfma(Op a, Op b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

template <class Pr>
__device__ __forceinline__ int drow_of(int g, int j) {
  return drow(Pr::f64, g, j);
}

// ---------------------------------------------------------------- arithmetic helpers
// fp32 pointwise physics uses the hardware reciprocal and square root (about one ulp);
// fp64 keeps correctly rounded division and square root.
__device__ __forceinline__ float prec_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double prec_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float prec_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double prec_sqrt(double x) { return sqrt(x); }

// double -> bf16 / fp16 operand through float.  Rounding to float first and then to the
// operand type equals a single correct rounding (float carries at least 2p + 2 bits of
// either target), but the compiler folds the two conversions into one double -> 16-bit
// truncation that it expands into a ten-instruction round-to-odd sequence; the empty asm
// makes the float opaque, so each step is one conversion instruction.
template <class E1>
__device__ __forceinline__ E1 to_operand(double x) {
  float f = (float)x;
  asm("" : "+v"(f));
  return (E1)f;
}

// ---------------------------------------------------------------- Euler physics
// The pointwise physics is written with explicit fused multiply-adds and compiled without
// letting the compiler contract any other product into a sum: every inlined copy of a
// function then rounds identically, so a point whose state equals the cell mean reproduces
// the cell-mean flux bit for bit (the mixed modes rely on this for exact free-stream
// preservation).  Two-sided sums in the face fluxes add one-sided terms, which keeps the
// flux exactly antisymmetric under exchanging the two states and negating the normal.
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Contravariant flux rows y_d = sum_e M[d][e] F_e(U) for d = 0..2, where F_e is the
// Euler flux in direction e (eq. 2, 3-D) and M = |det J| J^-1:
//   theta_d = M_d . v,  y_d = (rho theta_d, m theta_d + p M_d, (E + p) theta_d).
template <class T>
__device__ __forceinline__ void contra_flux(const T u[5], const T M[9], T gm1, T y[3][5]) {
#pragma clang fp contract(off)
  const T rho = u[0];
  const T ir = prec_rcp(rho);
  const T vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
  const T mv = fmaT(u[1], vx, fmaT(u[2], vy, u[3] * vz));
  const T p = gm1 * fmaT(T(-0.5), mv, u[4]);
  const T ep = u[4] + p;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T th = fmaT(M[3 * d + 0], vx, fmaT(M[3 * d + 1], vy, M[3 * d + 2] * vz));
    y[d][0] = rho * th;
    y[d][1] = fmaT(u[1], th, p * M[3 * d + 0]);
    y[d][2] = fmaT(u[2], th, p * M[3 * d + 1]);
    y[d][3] = fmaT(u[3], th, p * M[3 * d + 2]);
    y[d][4] = ep * th;
  }
}

// Rusanov flux through an area-weighted normal N (|N| = nn):
//   Fhat = (F(um).N + F(up).N)/2 - max(|um.N| + c- nn, |up.N| + c+ nn)/2 (up - um)
template <class T>
__device__ __forceinline__ void rusanov_n(const T um[5], const T up[5], const T N[3], T nn, T gamma, T out[5]) {
#pragma clang fp contract(off)
  const T gm1 = gamma - T(1);
  const T irm = prec_rcp(um[0]), irp = prec_rcp(up[0]);
  const T unm = fmaT(um[1], N[0], fmaT(um[2], N[1], um[3] * N[2])) * irm;
  const T unp = fmaT(up[1], N[0], fmaT(up[2], N[1], up[3] * N[2])) * irp;
  const T km = fmaT(um[1], um[1], fmaT(um[2], um[2], um[3] * um[3]));
  const T kp = fmaT(up[1], up[1], fmaT(up[2], up[2], up[3] * up[3]));
  const T pm = gm1 * fmaT(T(-0.5) * km, irm, um[4]);
  const T pp = gm1 * fmaT(T(-0.5) * kp, irp, up[4]);
  const T cm = prec_sqrt(gamma * pm * irm), cp = prec_sqrt(gamma * pp * irp);
  const T lm = fmaT(cm, nn, fabs(unm)), lp = fmaT(cp, nn, fabs(unp));
  const T hl = T(0.5) * (lm > lp ? lm : lp);
  const T h = T(0.5);
  out[0] = fmaT(h, um[0] * unm + up[0] * unp, -(hl * (up[0] - um[0])));
#pragma unroll
  for (int d = 0; d < 3; ++d)
    out[1 + d] = fmaT(h, fmaT(um[1 + d], unm, pm * N[d]) + fmaT(up[1 + d], unp, pp * N[d]),
                      -(hl * (up[1 + d] - um[1 + d])));
  out[4] = fmaT(h, (um[4] + pm) * unm + (up[4] + pp) * unp, -(hl * (up[4] - um[4])));
}

// Roe flux through an area-weighted normal N (|N| = nn): central part minus
// |N|/2 sum_k |lambda_k| alpha_k r_k with Roe averages (sqrt(rho) weights), acoustic
// waves u.n -+ c (Harten entropy fix of width 0.1 c), entropy and shear waves at u.n.
// The sum over the waves is regrouped with the acoustic pair's sum k1 + k4 and
// difference k4 - k1 (r_{1,4} = r_2 -+ c (0, n, u.n)), and every sum of one-sided
// terms is symmetric in the two states, so that, as for Rusanov's flux, exchanging the
// states and negating the normal negates the flux exactly.
template <class T>
__device__ __forceinline__ void roe_n(const T um[5], const T up[5], const T N[3], T nn, T gamma, T out[5]) {
#pragma clang fp contract(off)
  const T gm1 = gamma - T(1);
  const T inn = prec_rcp(nn);
  const T n[3] = {N[0] * inn, N[1] * inn, N[2] * inn};
  const T irl = prec_rcp(um[0]), irr = prec_rcp(up[0]);
  const T ul[3] = {um[1] * irl, um[2] * irl, um[3] * irl};
  const T ur[3] = {up[1] * irr, up[2] * irr, up[3] * irr};
  // p = (gamma - 1) (E - m.u / 2); el, er = E + p = rho H
  const T pl = gm1 * fmaT(T(-0.5), fmaT(um[1], ul[0], fmaT(um[2], ul[1], um[3] * ul[2])), um[4]);
  const T pr = gm1 * fmaT(T(-0.5), fmaT(up[1], ur[0], fmaT(up[2], ur[1], up[3] * ur[2])), up[4]);
  const T el = um[4] + pl, er = up[4] + pr;
  const T sl = prec_sqrt(um[0]), sr = prec_sqrt(up[0]);
  const T iw = prec_rcp(sl + sr);
  const T wl = sl * iw, wr = sr * iw;
  const T rho = sl * sr;
  T u[3], du[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    u[d] = wl * ul[d] + wr * ur[d];
    du[d] = ur[d] - ul[d];
  }
  const T h = wl * (el * irl) + wr * (er * irr);
  const T q2 = fmaT(u[0], u[0], fmaT(u[1], u[1], u[2] * u[2]));
  const T c = prec_sqrt(gm1 * fmaT(T(-0.5), q2, h));
  const T hic2 = T(0.5) * prec_rcp(c * c);
  const T un = fmaT(u[0], n[0], fmaT(u[1], n[1], u[2] * n[2]));
  const T dr = up[0] - um[0], dp = pr - pl;
  const T dun = fmaT(du[0], n[0], fmaT(du[1], n[1], du[2] * n[2]));
  // Harten: |lambda| -> (lambda^2 + del^2) / (2 del) inside |lambda| < del
  const T del = T(0.1) * c;
  const T dd = del * del, hid = T(0.5) * prec_rcp(del);
  auto fix = [&](T lam) {
    const T a = fabs(lam);
    return a < del ? fmaT(lam, lam, dd) * hid : a;
  };
  const T l1 = fix(un - c), l2 = fabs(un), l4 = fix(un + c);
  const T rc = rho * c;
  const T a1 = fmaT(-rc, dun, dp) * hic2;
  const T a2 = fmaT(-dp, T(2) * hic2, dr);
  const T a4 = fmaT(rc, dun, dp) * hic2;
  const T k1 = l1 * a1, k2 = l2 * a2, k3 = l2 * rho, k4 = l4 * a4;
  const T ks = k1 + k4, kdc = (k4 - k1) * c;
  const T udu = fmaT(u[0], du[0], fmaT(u[1], du[1], u[2] * du[2]));
  T diss[5];
  diss[0] = ks + k2;
#pragma unroll
  for (int d = 0; d < 3; ++d) diss[1 + d] = fmaT(diss[0], u[d], fmaT(kdc, n[d], k3 * fmaT(-dun, n[d], du[d])));
  diss[4] = fmaT(ks, h, fmaT(kdc, un, fmaT(k2, T(0.5) * q2, k3 * fmaT(-un, dun, udu))));
  // central part with the area-weighted normal
  const T unl = fmaT(ul[0], N[0], fmaT(ul[1], N[1], ul[2] * N[2]));
  const T unr = fmaT(ur[0], N[0], fmaT(ur[1], N[1], ur[2] * N[2]));
  const T hn = T(0.5) * nn;
  out[0] = fmaT(T(0.5), um[0] * unl + up[0] * unr, -(hn * diss[0]));
#pragma unroll
  for (int d = 0; d < 3; ++d)
    out[1 + d] = fmaT(T(0.5), fmaT(um[1 + d], unl, pl * N[d]) + fmaT(up[1 + d], unr, pr * N[d]), -(hn * diss[1 + d]));
  out[4] = fmaT(T(0.5), el * unl + er * unr, -(hn * diss[4]));
}

// Numerical flux chosen at compile time (Roe when kRoe, else Rusanov).
template <bool kRoe, class T>
__device__ __forceinline__ void num_flux(const T um[5], const T up[5], const T N[3], T nn, T gamma, T out[5]) {
  if constexpr (kRoe)
    roe_n<T>(um, up, N, nn, gamma, out);
  else
    rusanov_n<T>(um, up, N, nn, gamma, out);
}

// Ghost state on a boundary face: tag 1 farfield (given state), tag 2 slip wall
// (density and energy kept, normal momentum mirrored).
template <class T>
__device__ __forceinline__ void ghost_state(int tag, const T um[5], const T N[3], const T far[5], T up[5]) {
#pragma clang fp contract(off)
  if (tag == 2) {
    const T nn2 = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
    const T mn = (um[1] * N[0] + um[2] * N[1] + um[3] * N[2]) * prec_rcp(nn2);
    up[0] = um[0];
    up[1] = um[1] - T(2) * mn * N[0];
    up[2] = um[2] - T(2) * mn * N[1];
    up[3] = um[3] - T(2) * mn * N[2];
    up[4] = um[4];
  } else {
#pragma unroll
    for (int v = 0; v < 5; ++v) up[v] = far[v];
  }
}

// Area-weighted outward normal of local face f: N_f = M^T (2 A n)_ref with the
// reference vectors (1,1,1), (-1,0,0), (0,-1,0), (0,0,-1).
template <class T>
__device__ __forceinline__ void face_normal(int f, const double M[9], T N[3]) {
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const double v = f == 0 ? (M[e] + M[3 + e] + M[6 + e]) : f == 1 ? -M[e] : f == 2 ? -M[3 + e] : -M[6 + e];
    N[e] = T(v);
  }
}

}  // namespace tetdg
