// Vector-Jacobian product of the DG residual, Ubar = (dR/dU)^T W, for gfx950.
//
// R_e = (V_e - S_e)/|K_e| with V_e = sum_q,d G_d^T Y_d(U_q), Y_d = sum_c M[d][c] F_c,
// S_e = sum_f sum_q L_f^T Fhat_N(U-_fq, U+_fq).  With Wt = W/|K| per element:
//   volume: Gbar_d(q) = sum_i w_q dphi_i/dxi_d(q) Wt_i           (points x modes MFMA)
//           Ubar_q   = sum_c A_c(U_q)^T Z_c,  Z_c = sum_d M[d][c] Gbar_d
//           Ubar    += B^T Ubar_q                                   (modes x points MFMA)
//   faces:  fb_e(q)  = sum_i w^f_q phi_i(xi_f(q)) Wt_e,i  and the same for the neighbour
//           with its own face table (f+, selected per column by masked operands);
//           the neighbour's residual sees this element's trace through
//           Fhat(U+, U-, -N) = -Fhat(U-, U+, N), so
//           Ubar-_q  = (dFhat/dU-)^T (fb_nbr(q) - fb_e(q))          (interior)
//           Ubar-_q  = -(dFhat/dU- + dFhat/dU+ dghost/dU-)^T fb_e(q) (boundary)
//           Ubar    += B_f^T Ubar-_q
// Every element gathers its neighbours' U and W and writes only its own Ubar: no
// atomics.  Ties of max(lambda-, lambda+) split the derivative evenly; d|x| = 0 at 0.
// Rusanov's and Roe's fluxes are both antisymmetric under exchanging the states and
// negating the normal, which the interior-face rule above relies on.
#include <hip/hip_runtime.h>

#include "dg_kernels.hpp"
#include "dg_launch.hpp"

namespace tetdg {

namespace {

// g . (dF_N/dU)(U) for one state: returns the gradient of phi(U) = g . F_N(U).
template <class T>
__device__ __forceinline__ void flux_n_vjp(const T U[5], const T N[3], const T g[5], T gm1, T out[5]) {
  const T rho = U[0], ir = T(1) / rho;
  const T u[3] = {U[1] * ir, U[2] * ir, U[3] * ir};
  const T un = u[0] * N[0] + u[1] * N[1] + u[2] * N[2];
  const T q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T p = gm1 * (U[4] - T(0.5) * rho * q2);
  const T Q = g[0] * rho + g[1] * U[1] + g[2] * U[2] + g[3] * U[3] + g[4] * U[4];
  const T H = g[1] * N[0] + g[2] * N[1] + g[3] * N[2] + g[4] * un;
  out[0] = -un * ir * Q + un * g[0] + gm1 * T(0.5) * q2 * H - p * g[4] * un * ir;
#pragma unroll
  for (int a = 0; a < 3; ++a) out[1 + a] = N[a] * ir * Q + un * g[1 + a] - gm1 * u[a] * H + p * g[4] * N[a] * ir;
  out[4] = un * g[4] + gm1 * H;
}

// sum_c Z_c . (dF_c/dU)(U): gradient of phi(U) = sum_c Z_c . F_c(U).
template <class T>
__device__ __forceinline__ void flux_vjp(const T U[5], const T Z[3][5], T gm1, T out[5]) {
  const T rho = U[0], ir = T(1) / rho;
  const T u[3] = {U[1] * ir, U[2] * ir, U[3] * ir};
  const T q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T p = gm1 * (U[4] - T(0.5) * rho * q2);
  T H = T(0), a0 = T(0), a4 = T(0), uq = T(0), z4u = T(0);
  T Qc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Qc[c] = Z[c][0] * rho + Z[c][1] * U[1] + Z[c][2] * U[2] + Z[c][3] * U[3] + Z[c][4] * U[4];
    H += Z[c][1 + c] + Z[c][4] * u[c];
    uq += u[c] * Qc[c];
    a0 += u[c] * Z[c][0];
    a4 += u[c] * Z[c][4];
    z4u += Z[c][4] * u[c];
  }
  out[0] = -uq * ir + a0 + gm1 * T(0.5) * q2 * H - p * z4u * ir;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T zm = u[0] * Z[0][1 + a] + u[1] * Z[1][1 + a] + u[2] * Z[2][1 + a];
    out[1 + a] = Qc[a] * ir + zm - gm1 * u[a] * H + p * Z[a][4] * ir;
  }
  out[4] = a4 + gm1 * H;
}

// Wave speed lambda = |u.N| + c |N| and its gradient with respect to U.
template <class T>
__device__ __forceinline__ T wave_speed_grad(const T U[5], const T N[3], T nn, T gamma, T grad[5]) {
  const T gm1 = gamma - T(1);
  const T rho = U[0], ir = T(1) / rho;
  const T u[3] = {U[1] * ir, U[2] * ir, U[3] * ir};
  const T un = u[0] * N[0] + u[1] * N[1] + u[2] * N[2];
  const T q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T p = gm1 * (U[4] - T(0.5) * rho * q2);
  const T c = sqrt(gamma * p * ir);
  const T sg = un > T(0) ? T(1) : (un < T(0) ? T(-1) : T(0));
  const T k = gamma / (T(2) * c * rho);  // dc/dp_eff
  grad[0] = sg * (-un * ir) + nn * k * (gm1 * T(0.5) * q2 - p * ir);
#pragma unroll
  for (int a = 0; a < 3; ++a) grad[1 + a] = sg * N[a] * ir + nn * k * (-gm1 * u[a]);
  grad[4] = nn * k * gm1;
  return fabs(un) + c * nn;
}

// (dFhat/da)^T g and (dFhat/db)^T g for the Rusanov flux Fhat_N(a, b).
template <class T>
__device__ __forceinline__ void rusanov_vjp(const T a[5], const T b[5], const T N[3], T nn, T gamma, const T g[5],
                                            T ga[5], T gb[5], bool need_b) {
  const T gm1 = gamma - T(1);
  T la_g[5], lb_g[5];
  const T la = wave_speed_grad<T>(a, N, nn, gamma, la_g);
  const T lb = wave_speed_grad<T>(b, N, nn, gamma, lb_g);
  const T lam = la > lb ? la : lb;
  const T wa = la > lb ? T(1) : (la < lb ? T(0) : T(0.5));
  const T wb = T(1) - wa;
  T gd = T(0);
#pragma unroll
  for (int v = 0; v < 5; ++v) gd += g[v] * (b[v] - a[v]);
  T fa[5];
  flux_n_vjp<T>(a, N, g, gm1, fa);
#pragma unroll
  for (int v = 0; v < 5; ++v) ga[v] = T(0.5) * fa[v] + T(0.5) * lam * g[v] - T(0.5) * gd * wa * la_g[v];
  if (need_b) {
    T fb[5];
    flux_n_vjp<T>(b, N, g, gm1, fb);
#pragma unroll
    for (int v = 0; v < 5; ++v) gb[v] = T(0.5) * fb[v] - T(0.5) * lam * g[v] - T(0.5) * gd * wb * lb_g[v];
  }
}

// (dFhat/da)^T g and (dFhat/db)^T g for the Roe flux Fhat_N(a, b) (the forward
// evaluation in roe_n, differentiated in reverse order).  The central part reuses
// flux_n_vjp; the dissipation -|N|/2 sum_k |lambda_k| alpha_k r_k is taken through the
// Roe averages back to both states.  Harten's fix is C1 at |lambda| = delta, and d|x| = 0
// at x = 0 for the entropy/shear waves.
template <class T>
__device__ __forceinline__ void roe_vjp(const T a[5], const T b[5], const T N[3], T nn, T gamma, const T g[5], T ga[5],
                                        T gb[5], bool need_b) {
  const T gm1 = gamma - T(1), hf = T(0.5);
  const T inn = T(1) / nn;
  const T n[3] = {N[0] * inn, N[1] * inn, N[2] * inn};
  // ---- forward
  const T rl = a[0], rr = b[0];
  const T irl = T(1) / rl, irr = T(1) / rr;
  const T ul[3] = {a[1] * irl, a[2] * irl, a[3] * irl};
  const T ur[3] = {b[1] * irr, b[2] * irr, b[3] * irr};
  const T kl = ul[0] * ul[0] + ul[1] * ul[1] + ul[2] * ul[2];
  const T kr = ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2];
  const T pl = gm1 * (a[4] - hf * rl * kl), pr = gm1 * (b[4] - hf * rr * kr);
  const T hl = (a[4] + pl) * irl, hr = (b[4] + pr) * irr;
  const T sl = sqrt(rl), sr = sqrt(rr);
  const T iw = T(1) / (sl + sr);
  const T rho = sl * sr;
  T u[3], du[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    u[d] = (sl * ul[d] + sr * ur[d]) * iw;
    du[d] = ur[d] - ul[d];
  }
  const T h = (sl * hl + sr * hr) * iw;
  const T q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T c = sqrt(gm1 * (h - hf * q2));
  const T ic2 = T(1) / (c * c);
  const T un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
  const T dr = rr - rl, dp = pr - pl;
  const T dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  const T del = T(0.1) * c;
  const T lm1 = un - c, lm4 = un + c;
  const bool f1 = fabs(lm1) < del, f4 = fabs(lm4) < del;
  const T l1 = f1 ? (lm1 * lm1 + del * del) * hf / del : fabs(lm1);
  const T l4 = f4 ? (lm4 * lm4 + del * del) * hf / del : fabs(lm4);
  const T l2 = fabs(un);
  const T s = hf * ic2;
  const T a1 = (dp - rho * c * dun) * s;
  const T a2 = dr - dp * ic2;
  const T a4 = (dp + rho * c * dun) * s;
  const T k1 = l1 * a1, k2 = l2 * a2, k3 = l2 * rho, k4 = l4 * a4;
  const T udu = u[0] * du[0] + u[1] * du[1] + u[2] * du[2];
  // ---- reverse: the dissipation enters the flux as -|N|/2 diss
  T G[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) G[v] = -hf * nn * g[v];
  const T Gn = G[1] * n[0] + G[2] * n[1] + G[3] * n[2];
  T gu[3], gdu[3];
  T gk1 = G[0] + G[4] * (h - un * c), gk2 = G[0] + G[4] * hf * q2;
  T gk3 = G[4] * (udu - un * dun), gk4 = G[0] + G[4] * (h + un * c);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    gk1 += G[1 + d] * (u[d] - c * n[d]);
    gk2 += G[1 + d] * u[d];
    gk3 += G[1 + d] * (du[d] - dun * n[d]);
    gk4 += G[1 + d] * (u[d] + c * n[d]);
    gu[d] = G[1 + d] * (k1 + k2 + k4) + G[4] * k3 * du[d];
    gdu[d] = G[1 + d] * k3 + G[4] * k3 * u[d];
  }
  T gc = (k4 - k1) * Gn + G[4] * un * (k4 - k1);
  T gdun = -k3 * Gn - G[4] * k3 * un;
  T gun = G[4] * c * (k4 - k1) - G[4] * k3 * dun;
  T gh = G[4] * (k1 + k4);
  T gq2 = G[4] * hf * k2;
  const T gl1 = gk1 * a1, gl2 = gk2 * a2 + gk3 * rho, gl4 = gk4 * a4;
  const T ga1 = gk1 * l1, ga2 = gk2 * l2, ga4 = gk4 * l4;
  T grho = gk3 * l2;
  // alpha_k
  T gdp = (ga1 + ga4) * s - ga2 * ic2;
  const T gdr = ga2;
  grho += (ga4 - ga1) * c * dun * s;
  gc += (ga4 - ga1) * rho * dun * s;
  gdun += (ga4 - ga1) * rho * c * s;
  const T gic2 = hf * (ga1 * (dp - rho * c * dun) + ga4 * (dp + rho * c * dun)) - ga2 * dp;
  // wave speeds (Harten: fix = (lam^2 + del^2) / (2 del), del = 0.1 c)
  {
    const T sg2 = un > T(0) ? T(1) : (un < T(0) ? T(-1) : T(0));
    gun += gl2 * sg2;
    const T d1 = f1 ? lm1 / del : (lm1 > T(0) ? T(1) : (lm1 < T(0) ? T(-1) : T(0)));
    const T d4 = f4 ? lm4 / del : (lm4 > T(0) ? T(1) : (lm4 < T(0) ? T(-1) : T(0)));
    gun += gl1 * d1 + gl4 * d4;
    gc += -gl1 * d1 + gl4 * d4;
    if (f1) gc += gl1 * (del * del - lm1 * lm1) * hf / (del * del) * T(0.1);
    if (f4) gc += gl4 * (del * del - lm4 * lm4) * hf / (del * del) * T(0.1);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    gu[d] += gun * n[d];
    gdu[d] += gdun * n[d];
  }
  gc += gic2 * (-T(2) * ic2 / c);
  // c = sqrt(gm1 (h - q2 / 2))
  gh += gc * gm1 * hf / c;
  gq2 += -gc * gm1 * T(0.25) / c;
#pragma unroll
  for (int d = 0; d < 3; ++d) gu[d] += T(2) * u[d] * gq2;
  // Roe averages
  T gsl = gh * hl * iw + grho * sr, gsr = gh * hr * iw + grho * sl;
  const T ghl = gh * sl * iw, ghr = gh * sr * iw;
  T giw = gh * (sl * hl + sr * hr);
  T gul[3], gur[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    gsl += iw * gu[d] * ul[d];
    gsr += iw * gu[d] * ur[d];
    gul[d] = gu[d] * sl * iw - gdu[d];
    gur[d] = gu[d] * sr * iw + gdu[d];
    giw += gu[d] * (sl * ul[d] + sr * ur[d]);
  }
  gsl += -giw * iw * iw;
  gsr += -giw * iw * iw;
  T grl = gsl * hf / sl - gdr, grr = gsr * hf / sr + gdr;
  T gpl = -gdp + ghl * irl, gpr = gdp + ghr * irr;
  T gal4 = ghl * irl, gbr4 = ghr * irr;
  T girl = ghl * (a[4] + pl), girr = ghr * (b[4] + pr);
  // pressures
  gal4 += gpl * gm1;
  gbr4 += gpr * gm1;
  grl += -gpl * gm1 * hf * kl;
  grr += -gpr * gm1 * hf * kr;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    gul[d] += -gpl * gm1 * rl * ul[d];
    gur[d] += -gpr * gm1 * rr * ur[d];
    girl += gul[d] * a[1 + d];
    girr += gur[d] * b[1 + d];
  }
  grl += -girl * irl * irl;
  grr += -girr * irr * irr;
  // central part (F(a).N + F(b).N) / 2
  T fa[5];
  flux_n_vjp<T>(a, N, g, gm1, fa);
  ga[0] = hf * fa[0] + grl;
#pragma unroll
  for (int d = 0; d < 3; ++d) ga[1 + d] = hf * fa[1 + d] + gul[d] * irl;
  ga[4] = hf * fa[4] + gal4;
  if (need_b) {
    T fb[5];
    flux_n_vjp<T>(b, N, g, gm1, fb);
    gb[0] = hf * fb[0] + grr;
#pragma unroll
    for (int d = 0; d < 3; ++d) gb[1 + d] = hf * fb[1 + d] + gur[d] * irr;
    gb[4] = hf * fb[4] + gbr4;
  }
}

template <class Pr, int NP, int KS>
__device__ __forceinline__ void load_ops(const char* __restrict__ base, uint32_t var_bytes, uint32_t elem_off,
                                         const uint32_t (&off)[KS], const bool (&keep)[KS], typename Pr::T scale,
                                         typename Pr::Op (&b)[5][KS]) {
  using S = typename Pr::S;
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const S x = *reinterpret_cast<const S*>(base + (size_t)v * var_bytes + off[s] + elem_off);
      b[v][s] = keep[s] ? typename Pr::Op(scale * x) : typename Pr::Op(0);
    }
}

template <int P, class Pr>
constexpr int vjp_min_blocks() {
  return (!Pr::f64 && P <= 2) ? 2 : 1;
}

// kRoe selects the face flux at compile time (Roe's adjoint needs more registers).  FP32 up
// to P2 fits two waves per SIMD; FP64 and higher orders take one.  kLds: the operand tables
// are copied into LDS once per workgroup (every MFMA A operand is then an LDS read instead
// of an L1/L2 access); P4 FP64 (320 KB) and P4 FP32 (160 KB) read them from global memory.
template <int P, class Pr, bool kRoe, bool kLds>
__global__ __launch_bounds__(256, (vjp_min_blocks<P, Pr>())) void vjp_kernel(VjpArgs a) {
  using O = Ord<P>;
  using V = VjpLayout<P>;
  using S = typename Pr::S;
  using T = typename Pr::T;
  using Op = typename Pr::Op;
  using Acc = typename Pr::Acc;
  constexpr int NP = O::NP, NQ = O::NQ, NF = O::NF, MT = O::MT, QT = O::QT, FT = O::FT, KS = V::KS;
  static_assert(Pr::KW == 1, "the adjoint uses the f64/f32 instructions");

  __shared__ Op lds_tab[kLds ? V::n_slots * 64 : 1];
  const Op* __restrict__ vt;
  if constexpr (kLds) {
    const Op* src = reinterpret_cast<const Op*>(a.tab);
    for (int i = threadIdx.x; i < V::n_slots * 64; i += blockDim.x) lds_tab[i] = src[i];
    __syncthreads();
    vt = lds_tab;
  } else {
    vt = reinterpret_cast<const Op*>(a.tab);
  }
  const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
  const char* __restrict__ ubase = reinterpret_cast<const char*>(a.u);
  const char* __restrict__ wbase = reinterpret_cast<const char*>(a.w);
  char* __restrict__ obase = reinterpret_cast<char*>(a.ubar);
  const MeshView& mv = a.mesh;
  const int64_t epad = mv.epad;
  constexpr int NPQ = npq_of(NP);
  const uint32_t quad_bytes = (uint32_t)(epad * 4 * sizeof(S));
  const uint32_t var_bytes = quad_bytes * NPQ;
  auto moff = [&](int mode) { return (uint32_t)(mode >> 2) * quad_bytes + (uint32_t)(mode & 3) * sizeof(S); };
  const T gamma = T(a.gamma), gm1 = T(a.gamma - 1.0);
  T far[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) far[v] = T(a.far[v]);
  uint32_t off[KS];
  bool keep[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int mode = 4 * s + g;
    keep[s] = mode < NP;
    off[s] = moff(mode < NP ? mode : NP - 1);
  }

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
    T Mt[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Mt[i] = T(Md[i]);
    const T ivol = T(mv.inv_vol[e]);
    const int fcode = mv.fcode[e];
    // the four neighbours, requested with the element's own data (not at each face)
    int nbr[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) nbr[f] = mv.nbr[f * epad + e];

    Op bc[5][KS], bw[5][KS];
    load_ops<Pr, NP, KS>(ubase, var_bytes, eoff, off, keep, T(1), bc);
    load_ops<Pr, NP, KS>(wbase, var_bytes, eoff, off, keep, ivol, bw);

    Acc acc[MT][5];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[mt][v] = Acc{0, 0, 0, 0};

    // ------------------------------------------------------------ volume
#pragma unroll 1
    for (int qt = 0; qt < QT; ++qt) {
      Acc du[5], dg[3][5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        du[v] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int d = 0; d < 3; ++d) dg[d][v] = Acc{0, 0, 0, 0};
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const Op av = vt[V::interp(qt, s) * 64 + lane];
#pragma unroll
        for (int v = 0; v < 5; ++v) du[v] = Pr::mfma(av, bc[v][s], du[v]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const Op ad = vt[V::tinterp(qt, d, s) * 64 + lane];
#pragma unroll
          for (int v = 0; v < 5; ++v) dg[d][v] = Pr::mfma(ad, bw[v][s], dg[d][v]);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = 16 * qt + drow_of<Pr>(g, j);
        T ub[5];
        if (q < NQ) {
          T U[5], Z[3][5];
#pragma unroll
          for (int v = 0; v < 5; ++v) U[v] = T(du[v][j]);
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int v = 0; v < 5; ++v)
              Z[c][v] = Mt[c] * T(dg[0][v][j]) + Mt[3 + c] * T(dg[1][v][j]) + Mt[6 + c] * T(dg[2][v][j]);
          flux_vjp<T>(U, Z, gm1, ub);
        } else {
#pragma unroll
          for (int v = 0; v < 5; ++v) ub[v] = T(0);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const Op av = vt[V::tproj(mt, qt, j) * 64 + lane];
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[mt][v] = Pr::mfma(av, Pr::op1(ub[v]), acc[mt][v]);
        }
      }
    }

    // ------------------------------------------------------------ faces
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      T N[3];
      face_normal<T>(f, Md, N);
      const T nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
      const int nbf = f == 0 ? nbr[0] : f == 1 ? nbr[1] : f == 2 ? nbr[2] : nbr[3];
      const int fpl = (fcode >> (2 * f)) & 3;
      const int en = nbf >= 0 ? nbf : e;
      const uint32_t enoff = (uint32_t)en * 4 * sizeof(S);
      const T ivn = T(mv.inv_vol[en]);
      Op bn[5][KS], bwn[5][KS];
      load_ops<Pr, NP, KS>(ubase, var_bytes, enoff, off, keep, T(1), bn);
      load_ops<Pr, NP, KS>(wbase, var_bytes, enoff, off, keep, ivn, bwn);
#pragma unroll 1
      for (int ft = 0; ft < FT; ++ft) {
        Acc dm[5], dp[5], wm[5], wp[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) dm[v] = dp[v] = wm[v] = wp[v] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const Op av = vt[V::trace(f, ft, s) * 64 + lane];
          const Op aw = vt[V::ttrace(f, ft, s) * 64 + lane];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            dm[v] = Pr::mfma(av, bc[v][s], dm[v]);
            wm[v] = Pr::mfma(aw, bw[v][s], wm[v]);
          }
        }
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
          const bool mine = nbf >= 0 && fpl == c;
          if (__any(mine)) {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
              const Op av = vt[V::trace(c, ft, s) * 64 + lane];
              const Op aw = vt[V::ttrace(c, ft, s) * 64 + lane];
#pragma unroll
              for (int v = 0; v < 5; ++v) {
                dp[v] = Pr::mfma(av, mine ? bn[v][s] : Op(0), dp[v]);
                wp[v] = Pr::mfma(aw, mine ? bwn[v][s] : Op(0), wp[v]);
              }
            }
          }
        }
        T ubf[5][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int q = 16 * ft + drow_of<Pr>(g, j);
          T um[5], up[5], gcot[5], ga[5], gb[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            um[v] = T(dm[v][j]);
            up[v] = T(dp[v][j]);
          }
          const bool bnd = nbf < 0;
          if (bnd) ghost_state<T>(-nbf, um, N, far, up);
#pragma unroll
          for (int v = 0; v < 5; ++v) gcot[v] = bnd ? -T(wm[v][j]) : T(wp[v][j]) - T(wm[v][j]);
          if (q < NF) {
            if constexpr (kRoe)
              roe_vjp<T>(um, up, N, nn, gamma, gcot, ga, gb, bnd);
            else
              rusanov_vjp<T>(um, up, N, nn, gamma, gcot, ga, gb, bnd);
            if (bnd) {
              if (-nbf == 2) {  // slip wall: ghost = (rho, m - 2 (m.n) n, E), symmetric Jacobian
                const T nn2 = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
                const T gn = (gb[1] * N[0] + gb[2] * N[1] + gb[3] * N[2]) / nn2;
                ga[0] += gb[0];
#pragma unroll
                for (int d = 0; d < 3; ++d) ga[1 + d] += gb[1 + d] - T(2) * gn * N[d];
                ga[4] += gb[4];
              }
            }
          } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) ga[v] = T(0);
          }
#pragma unroll
          for (int v = 0; v < 5; ++v) ubf[v][j] = ga[v];
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const Op av = vt[V::tlift(mt, f, ft, j) * 64 + lane];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[mt][v] = Pr::mfma(av, Pr::op1(ubf[v][j]), acc[mt][v]);
          }
      }
    }

    if (e < mv.n_elem) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int mode = 16 * mt + drow_of<Pr>(g, j);
          // padding modes of the last quad are written 0
          if ((mode >> 2) < npq_of(NP)) {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
              const size_t o = (size_t)v * var_bytes + moff(mode) + eoff;
              double r = 0.0;
              if (mode < NP) {
                r = a.c * double(acc[mt][v][j]);
                for (int k = 0; k < a.n_terms; ++k)
                  r += a.ya[k] * double(*reinterpret_cast<const S*>(reinterpret_cast<const char*>(a.y[k]) + o));
              }
              *reinterpret_cast<S*>(obase + o) = S(r);
            }
          }
        }
    }
  }
}

template <int P, class Pr>
hipError_t launch_vjp_impl(const VjpArgs& a, hipStream_t stream) {
  // tables in LDS when they fit in the share of one workgroup (160 KB per CU over the
  // workgroups resident per CU)
  constexpr bool lds = sizeof(typename Pr::Op) * VjpLayout<P>::n_slots * 64 <= 160 * 1024 / vjp_min_blocks<P, Pr>();
  auto kern = a.flux == 1 ? vjp_kernel<P, Pr, true, lds> : vjp_kernel<P, Pr, false, lds>;
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

}  // namespace

hipError_t launch_vjp(int p, int prec, const VjpArgs& a, hipStream_t stream) {
  const bool f32 = prec == 1;  // the mixed modes keep an fp64 state: their adjoint is fp64
  switch (p) {
    case 1: return f32 ? launch_vjp_impl<1, PrecF32>(a, stream) : launch_vjp_impl<1, PrecF64>(a, stream);
    case 2: return f32 ? launch_vjp_impl<2, PrecF32>(a, stream) : launch_vjp_impl<2, PrecF64>(a, stream);
    case 3: return f32 ? launch_vjp_impl<3, PrecF32>(a, stream) : launch_vjp_impl<3, PrecF64>(a, stream);
    case 4: return f32 ? launch_vjp_impl<4, PrecF32>(a, stream) : launch_vjp_impl<4, PrecF64>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tetdg
