// Launch interfaces between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "dg_common.hpp"
#include "tetdg.h"

namespace tetdg {

struct StageArgs {
  const void* u_in;   // internal state read (and whose neighbours are read)
  const void* u0;     // RK stage base state (may be null when alpha == 0)
  void* u_out;        // residual or stage result
  double alpha, dt;   // U_out = alpha U0 + (1 - alpha)(U_in + dt R)
  const void* r_add;  // when non-null, a residual part added to R (state layout, S): the viscous terms
  const double* dt_dev;  // when non-null, dt is read from this device scalar instead
  int rk;             // 0: store R, 1: store the stage update
  int max_blocks;     // 0: fill the device once
  MeshView mesh;
  const void* tab;    // packed MFMA operand tables
  const double* mom;       // mixed modes: [7][N_p] fp64 moments of the volume and face tables
  const double* mean_tab;  // mixed modes: the moments as fp64 MFMA A operands, [MT][2][64]
  double gamma;
  double far[5];      // farfield conserved state
  int flux;           // 0 Rusanov, 1 Roe
  // mixed modes: low-precision operand companion of u_in (modes 1.. as bf16/fp16,
  // [E][5][32 KS]) and its fp32 cell means ([5][E]); the stage result's companion is
  // written to q_out / c0_out when they are non-null
  const void* q_in;
  const float* c0_in;
  void* q_out;
  float* c0_out;
  // mixed modes, SSP-RK3 through rk_step (the update's algebra regrouped so that the third
  // stage does not read U0): dt is multiplied by dt_scale; when alpha_w != 0 the stored
  // result is alpha_w U0 + (1 - alpha_w) times the stage result, while the companion and
  // mean_out ([5][E_pad] fp64 cell means) are of the stage result itself; when mean_in is
  // non-null it holds the fp64 cell means of the state whose companion is q_in (u_in then
  // holds another combination)
  double dt_scale;
  double alpha_w;
  const double* mean_in;
  double* mean_out;
};

struct VjpArgs {
  const void* u;      // state (internal layout, S)
  const void* w;      // cotangent (internal layout, S)
  void* ubar;         // result (internal layout, S): c J^T W + sum_k a_k Y_k
  double c;
  int n_terms;
  const void* y[3];
  double ya[3];
  int max_blocks;
  MeshView mesh;
  const void* tab;    // packed VJP operand tables (f64 or f32)
  double gamma;
  double far[5];
  int flux;           // numerical flux: 0 Rusanov, 1 Roe
};

// Viscous (BR1) kernels: grad_kernel writes Z = grad U (15 state-layout variables,
// index 5 k + v) to out; visc_kernel reads U and Z and writes the viscous residual part
// Rv (5 variables) to out.  FP64 and FP32 (S = T = the mode's state type).
struct ViscArgs {
  const void* u;
  const void* z;
  void* out;
  int max_blocks;
  MeshView mesh;
  const void* tab;    // the stage kernel's operand tables (16x16x4 layout)
  double gamma, mu, prandtl;
  double far[5];      // farfield conserved state
  void* hbuf;         // own-half viscous face fluxes, [E_pad][4 faces][5][16 FT] (state precision)
};

struct RefView {
  const double* qx;   // [N_q][3]
  const double* qw;   // [N_q]
  const double* B;    // [N_q][N_p]
  const double* fw;   // [N_f]
  const double* Bf;   // [4][N_f][N_p]
};

hipError_t launch_stage(int p, int prec, const StageArgs& a, hipStream_t stream);
hipError_t launch_grad(int p, int prec, const ViscArgs& a, hipStream_t stream);
hipError_t launch_visc(int p, int prec, const ViscArgs& a, hipStream_t stream);
hipError_t launch_visc_nbr(int p, int prec, const ViscArgs& a, hipStream_t stream);
// Build the operand companion (q, c0) of an fp64 state for the mixed modes.
hipError_t launch_pack(int p, int prec, const MeshView& m, const void* u, void* q, float* c0, hipStream_t s);
// Bytes of one operand companion (q and c0) for the mixed modes.
size_t companion_bytes(int p, int64_t epad);
hipError_t launch_vjp(int p, int prec, const VjpArgs& a, hipStream_t stream);
hipError_t launch_set_state(int p, int prec, const MeshView& m, const double* user, void* internal, hipStream_t s);
hipError_t launch_get_state(int p, int prec, const MeshView& m, const void* internal, double* user, hipStream_t s);
hipError_t launch_volume_points(int p, const MeshView& m, const RefView& r, double* xyz, hipStream_t s);
hipError_t launch_wall_pressure(int p, int prec, const MeshView& m, const RefView& r, double gamma, const void* u,
                                double* J, void* grad, hipStream_t s);
hipError_t launch_check_state(int p, int prec, const MeshView& m, const RefView& r, double gamma, const void* u,
                              int64_t* n_bad, hipStream_t s);
hipError_t launch_local_dt(int p, int prec, const MeshView& m, double gamma, double cfl, const void* u, double* dt,
                           hipStream_t s);
hipError_t launch_stream_probe(int kind, const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_project(int p, int prec, const MeshView& m, const RefView& r, double gamma, const double* prim,
                          void* internal, hipStream_t s);
// Set a context's last-error text and return code (entry points outside api.cpp).
int ctx_fail(::tdg_ctx* c, int code, const char* msg);

}  // namespace tetdg
