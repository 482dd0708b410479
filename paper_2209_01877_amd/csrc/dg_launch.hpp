// Launch interfaces between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "dg_common.hpp"

namespace tetdg {

struct StageArgs {
  const void* u_in;   // internal state read (and whose neighbours are read)
  const void* u0;     // RK stage base state (may be null when alpha == 0)
  void* u_out;        // residual or stage result
  double alpha, dt;   // U_out = alpha U0 + (1 - alpha)(U_in + dt R)
  int rk;             // 0: store R, 1: store the stage update
  int max_blocks;     // 0: fill the device once
  MeshView mesh;
  const void* tab;    // packed MFMA operand tables
  const double* mom;  // mixed modes: [7][N_p] fp64 moments of the volume and face tables
  double gamma;
  double far[5];      // farfield conserved state
};

struct VjpArgs {
  const void* u;      // state (internal layout, S)
  const void* w;      // cotangent (internal layout, S)
  void* ubar;         // result (internal layout, S)
  int max_blocks;
  MeshView mesh;
  const void* tab;    // packed VJP operand tables (f64 or f32)
  double gamma;
  double far[5];
};

struct RefView {
  const double* qx;   // [N_q][3]
  const double* qw;   // [N_q]
  const double* B;    // [N_q][N_p]
};

hipError_t launch_stage(int p, int prec, const StageArgs& a, hipStream_t stream);
hipError_t launch_vjp(int p, int prec, const VjpArgs& a, hipStream_t stream);
hipError_t launch_set_state(int p, int prec, const MeshView& m, const double* user, void* internal, hipStream_t s);
hipError_t launch_get_state(int p, int prec, const MeshView& m, const void* internal, double* user, hipStream_t s);
hipError_t launch_volume_points(int p, const MeshView& m, const RefView& r, double* xyz, hipStream_t s);
hipError_t launch_project(int p, int prec, const MeshView& m, const RefView& r, double gamma, const double* prim,
                          void* internal, hipStream_t s);

}  // namespace tetdg
