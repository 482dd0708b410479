/*
 * tetdg — explicit modal DG residual and SSP-RK3 stage update for the 3-D
 * compressible Euler equations on affine tetrahedra, on one MI355X (gfx950).
 *
 * The method is the one of arXiv 2209.01877, Sec. II: conserved variables
 * U = (rho, rho u, rho v, rho w, E) (Sec. II.A, eqs. 1-4, inviscid), a modal
 * expansion U_h = sum_j c_j(t) phi_j(x) per element (Sec. II.B, eq. 10) and the
 * weak form of eq. 11 with element and face Gaussian integrals, advanced by an
 * explicit Runge-Kutta scheme (Sec. III).  The choices the paper leaves open are
 * fixed as follows and are part of this interface:
 *
 *   basis       orthonormal PKD polynomials of total degree <= p on the unit tet
 *               (0,0,0),(1,0,0),(0,1,0),(0,0,1), scaled so 6*int phi_m phi_n = delta_mn
 *               (phi_0 = 1, so c_0 is the cell mean); ordering by total degree d,
 *               then k = 0..d, j = 0..d-k, i = d-j-k of the collapsed-coordinate form.
 *   element map each tet's vertices taken in ascending global vertex id,
 *               x = X0 + [X1-X0 | X2-X0 | X3-X0] xi.  Coefficients refer to this map.
 *   quadrature  collapsed Gauss-Jacobi, n = p+1 points per direction (tet n^3,
 *               triangle n^2), exact to degree 2p+1.
 *   face flux   Rusanov (local Lax-Friedrichs), lambda = max(|u.n|+c) over both
 *               sides per quadrature point; Roe (the paper's flux) as an option.
 *   boundaries  ghost states: farfield = free stream, slip wall = mirrored normal
 *               momentum (eq. 11 boundary-face term).
 *   time        SSP-RK3 in Shu-Osher form (the paper uses explicit 2nd-order RK).
 *
 * Conventions for every call:
 *   - The return value is a tdg_status; nothing throws across this interface.
 *     On failure tdg_last_error(ctx) describes it (valid until the next call on ctx).
 *   - "device" pointers are HIP device memory owned by the caller (e.g. torch
 *     tensors); "host" pointers are ordinary host memory, read during the call.
 *   - Compute calls are asynchronous on the given hipStream_t (passed as void*,
 *     NULL = the null stream).  Kernel-side faults surface on the next
 *     synchronisation; tdg_sync_check() synchronises and reports them.
 *   - The library allocates no device memory after tdg_mesh_bind().  The mixed modes (an
 *     operand companion) and the viscous terms (Z, the viscous residual part, face fluxes)
 *     keep scratch inside the bound mesh buffer, so calls on one context must not overlap
 *     in time (on different streams).
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - U, R, W and Ubar must not alias, except U in tdg_rk_step (updated in place).
 */
#ifndef TETDG_H
#define TETDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdg_ctx tdg_ctx;

typedef enum {
  TDG_OK = 0,
  TDG_ERR_INVALID_ARG = -1, /* bad argument: null pointer, size, enum, order */
  TDG_ERR_MESH = -2,        /* degenerate element, unmatched or over-shared face */
  TDG_ERR_STATE = -3,       /* call out of order (no mesh, not bound) */
  TDG_ERR_HIP = -4,         /* HIP runtime error (launch, copy, async fault) */
  TDG_ERR_UNSUPPORTED = -5, /* valid request this build does not implement */
  TDG_ERR_NOMEM = -6        /* host allocation failed or device buffer too small */
} tdg_status;

typedef enum {
  TDG_FP64 = 0,       /* state, contractions and fluxes in double */
  TDG_FP32 = 1,       /* state, contractions and fluxes in float */
  TDG_MIXED_BF16 = 2, /* FP64 state; contractions bf16 x bf16 -> fp32 on MFMA; fluxes fp32 */
  TDG_MIXED_FP16 = 3  /* as above with fp16 operands */
} tdg_precision;

typedef enum {
  TDG_RENUM_NONE = 0,   /* keep the caller's element order */
  TDG_RENUM_RCM = 1,    /* reverse Cuthill-McKee on the face-adjacency graph (Sec. III.B) */
  TDG_RENUM_MORTON = 2, /* Morton (Z-order) curve of element centroids */
  TDG_RENUM_HILBERT = 3 /* Hilbert curve of element centroids */
} tdg_renumber;

typedef enum { TDG_BC_FARFIELD = 1, TDG_BC_SLIPWALL = 2 } tdg_bc;

typedef enum {
  TDG_FLUX_RUSANOV = 0, /* local Lax-Friedrichs (default) */
  TDG_FLUX_ROE = 1      /* Roe's flux (the paper's, Sec. II.B), Harten entropy fix 0.1 c */
} tdg_flux;

/* ------------------------------------------------------------------ context */

/* Create a context for polynomial order p (1..4) and a precision mode.  gamma is the
 * ratio of specific heats (Sec. II.A, eq. 4).  *out receives the new context.
 * Errors: TDG_ERR_INVALID_ARG (p, precision, gamma <= 1, out NULL), TDG_ERR_NOMEM. */
int tdg_create(int order_p, int precision, double gamma, tdg_ctx** out);

/* Release a context and its host memory; device memory stays with the caller. NULL is a no-op. */
void tdg_destroy(tdg_ctx* ctx);

/* Text of the last error on ctx ("" if none).  ctx may be NULL (then a static message). */
const char* tdg_last_error(const tdg_ctx* ctx);

/* Problem sizes: modes N_p, volume points N_q, points per face N_f. */
int tdg_sizes(const tdg_ctx* ctx, int* n_modes, int* n_vol_points, int* n_face_points);

/* ------------------------------------------------------------------ mesh */

/* Upload a tetrahedral mesh (host arrays, copied).  Builds the face adjacency by
 * matching sorted vertex-id triples, tags boundary faces, computes FP64 geometry and
 * renumbers the elements (the grid renumbering of Sec. III.B: RCM, or a space-filling
 * curve).  The renumbering runs once, before time stepping.  For the FP64 and FP32 modes
 * the RCM and curve orders are then refined inside windows of 256 elements by grouping
 * elements with equal neighbour face codes (fewer distinct face tables per 16-element
 * tile in the stage kernel); the mixed modes keep the plain order.
 *   elem_vid   host int64 [n_elem][4]   global vertex ids (on a torus: periodic ids)
 *   elem_xyz   host double [n_elem][4][3] vertex coordinates, per element, unwrapped
 *   bface_vid  host int64 [n_bface][3]  boundary faces (any vertex order), may be NULL if 0
 *   bface_tag  host int32 [n_bface]     TDG_BC_FARFIELD or TDG_BC_SLIPWALL
 *   renumber   a tdg_renumber value
 *   perm_new_to_old  host int64 [n_elem] out (may be NULL): internal index -> caller index
 * Errors: TDG_ERR_INVALID_ARG; TDG_ERR_MESH for a zero-volume element, a face shared by
 * more than two elements, or an unmatched face that is not a listed boundary face. */
int tdg_mesh_upload(tdg_ctx* ctx, int64_t n_elem, const int64_t* elem_vid, const double* elem_xyz,
                    int64_t n_bface, const int64_t* bface_vid, const int32_t* bface_tag, int renumber,
                    int64_t* perm_new_to_old);

/* Bytes of device memory the uploaded mesh and reference tables need (caller allocates). */
int tdg_mesh_device_bytes(const tdg_ctx* ctx, size_t* bytes);

/* Copy mesh arrays and reference tables into dev_buf (device, >= the size above, 256-byte
 * aligned) on the stream and wait for the copy.  dev_buf must stay allocated while the
 * context computes.  Errors: TDG_ERR_STATE (no mesh), TDG_ERR_INVALID_ARG, TDG_ERR_HIP. */
int tdg_mesh_bind(tdg_ctx* ctx, void* dev_buf, size_t bytes, void* hip_stream);

/* Interface flux of eq. 11 (a tdg_flux value; default Rusanov).  The residual, the RK
 * stages and the adjoint entry points all use the selected flux. */
int tdg_set_flux(tdg_ctx* ctx, int flux);

/* Viscous (Navier-Stokes) terms of eqs. 1 and 11 with constant dynamic viscosity mu and
 * Prandtl number Pr (mu = 0: Euler, the default).  The paper's BR1 form: the auxiliary
 * variable Z = grad U is lifted with central interface values, and the viscous interface
 * flux is the average of both sides' viscous fluxes; boundary faces use the inviscid
 * ghost state with Z+ = Z-.  Stress by Stokes' hypothesis, heat flux -kappa grad T with
 * kappa = mu gamma / ((gamma - 1) Pr) and T = p / rho.  Every residual and RK entry point
 * then includes them (three more launches per stage: the lifting, the volume and own-side
 * face part of the viscous residual, and the neighbours' face halves; the stage kernel adds
 * the result).  Must be called before tdg_mesh_upload (the device buffer then holds their
 * scratch: four more states and each element's own-side viscous face fluxes at its face
 * points, 4 x 5 x 16 ceil(N_f / 16) values).  FP64 and FP32 modes; the mixed
 * modes return TDG_ERR_UNSUPPORTED, and so do the adjoint entry points while mu > 0.
 * tdg_stable_dt stays the inviscid rule (the caller bounds dt by the viscous limit).
 * Errors: TDG_ERR_INVALID_ARG (mu < 0, Pr <= 0), TDG_ERR_STATE (mesh already uploaded). */
int tdg_set_viscosity(tdg_ctx* ctx, double mu, double prandtl);

/* Free-stream primitive state (rho, u, v, w, p) used as the farfield ghost (host array). */
int tdg_set_farfield(tdg_ctx* ctx, const double prim[5]);

/* Mesh statistics after renumbering (host int64 out[7]): n_elem, n_elem_pad,
 * interior faces, boundary faces, max |i - j| over face neighbours (bandwidth),
 * the number of neighbour pairs with |i - j| < 64, and the number of distinct neighbour
 * face tables summed over (16-element tile, face) pairs (MFMA chains of the stage kernel). */
int tdg_mesh_stats(const tdg_ctx* ctx, int64_t out[7]);

/* ------------------------------------------------------------------ state */

/* Internal state: [5][ceil(N_p/4)][n_elem_pad][4] in renumbered element order: for each
 * variable, quads of four consecutive modes, element index next, the four modes of a quad
 * innermost (modes past N_p are padding, written as zero by set_state/project).  double for
 * TDG_FP64 and the mixed modes, float for TDG_FP32.  Elements n_elem .. n_elem_pad - 1 pad
 * the arrays to the kernels' tile width and carry no result: the compute calls leave them
 * unchanged in their outputs or write zeros there.
 * User state:     [n_elem][5][N_p] double, caller's element order. */
int tdg_state_elems(const tdg_ctx* ctx, int64_t* n_elem_pad);
int tdg_state_bytes(const tdg_ctx* ctx, size_t* bytes);

/* The state is the set of coefficients c_j of the modal expansion U_h = sum_j c_j phi_j of
 * each conserved variable on each element (Sec. II.B, eq. 10); these two calls only move
 * it between the caller's layout and the internal one, without arithmetic.
 * User (device, double) -> internal (device): padding elements are set to a copy of
 * element 0 (FP32 mode: each coefficient rounded to float).  U_user: device double
 * [n_elem][5][N_p], caller-owned, read; U_int: device, tdg_state_bytes() bytes, written.
 * Errors: TDG_ERR_STATE (no bound mesh), TDG_ERR_INVALID_ARG (NULL), TDG_ERR_HIP. */
int tdg_set_state(tdg_ctx* ctx, const double* U_user, void* U_int, void* hip_stream);
/* Internal (device) -> user (device, double [n_elem][5][N_p], caller's element order,
 * overwritten).  Errors as tdg_set_state. */
int tdg_get_state(tdg_ctx* ctx, const void* U_int, double* U_user, void* hip_stream);

/* Physical coordinates of the volume quadrature points, device double [n_elem][N_q][3],
 * caller's element order (for evaluating initial fields). */
int tdg_volume_points(tdg_ctx* ctx, double* xyz_user, void* hip_stream);

/* L2 projection of a primitive field sampled at the volume points (device double
 * [n_elem][N_q][5], caller's order) onto the basis: c_i = 6 sum_q w_q U(prim_q) phi_i(xi_q),
 * written as an internal state. */
int tdg_project(tdg_ctx* ctx, const double* prim_user, void* U_int, void* hip_stream);

/* ------------------------------------------------------------------ hot path */

/* R = M^-1 (V - S) for internal state U (Sec. II.B, eq. 11, inviscid):
 *   V_i = int_K F(U_h) . grad phi_i,  S_i = sum_f int_f Fhat(U-, U+, n) phi_i,  M = |K| I.
 * Each element evaluates its own four faces, reading its neighbours' coefficients, so
 * the face integral reaches both neighbours without atomics.  R has U's layout. */
int tdg_residual(tdg_ctx* ctx, const void* U, void* R, void* hip_stream);

/* The time loop of Sec. III (opening passage): the semi-discrete system dc/dt = R(c) of
 * eq. 11 is advanced by an explicit Runge-Kutta scheme with one right-hand-side evaluation
 * per stage (the paper uses second order; this library the three-stage SSP scheme).
 * n_steps SSP-RK3 steps of size dt on U (internal, in place):
 *   U1 = U + dt R(U);  U2 = 3/4 U + 1/4 (U1 + dt R(U1));  U <- 1/3 U + 2/3 (U2 + dt R(U2)).
 * work: device buffer of tdg_work_bytes() bytes (two internal states, plus in the mixed
 * modes three low-precision operand companions, and up to P3 one array of fp64 cell
 * means).  One fused residual+update launch per stage (mixed modes: plus one companion
 * pass over U per call).  In the mixed modes up to P3 the second stage stores
 * W2 = 1/3 U + 2/3 U2 instead of U2 and the third computes U <- W2 + 2/3 dt R(U2) (the same
 * update, rounded differently), so that it reads no U; U2 itself enters only through its
 * companion and its cell means.
 * Errors: TDG_ERR_INVALID_ARG (NULL U or work, n_steps < 0), TDG_ERR_STATE, TDG_ERR_HIP. */
int tdg_rk_step(tdg_ctx* ctx, void* U, void* work, double dt, int n_steps, void* hip_stream);

/* n_steps SSP-RK3 steps with the step size chosen on the device before every step
 * (Sec. III.C: the global minimum of the local time steps):
 *   dt_k = min_K cfl d_K / ((2p+1)(|u_K| + c_K)),  d_K = 6|K| / sum_f A_f,
 * with the cell means of the current U (as tdg_stable_dt), then one step as tdg_rk_step.
 * dt_k is written to dt_hist[k] (device, n_steps doubles) and read there by the stage
 * kernels, so the loop needs no host round trip.  U, work: as tdg_rk_step.
 * dt_hist[k] = 0 reports that the state entering step k had an inadmissible cell mean
 * (density or pressure not positive, or a value not finite): the run is invalid from that
 * step on, and since the loop does not synchronise, the caller checks dt_hist afterwards.
 * Errors: TDG_ERR_INVALID_ARG (null pointers, cfl <= 0, n_steps < 0). */
int tdg_rk_step_adaptive(tdg_ctx* ctx, void* U, void* work, double cfl, int n_steps, double* dt_hist,
                         void* hip_stream);

/* Bytes of the work buffer tdg_rk_step needs. */
int tdg_work_bytes(const tdg_ctx* ctx, size_t* bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tdg_rk_step with the work buffer taken
 * from a fixed 64 MiB device array of the library (one per GPU, held from the library's
 * load on that device until the process ends) instead of a caller buffer.  Same kernels and
 * results as tdg_rk_step; allocates nothing.  The array is shared by every call on a GPU
 * and keeps the last call's contents (nothing in it needs to start at zero): calls that
 * overlap in time on one GPU race, so callers serialise them.
 * Errors: TDG_ERR_NOMEM when tdg_work_bytes() exceeds 64 MiB (e.g. above ~25,000 P3 FP64
 * elements), checked before any device work; otherwise as tdg_rk_step. */
int tdg_rk_step_noalloc(tdg_ctx* ctx, void* U, double dt, int n_steps, void* hip_stream);

/* Vector-Jacobian product Ubar = (dR/dU)^T W at U (all internal layout; Ubar overwritten).
 * Element-centric: each element gathers U and W of its neighbours and applies the
 * transposed interpolation, flux Jacobians and transposed lift of its own and its
 * neighbours' shared faces; no atomics.  FP64 and FP32 modes; the mixed modes compute
 * the adjoint in FP64.  At exact ties of max(lambda-, lambda+) the derivative is split
 * evenly, and d|x|/dx = 0 at x = 0. */
int tdg_residual_vjp(tdg_ctx* ctx, const void* U, const void* W, void* Ubar, void* hip_stream);

/* One SSP-RK3 stage: U_out = alpha U0 + (1 - alpha)(U_in + dt R(U_in)) (internal states;
 * U0 may be NULL when alpha == 0; U_out may alias U0 but not U_in).  The same fused
 * kernel as tdg_rk_step; exposed so an adjoint can recompute stage states. */
int tdg_rk_stage(tdg_ctx* ctx, const void* U_in, const void* U0, void* U_out, double alpha, double dt,
                 void* hip_stream);

/* Accumulating VJP: Out = c (dR/dU)^T(U) W + sum_{k < n_terms} a[k] Y[k], all internal
 * states (Y[k] may alias W; Out must not alias U, W or any Y[k]).  n_terms in 0..3.
 * This is the per-stage operation of the discrete SSP-RK3 adjoint (reverse step):
 *   Ub2 = (2/3) dt J(U2)^T Ub3 + (2/3) Ub3;   Ub1 = (1/4) dt J(U1)^T Ub2 + (1/4) Ub2;
 *   Ub0 = dt J(U0)^T Ub1 + Ub1 + (3/4) Ub2 + (1/3) Ub3. */
int tdg_residual_vjp_axpy(tdg_ctx* ctx, const void* U, const void* W, double c, int n_terms, const void* const* Y,
                          const double* a, void* Out, void* hip_stream);

/* Admissibility of internal state U: the number of elements where, at some volume
 * quadrature point, a conserved variable is not finite or the density or pressure is not
 * positive (n_bad: device int64, overwritten).  The pressure is the one of the equation of
 * state with the energy relation of Sec. II.A (eq. 4 and the energy definition after it);
 * the flux Jacobian's sound speed sqrt(gamma p / rho) of Sec. II.B needs both positive.
 * A run's failure detector: call it every few steps and stop when it is non-zero.
 * Errors: TDG_ERR_INVALID_ARG (NULL), TDG_ERR_STATE, TDG_ERR_HIP. */
int tdg_check_state(tdg_ctx* ctx, const void* U, int64_t* n_bad, void* hip_stream);

/* Integrated slip-wall pressure J = sum over slip-wall faces of int_f p(U-) dA (boundary-face
 * quadrature of eq. 11) at internal state U, and optionally dJ/dU (internal layout, overwritten;
 * NULL to skip).  J: device double, overwritten.  The objective of the full configuration's
 * adjoint (its gradient seeds the trajectory adjoint). */
int tdg_wall_pressure(tdg_ctx* ctx, const void* U, double* J, void* dJdU, void* hip_stream);

/* Explicit time step as the global minimum of local steps (the paper's minimum over the
 * local time steps of all cells, Sec. III.C, computed by a GPU reduction):
 *   dt = min_K cfl d_K / ((2p+1)(|u_K| + c_K)),  d_K = 6|K| / sum_f A_f,
 * with u_K, c_K from the cell means of U.  dt: device double, overwritten; 0 when some
 * cell mean is inadmissible (density or pressure not positive, or a value not finite). */
int tdg_stable_dt(tdg_ctx* ctx, const void* U, double cfl, double* dt, void* hip_stream);

/* Synchronise the stream; map a pending asynchronous HIP error to TDG_ERR_HIP. */
int tdg_sync_check(tdg_ctx* ctx, void* hip_stream);

/* Streaming probe: the practical DRAM bandwidth that the roofline model of Sec. IV.A bounds
 * a memory-bound kernel by, measured with 16-byte non-temporal accesses over caller device
 * buffers (grid-strided, 512-thread workgroups).  kind 0 copies src to dst, kind 1 only reads
 * src (dst: at least 16 bytes, whose first 16 may be overwritten), kind 2 zero-fills dst,
 * kind 3 reads like kind 1 with ordinary cache-allocating loads (over a buffer that fits the
 * last-level cache, repeated calls measure that cache's bandwidth).
 * bytes: a positive multiple of 16; src and dst 16-byte aligned and not overlapping (src may
 * be NULL for kind 2).  Asynchronous on hip_stream; no context, no allocation.  Errors:
 * TDG_ERR_INVALID_ARG (checked before any device call), TDG_ERR_HIP (launch failure). */
int tdg_stream_probe(int kind, const void* src, void* dst, size_t bytes, void* hip_stream);

/* ------------------------------------------------------------------ host-only checks */

/* Reference tables computed by this library, no GPU needed.  which:
 *   0 volume points [N_q][3]      1 volume weights [N_q]
 *   2 face points (s,t) [N_f][2]  3 face weights [N_f]
 *   4 basis at volume points [N_q][N_p]
 *   5 reference gradients [3][N_q][N_p]
 *   6 basis at face points [4][N_f][N_p]
 * out may be NULL to query *need (element count).  Errors: TDG_ERR_INVALID_ARG,
 * TDG_ERR_NOMEM when cap < need. */
int tdg_debug_tables(int order_p, int which, double* out, size_t cap, size_t* need);

#ifdef __cplusplus
}
#endif
#endif /* TETDG_H */
