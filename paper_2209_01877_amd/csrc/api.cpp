// C ABI of libtetdg (declared in include/tetdg.h): context, mesh upload and
// renumbering, operand-table packing, device binding and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dg_common.hpp"
#include "dg_launch.hpp"
#include "mesh.hpp"
#include "refelem.hpp"
#include "tetdg.h"

using namespace tetdg;

struct tdg_ctx {
  int p = 1, prec = 0;
  double gamma = 1.4;
  RefElem ref;
  std::string err;
  bool has_mesh = false, bound = false;
  int64_t n = 0, epad = 0, n_interior = 0, n_boundary = 0, bandwidth = 0, near64 = 0, tile_tables = 0;
  // host images of the device arrays (internal element order)
  std::vector<double> M, inv_vol, x0j;
  std::vector<int32_t> nbr, fcode, perm;
  std::vector<unsigned char> stage_tab, vjp_tab;
  std::vector<double> mom, mean_tab;
  // device buffer (caller-owned) and offsets into it
  char* dev = nullptr;
  size_t dev_bytes = 0;
  size_t off_M = 0, off_iv = 0, off_x0j = 0, off_nbr = 0, off_fcode = 0, off_perm = 0, off_stab = 0, off_vtab = 0,
         off_mom = 0, off_mtab = 0, off_qx = 0, off_qw = 0, off_B = 0, off_fw = 0, off_Bf = 0, off_comp = 0, total = 0;
  double far[5] = {1.0, 0.0, 0.0, 0.0, 2.5};
  int flux = TDG_FLUX_RUSANOV;
  // viscous (Navier-Stokes, BR1) terms: off when mu == 0; scratch Z (3 states) and Rv
  double mu = 0.0, prandtl = 0.72;
  size_t off_z = 0, off_rv = 0, off_hb = 0;
};

namespace {

int fail(tdg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(tdg_ctx* c, hipError_t e, const char* what) {
  return fail(c, TDG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

uint16_t to_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                           // round to nearest even
  return (uint16_t)(u >> 16);
}

uint16_t to_fp16(float x) {
  _Float16 h = (_Float16)x;
  uint16_t r;
  std::memcpy(&r, &h, 2);
  return r;
}

// Append one value of the operand type of `prec` to a byte vector.
void put(std::vector<unsigned char>& out, int prec, double v) {
  if (prec == TDG_FP64) {
    unsigned char b[8];
    std::memcpy(b, &v, 8);
    out.insert(out.end(), b, b + 8);
  } else if (prec == TDG_FP32) {
    float f = (float)v;
    unsigned char b[4];
    std::memcpy(b, &f, 4);
    out.insert(out.end(), b, b + 4);
  } else {
    const uint16_t h = prec == TDG_MIXED_BF16 ? to_bf16((float)v) : to_fp16((float)v);
    out.push_back((unsigned char)(h & 0xff));
    out.push_back((unsigned char)(h >> 8));
  }
}

// Stage-kernel operand tables (slot layout of Layout<P, KW>).
template <int P>
void pack_stage(const RefElem& R, int prec, std::vector<unsigned char>& out) {
  using O = Ord<P>;
  const bool mixed = prec >= TDG_MIXED_BF16;
  const int KW = mixed ? 8 : 1;
  const int K = mixed ? 32 : 4;
  const bool f64 = prec == TDG_FP64;
  const int KS = mixed ? Layout<P, 8>::KS : Layout<P, 1>::KS;
  const int NP = O::NP, NQ = O::NQ, NF = O::NF;
  out.clear();
  // value(row, g, m) for one slot, written lane-major
  auto slot = [&](auto&& A) {
    for (int l = 0; l < 64; ++l)
      for (int m = 0; m < KW; ++m) put(out, prec, A(l % 16, l / 16, m));
  };
  auto kmode = [&](int s, int g, int m) { return KW == 1 ? K * s + g : K * s + 8 * g + m; };
  auto mode_ok = [&](int mode) { return mode < NP && !(mixed && mode == 0); };
  // FP32 / FP64, last mode tile of at most 4 modes: lane row r supplies mode 16 mt + r % 4
  // (4x4x1 block operands in fp32; in fp64 lanes 16 g + 0..3 hold the four values of lane
  // group g's point; the stage kernel's kTail4)
  const bool tail4 = !mixed && NP - 16 * (O::MT - 1) <= 4;
  // mixed, P3 / P4: last mode tile of at most 4 modes spread over the lane groups, row 4 g
  // holding mode 16 mt + g and the other rows zero (the stage kernel's kSpread)
  const bool spread = mixed && O::MT >= 2 && NP - 16 * (O::MT - 1) <= 4;
  auto tile_mode = [&](int mt, int r) {
    if (spread && mt == O::MT - 1) return r % 4 == 0 ? 16 * mt + r / 4 : NP;
    return 16 * mt + ((tail4 && mt == O::MT - 1) ? r % 4 : r);
  };
  // interp
  for (int qt = 0; qt < O::QT; ++qt)
    for (int s = 0; s < KS; ++s)
      slot([&](int r, int g, int m) {
        const int q = 16 * qt + r, mode = kmode(s, g, m);
        return (q < NQ && mode_ok(mode)) ? R.B[(size_t)q * NP + mode] : 0.0;
      });
  // trace
  for (int f = 0; f < 4; ++f)
    for (int ft = 0; ft < O::FT; ++ft)
      for (int s = 0; s < KS; ++s)
        slot([&](int r, int g, int m) {
          const int q = 16 * ft + r, mode = kmode(s, g, m);
          return (q < NF && mode_ok(mode)) ? R.Bf[((size_t)f * NF + q) * NP + mode] : 0.0;
        });
  // projection: rows = modes, k = (direction, point) in the accumulator order of the interp.
  // f64/f32: k-step pk = 4 d + j.  bf16/f16: k-step jp covers points j = 2 jp (m = 0..2 -> d = m)
  // and j = 2 jp + 1 (m = 4..6 -> d = m - 4); m = 3, 7 are zero.
  const int PK = mixed ? 2 : 12;
  for (int mt = 0; mt < O::MT; ++mt)
    for (int qt = 0; qt < O::QT; ++qt)
      for (int pk = 0; pk < PK; ++pk)
        slot([&](int r, int g, int m) {
          const int mode = tile_mode(mt, r);
          int d, j;
          if (!mixed) {
            d = pk / 4;
            j = pk % 4;
          } else {
            if ((m & 3) == 3) return 0.0;
            d = m & 3;
            j = 2 * pk + (m >> 2);
          }
          const int q = 16 * qt + drow(f64, g, j);
          if (q >= NQ || mode >= NP) return 0.0;
          return R.qw[q] * R.G[((size_t)d * NQ + q) * NP + mode];
        });
  // lift (negated: the face integral is subtracted)
  const int LK = mixed ? 1 : 4;
  for (int mt = 0; mt < O::MT; ++mt)
    for (int f = 0; f < 4; ++f)
      for (int ft = 0; ft < O::FT; ++ft)
        for (int lk = 0; lk < LK; ++lk)
          slot([&](int r, int g, int m) {
            const int mode = tile_mode(mt, r);
            int j = lk;
            if (mixed) {
              if (m >= 4) return 0.0;
              j = m;
            }
            const int q = 16 * ft + drow(f64, g, j);
            if (q >= NF || mode >= NP) return 0.0;
            return -R.fw[q] * R.Bf[((size_t)f * NF + q) * NP + mode];
          });
}

// VJP operand tables (slot layout of VjpLayout<P>), f64 or f32.
template <int P>
void pack_vjp(const RefElem& R, int prec, std::vector<unsigned char>& out) {
  using O = Ord<P>;
  using V = VjpLayout<P>;
  const bool f64 = prec == TDG_FP64;
  const int NP = O::NP, NQ = O::NQ, NF = O::NF;
  out.clear();
  auto slot = [&](auto&& A) {
    for (int l = 0; l < 64; ++l) put(out, f64 ? TDG_FP64 : TDG_FP32, A(l % 16, l / 16));
  };
  // interp(qt, s) and trace(f, ft, s): the forward interpolation tables
  for (int qt = 0; qt < O::QT; ++qt)
    for (int s = 0; s < V::KS; ++s)
      slot([&](int r, int g) {
        const int q = 16 * qt + r, mode = 4 * s + g;
        return (q < NQ && mode < NP) ? R.B[(size_t)q * NP + mode] : 0.0;
      });
  for (int f = 0; f < 4; ++f)
    for (int ft = 0; ft < O::FT; ++ft)
      for (int s = 0; s < V::KS; ++s)
        slot([&](int r, int g) {
          const int q = 16 * ft + r, mode = 4 * s + g;
          return (q < NF && mode < NP) ? R.Bf[((size_t)f * NF + q) * NP + mode] : 0.0;
        });
  // tinterp(qt, d, s): rows = points, k = modes: w_q dphi/dxi_d
  for (int qt = 0; qt < O::QT; ++qt)
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < V::KS; ++s)
        slot([&](int r, int g) {
          const int q = 16 * qt + r, mode = 4 * s + g;
          return (q < NQ && mode < NP) ? R.qw[q] * R.G[((size_t)d * NQ + q) * NP + mode] : 0.0;
        });
  // ttrace(f, ft, s): rows = face points, k = modes: w^f_q phi(xi_f(q))
  for (int f = 0; f < 4; ++f)
    for (int ft = 0; ft < O::FT; ++ft)
      for (int s = 0; s < V::KS; ++s)
        slot([&](int r, int g) {
          const int q = 16 * ft + r, mode = 4 * s + g;
          return (q < NF && mode < NP) ? R.fw[q] * R.Bf[((size_t)f * NF + q) * NP + mode] : 0.0;
        });
  // tproj(mt, qt, j): rows = modes, k = points in accumulator order: phi(xi_q)
  for (int mt = 0; mt < O::MT; ++mt)
    for (int qt = 0; qt < O::QT; ++qt)
      for (int j = 0; j < 4; ++j)
        slot([&](int r, int g) {
          const int mode = 16 * mt + r, q = 16 * qt + drow(f64, g, j);
          return (q < NQ && mode < NP) ? R.B[(size_t)q * NP + mode] : 0.0;
        });
  // tlift(mt, f, ft, j): rows = modes, k = face points: phi(xi_f(q))
  for (int mt = 0; mt < O::MT; ++mt)
    for (int f = 0; f < 4; ++f)
      for (int ft = 0; ft < O::FT; ++ft)
        for (int j = 0; j < 4; ++j)
          slot([&](int r, int g) {
            const int mode = 16 * mt + r, q = 16 * ft + drow(f64, g, j);
            return (q < NF && mode < NP) ? R.Bf[((size_t)f * NF + q) * NP + mode] : 0.0;
          });
}

void build_tables(tdg_ctx* c) {
  switch (c->p) {
    case 1: pack_stage<1>(c->ref, c->prec, c->stage_tab); break;
    case 2: pack_stage<2>(c->ref, c->prec, c->stage_tab); break;
    case 3: pack_stage<3>(c->ref, c->prec, c->stage_tab); break;
    case 4: pack_stage<4>(c->ref, c->prec, c->stage_tab); break;
  }
  const int vprec = c->prec == TDG_FP32 ? TDG_FP32 : TDG_FP64;
  switch (c->p) {
    case 1: pack_vjp<1>(c->ref, vprec, c->vjp_tab); break;
    case 2: pack_vjp<2>(c->ref, vprec, c->vjp_tab); break;
    case 3: pack_vjp<3>(c->ref, vprec, c->vjp_tab); break;
    case 4: pack_vjp<4>(c->ref, vprec, c->vjp_tab); break;
  }
  const int NP = c->ref.np, NQ = c->ref.nq, NF = c->ref.nf;
  c->mom.assign(7 * NP, 0.0);
  for (int i = 0; i < NP; ++i) {
    for (int d = 0; d < 3; ++d)
      for (int q = 0; q < NQ; ++q) c->mom[d * NP + i] += c->ref.qw[q] * c->ref.G[((size_t)d * NQ + q) * NP + i];
    for (int f = 0; f < 4; ++f)
      for (int q = 0; q < NF; ++q) c->mom[(3 + f) * NP + i] += c->ref.fw[q] * c->ref.Bf[((size_t)f * NF + q) * NP + i];
  }
  // mean-flux projection as fp64 MFMA A operands: slot (mt, step), lane l holds A[r][k] with
  // r = l % 16, k = 4 step + l / 16; the row r = g + 4 j holds mode 16 mt + 4 g + j so that the
  // fp64 accumulator element j of lane group g is the same mode as in the fp32 accumulators.
  // k = 0..2: volume moments (+); k = 3: face 0; k = 4..6: faces 1..3 (face moments negated).
  const int MT = (NP + 15) / 16;
  // the last tile of at most 4 modes (P3, P4): row r < 4 holds mode 16 mt + r (register 0 of
  // lane group r), as in the spread fp32 tables
  const bool spread = MT >= 2 && NP - 16 * (MT - 1) <= 4;
  c->mean_tab.assign((size_t)MT * 2 * 64, 0.0);
  for (int mt = 0; mt < MT; ++mt)
    for (int step = 0; step < 2; ++step)
      for (int l = 0; l < 64; ++l) {
        const int r = l % 16, k = 4 * step + l / 16;
        const int mode = (spread && mt == MT - 1) ? (r < 4 ? 16 * mt + r : NP) : 16 * mt + 4 * (r % 4) + r / 4;
        double v = 0.0;
        if (mode < NP && k < 7) {
          const int face = k == 3 ? 0 : k - 3;
          v = k < 3 ? c->mom[k * NP + mode] : -c->mom[(3 + face) * NP + mode];
        }
        c->mean_tab[((size_t)mt * 2 + step) * 64 + l] = v;
      }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

MeshView view(const tdg_ctx* c) {
  MeshView m;
  m.M = (const double*)(c->dev + c->off_M);
  m.inv_vol = (const double*)(c->dev + c->off_iv);
  m.nbr = (const int32_t*)(c->dev + c->off_nbr);
  m.fcode = (const int32_t*)(c->dev + c->off_fcode);
  m.perm = (const int32_t*)(c->dev + c->off_perm);
  m.x0j = (const double*)(c->dev + c->off_x0j);
  m.n_elem = c->n;
  m.epad = c->epad;
  return m;
}

RefView refview(const tdg_ctx* c) {
  RefView r;
  r.qx = (const double*)(c->dev + c->off_qx);
  r.qw = (const double*)(c->dev + c->off_qw);
  r.B = (const double*)(c->dev + c->off_B);
  r.fw = (const double*)(c->dev + c->off_fw);
  r.Bf = (const double*)(c->dev + c->off_Bf);
  return r;
}

int require_bound(tdg_ctx* c) {
  if (!c) return TDG_ERR_INVALID_ARG;
  if (!c->has_mesh) return fail(c, TDG_ERR_STATE, "no mesh uploaded");
  if (!c->bound) return fail(c, TDG_ERR_STATE, "mesh not bound to device memory (tdg_mesh_bind)");
  return TDG_OK;
}

size_t state_bytes(const tdg_ctx* c) {
  return (size_t)5 * 4 * npq_of(c->ref.np) * c->epad * (c->prec == TDG_FP32 ? sizeof(float) : sizeof(double));
}

bool is_mixed(const tdg_ctx* c) { return c->prec >= TDG_MIXED_BF16; }

size_t comp_bytes(const tdg_ctx* c) { return is_mixed(c) ? companion_bytes(c->p, c->epad) : 0; }

// Companion (q, c0) pointers inside a buffer of companion_bytes().
void comp_ptrs(const tdg_ctx* c, char* base, void** q, float** c0) {
  const size_t qb = ((size_t)c->epad * 5 * 32 * ((c->ref.np + 31) / 32) * 2 + 255) & ~(size_t)255;
  *q = base;
  *c0 = (float*)(base + qb);
}

// Mixed modes up to P3: rk_step's second stage stores W2 = U0/3 + 2 U2/3 instead of U2, so
// that the third stage reads no U0 (at P4, whose stage kernel runs one wave per SIMD, that
// measured no faster).
bool split_rk3(const tdg_ctx* c) { return is_mixed(c) && c->p <= 3; }

// rk_step's work buffer: the states U1 and U2, then (mixed modes) the companions of U, U1,
// U2, then (split_rk3) the fp64 cell means of U2 ([5][E_pad]).
size_t work_bytes(const tdg_ctx* c) {
  return 2 * state_bytes(c) + 3 * comp_bytes(c) + (split_rk3(c) ? 5 * (size_t)c->epad * sizeof(double) : 0);
}

}  // namespace

namespace tetdg {
// Record an error on a context for the entry points defined in other source files.
int ctx_fail(tdg_ctx* c, int code, const char* msg) { return fail(c, code, msg ? msg : ""); }
}  // namespace tetdg

extern "C" {

int tdg_create(int order_p, int precision, double gamma, tdg_ctx** out) {
  if (!out) return TDG_ERR_INVALID_ARG;
  *out = nullptr;
  if (order_p < 1 || order_p > 4) return TDG_ERR_INVALID_ARG;
  if (precision < TDG_FP64 || precision > TDG_MIXED_FP16) return TDG_ERR_INVALID_ARG;
  if (!(gamma > 1.0)) return TDG_ERR_INVALID_ARG;
  tdg_ctx* c = new (std::nothrow) tdg_ctx;
  if (!c) return TDG_ERR_NOMEM;
  c->p = order_p;
  c->prec = precision;
  c->gamma = gamma;
  try {
    c->ref = build_refelem(order_p);
    build_tables(c);
  } catch (...) {
    delete c;
    return TDG_ERR_NOMEM;
  }
  // default farfield: rho = 1, u = 0, p = 1
  c->far[0] = 1.0;
  c->far[1] = c->far[2] = c->far[3] = 0.0;
  c->far[4] = 1.0 / (gamma - 1.0);
  *out = c;
  return TDG_OK;
}

void tdg_destroy(tdg_ctx* ctx) { delete ctx; }

const char* tdg_last_error(const tdg_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

int tdg_sizes(const tdg_ctx* c, int* np, int* nq, int* nf) {
  if (!c) return TDG_ERR_INVALID_ARG;
  if (np) *np = c->ref.np;
  if (nq) *nq = c->ref.nq;
  if (nf) *nf = c->ref.nf;
  return TDG_OK;
}

int tdg_mesh_upload(tdg_ctx* c, int64_t n_elem, const int64_t* elem_vid, const double* elem_xyz, int64_t n_bface,
                    const int64_t* bface_vid, const int32_t* bface_tag, int renumber_mode, int64_t* perm_new_to_old) {
  if (!c) return TDG_ERR_INVALID_ARG;
  c->err.clear();
  if (n_elem <= 0 || n_elem > (int64_t)INT32_MAX - 64) return fail(c, TDG_ERR_INVALID_ARG, "n_elem out of range");
  if (!elem_vid || !elem_xyz) return fail(c, TDG_ERR_INVALID_ARG, "null mesh array");
  if (n_bface < 0 || (n_bface > 0 && (!bface_vid || !bface_tag)))
    return fail(c, TDG_ERR_INVALID_ARG, "boundary face arrays missing");
  if (renumber_mode < TDG_RENUM_NONE || renumber_mode > TDG_RENUM_HILBERT)
    return fail(c, TDG_ERR_INVALID_ARG, "unknown renumbering mode");
  try {
    HostMesh hm;
    std::string msg = build_topology(n_elem, elem_vid, elem_xyz, n_bface, bface_vid, bface_tag, hm);
    if (!msg.empty()) return fail(c, TDG_ERR_MESH, msg);
    std::vector<double> M, iv, x0j;
    msg = build_geometry(hm, M, iv, x0j);
    if (!msg.empty()) return fail(c, TDG_ERR_MESH, msg);
    // the compute-bound fp64/fp32 kernels gain from fewer neighbour face tables per tile, and
    // so do the mixed kernels at P4 (two operand slots per table); the memory-bound mixed
    // kernels up to P3 keep the tighter spatial order
    const bool group_codes = !is_mixed(c) || c->p >= 4;
    const std::vector<int64_t> order = renumber(hm, renumber_mode, group_codes);  // new -> old
    std::vector<int64_t> inv(n_elem);
    for (int64_t i = 0; i < n_elem; ++i) inv[order[i]] = i;
    const int64_t epad = (n_elem + 63) / 64 * 64;
    const double var_bytes = 4.0 * npq_of(c->ref.np) * (double)epad * (c->prec == TDG_FP32 ? 4 : 8);
    if (var_bytes >= 4294967296.0)
      return fail(c, TDG_ERR_UNSUPPORTED, "mesh too large: one variable of the state exceeds 4 GiB (32-bit offsets)");
    c->n = n_elem;
    c->epad = epad;
    c->n_interior = hm.n_interior;
    c->n_boundary = hm.n_boundary;
    c->M.assign(9 * epad, 0.0);
    c->inv_vol.assign(epad, 0.0);
    c->x0j.assign(12 * epad, 0.0);
    c->nbr.assign(4 * epad, 0);
    c->fcode.assign(epad, 0);
    c->perm.assign(epad, 0);
    int64_t bw = 0, near = 0;
    for (int64_t i = 0; i < epad; ++i) {
      const int64_t o = i < n_elem ? order[i] : order[0];
      for (int k = 0; k < 9; ++k) c->M[k * epad + i] = M[9 * o + k];
      c->inv_vol[i] = iv[o];
      for (int k = 0; k < 12; ++k) c->x0j[k * epad + i] = x0j[12 * o + k];
      c->perm[i] = (int32_t)(i < n_elem ? o : order[0]);
      int32_t code = 0;
      for (int f = 0; f < 4; ++f) {
        const int64_t nb = hm.nbr[4 * o + f];
        int32_t val;
        if (i >= n_elem) {
          val = (int32_t)i;  // padding: its own (valid) index
        } else if (nb >= 0) {
          val = (int32_t)inv[nb];
          const int64_t d = std::llabs(val - i);
          bw = std::max(bw, d);
          near += d < 64;
          code |= (int32_t)hm.nface[4 * o + f] << (2 * f);
        } else {
          val = (int32_t)nb;  // -1 farfield, -2 slip wall
        }
        c->nbr[f * epad + i] = val;
      }
      c->fcode[i] = i < n_elem ? code : 0;
    }
    c->bandwidth = bw;
    c->near64 = near;
    // distinct neighbour face tables per (16-element tile, face), summed over tiles and faces
    int64_t tt = 0;
    for (int64_t t0 = 0; t0 < epad; t0 += 16)
      for (int f = 0; f < 4; ++f) {
        int mask = 0;
        for (int64_t i = t0; i < t0 + 16 && i < n_elem; ++i)
          if (c->nbr[f * epad + i] >= 0) mask |= 1 << ((c->fcode[i] >> (2 * f)) & 3);
        tt += __builtin_popcount(mask);
      }
    c->tile_tables = tt;
    if (perm_new_to_old)
      for (int64_t i = 0; i < n_elem; ++i) perm_new_to_old[i] = order[i];
    // device layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off = align256(off + bytes);
      return o;
    };
    c->off_M = take(9 * epad * sizeof(double));
    c->off_iv = take(epad * sizeof(double));
    c->off_x0j = take(12 * epad * sizeof(double));
    c->off_nbr = take(4 * epad * sizeof(int32_t));
    c->off_fcode = take(epad * sizeof(int32_t));
    c->off_perm = take(epad * sizeof(int32_t));
    c->off_stab = take(c->stage_tab.size());
    c->off_vtab = take(c->vjp_tab.size());
    c->off_mom = take(c->mom.size() * sizeof(double));
    c->off_mtab = take(c->mean_tab.size() * sizeof(double));
    c->off_qx = take(c->ref.qx.size() * sizeof(double));
    c->off_qw = take(c->ref.qw.size() * sizeof(double));
    c->off_B = take(c->ref.B.size() * sizeof(double));
    c->off_fw = take(c->ref.fw.size() * sizeof(double));
    c->off_Bf = take(c->ref.Bf.size() * sizeof(double));
    // mixed modes: scratch operand companion for single residual / stage calls
    c->off_comp = take(c->prec >= TDG_MIXED_BF16 ? companion_bytes(c->p, epad) : 0);
    // viscous scratch: Z = grad U (15 state-layout variables) and the viscous residual part
    {
      const size_t sb = (size_t)5 * ((c->ref.np + 3) / 4) * epad * 4 * (c->prec == TDG_FP32 ? 4 : 8);
      c->off_z = take(c->mu > 0.0 ? 3 * sb : 0);
      c->off_rv = take(c->mu > 0.0 ? sb : 0);
      // own-half viscous face fluxes at the face points (padded to whole 16-point tiles),
      // 4 faces x 5 variables per element
      const size_t nfp = (c->ref.fw.size() + 15) / 16 * 16;
      const size_t hb = (size_t)epad * 4 * 5 * nfp * (c->prec == TDG_FP32 ? 4 : 8);
      c->off_hb = take(c->mu > 0.0 ? hb : 0);
    }
    c->total = off;
    c->has_mesh = true;
    c->bound = false;
    c->dev = nullptr;
  } catch (const std::bad_alloc&) {
    return fail(c, TDG_ERR_NOMEM, "host allocation failed");
  }
  return TDG_OK;
}

int tdg_mesh_device_bytes(const tdg_ctx* c, size_t* bytes) {
  if (!c || !bytes) return TDG_ERR_INVALID_ARG;
  if (!c->has_mesh) return TDG_ERR_STATE;
  *bytes = c->total;
  return TDG_OK;
}

int tdg_mesh_bind(tdg_ctx* c, void* dev_buf, size_t bytes, void* hip_stream) {
  if (!c) return TDG_ERR_INVALID_ARG;
  if (!c->has_mesh) return fail(c, TDG_ERR_STATE, "no mesh uploaded");
  if (!dev_buf || ((uintptr_t)dev_buf & 255)) return fail(c, TDG_ERR_INVALID_ARG, "device buffer null or not 256-byte aligned");
  if (bytes < c->total) return fail(c, TDG_ERR_NOMEM, "device buffer smaller than tdg_mesh_device_bytes");
  hipStream_t s = (hipStream_t)hip_stream;
  char* d = (char*)dev_buf;
  struct Piece {
    size_t off;
    const void* src;
    size_t n;
  } pieces[] = {
      {c->off_M, c->M.data(), c->M.size() * sizeof(double)},
      {c->off_iv, c->inv_vol.data(), c->inv_vol.size() * sizeof(double)},
      {c->off_x0j, c->x0j.data(), c->x0j.size() * sizeof(double)},
      {c->off_nbr, c->nbr.data(), c->nbr.size() * sizeof(int32_t)},
      {c->off_fcode, c->fcode.data(), c->fcode.size() * sizeof(int32_t)},
      {c->off_perm, c->perm.data(), c->perm.size() * sizeof(int32_t)},
      {c->off_stab, c->stage_tab.data(), c->stage_tab.size()},
      {c->off_vtab, c->vjp_tab.data(), c->vjp_tab.size()},
      {c->off_mom, c->mom.data(), c->mom.size() * sizeof(double)},
      {c->off_mtab, c->mean_tab.data(), c->mean_tab.size() * sizeof(double)},
      {c->off_qx, c->ref.qx.data(), c->ref.qx.size() * sizeof(double)},
      {c->off_qw, c->ref.qw.data(), c->ref.qw.size() * sizeof(double)},
      {c->off_B, c->ref.B.data(), c->ref.B.size() * sizeof(double)},
      {c->off_fw, c->ref.fw.data(), c->ref.fw.size() * sizeof(double)},
      {c->off_Bf, c->ref.Bf.data(), c->ref.Bf.size() * sizeof(double)},
  };
  for (const Piece& pc : pieces) {
    if (pc.n == 0) continue;
    hipError_t e = hipMemcpyAsync(d + pc.off, pc.src, pc.n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "mesh copy");
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "mesh copy sync");
  c->dev = d;
  c->dev_bytes = bytes;
  c->bound = true;
  return TDG_OK;
}

int tdg_set_flux(tdg_ctx* c, int flux) {
  if (!c) return TDG_ERR_INVALID_ARG;
  if (flux != TDG_FLUX_RUSANOV && flux != TDG_FLUX_ROE) return fail(c, TDG_ERR_INVALID_ARG, "unknown flux");
  c->flux = flux;
  return TDG_OK;
}

int tdg_set_viscosity(tdg_ctx* c, double mu, double prandtl) {
  if (!c) return TDG_ERR_INVALID_ARG;
  if (!(mu >= 0.0) || !std::isfinite(mu) || !(prandtl > 0.0) || !std::isfinite(prandtl))
    return fail(c, TDG_ERR_INVALID_ARG, "mu must be >= 0 and the Prandtl number > 0");
  if (c->has_mesh) return fail(c, TDG_ERR_STATE, "set the viscosity before tdg_mesh_upload (it sizes the device buffer)");
  if (mu > 0.0 && c->prec >= TDG_MIXED_BF16)
    return fail(c, TDG_ERR_UNSUPPORTED, "viscous terms are implemented for the FP64 and FP32 modes");
  c->mu = mu;
  c->prandtl = prandtl;
  return TDG_OK;
}

int tdg_set_farfield(tdg_ctx* c, const double prim[5]) {
  if (!c || !prim) return TDG_ERR_INVALID_ARG;
  if (!(prim[0] > 0.0) || !(prim[4] > 0.0)) return fail(c, TDG_ERR_INVALID_ARG, "farfield density and pressure must be positive");
  const double rho = prim[0], u = prim[1], v = prim[2], w = prim[3], p = prim[4];
  c->far[0] = rho;
  c->far[1] = rho * u;
  c->far[2] = rho * v;
  c->far[3] = rho * w;
  c->far[4] = p / (c->gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
  return TDG_OK;
}

int tdg_mesh_stats(const tdg_ctx* c, int64_t out[7]) {
  if (!c || !out) return TDG_ERR_INVALID_ARG;
  if (!c->has_mesh) return TDG_ERR_STATE;
  out[0] = c->n;
  out[1] = c->epad;
  out[2] = c->n_interior;
  out[3] = c->n_boundary;
  out[4] = c->bandwidth;
  out[5] = c->near64;
  out[6] = c->tile_tables;
  return TDG_OK;
}

int tdg_state_elems(const tdg_ctx* c, int64_t* n_elem_pad) {
  if (!c || !n_elem_pad) return TDG_ERR_INVALID_ARG;
  if (!c->has_mesh) return TDG_ERR_STATE;
  *n_elem_pad = c->epad;
  return TDG_OK;
}

int tdg_state_bytes(const tdg_ctx* c, size_t* bytes) {
  if (!c || !bytes) return TDG_ERR_INVALID_ARG;
  if (!c->has_mesh) return TDG_ERR_STATE;
  *bytes = state_bytes(c);
  return TDG_OK;
}

int tdg_set_state(tdg_ctx* c, const double* U_user, void* U_int, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!U_user || !U_int) return fail(c, TDG_ERR_INVALID_ARG, "null state pointer");
  hipError_t e = launch_set_state(c->p, c->prec, view(c), U_user, U_int, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "set_state launch");
}

int tdg_get_state(tdg_ctx* c, const void* U_int, double* U_user, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!U_user || !U_int) return fail(c, TDG_ERR_INVALID_ARG, "null state pointer");
  hipError_t e = launch_get_state(c->p, c->prec, view(c), U_int, U_user, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "get_state launch");
}

int tdg_volume_points(tdg_ctx* c, double* xyz_user, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!xyz_user) return fail(c, TDG_ERR_INVALID_ARG, "null output");
  hipError_t e = launch_volume_points(c->p, view(c), refview(c), xyz_user, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "volume_points launch");
}

int tdg_project(tdg_ctx* c, const double* prim_user, void* U_int, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!prim_user || !U_int) return fail(c, TDG_ERR_INVALID_ARG, "null pointer");
  hipError_t e = launch_project(c->p, c->prec, view(c), refview(c), c->gamma, prim_user, U_int, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "project launch");
}

static StageArgs stage_args(const tdg_ctx* c) {
  StageArgs a;
  std::memset(&a, 0, sizeof(a));
  a.mesh = view(c);
  a.tab = c->dev + c->off_stab;
  a.mom = (const double*)(c->dev + c->off_mom);
  a.mean_tab = (const double*)(c->dev + c->off_mtab);
  a.gamma = c->gamma;
  for (int v = 0; v < 5; ++v) a.far[v] = c->far[v];
  a.flux = c->flux;
  a.dt_scale = 1.0;
  return a;
}

// Mixed modes: build the operand companion of U in the context's scratch area.
static hipError_t pack_scratch(tdg_ctx* c, const void* U, StageArgs& a, hipStream_t s) {
  void* q;
  float* c0;
  comp_ptrs(c, c->dev + c->off_comp, &q, &c0);
  a.q_in = q;
  a.c0_in = c0;
  return launch_pack(c->p, c->prec, view(c), U, q, c0, s);
}

int tdg_work_bytes(const tdg_ctx* c, size_t* bytes) {
  if (!c || !bytes) return TDG_ERR_INVALID_ARG;
  if (!c->has_mesh) return TDG_ERR_STATE;
  *bytes = work_bytes(c);
  return TDG_OK;
}

// Viscous terms of U (mu > 0): Z = grad U, then the viscous residual part into the
// context's scratch, which the next stage launch adds to R through a.r_add.
static hipError_t viscous_part(tdg_ctx* c, const void* U, StageArgs& a, hipStream_t s) {
  a.r_add = nullptr;
  if (!(c->mu > 0.0)) return hipSuccess;
  ViscArgs v;
  std::memset(&v, 0, sizeof(v));
  v.u = U;
  v.z = c->dev + c->off_z;
  v.out = c->dev + c->off_z;
  v.mesh = view(c);
  v.tab = c->dev + c->off_stab;
  v.gamma = c->gamma;
  v.mu = c->mu;
  v.prandtl = c->prandtl;
  for (int k = 0; k < 5; ++k) v.far[k] = c->far[k];
  v.hbuf = c->dev + c->off_hb;
  hipError_t e = launch_grad(c->p, c->prec, v, s);
  if (e != hipSuccess) return e;
  v.out = c->dev + c->off_rv;
  e = launch_visc(c->p, c->prec, v, s);
  if (e != hipSuccess) return e;
  e = launch_visc_nbr(c->p, c->prec, v, s);
  a.r_add = c->dev + c->off_rv;
  return e;
}

int tdg_residual(tdg_ctx* c, const void* U, void* R, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!U || !R || U == R) return fail(c, TDG_ERR_INVALID_ARG, "U and R must be distinct device arrays");
  StageArgs a = stage_args(c);
  if (is_mixed(c)) {
    hipError_t e = pack_scratch(c, U, a, (hipStream_t)s);
    if (e != hipSuccess) return hip_fail(c, e, "pack launch");
  }
  hipError_t ev = viscous_part(c, U, a, (hipStream_t)s);
  if (ev != hipSuccess) return hip_fail(c, ev, "viscous launch");
  a.u_in = U;
  a.u0 = U;
  a.u_out = R;
  a.rk = 0;
  hipError_t e = launch_stage(c->p, c->prec, a, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "residual launch");
}

int tdg_rk_step(tdg_ctx* c, void* U, void* work, double dt, int n_steps, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!U || !work) return fail(c, TDG_ERR_INVALID_ARG, "null state or work pointer");
  if (n_steps < 0 || !std::isfinite(dt)) return fail(c, TDG_ERR_INVALID_ARG, "bad dt or n_steps");
  char* w = (char*)work;
  void* U1 = w;
  void* U2 = w + state_bytes(c);
  // mixed: operand companions of U, U1, U2 follow the two states
  void* q[3] = {nullptr, nullptr, nullptr};
  float* c0[3] = {nullptr, nullptr, nullptr};
  // split_rk3: the fp64 cell means of U2 (the third stage's u_in holds W2, see below)
  double* const means = split_rk3(c) ? (double*)(w + 2 * state_bytes(c) + 3 * comp_bytes(c)) : nullptr;
  if (is_mixed(c)) {
    for (int k = 0; k < 3; ++k) comp_ptrs(c, w + 2 * state_bytes(c) + k * comp_bytes(c), &q[k], &c0[k]);
    if (n_steps > 0) {
      hipError_t e = launch_pack(c->p, c->prec, view(c), U, q[0], c0[0], (hipStream_t)s);
      if (e != hipSuccess) return hip_fail(c, e, "pack launch");
    }
  }
  StageArgs a = stage_args(c);
  a.rk = 1;
  a.dt = dt;
  for (int k = 0; k < n_steps; ++k) {
    const void* ins[3] = {U, U1, U2};
    const void* base[3] = {nullptr, U, U};
    void* outs[3] = {U1, U2, U};
    const double alphas[3] = {0.0, 0.75, 1.0 / 3.0};
    const int qin[3] = {0, 1, 2}, qout[3] = {1, 2, 0};
    for (int stg = 0; stg < 3; ++stg) {
      a.u_in = ins[stg];
      a.u0 = base[stg];
      a.u_out = outs[stg];
      a.alpha = alphas[stg];
      a.q_in = q[qin[stg]];
      a.c0_in = c0[qin[stg]];
      a.q_out = q[qout[stg]];
      a.c0_out = c0[qout[stg]];
      // split_rk3: the second stage stores W2 = U0/3 + 2 U2/3 in place of U2 (U2's
      // companion and fp64 cell means beside it), so that the third stage, U3 = W2 +
      // (2/3) dt R(U2), reads no U0 (the same update as U0/3 + 2/3 (U2 + dt R(U2)))
      a.alpha_w = means && stg == 1 ? 1.0 / 3.0 : 0.0;
      a.mean_out = means && stg == 1 ? means : nullptr;
      a.mean_in = means && stg == 2 ? means : nullptr;
      a.dt_scale = means && stg == 2 ? 2.0 / 3.0 : 1.0;
      if (means && stg == 2) {
        a.alpha = 0.0;
        a.u0 = nullptr;
      }
      hipError_t e = viscous_part(c, a.u_in, a, (hipStream_t)s);
      if (e != hipSuccess) return hip_fail(c, e, "viscous launch");
      e = launch_stage(c->p, c->prec, a, (hipStream_t)s);
      if (e != hipSuccess) return hip_fail(c, e, "rk stage launch");
    }
  }
  return TDG_OK;
}

int tdg_rk_step_adaptive(tdg_ctx* c, void* U, void* work, double cfl, int n_steps, double* dt_hist, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!U || !work || !dt_hist) return fail(c, TDG_ERR_INVALID_ARG, "null state, work or dt pointer");
  if (n_steps < 0 || !(cfl > 0.0) || !std::isfinite(cfl)) return fail(c, TDG_ERR_INVALID_ARG, "bad cfl or n_steps");
  char* w = (char*)work;
  void* U1 = w;
  void* U2 = w + state_bytes(c);
  void* q[3] = {nullptr, nullptr, nullptr};
  float* c0[3] = {nullptr, nullptr, nullptr};
  // split_rk3: the fp64 cell means of U2 (the third stage's u_in holds W2, see below)
  double* const means = split_rk3(c) ? (double*)(w + 2 * state_bytes(c) + 3 * comp_bytes(c)) : nullptr;
  if (is_mixed(c)) {
    for (int k = 0; k < 3; ++k) comp_ptrs(c, w + 2 * state_bytes(c) + k * comp_bytes(c), &q[k], &c0[k]);
    if (n_steps > 0) {
      hipError_t e = launch_pack(c->p, c->prec, view(c), U, q[0], c0[0], (hipStream_t)s);
      if (e != hipSuccess) return hip_fail(c, e, "pack launch");
    }
  }
  StageArgs a = stage_args(c);
  a.rk = 1;
  a.dt = 0.0;
  for (int k = 0; k < n_steps; ++k) {
    // dt_k = min over elements of the local stable step of the current U, on the device
    hipError_t e = launch_local_dt(c->p, c->prec, view(c), c->gamma, cfl, U, dt_hist + k, (hipStream_t)s);
    if (e != hipSuccess) return hip_fail(c, e, "stable dt launch");
    a.dt_dev = dt_hist + k;
    const void* ins[3] = {U, U1, U2};
    const void* base[3] = {nullptr, U, U};
    void* outs[3] = {U1, U2, U};
    const double alphas[3] = {0.0, 0.75, 1.0 / 3.0};
    const int qin[3] = {0, 1, 2}, qout[3] = {1, 2, 0};
    for (int stg = 0; stg < 3; ++stg) {
      a.u_in = ins[stg];
      a.u0 = base[stg];
      a.u_out = outs[stg];
      a.alpha = alphas[stg];
      a.q_in = q[qin[stg]];
      a.c0_in = c0[qin[stg]];
      a.q_out = q[qout[stg]];
      a.c0_out = c0[qout[stg]];
      // split_rk3: the second stage stores W2 = U0/3 + 2 U2/3 in place of U2 (U2's
      // companion and fp64 cell means beside it), so that the third stage, U3 = W2 +
      // (2/3) dt R(U2), reads no U0 (the same update as U0/3 + 2/3 (U2 + dt R(U2)))
      a.alpha_w = means && stg == 1 ? 1.0 / 3.0 : 0.0;
      a.mean_out = means && stg == 1 ? means : nullptr;
      a.mean_in = means && stg == 2 ? means : nullptr;
      a.dt_scale = means && stg == 2 ? 2.0 / 3.0 : 1.0;
      if (means && stg == 2) {
        a.alpha = 0.0;
        a.u0 = nullptr;
      }
      e = viscous_part(c, a.u_in, a, (hipStream_t)s);
      if (e != hipSuccess) return hip_fail(c, e, "viscous launch");
      e = launch_stage(c->p, c->prec, a, (hipStream_t)s);
      if (e != hipSuccess) return hip_fail(c, e, "rk stage launch");
    }
  }
  return TDG_OK;
}

int tdg_rk_stage(tdg_ctx* c, const void* U_in, const void* U0, void* U_out, double alpha, double dt, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!U_in || !U_out || U_in == U_out || (alpha != 0.0 && !U0))
    return fail(c, TDG_ERR_INVALID_ARG, "bad stage arrays (U_out must differ from U_in; U0 needed when alpha != 0)");
  if (!std::isfinite(dt) || !std::isfinite(alpha)) return fail(c, TDG_ERR_INVALID_ARG, "bad dt or alpha");
  StageArgs a = stage_args(c);
  if (is_mixed(c)) {
    hipError_t e = pack_scratch(c, U_in, a, (hipStream_t)s);
    if (e != hipSuccess) return hip_fail(c, e, "pack launch");
  }
  a.rk = 1;
  a.dt = dt;
  a.alpha = alpha;
  a.u_in = U_in;
  a.u0 = U0;
  a.u_out = U_out;
  hipError_t ev = viscous_part(c, U_in, a, (hipStream_t)s);
  if (ev != hipSuccess) return hip_fail(c, ev, "viscous launch");
  hipError_t e = launch_stage(c->p, c->prec, a, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "rk stage launch");
}

int tdg_residual_vjp_axpy(tdg_ctx* c, const void* U, const void* W, double cw, int n_terms, const void* const* Y,
                          const double* ya, void* Out, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (c->mu > 0.0) return fail(c, TDG_ERR_UNSUPPORTED, "the adjoint covers the inviscid residual (viscosity is set)");
  if (!U || !W || !Out || Out == U || Out == W) return fail(c, TDG_ERR_INVALID_ARG, "U, W, Out must be distinct");
  if (n_terms < 0 || n_terms > 3 || (n_terms > 0 && (!Y || !ya))) return fail(c, TDG_ERR_INVALID_ARG, "bad terms");
  VjpArgs a;
  std::memset(&a, 0, sizeof(a));
  for (int k = 0; k < n_terms; ++k) {
    if (!Y[k] || Y[k] == Out) return fail(c, TDG_ERR_INVALID_ARG, "term array null or aliasing Out");
    a.y[k] = Y[k];
    a.ya[k] = ya[k];
  }
  a.n_terms = n_terms;
  a.c = cw;
  a.u = U;
  a.w = W;
  a.ubar = Out;
  a.mesh = view(c);
  a.tab = c->dev + c->off_vtab;
  a.gamma = c->gamma;
  a.flux = c->flux;
  for (int v = 0; v < 5; ++v) a.far[v] = c->far[v];
  hipError_t e = launch_vjp(c->p, c->prec, a, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "vjp launch");
}

int tdg_residual_vjp(tdg_ctx* c, const void* U, const void* W, void* Ubar, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (c->mu > 0.0) return fail(c, TDG_ERR_UNSUPPORTED, "the adjoint covers the inviscid residual (viscosity is set)");
  if (!U || !W || !Ubar || Ubar == U || Ubar == W) return fail(c, TDG_ERR_INVALID_ARG, "U, W, Ubar must be distinct");
  VjpArgs a;
  std::memset(&a, 0, sizeof(a));
  a.c = 1.0;
  a.u = U;
  a.w = W;
  a.ubar = Ubar;
  a.mesh = view(c);
  a.tab = c->dev + c->off_vtab;
  a.gamma = c->gamma;
  a.flux = c->flux;
  for (int v = 0; v < 5; ++v) a.far[v] = c->far[v];
  hipError_t e = launch_vjp(c->p, c->prec, a, (hipStream_t)s);
  if (e == hipErrorNotSupported) return fail(c, TDG_ERR_UNSUPPORTED, "VJP not available for this mode");
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "vjp launch");
}

int tdg_wall_pressure(tdg_ctx* c, const void* U, double* J, void* dJdU, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!U || !J || (dJdU && dJdU == U)) return fail(c, TDG_ERR_INVALID_ARG, "bad pointers");
  hipError_t e = launch_wall_pressure(c->p, c->prec, view(c), refview(c), c->gamma, U, J, dJdU, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "wall pressure launch");
}

int tdg_stable_dt(tdg_ctx* c, const void* U, double cfl, double* dt, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!U || !dt || !(cfl > 0.0)) return fail(c, TDG_ERR_INVALID_ARG, "bad arguments");
  hipError_t e = launch_local_dt(c->p, c->prec, view(c), c->gamma, cfl, U, dt, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "stable dt launch");
}

int tdg_check_state(tdg_ctx* c, const void* U, int64_t* n_bad, void* s) {
  int st = require_bound(c);
  if (st) return st;
  if (!U || !n_bad) return fail(c, TDG_ERR_INVALID_ARG, "null state or count pointer");
  hipError_t e = launch_check_state(c->p, c->prec, view(c), refview(c), c->gamma, U, n_bad, (hipStream_t)s);
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "check state launch");
}

int tdg_sync_check(tdg_ctx* c, void* s) {
  if (!c) return TDG_ERR_INVALID_ARG;
  hipError_t e = hipStreamSynchronize((hipStream_t)s);
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? TDG_OK : hip_fail(c, e, "stream synchronize");
}

int tdg_stream_probe(int kind, const void* src, void* dst, size_t bytes, void* s) {
  if (kind < 0 || kind > 3 || bytes == 0 || bytes % 16 != 0 || !dst || (kind != 2 && !src)) return TDG_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0) return TDG_ERR_INVALID_ARG;
  return launch_stream_probe(kind, src, dst, bytes, (hipStream_t)s) == hipSuccess ? TDG_OK : TDG_ERR_HIP;
}

int tdg_debug_tables(int order_p, int which, double* out, size_t cap, size_t* need) {
  if (order_p < 1 || order_p > 4 || which < 0 || which > 6 || !need) return TDG_ERR_INVALID_ARG;
  RefElem R;
  try {
    R = build_refelem(order_p);
  } catch (...) {
    return TDG_ERR_NOMEM;
  }
  const std::vector<double>* src[7] = {&R.qx, &R.qw, &R.fx, &R.fw, &R.B, &R.G, &R.Bf};
  const std::vector<double>& v = *src[which];
  *need = v.size();
  if (!out) return TDG_OK;
  if (cap < v.size()) return TDG_ERR_NOMEM;
  std::copy(v.begin(), v.end(), out);
  return TDG_OK;
}

}  // extern "C"
