// Reference-element data: collapsed Gauss-Jacobi quadrature and the orthonormal
// PKD modal basis on the unit tetrahedron (the Gaussian element/face integrals and
// the modal expansion of arXiv 2209.01877, Sec. II.B, eqs. 10-11).  Host code, FP64.
#pragma once
#include <vector>

namespace tetdg {

struct RefElem {
  int p = 0, np = 0, nq = 0, nf = 0;
  std::vector<double> qx;   // [nq][3] volume points (xi, eta, zeta)
  std::vector<double> qw;   // [nq]    volume weights, sum 1/6
  std::vector<double> fx;   // [nf][2] face points (s, t)
  std::vector<double> fw;   // [nf]    face weights, sum 1/2
  std::vector<double> B;    // [nq][np] phi at volume points
  std::vector<double> G;    // [3][nq][np] d phi / d xi_d at volume points
  std::vector<double> Bf;   // [4][nf][np] phi at the points of local face f
};

// Gauss-Jacobi rule with n points for the weight (1-x)^alpha (1+x)^beta on [-1, 1].
void gauss_jacobi(int n, double alpha, double beta, double* x, double* w);

// Standard Jacobi polynomial P_n^(alpha,beta)(x) and its derivative.
double jacobi_p(int n, double alpha, double beta, double x);
double jacobi_dp(int n, double alpha, double beta, double x);

// Basis values (np) and optionally reference gradients (3*np, layout [d][m]) at xi.
void pkd_eval(int p, const double xi[3], double* val, double* grad);

// Reference point of local face f (opposite vertex f) at face parameter (s, t).
void face_point(int f, double s, double t, double xi[3]);

int n_modes(int p);
RefElem build_refelem(int p);

}  // namespace tetdg
