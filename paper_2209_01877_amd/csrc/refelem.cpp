// Collapsed Gauss-Jacobi quadrature and PKD basis (see refelem.hpp).
#include "refelem.hpp"

#include <cmath>
#include <stdexcept>

namespace tetdg {

double jacobi_p(int n, double a, double b, double x) {
  // three-term recurrence of the classical Jacobi polynomials
  if (n == 0) return 1.0;
  double p0 = 1.0;
  double p1 = 0.5 * (a - b) + 0.5 * (a + b + 2.0) * x;
  for (int k = 2; k <= n; ++k) {
    const double s = 2.0 * k + a + b;
    const double c1 = 2.0 * k * (k + a + b) * (s - 2.0);
    const double c2 = (s - 1.0) * (s * (s - 2.0) * x + a * a - b * b);
    const double c3 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * s;
    const double p2 = (c2 * p1 - c3 * p0) / c1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

double jacobi_dp(int n, double a, double b, double x) {
  // d/dx P_n^(a,b) = (n + a + b + 1)/2 P_{n-1}^(a+1,b+1)
  if (n == 0) return 0.0;
  return 0.5 * (n + a + b + 1.0) * jacobi_p(n - 1, a + 1.0, b + 1.0, x);
}

void gauss_jacobi(int n, double a, double b, double* x, double* w) {
  // Newton iteration with deflation by the roots already found; initial guesses
  // from the Chebyshev-like angle of the k-th root.
  for (int k = 0; k < n; ++k) {
    double r = -std::cos((2.0 * k + 1.0) * M_PI / (2.0 * n));
    for (int it = 0; it < 100; ++it) {
      double defl = 0.0;
      for (int j = 0; j < k; ++j) defl += 1.0 / (r - x[j]);
      const double f = jacobi_p(n, a, b, r);
      const double df = jacobi_dp(n, a, b, r);
      const double step = f / (df - f * defl);
      r -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[k] = r;
  }
  // weights: 2^(a+b+1) Gamma(n+a+1) Gamma(n+b+1) / (Gamma(n+a+b+1) n! (1-x^2) P_n'(x)^2)
  const double c = std::exp((a + b + 1.0) * std::log(2.0) + std::lgamma(n + a + 1.0) + std::lgamma(n + b + 1.0) -
                            std::lgamma(n + a + b + 1.0) - std::lgamma(n + 1.0));
  for (int k = 0; k < n; ++k) {
    const double d = jacobi_dp(n, a, b, x[k]);
    w[k] = c / ((1.0 - x[k] * x[k]) * d * d);
  }
  // ascending order
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (x[j] < x[i]) {
        std::swap(x[i], x[j]);
        std::swap(w[i], w[j]);
      }
}

int n_modes(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

void pkd_eval(int p, const double xi[3], double* val, double* grad) {
  const double r = 2.0 * xi[0] - 1.0, s = 2.0 * xi[1] - 1.0, t = 2.0 * xi[2] - 1.0;
  const double a = (s + t != 0.0) ? 2.0 * (1.0 + r) / (-s - t) - 1.0 : -1.0;
  const double b = (t != 1.0) ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
  const double c = t;
  // collapsed-map derivatives
  const double da_dr = 2.0 / (-s - t);
  const double da_ds = 2.0 * (1.0 + r) / ((s + t) * (s + t));
  const double da_dt = da_ds;
  const double db_ds = 2.0 / (1.0 - t);
  const double db_dt = 2.0 * (1.0 + s) / ((1.0 - t) * (1.0 - t));
  int m = 0;
  for (int d = 0; d <= p; ++d)
    for (int k = 0; k <= d; ++k)
      for (int j = 0; j <= d - k; ++j, ++m) {
        const int i = d - j - k;
        const double norm = std::sqrt((2.0 * i + 1.0) * (2.0 * i + 2.0 * j + 2.0) * (2.0 * i + 2.0 * j + 2.0 * k + 3.0) / 6.0);
        const double hb = 0.5 * (1.0 - b), hc = 0.5 * (1.0 - c);
        const double fa = jacobi_p(i, 0.0, 0.0, a);
        const double pj = jacobi_p(j, 2.0 * i + 1.0, 0.0, b);
        const double pk = jacobi_p(k, 2.0 * i + 2.0 * j + 2.0, 0.0, c);
        const double gb = std::pow(hb, i) * pj;
        const double hcv = std::pow(hc, i + j) * pk;
        val[m] = norm * fa * gb * hcv;
        if (grad) {
          const double dfa = jacobi_dp(i, 0.0, 0.0, a);
          const double dgb = (i > 0 ? -0.5 * i * std::pow(hb, i - 1) * pj : 0.0) +
                             std::pow(hb, i) * jacobi_dp(j, 2.0 * i + 1.0, 0.0, b);
          const double dhc = (i + j > 0 ? -0.5 * (i + j) * std::pow(hc, i + j - 1) * pk : 0.0) +
                             std::pow(hc, i + j) * jacobi_dp(k, 2.0 * i + 2.0 * j + 2.0, 0.0, c);
          const double dr = dfa * gb * hcv * da_dr;
          const double ds = dfa * gb * hcv * da_ds + fa * dgb * hcv * db_ds;
          const double dt = dfa * gb * hcv * da_dt + fa * dgb * hcv * db_dt + fa * gb * dhc;
          // d/dxi = 2 d/dr, etc.
          grad[0 * (n_modes(p)) + m] = 2.0 * norm * dr;
          grad[1 * (n_modes(p)) + m] = 2.0 * norm * ds;
          grad[2 * (n_modes(p)) + m] = 2.0 * norm * dt;
        }
      }
}

void face_point(int f, double s, double t, double xi[3]) {
  static const double V[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  int vs[3], n = 0;
  for (int v = 0; v < 4; ++v)
    if (v != f) vs[n++] = v;
  for (int d = 0; d < 3; ++d)
    xi[d] = V[vs[0]][d] + s * (V[vs[1]][d] - V[vs[0]][d]) + t * (V[vs[2]][d] - V[vs[0]][d]);
}

RefElem build_refelem(int p) {
  if (p < 0 || p > 6) throw std::invalid_argument("order out of range");
  RefElem R;
  R.p = p;
  R.np = n_modes(p);
  const int n = p + 1;
  R.nq = n * n * n;
  R.nf = n * n;
  std::vector<double> xa(n), wa(n), xb(n), wb(n), xc(n), wc(n), xb1(n), wb1(n);
  gauss_jacobi(n, 0.0, 0.0, xa.data(), wa.data());
  gauss_jacobi(n, 1.0, 0.0, xb.data(), wb.data());
  gauss_jacobi(n, 2.0, 0.0, xc.data(), wc.data());
  // tet: a fastest, then b, then c
  for (int kc = 0; kc < n; ++kc)
    for (int jb = 0; jb < n; ++jb)
      for (int ia = 0; ia < n; ++ia) {
        const double A = xa[ia], Bc = xb[jb], C = xc[kc];
        R.qx.push_back((1.0 + A) * (1.0 - Bc) * (1.0 - C) / 8.0);
        R.qx.push_back((1.0 + Bc) * (1.0 - C) / 4.0);
        R.qx.push_back((1.0 + C) / 2.0);
        R.qw.push_back(wa[ia] * wb[jb] * wc[kc] / 64.0);
      }
  for (int jb = 0; jb < n; ++jb)
    for (int ia = 0; ia < n; ++ia) {
      R.fx.push_back((1.0 + xa[ia]) * (1.0 - xb[jb]) / 4.0);
      R.fx.push_back((1.0 + xb[jb]) / 2.0);
      R.fw.push_back(wa[ia] * wb[jb] / 8.0);
    }
  R.B.assign((size_t)R.nq * R.np, 0.0);
  R.G.assign((size_t)3 * R.nq * R.np, 0.0);
  R.Bf.assign((size_t)4 * R.nf * R.np, 0.0);
  std::vector<double> val(R.np), grad(3 * R.np);
  for (int q = 0; q < R.nq; ++q) {
    pkd_eval(p, &R.qx[3 * q], val.data(), grad.data());
    for (int m = 0; m < R.np; ++m) {
      R.B[(size_t)q * R.np + m] = val[m];
      for (int d = 0; d < 3; ++d) R.G[((size_t)d * R.nq + q) * R.np + m] = grad[d * R.np + m];
    }
  }
  for (int f = 0; f < 4; ++f)
    for (int q = 0; q < R.nf; ++q) {
      double xi[3];
      face_point(f, R.fx[2 * q], R.fx[2 * q + 1], xi);
      pkd_eval(p, xi, val.data(), nullptr);
      for (int m = 0; m < R.np; ++m) R.Bf[((size_t)f * R.nf + q) * R.np + m] = val[m];
    }
  return R;
}

}  // namespace tetdg
