/*
 * recon.cpp -- oracle: spatial reconstruction (arXiv 2508.19911, Sec. 3.2 and 3.3).
 * TEST INFRASTRUCTURE ONLY.
 *
 * CGKS-5th (Sec. 3.2): P^4 = Q0 + sum_{1<=|d|<=4} a_d p_d with the zero-mean basis of
 * eq. (base) in normalised coordinates on the 19-cell compact stencil, found by the
 * constrained least squares of eq. (compact-big-5): the 18 neighbour averages are matched
 * exactly, gradient data in the least-squares sense.  Readings:
 *  R1  data = cell averages + cell-averaged gradients of all 19 cells; every cell (the target,
 *      the 6 face and the 12 edge neighbours) contributes all 3 gradient components;
 *  R2  all least-squares rows use normalised derivatives h_e d/dx_e with unit weight;
 *  R3  sub-stencil P^1_m of eq. (p1): slope across face m from the neighbour difference,
 *      tangential slopes from the target's own cell-averaged gradient;
 *  R4  GENO blend of eq. (weno-new): omega_m from the paper's formula, evaluated as
 *      1/sum_k((IS_m+eps)/(IS_k+eps))^5; chi = omega_H/d_H with the adaptive-order weights
 *      alpha_H = d_H(1+(tau_Z/(IS_H+e_chi))^2), alpha_L = (1-d_H)(1+(tau_Z/(IS_L+e_chi))^2),
 *      tau_Z = |IS_H-IS_L|, IS_H = sum_{1<=|alpha|<=4} int (D^alpha P^4)^2 over the unit cell,
 *      IS_L = |sum_m omega_m b^m|^2; applied per conservative component.  e_chi = eps + h^2 S with
 *      h the largest cell size and S the variable's scale (rho^2, 2 rho rhoE for a momentum,
 *      (rhoE)^2): at smooth critical points both indicators are O(h^4) and a bare eps would let
 *      chi leave 1 there (second order); a jump of relative size above h still sends chi to 0.
 * Each face carries 2x2 Gauss-Legendre points (weights 1/4, Sec. 2).
 *
 * GKS-2nd (Sec. 3.3): least-squares P^1 on the 7-cell stencil (central differences on a
 * uniform grid), optional Venkatakrishnan limiter phi_0 = min over the 6 faces, evaluated at
 * the face centres.  Reading R13: phi = ((d1^2+e2) + 2 d1 d2)/(d1^2 + 2 d2^2 + d1 d2 + e2),
 * e2 = (K h)^3, d1 = max/min over {Q0, face neighbours} minus Q0 by the sign of d2.
 */
#include "oracle_internal.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace cgkso {

struct Basis {
  int d[NB][3];
  double mean[NB];
};

static double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// integral of x^n over [o-1/2, o+1/2]
static double I1(int n, double o) {
  return (std::pow(o + 0.5, n + 1) - std::pow(o - 0.5, n + 1)) / (n + 1);
}

static Basis build_basis() {
  Basis B;
  {
    int n = 0;
    for (int deg = 1; deg <= 4; ++deg)
      for (int a = deg; a >= 0; --a)
        for (int b = deg - a; b >= 0; --b) {
          B.d[n][0] = a;
          B.d[n][1] = b;
          B.d[n][2] = deg - a - b;
          B.mean[n] = I1(a, 0) / fact(a) * I1(b, 0) / fact(b) * I1(deg - a - b, 0) / fact(deg - a - b);
          ++n;
        }
  }
  return B;
}

// thread-safe one-time initialisation (function-local static)
static const Basis& basis() {
  static const Basis B = build_basis();
  return B;
}

void stencil_offsets(int off[NSTEN][3]) {
  static const int o[NSTEN][3] = {
      {0, 0, 0},   {-1, 0, 0},  {1, 0, 0},   {0, -1, 0}, {0, 1, 0},  {0, 0, -1}, {0, 0, 1},
      {-1, -1, 0}, {-1, 1, 0},  {1, -1, 0},  {1, 1, 0},  {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1},
      {1, 0, 1},   {0, -1, -1}, {0, -1, 1},  {0, 1, -1}, {0, 1, 1}};
  std::memcpy(off, o, sizeof(o));
}

// cell average over the cell at offset o of the monomial delta^d / d!
static double avg_mono(const int d[3], const int o[3]) {
  double r = 1.0;
  for (int k = 0; k < 3; ++k) r *= I1(d[k], o[k]) / fact(d[k]);
  return r;
}

// value of the basis function p_n at the point x (normalised coordinates)
static double p_at(int n, const double x[3]) {
  const Basis& B = basis();
  double r = 1.0;
  for (int k = 0; k < 3; ++k) r *= std::pow(x[k], B.d[n][k]) / fact(B.d[n][k]);
  return r - B.mean[n];
}

// d p_n / d x_e at x (normalised)
static double dp_at(int n, int e, const double x[3]) {
  const Basis& B = basis();
  if (B.d[n][e] == 0) return 0.0;
  double r = 1.0;
  for (int k = 0; k < 3; ++k) {
    const int m = B.d[n][k] - (k == e ? 1 : 0);
    r *= std::pow(x[k], m) / fact(m);
  }
  return r;
}

static std::vector<double> build_operator() {
  std::vector<double> R;
  const Basis& B = basis();
  int off[NSTEN][3];
  stencil_offsets(off);
  // constraint rows C (18 x 34): averages of p_d over the neighbours
  // least-squares rows A (57 x 34): averages of d p_d / d delta_e over all 19 cells
  std::vector<double> C(18 * NB), A(57 * NB);
  for (int n = 0; n < 18; ++n)
    for (int j = 0; j < NB; ++j) C[n * NB + j] = avg_mono(B.d[j], off[n + 1]) - B.mean[j];
  for (int c = 0; c < NSTEN; ++c)
    for (int e = 0; e < 3; ++e)
      for (int j = 0; j < NB; ++j) {
        double v = 0.0;
        if (B.d[j][e] > 0) {
          int dm[3] = {B.d[j][0], B.d[j][1], B.d[j][2]};
          dm[e] -= 1;
          v = avg_mono(dm, off[c]);
        }
        A[(3 * c + e) * NB + j] = v;
      }
  // KKT system [A^T A, C^T; C, 0] [a; mu] = [A^T b; c]
  const int n = NB + 18;
  std::vector<double> K(n * n, 0.0), rhs(n * NCOL, 0.0);
  for (int i = 0; i < NB; ++i)
    for (int j = 0; j < NB; ++j) {
      double s = 0.0;
      for (int r = 0; r < 57; ++r) s += A[r * NB + i] * A[r * NB + j];
      K[i * n + j] = s;
    }
  for (int r = 0; r < 18; ++r)
    for (int j = 0; j < NB; ++j) {
      K[(NB + r) * n + j] = C[r * NB + j];
      K[j * n + NB + r] = C[r * NB + j];
    }
  for (int r = 0; r < 18; ++r) rhs[(NB + r) * NCOL + r] = 1.0;  // value differences
  for (int r = 0; r < 57; ++r)
    for (int i = 0; i < NB; ++i) rhs[i * NCOL + 18 + r] = A[r * NB + i];  // gradient rows
  solve_dense(n, K.data(), rhs.data(), NCOL);
  R.assign(NB * NCOL, 0.0);
  for (int i = 0; i < NB; ++i)
    for (int c = 0; c < NCOL; ++c) R[i * NCOL + c] = rhs[i * NCOL + c];
  return R;
}

const double* recon_operator() {
  static const std::vector<double> R = build_operator();
  return R.data();
}

void face_gauss_points(double gp[4][2]) {
  const double g = 0.5 / std::sqrt(3.0);  // 2-point Gauss-Legendre on [-1/2, 1/2]
  const double t[4][2] = {{-g, -g}, {-g, g}, {g, -g}, {g, g}};
  std::memcpy(gp, t, sizeof(t));
}

// point on face f (axis f/2, sign -1 for even f), Gauss point k; tangential axes are cyclic
static void face_point(int f, int k, double x[3]) {
  double gp[4][2];
  face_gauss_points(gp);
  const int e = f / 2;
  x[e] = (f % 2) ? 0.5 : -0.5;
  x[(e + 1) % 3] = gp[k][0];
  x[(e + 2) % 3] = gp[k][1];
}

// Gram matrix of the smoothness indicator: sum over 1<=|alpha|<=4 of the integral over the
// unit cell of D^alpha p_i D^alpha p_j (normalised coordinates).
static std::vector<double> build_gram() {
  std::vector<double> G;
  const Basis& B = basis();
  auto J = [](int n) { return (n % 2) ? 0.0 : 2.0 * std::pow(0.5, n + 1) / (n + 1); };
  G.assign(NB * NB, 0.0);
  for (int al = 0; al < NB; ++al)
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) {
        double r = 1.0;
        for (int k = 0; k < 3; ++k) {
          const int mi = B.d[i][k] - B.d[al][k], mj = B.d[j][k] - B.d[al][k];
          if (mi < 0 || mj < 0) {
            r = 0.0;
            break;
          }
          r *= J(mi + mj) / (fact(mi) * fact(mj));
        }
        G[i * NB + j] += r;
      }
  return G;
}

static const double* is_gram() {
  static const std::vector<double> G = build_gram();
  return G.data();
}

// The reconstruction of one cell as a polynomial: a (coefficients of P^4 on the zero-mean basis), and
// for GENO the blend weight chi and the combined linear slope bbar (chi = 1, bbar = 0 otherwise).
static void recon_poly(const cgkso_params& P, const double* q, const double (*g)[3], const double h[3],
                       double scale, int mode, double a[NB], double* chi_out, double bbar[3],
                       double info[4]) {
  const double* R = recon_operator();
  double data[NCOL];
  for (int n = 0; n < 18; ++n) data[n] = q[n + 1] - q[0];
  for (int c = 0; c < NSTEN; ++c)
    for (int e = 0; e < 3; ++e) data[18 + 3 * c + e] = h[e] * g[c][e];
  for (int i = 0; i < NB; ++i) {
    double s = 0.0;
    for (int c = 0; c < NCOL; ++c) s += R[i * NCOL + c] * data[c];
    a[i] = s;
  }

  double chi = 1.0, ISH = 0.0, ISL = 0.0;
  bbar[0] = bbar[1] = bbar[2] = 0.0;
  if (mode == 1) {
    const double eps = P.geno_eps;
    // six linear sub-stencil polynomials (R3)
    double b[6][3], IS[6];
    for (int m = 0; m < 6; ++m) {
      const int e = m / 2;
      const double s = (m % 2) ? 1.0 : -1.0;
      for (int t = 0; t < 3; ++t) b[m][t] = h[t] * g[0][t];
      b[m][e] = s * (q[1 + m] - q[0]);
      IS[m] = b[m][0] * b[m][0] + b[m][1] * b[m][1] + b[m][2] * b[m][2];
    }
    double om[6];
    for (int m = 0; m < 6; ++m) {
      double s = 0.0;
      for (int k = 0; k < 6; ++k) s += std::pow((IS[m] + eps) / (IS[k] + eps), 5.0);
      om[m] = 1.0 / s;
    }
    for (int t = 0; t < 3; ++t)
      for (int m = 0; m < 6; ++m) bbar[t] += om[m] * b[m][t];
    ISL = bbar[0] * bbar[0] + bbar[1] * bbar[1] + bbar[2] * bbar[2];
    const double* G = is_gram();
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) ISH += a[i] * G[i * NB + j] * a[j];
    const double dH = P.geno_dh;
    const double tz = std::fabs(ISH - ISL);
    const double hmax = std::fmax(h[0], std::fmax(h[1], h[2]));
    const double echi = eps + hmax * hmax * scale;
    const double aH = dH * (1.0 + std::pow(tz / (ISH + echi), 2.0));
    const double aL = (1.0 - dH) * (1.0 + std::pow(tz / (ISL + echi), 2.0));
    chi = (aH / (aH + aL)) / dH;
  }
  if (info) {
    info[0] = chi;
    info[1] = ISH;
    info[2] = ISL;
    info[3] = 0.0;
  }

  *chi_out = chi;
}

// value and physical derivatives of the reconstruction at the normalised point x:
// eq. (weno-new), Q = chi P^4 + (1-chi) sum_m omega_m P^1_m, the same for the derivatives
static void eval_poly(const double* q, const double h[3], const double a[NB], double chi,
                      const double bbar[3], const double x[3], double out[4]) {
  double val = 0.0, der[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < NB; ++i) {
    val += a[i] * p_at(i, x);
    for (int e = 0; e < 3; ++e) der[e] += a[i] * dp_at(i, e, x);
  }
  const double lin = bbar[0] * x[0] + bbar[1] * x[1] + bbar[2] * x[2];
  out[0] = q[0] + chi * val + (1.0 - chi) * lin;
  for (int e = 0; e < 3; ++e) out[1 + e] = (chi * der[e] + (1.0 - chi) * bbar[e]) / h[e];
}

void recon_cell(const cgkso_params& P, const double* q, const double (*g)[3], const double h[3],
                double scale, int mode, double out[6][4][4], double info[4]) {
  double a[NB], chi, bbar[3];
  recon_poly(P, q, g, h, scale, mode, a, &chi, bbar, info);
  for (int f = 0; f < 6; ++f)
    for (int k = 0; k < 4; ++k) {
      double x[3];
      face_point(f, k, x);
      eval_poly(q, h, a, chi, bbar, x, out[f][k]);
    }
}

void recon_cell_at(const cgkso_params& P, const double* q, const double (*g)[3], const double h[3],
                   double scale, int mode, int npts, const double (*x)[3], double (*out)[4]) {
  double a[NB], chi, bbar[3];
  recon_poly(P, q, g, h, scale, mode, a, &chi, bbar, nullptr);
  for (int n = 0; n < npts; ++n) eval_poly(q, h, a, chi, bbar, x[n], out[n]);
}

double geno_scale(const double* q5, int v) {
  if (v == 0) return q5[0] * q5[0];
  if (v == 4) return q5[4] * q5[4];
  return 2.0 * q5[0] * q5[4];
}

// GKS-2nd P^1: central slopes b (per unit of the normalised coordinate) and the limiter factor phi
static void gks2_slopes(const cgkso_params& P, const double* q7, const double h[3], int limited,
                        double b[3], double* phi_out) {
  for (int e = 0; e < 3; ++e) b[e] = 0.5 * (q7[2 + 2 * e] - q7[1 + 2 * e]);
  double phi = 1.0;
  if (limited) {
    double qmax = q7[0], qmin = q7[0];
    for (int m = 1; m < 7; ++m) {
      qmax = std::fmax(qmax, q7[m]);
      qmin = std::fmin(qmin, q7[m]);
    }
    const double hh = std::cbrt(h[0] * h[1] * h[2]);
    const double e2 = std::pow(P.vk_k * hh, 3.0);
    for (int f = 0; f < 6; ++f) {
      const double s = (f % 2) ? 0.5 : -0.5;
      const double d2 = s * b[f / 2];
      double pf = 1.0;
      if (d2 != 0.0) {
        const double d1 = (d2 > 0.0) ? (qmax - q7[0]) : (qmin - q7[0]);
        pf = ((d1 * d1 + e2) + 2.0 * d1 * d2) / (d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + e2);
      }
      phi = std::fmin(phi, pf);
    }
  }
  *phi_out = phi;
}

void recon_cell_gks2(const cgkso_params& P, const double* q7, const double h[3], int limited,
                     double out[6][4]) {
  double b[3], phi;
  gks2_slopes(P, q7, h, limited, b, &phi);
  for (int f = 0; f < 6; ++f) {
    const double s = (f % 2) ? 0.5 : -0.5;
    out[f][0] = q7[0] + phi * s * b[f / 2];
    for (int e = 0; e < 3; ++e) out[f][1 + e] = phi * b[e] / h[e];
  }
}

void recon_cell_gks2_at(const cgkso_params& P, const double* q7, const double h[3], int limited, int npts,
                        const double (*x)[3], double (*out)[4]) {
  double b[3], phi;
  gks2_slopes(P, q7, h, limited, b, &phi);
  for (int n = 0; n < npts; ++n) {
    out[n][0] = q7[0] + phi * (b[0] * x[n][0] + b[1] * x[n][1] + b[2] * x[n][2]);
    for (int e = 0; e < 3; ++e) out[n][1 + e] = phi * b[e] / h[e];
  }
}

}  // namespace cgkso

using namespace cgkso;

extern "C" {

void cgkso_recon_operator(double* coef) {
  const double* R = recon_operator();
  std::memcpy(coef, R, sizeof(double) * NB * NCOL);
}

void cgkso_stencil_offsets(int* offsets) { stencil_offsets(reinterpret_cast<int(*)[3]>(offsets)); }

void cgkso_recon_cell(const cgkso_params* p, const double* q, const double* g, const double* h,
                      double scale, int mode, double* out, double* info) {
  recon_cell(*p, q, reinterpret_cast<const double(*)[3]>(g), h, scale, mode,
             reinterpret_cast<double(*)[4][4]>(out), info);
}

void cgkso_face_gauss_points(double* gp) { face_gauss_points(reinterpret_cast<double(*)[2]>(gp)); }

double cgkso_geno_scale(const double* q5, int v) { return geno_scale(q5, v); }

void cgkso_recon_cell_gks2(const cgkso_params* p, const double* q7, const double* h, int limited,
                           double* out, double* phi) {
  double b[3], ph;
  gks2_slopes(*p, q7, h, limited, b, &ph);
  recon_cell_gks2(*p, q7, h, limited, reinterpret_cast<double(*)[4]>(out));
  if (phi) *phi = ph;
}

}  // extern "C"
