// recon.hpp -- compact fifth-order reconstruction on the device (arXiv 2508.19911, Sec. 3.2).
//
// P^4 = Q0 + sum_m a_m p_m (eq. base); a = R d with the constant operator of the constrained
// least-squares system (eq. compact-big-5) on a uniform cell, generated in exact arithmetic.  The
// GENO blend of eq. (weno-new) is folded into the coefficients: Q(x) = chi P^4 + (1 - chi) P_L with
// P_L = Q0 + bbar . delta is again a polynomial of the same basis, so the blended coefficients are
// chi a_m plus (1 - chi) bbar on the three linear basis functions.  Readings: the sub-stencil
// polynomial across face m takes the neighbour difference as its normal slope and the target's own
// cell-averaged gradient as its tangential slopes; omega_m = d_m/(IS_m+eps)^5 normalised (paper),
// evaluated relative to the smallest IS_m+eps so no power under- or overflows; chi = omega_H/d_H
// with adaptive-order weights alpha_H = d_H (1 + (tz/(IS_H+e))^2), alpha_L = (1-d_H)
// (1 + (tz/(IS_L+e))^2), tz = |IS_H - IS_L|, e = eps + h_max^2 S (S: rho^2, 2 rho rhoE for a
// momentum, (rhoE)^2), which keeps chi at 1 at smooth critical points where both indicators are
// O(h^4) while a jump of relative size above h still drives chi to 0.
#pragma once
#include <utility>

#include "common.hpp"
#include "recon_tables.hpp"

namespace cgks {

template <class T>
__host__ __device__ __forceinline__ T dfma(T a, T b, T c) {
  return fma(a, b, c);
}

// ---- a = R d, nonzeros only ------------------------------------------------------------------------
// column form: a[m] += R[m][C] x for the nonzero rows of column C (the datum is consumed at once)
template <int C, class T, int... M>
__host__ __device__ __forceinline__ void op_col(T x, T* a, std::integer_sequence<int, M...>) {
  ((tab::R[M][C] != 0.0 ? (void)(a[M] = dfma(T(tab::R[M][C]), x, a[M])) : (void)0), ...);
}
template <int C, class T>
__host__ __device__ __forceinline__ void op_col(T x, T* a) {
  op_col<C>(x, a, std::make_integer_sequence<int, tab::NB>{});
}

// ---- indices derived from the tables at compile time ------------------------------------------------
constexpr int stencil_index(int dx, int dy, int dz) {
  for (int s = 0; s < tab::NSTEN; ++s)
    if (tab::SOFF[s][0] == dx && tab::SOFF[s][1] == dy && tab::SOFF[s][2] == dz) return s;
  return -1;
}
constexpr int basis_index(int a, int b, int c) {
  for (int m = 0; m < tab::NB; ++m)
    if (tab::BD[m][0] == a && tab::BD[m][1] == b && tab::BD[m][2] == c) return m;
  return -1;
}
// data slot of the face neighbour across face f = (-x,+x,-y,+y,-z,+z)
constexpr int face_slot(int f) {
  const int e = f / 2, s = (f % 2) ? 1 : -1;
  return tab::NEIGH_SLOT[stencil_index(e == 0 ? s : 0, e == 1 ? s : 0, e == 2 ? s : 0)];
}
constexpr int LIN[3] = {basis_index(1, 0, 0), basis_index(0, 1, 0), basis_index(0, 0, 1)};
static_assert(LIN[0] >= 0 && LIN[1] >= 0 && LIN[2] >= 0, "linear basis functions missing");

// ---- IS_H = a^T GR a ---------------------------------------------------------------------------------
template <int I, class T, int... J>
__host__ __device__ __forceinline__ T gram_row(const T* a, std::integer_sequence<int, J...>) {
  T s = T(0);
  ((tab::GR[I][J] != 0.0 ? (void)(s = dfma(T(tab::GR[I][J]), a[J], s)) : (void)0), ...);
  return s;
}
template <class T, int... I>
__host__ __device__ __forceinline__ T gram_form(const T* a, std::integer_sequence<int, I...>) {
  T s = T(0);
  ((s = dfma(a[I], gram_row<I>(a, std::make_integer_sequence<int, tab::NB>{}), s)), ...);
  return s;
}

struct GenoParams {
  double dH;
  double eps;
  double hmax2;  // square of the largest cell size
};

// the magnitude scale S of variable v of a cell state (for the smoothness floor of chi)
__host__ __device__ __forceinline__ double geno_scale(const double* q5, int v) {
  return v == 0 ? q5[0] * q5[0] : (v == 4 ? q5[4] * q5[4] : 2.0 * q5[0] * q5[4]);
}

// GENO: blend the coefficients a (one conservative variable) in place.  dface[f]: Q(neighbour across
// face f) - Q0 for f = (-x,+x,-y,+y,-z,+z); g0: the cell's own normalised gradient h_e dQ/dx_e;
// echi: eps + h_max^2 S, the floor of the indicators in the path function.
template <class T>
__host__ __device__ __forceinline__ T geno_blend(const T* dface, const T* g0, T* a, const GenoParams& gp,
                                                 T echi) {
  const T eps = T(gp.eps);
  T b[6][3], ISe[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int e = f / 2;
#pragma unroll
    for (int t = 0; t < 3; ++t) b[f][t] = g0[t];
    b[f][e] = (f % 2) ? dface[f] : -dface[f];
    ISe[f] = b[f][0] * b[f][0] + b[f][1] * b[f][1] + b[f][2] * b[f][2] + eps;
  }
  T mn = ISe[0];
#pragma unroll
  for (int f = 1; f < 6; ++f) mn = fmin(mn, ISe[f]);
  T wr[6], ws = T(0);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const T r = mn / ISe[f];
    const T r2 = r * r;
    wr[f] = r2 * r2 * r;
    ws += wr[f];
  }
  const T iws = T(1) / ws;
  T bb[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const T w = wr[f] * iws;
#pragma unroll
    for (int t = 0; t < 3; ++t) bb[t] += w * b[f][t];
  }
  const T ISL = bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
  const T ISH = gram_form(a, std::make_integer_sequence<int, tab::NB>{});
  const T tz = fabs(ISH - ISL);
  const T dH = T(gp.dH);
  const T xh = tz / (ISH + echi), xl = tz / (ISL + echi);
  const T aH = dH * (T(1) + xh * xh);
  const T aL = (T(1) - dH) * (T(1) + xl * xl);
  const T chi = (aH / (aH + aL)) / dH;
#pragma unroll
  for (int m = 0; m < tab::NB; ++m) a[m] *= chi;
  const T c1 = T(1) - chi;
#pragma unroll
  for (int t = 0; t < 3; ++t) a[LIN[t]] = dfma(c1, bb[t], a[LIN[t]]);
  return chi;
}

// ---- evaluation at a face Gauss point (normalised derivatives) ------------------------------------
// On face F the four Gauss points differ only in the signs (s1, s2) of the two tangential
// coordinates.  With the basis values at the (+,+) point, every basis function contributes with the
// sign s1^(d_t1) s2^(d_t2) (its parity class); the cell mean only enters even-even functions.  So
// value = E + s1 O1 + s2 O2 + s1 s2 O12 with four compile-time sums, and likewise per derivative.
template <int F, int M, int AX>
constexpr int parity_class() {
  constexpr int e = F / 2, t1 = (e + 1) % 3, t2 = (e + 2) % 3;
  int d[3] = {tab::BD[M][0], tab::BD[M][1], tab::BD[M][2]};
  if (AX >= 0) d[AX] -= 1;
  return (d[t1] & 1) | ((d[t2] & 1) << 1);
}

template <int F, class T, int... M>
__host__ __device__ __forceinline__ void eval_gp_impl(const T* a, T s1, T s2, T& val, T* der,
                                             std::integer_sequence<int, M...>) {
  T v[4] = {T(0), T(0), T(0), T(0)};
  ((v[parity_class<F, M, -1>()] = dfma(T(tab::PV[F][3][M]), a[M], v[parity_class<F, M, -1>()])), ...);
  const T s12 = s1 * s2;
  val = v[0] + s1 * v[1] + s2 * v[2] + s12 * v[3];
  T w[3][4] = {{T(0), T(0), T(0), T(0)}, {T(0), T(0), T(0), T(0)}, {T(0), T(0), T(0), T(0)}};
  ((tab::BD[M][0] > 0 ? (void)(w[0][parity_class<F, M, 0>()] =
                                   dfma(T(tab::PD[F][3][0][M]), a[M], w[0][parity_class<F, M, 0>()]))
                      : (void)0), ...);
  ((tab::BD[M][1] > 0 ? (void)(w[1][parity_class<F, M, 1>()] =
                                   dfma(T(tab::PD[F][3][1][M]), a[M], w[1][parity_class<F, M, 1>()]))
                      : (void)0), ...);
  ((tab::BD[M][2] > 0 ? (void)(w[2][parity_class<F, M, 2>()] =
                                   dfma(T(tab::PD[F][3][2][M]), a[M], w[2][parity_class<F, M, 2>()]))
                      : (void)0), ...);
#pragma unroll
  for (int x = 0; x < 3; ++x) der[x] = w[x][0] + s1 * w[x][1] + s2 * w[x][2] + s12 * w[x][3];
}

// value and the three normalised derivatives of sum_m a_m p_m at the Gauss point of face F with
// tangential signs (s1, s2)
template <int F, class T>
__host__ __device__ __forceinline__ void eval_gp(const T* a, T s1, T s2, T& val, T* der) {
  static_assert(tab::GP_SIGN[3][0] == 1 && tab::GP_SIGN[3][1] == 1, "table point 3 must be (+,+)");
  eval_gp_impl<F>(a, s1, s2, val, der, std::make_integer_sequence<int, tab::NB>{});
}

// ---- all four Gauss points of a face, either side -------------------------------------------------------
// Evaluated at the (+,+) point of face F = 2e+1 (normal coordinate +1/2), a basis function's value
// changes sign with the normal coordinate when its normal exponent is odd and with a tangential
// sign when that exponent is odd; the zero-mean shift is nonzero only for all-even exponents.  So
// eight parity-class sums give the values at the four points of the + face (sn = +1) and, with
// sn = -1, of the - face of the same axis.  Class bits: 1 = t1 odd, 2 = t2 odd, 4 = normal odd.
template <int F, int M, int AX>
constexpr int parity_class8() {
  constexpr int e = F / 2, t1 = (e + 1) % 3, t2 = (e + 2) % 3;
  int d[3] = {tab::BD[M][0], tab::BD[M][1], tab::BD[M][2]};
  if (AX >= 0) d[AX] -= 1;
  return (d[t1] & 1) | ((d[t2] & 1) << 1) | ((d[e] & 1) << 2);
}

// the four point values from the eight class sums, in the table's point order (-,-), (-,+), (+,-), (+,+)
template <class T>
__host__ __device__ __forceinline__ void gp_combine(const T v[8], T sn, T out[4]) {
  T u[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) u[t] = dfma(sn, v[4 + t], v[t]);
  const T A = u[0] + u[3], B = u[1] + u[2], C = u[0] - u[3], D = u[1] - u[2];
  out[0] = A - B;
  out[1] = C - D;
  out[2] = C + D;
  out[3] = A + B;
}

template <int F, class T, int... M>
__host__ __device__ __forceinline__ void eval_face_impl(const T* a, T sn, T* val, T (*der)[3],
                                                        std::integer_sequence<int, M...>) {
  T v[8] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  ((v[parity_class8<F, M, -1>()] = dfma(T(tab::PV[F][3][M]), a[M], v[parity_class8<F, M, -1>()])), ...);
  gp_combine(v, sn, val);
  T w[3][8];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int c = 0; c < 8; ++c) w[x][c] = T(0);
  ((tab::BD[M][0] > 0 ? (void)(w[0][parity_class8<F, M, 0>()] =
                                   dfma(T(tab::PD[F][3][0][M]), a[M], w[0][parity_class8<F, M, 0>()]))
                      : (void)0), ...);
  ((tab::BD[M][1] > 0 ? (void)(w[1][parity_class8<F, M, 1>()] =
                                   dfma(T(tab::PD[F][3][1][M]), a[M], w[1][parity_class8<F, M, 1>()]))
                      : (void)0), ...);
  ((tab::BD[M][2] > 0 ? (void)(w[2][parity_class8<F, M, 2>()] =
                                   dfma(T(tab::PD[F][3][2][M]), a[M], w[2][parity_class8<F, M, 2>()]))
                      : (void)0), ...);
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    T o[4];
    gp_combine(w[x], sn, o);
#pragma unroll
    for (int g = 0; g < 4; ++g) der[g][x] = o[g];
  }
}

// value and the three normalised derivatives of sum_m a_m p_m at the four Gauss points of the face
// of axis e = F/2 on the + side (sn = +1) or the - side (sn = -1); F must be the + face
template <int F, class T>
__host__ __device__ __forceinline__ void eval_face(const T* a, T sn, T val[4], T der[4][3]) {
  static_assert(F % 2 == 1, "tables of the + face");
  static_assert(tab::GP_SIGN[0][0] == -1 && tab::GP_SIGN[0][1] == -1 && tab::GP_SIGN[1][0] == -1 &&
                    tab::GP_SIGN[1][1] == 1 && tab::GP_SIGN[2][0] == 1 && tab::GP_SIGN[2][1] == -1 &&
                    tab::GP_SIGN[3][0] == 1 && tab::GP_SIGN[3][1] == 1,
                "Gauss point order");
  eval_face_impl<F>(a, sn, val, der, std::make_integer_sequence<int, tab::NB>{});
}

}  // namespace cgks
