// gks_flux.hpp -- gas-kinetic interface flux at one Gauss point (arXiv 2508.19911, Sec. 2).
//
// Device routine, templated on the bulk arithmetic type T (double, or float in the FP32-bulk
// form).  The Gauss-point states arrive as FP64 conservative values plus T derivatives; the
// conversion to primitive variables is done in FP64 and everything after it in T.
//
// f at the interface is eq. (flux): an equilibrium part built on g0 and the left/right parts on
// g_l (u > 0) and g_r (u < 0).  Its time integrals over [0, dt/2] and [0, dt] give the linearised
// f^n and f_t^n, whose moments are F^n, F_t^n (eq. deri-t-f) and Q^n, Q_t^n (eq. deri-t-q).  The
// coefficients of the six time functions are used in closed form (no cancellation).
//
// Readings where the paper defers to its references:
//  * g0 is the half-space split of the two sides, W0 = rho_l <psi>_{l,u>0} + rho_r <psi>_{r,u<0};
//    its slopes are the kinetic weighting rho_l <a^l psi>_{l,u>0} + rho_r <a^r psi>_{r,u<0};
//  * micro-slopes a solve <a psi> = dW/rho; time slopes A solve <(a.u + A) psi> = 0;
//  * collision time tau = mu(T0)/p0 + C |p_l-p_r|/(p_l+p_r) dt (viscous) or eps dt + C|..| dt;
//  * Prandtl number: F^n_E gains (1/Pr - 1) times the heat flux of f^n in the g0 frame;
//  * l/r interface values Q^s = (1-w) Q^e + w (W^s, Euler time derivative of side s),
//    w = exp(-dt/tau0), tau0 = C |p_l-p_r|/(p_l+p_r) dt.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace cgks {

// primitive state of a Maxwellian; var = 1/(2 lam) = p/rho is kept beside lam
template <class T>
struct Prim {
  T rho, U, V, W, lam, var;
};

// Moment products in a tangentially co-moving frame.
//
// Seen from the frame that moves with a Maxwellian's tangential velocity (V, W), its normal velocity
// u keeps the mean U (the half-space split is at u = 0 in either frame) while v, w and xi are
// centred.  Every moment odd in v or w then vanishes, and the products <u^A (s.psi) psi> and
// <u^A v (s.psi) psi> of a slope polynomial s = s0 + s1 u + s2 v + s3 w + s4 psi4 need only these
// sums over the normal moments u_k = <u^k> (half or full range):
//   vu[k] = <u^k v^2>     = var u_k
//   ph[k] = <u^k psi4>    = (u_{k+2} + r1 u_k) / 2
//   qq[k] = <u^k psi4^2>  = (u_{k+4} + 2 r1 u_{k+2} + r2 u_k) / 4
//   vh[k] = <u^k v^2 psi4> = (vu_{k+2} + (K+4) var vu_k) / 2
// with psi4 = (u^2 + r)/2, r = v^2 + w^2 + xi^2, r1 = <r> = (K+2) var and
// r2 = <r^2> = (K+2)(K+4) var^2 (K internal degrees of freedom, <xi^2> = K var,
// <xi^4> = K (K+2) var^2).  Moment vectors computed here are of psi' = (1, u, v', w', psi4') in the
// frame; from_frame / to_frame carry them to and from the lab.
template <class T>
struct FrameMom {
  T u[7], vu[4], ph[4], qq[3], vh[2];
};

// sqrt(lam) and sqrt(var) = sqrt(1 / (2 lam)); the FP32 form takes both from one reciprocal square
// root
template <class T>
__host__ __device__ __forceinline__ void lam_roots(T lam, T var, T& sl, T& sv) {
  sl = dsqrt(lam);
  sv = dsqrt(var);
}
__host__ __device__ __forceinline__ void lam_roots(float lam, float, float& sl, float& sv) {
  const float r = drsq(lam);
  sl = lam * r;
  sv = 0.70710678118654752f * r;
}

// normal moments by the Gaussian recursion u_k = U u_{k-1} + (k-1) var u_{k-2} (exact on a half
// range bounded at 0 once k >= 2); HALF = +1 (u > 0), -1 (u < 0) or 0 (full range)
template <int HALF, class T>
__host__ __device__ __forceinline__ void frame_moments(const Prim<T>& p, T Kdof, FrameMom<T>& m) {
  const T var = p.var;
  if constexpr (HALF == 0) {
    m.u[0] = T(1);
    m.u[1] = p.U;
  } else {
    T sl, sv;
    lam_roots(p.lam, var, sl, sv);
    // e^{-lam U^2} / (2 sqrt(pi lam)) = e^{-lam U^2} sqrt(var / (2 pi))
    const T tail = dexp(-p.lam * p.U * p.U) * (T(0.39894228040143267794) * sv);
    if constexpr (HALF > 0) {
      m.u[0] = T(0.5) * derfc(-sl * p.U);
      m.u[1] = p.U * m.u[0] + tail;
    } else {
      m.u[0] = T(0.5) * derfc(sl * p.U);
      m.u[1] = p.U * m.u[0] - tail;
    }
  }
#pragma unroll
  for (int k = 2; k < 7; ++k) m.u[k] = p.U * m.u[k - 1] + T(k - 1) * var * m.u[k - 2];
  const T hr1 = T(0.5) * (Kdof + T(2)) * var;
  const T qr2 = T(0.25) * (Kdof + T(2)) * (Kdof + T(4)) * var * var;
  const T hk4 = T(0.5) * (Kdof + T(4)) * var;
#pragma unroll
  for (int k = 0; k < 4; ++k) m.vu[k] = var * m.u[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) m.ph[k] = T(0.5) * m.u[k + 2] + hr1 * m.u[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) m.qq[k] = T(0.25) * m.u[k + 4] + hr1 * m.u[k + 2] + qr2 * m.u[k];
#pragma unroll
  for (int k = 0; k < 2; ++k) m.vh[k] = T(0.5) * m.vu[k + 2] + hk4 * m.vu[k];
}

// o = x (SET) or o + x
template <bool SET, class T>
__host__ __device__ __forceinline__ T first(T o, T a, T b) {
  if constexpr (SET)
    return a * b;
  else
    return o + a * b;
}

// o (=|+=) <u^A (s.psi') psi'>
template <int A, bool SET = false, class T>
__host__ __device__ __forceinline__ void tslope(const FrameMom<T>& m, const T s[5], T o[5]) {
  o[0] = first<SET>(o[0], s[0], m.u[A]);
  o[0] = o[0] + s[1] * m.u[A + 1];
  o[0] = o[0] + s[4] * m.ph[A];
  o[1] = first<SET>(o[1], s[0], m.u[A + 1]);
  o[1] = o[1] + s[1] * m.u[A + 2];
  o[1] = o[1] + s[4] * m.ph[A + 1];
  o[2] = first<SET>(o[2], s[2], m.vu[A]);
  o[3] = first<SET>(o[3], s[3], m.vu[A]);
  o[4] = first<SET>(o[4], s[0], m.ph[A]);
  o[4] = o[4] + s[1] * m.ph[A + 1];
  o[4] = o[4] + s[4] * m.qq[A];
}

// o += <u^A t (s.psi') psi'> for a tangential velocity t = v' (AX = 2) or w' (AX = 3)
template <int A, int AX, class T>
__host__ __device__ __forceinline__ void tslope_t(const FrameMom<T>& m, const T s[5], T o[5]) {
  o[0] = o[0] + s[AX] * m.vu[A];
  o[1] = o[1] + s[AX] * m.vu[A + 1];
  o[AX] = o[AX] + s[0] * m.vu[A];
  o[AX] = o[AX] + s[1] * m.vu[A + 1];
  o[AX] = o[AX] + s[4] * m.vh[A];
  o[4] = o[4] + s[AX] * m.vh[A];
}

// o (=|+=) rho <u^A psi'> = rho (u_A, u_{A+1}, 0, 0, ph_A)
template <int A, class T>
__host__ __device__ __forceinline__ void tpsi(const FrameMom<T>& m, T rho, T o[5]) {
  o[0] = rho * m.u[A];
  o[1] = rho * m.u[A + 1];
  o[2] = T(0);
  o[3] = T(0);
  o[4] = rho * m.ph[A];
}

// Galilean shift by the tangential velocity (V, W), kv = (V^2 + W^2)/2:
// lab moments R -> frame moments R' (psi4 = psi4' + V v' + W w' + kv)
template <class T>
__host__ __device__ __forceinline__ void to_frame(const T* R, T V, T W, T kv, T o[5]) {
  o[0] = R[0];
  o[1] = R[1];
  o[2] = R[2] - V * R[0];
  o[3] = R[3] - W * R[0];
  o[4] = R[4] - V * R[2] - W * R[3] + kv * R[0];
}
// frame moments o' -> lab, stored (SET) or added into L; ZT: o'[2] = o'[3] = 0
template <bool SET, bool ZT = false, class T>
__host__ __device__ __forceinline__ void from_frame(const T o[5], T V, T W, T kv, T L[5]) {
  if constexpr (SET) {
    L[0] = o[0];
    L[1] = o[1];
    if constexpr (ZT) {
      L[2] = V * o[0];
      L[3] = W * o[0];
      L[4] = o[4] + kv * o[0];
    } else {
      L[2] = o[2] + V * o[0];
      L[3] = o[3] + W * o[0];
      L[4] = o[4] + V * o[2] + W * o[3] + kv * o[0];
    }
  } else {
    L[0] = L[0] + o[0];
    L[1] = L[1] + o[1];
    if constexpr (ZT) {
      L[2] = L[2] + V * o[0];
      L[3] = L[3] + W * o[0];
      L[4] = L[4] + o[4] + kv * o[0];
    } else {
      L[2] = L[2] + o[2] + V * o[0];
      L[3] = L[3] + o[3] + W * o[0];
      L[4] = L[4] + o[4] + V * o[2] + W * o[3] + kv * o[0];
    }
  }
}

// Micro-slope solver in the frame (tangential means zero): the polynomial a with <a psi'> = R for the
// full-range Maxwellian.  Closed form of the 5x5 moment system; uniform per Maxwellian:
// tl = 2 lam, c4 = 8 lam^2 / (K+3), hq = (U^2 + (K+3) var)/2.
template <class T>
struct SlopeSolver {
  T U, tl, c4, hq;
  __host__ __device__ __forceinline__ void init(const Prim<T>& p, T Kdof, T ik3) {
    U = p.U;
    tl = T(2) * p.lam;
    c4 = T(8) * p.lam * p.lam * ik3;
    hq = T(0.5) * (p.U * p.U + (Kdof + T(3)) * p.var);
  }
  __host__ __device__ __forceinline__ void solve(const T R[5], T a[5]) const {
    const T Ad = R[1] - U * R[0];
    a[4] = c4 * (R[4] - hq * R[0] - U * Ad);
    a[1] = tl * Ad - U * a[4];
    a[2] = tl * R[2];
    a[3] = tl * R[3];
    a[0] = R[0] - U * a[1] - hq * a[4];
  }
};

struct FluxParams {
  double gamma;
  double Kdof;       // internal degrees of freedom
  double mu0;        // 0 => inviscid collision time
  double tref;       // Sutherland reference temperature (<= 0: constant mu0)
  double prandtl;
  double tau_eps, tau_c;
  double ik3;        // 1 / (Kdof + 3)
  double itref;      // 1 / tref (0 when tref <= 0)
};

inline FluxParams make_flux_params(double gamma, double mu0, double tref, double prandtl,
                                   double tau_eps, double tau_c) {
  FluxParams f;
  f.gamma = gamma;
  f.Kdof = (5.0 - 3.0 * gamma) / (gamma - 1.0);
  f.mu0 = mu0;
  f.tref = tref;
  f.prandtl = prandtl;
  f.tau_eps = tau_eps;
  f.tau_c = tau_c;
  f.ik3 = 1.0 / (f.Kdof + 3.0);
  f.itref = tref > 0.0 ? 1.0 / tref : 0.0;
  return f;
}

template <class T>
__host__ __device__ __forceinline__ T viscosity(const FluxParams& P, T Temp) {
  if (P.tref > 0.0) {
    const T th = Temp * T(P.itref);
    return T(P.mu0) * T(1.4042) * th * dsqrt(th) * drcp(th + T(0.4042));
  }
  return T(P.mu0);
}

// Interface flux at one point in the face frame (first axis = face normal).
// WL/WR: conservative values (FP64); DL/DR[d*5+v]: derivative of variable v along face-frame axis d.
// out: Fn[5], Ft[5], QLn[5], QLt[5], QRn[5], QRt[5].  NOUT = 10 skips the interface values.
//
// Each Maxwellian (the two sides, then g0) is handled in its own tangentially co-moving frame, where
// the moment products are sparse; the results are shifted back to the lab before they are summed.
// Slopes are solved from the density-weighted derivatives directly (b = rho a), so every piece comes
// out density-weighted without a division.
template <class T, int NOUT>
__host__ __device__ __forceinline__ void gks_flux(const FluxParams& P, double dt, const double* WL,
                                         const T* DL, const double* WR, const T* DR, T* out) {
  const T K = T(P.Kdof);
  const T ik3 = T(P.ik3);
  const double gm1 = P.gamma - 1.0;
  // primitive variables in FP64
  double pres[2];
  Prim<T> pr[2];
  {
    const double* Ws[2] = {WL, WR};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const double rho = Ws[s][0];
      const double ir = 1.0 / rho;
      const double U = Ws[s][1] * ir, V = Ws[s][2] * ir, W = Ws[s][3] * ir;
      const double p = gm1 * (Ws[s][4] - 0.5 * rho * (U * U + V * V + W * W));
      pres[s] = p;
      pr[s].rho = data<T>(rho);
      pr[s].U = data<T>(U);
      pr[s].V = data<T>(V);
      pr[s].W = data<T>(W);
      pr[s].var = data<T>(p * ir);
      pr[s].lam = T(0.5) * drcp(pr[s].var);
    }
  }

  // lab sums over the two sides, each piece density-weighted on its half space:
  // W0 = <psi>, dW0[d] = <a_d psi>, SP = {<u psi>, <u (a.u) psi>, <u A psi>, -, <(a.u) psi>, <A psi>}
  T W0[5], dW0[3][5], SP[6][5];
  T eul[2][5];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const Prim<T>& p = pr[s];
    const T* D = s ? DR : DL;
    const T V = p.V, W = p.W, kv = T(0.5) * (V * V + W * W);
    FrameMom<T> mh, mf;
    if (s == 0)
      frame_moments<+1>(p, K, mh);
    else
      frame_moments<-1>(p, K, mh);
    frame_moments<0>(p, K, mf);
    SlopeSolver<T> sv;
    sv.init(p, K, ik3);
    // b[d] = rho a_d: <b[d] psi'> = D'[d] over the full range
    T Dp[3][5], b[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      to_frame(D + 5 * d, V, W, kv, Dp[d]);
      sv.solve(Dp[d], b[d]);
    }
    // Euler time derivative of the side: rho E = <(a.u) psi> over the full range, with the lab
    // tangential velocities v = v' + V, w = w' + W (and <b[d] psi'> = D'[d]); A from compatibility
    T E[5], B[5];
    tslope<1, true>(mf, b[0], E);
    tslope_t<0, 2>(mf, b[1], E);
    tslope_t<0, 3>(mf, b[2], E);
#pragma unroll
    for (int v = 0; v < 5; ++v) E[v] = E[v] + V * Dp[1][v] + W * Dp[2][v];
    {
      T RA[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) RA[v] = -E[v];
      sv.solve(RA, B);
    }
    // the side's pieces on its half space
    T w0[5], dw[3][5], s0[5], s1[5], s2[5], s4[5], s5[5];
    tpsi<0>(mh, p.rho, w0);
    tpsi<1>(mh, p.rho, s0);
#pragma unroll
    for (int d = 0; d < 3; ++d) tslope<0, true>(mh, b[d], dw[d]);
    {
      // the lab-velocity parts V b1 + W b2 of the tangential transport share one product
      T VW[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) VW[v] = V * b[1][v] + W * b[2][v];
      tslope<2, true>(mh, b[0], s1);
      tslope_t<1, 2>(mh, b[1], s1);
      tslope_t<1, 3>(mh, b[2], s1);
      tslope<1>(mh, VW, s1);
    }
    tslope<1, true>(mh, B, s2);
    tslope<1, true>(mh, b[0], s4);
    tslope_t<0, 2>(mh, b[1], s4);
    tslope_t<0, 3>(mh, b[2], s4);
#pragma unroll
    for (int v = 0; v < 5; ++v) s4[v] = s4[v] + V * dw[1][v] + W * dw[2][v];
    tslope<0, true>(mh, B, s5);
    if (s == 0) {
      from_frame<true, true>(w0, V, W, kv, W0);
      from_frame<true, true>(s0, V, W, kv, SP[0]);
#pragma unroll
      for (int d = 0; d < 3; ++d) from_frame<true>(dw[d], V, W, kv, dW0[d]);
      from_frame<true>(s1, V, W, kv, SP[1]);
      from_frame<true>(s2, V, W, kv, SP[2]);
      from_frame<true>(s4, V, W, kv, SP[4]);
      from_frame<true>(s5, V, W, kv, SP[5]);
    } else {
      from_frame<false, true>(w0, V, W, kv, W0);
      from_frame<false, true>(s0, V, W, kv, SP[0]);
#pragma unroll
      for (int d = 0; d < 3; ++d) from_frame<false>(dw[d], V, W, kv, dW0[d]);
      from_frame<false>(s1, V, W, kv, SP[1]);
      from_frame<false>(s2, V, W, kv, SP[2]);
      from_frame<false>(s4, V, W, kv, SP[4]);
      from_frame<false>(s5, V, W, kv, SP[5]);
    }
    if constexpr (NOUT > 10) {
      from_frame<true>(E, V, W, kv, eul[s]);
#pragma unroll
      for (int v = 0; v < 5; ++v) eul[s][v] = -eul[s][v];
    }
  }

  // interface equilibrium g0, in its own tangential frame
  Prim<T> p0;
  p0.rho = W0[0];
  const T ir0 = drcp(W0[0]);
  p0.U = W0[1] * ir0;
  p0.V = W0[2] * ir0;
  p0.W = W0[3] * ir0;
  const T pe = T(gm1) * (W0[4] - T(0.5) * W0[0] * (p0.U * p0.U + p0.V * p0.V + p0.W * p0.W));
  p0.var = pe * ir0;
  p0.lam = T(0.5) * drcp(p0.var);
  // G = rho0 x {<u psi>, <u (ab.u) psi>, <u Ab psi>, -, <(ab.u) psi>}; <Ab psi> = -<(ab.u) psi>
  T G[5][5];
  {
    const T V = p0.V, W = p0.W, kv = T(0.5) * (V * V + W * W);
    FrameMom<T> m0;
    frame_moments<0>(p0, K, m0);
    SlopeSolver<T> sv;
    sv.init(p0, K, ik3);
    T Dp[3][5], bb[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      to_frame(dW0[d], V, W, kv, Dp[d]);
      sv.solve(Dp[d], bb[d]);
    }
    T E[5], Bb[5];
    tslope<1, true>(m0, bb[0], E);
    tslope_t<0, 2>(m0, bb[1], E);
    tslope_t<0, 3>(m0, bb[2], E);
#pragma unroll
    for (int v = 0; v < 5; ++v) E[v] = E[v] + V * Dp[1][v] + W * Dp[2][v];
    {
      T RA[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) RA[v] = -E[v];
      sv.solve(RA, Bb);
    }
    T g0[5], g1[5], g2[5];
    tpsi<1>(m0, p0.rho, g0);
    {
      T VW[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) VW[v] = V * bb[1][v] + W * bb[2][v];
      tslope<2, true>(m0, bb[0], g1);
      tslope_t<1, 2>(m0, bb[1], g1);
      tslope_t<1, 3>(m0, bb[2], g1);
      tslope<1>(m0, VW, g1);
    }
    tslope<1, true>(m0, Bb, g2);
    from_frame<true, true>(g0, V, W, kv, G[0]);
    from_frame<true>(g1, V, W, kv, G[1]);
    from_frame<true>(g2, V, W, kv, G[2]);
    from_frame<true>(E, V, W, kv, G[4]);
  }

  // collision time (Sec. 4 opening)
  // relative pressure jump |p_l - p_r| / (p_l + p_r): the difference in FP64, the ratio in T
  const T jump = data<T>(fabs(pres[0] - pres[1])) * drcp(data<T>(pres[0] + pres[1]));
  const T Dt = T(dt);
  T tau;
  if (P.mu0 > 0.0)
    tau = viscosity(P, p0.var) * drcp(pe) + T(P.tau_c) * jump * Dt;
  else
    tau = (T(P.tau_eps) + T(P.tau_c) * jump) * Dt;

  // closed-form coefficients of f^n and f_t^n (time integrals over [0,dt/2] and [0,dt] combined);
  // the g0 and side weights of <psi> sum to 1 in f^n and to 0 in f_t^n (cn[0] + cn[3], ct[0] + ct[3])
  const T iDt = T(1.0 / dt);
  const T om = -dexpm1(T(-0.5) * Dt * drcp(tau));  // 1 - e^{-dt/(2 tau)}; tau = 0 gives 1
  const T e1 = T(1) - om;
  const T r = tau * iDt;
  const T rq = r * om * (T(3) - e1);
  T cn[6], ct[6];
  cn[0] = T(1) - rq;
  cn[1] = T(2) * tau * rq + tau * (e1 * e1 - T(2) * e1 - T(1));
  cn[2] = tau * (rq - T(1));
  cn[3] = rq;
  cn[4] = tau * e1 * (T(2) - e1) - T(2) * tau * rq;
  cn[5] = -tau * rq;
  const T rom = r * om;
  ct[0] = T(4) * rom * om * iDt;
  ct[1] = T(4) * rom * (e1 - T(2) * rom);
  ct[2] = T(1) - T(4) * rom * rom;
  ct[4] = -ct[1];
  ct[5] = T(4) * rom * rom;

  T Fn[5], Ft[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Fn[v] = cn[0] * G[0][v] + cn[1] * G[1][v] + cn[2] * G[2][v] + cn[3] * SP[0][v] +
            cn[4] * SP[1][v] + cn[5] * SP[2][v];
    Ft[v] = ct[0] * (G[0][v] - SP[0][v]) + ct[1] * G[1][v] + ct[2] * G[2][v] + ct[4] * SP[1][v] +
            ct[5] * SP[2][v];
  }
  // Q: g0 contributes W0 (<psi>) and (cn1 - cn2) <(ab.u) psi>; the sides their own pieces
  const T cq = cn[1] - cn[2];
  T Qn[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) Qn[v] = W0[v] + cq * G[4][v] + cn[4] * SP[4][v] + cn[5] * SP[5][v];
  if (P.mu0 > 0.0 && P.prandtl > 0.0 && P.prandtl != 1.0) {
    const T k2 = T(0.5) * (p0.U * p0.U + p0.V * p0.V + p0.W * p0.W);
    const T qf = Fn[4] - (p0.U * Fn[1] + p0.V * Fn[2] + p0.W * Fn[3]) + k2 * Fn[0];
    const T qq = Qn[4] - (p0.U * Qn[1] + p0.V * Qn[2] + p0.W * Qn[3]) + k2 * Qn[0];
    Fn[4] += T(1.0 / P.prandtl - 1.0) * (qf - p0.U * qq);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    out[v] = Fn[v];
    out[5 + v] = Ft[v];
  }
  if constexpr (NOUT > 10) {
    const T ctq = ct[1] - ct[2];
    T Qt[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Qt[v] = ctq * G[4][v] + ct[4] * SP[4][v] + ct[5] * SP[5][v];
    // w = e^{-dt/tau0}, tau0 = C jump dt; a zero jump gives w = 0
    const T w = dexp(-drcp(T(P.tau_c) * jump));
    const T w1 = T(1) - w;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      out[10 + v] = w1 * Qn[v] + w * data<T>(WL[v]);
      out[15 + v] = w1 * Qt[v] + w * eul[0][v];
      out[20 + v] = w1 * Qn[v] + w * data<T>(WR[v]);
      out[25 + v] = w1 * Qt[v] + w * eul[1][v];
    }
  }
}

}  // namespace cgks
