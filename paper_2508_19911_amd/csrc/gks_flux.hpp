// gks_flux.hpp -- gas-kinetic interface flux at one Gauss point (arXiv 2508.19911, Sec. 2).
//
// Device routine, templated on the bulk arithmetic type T (double, or float in the FP32-bulk
// form).  The Gauss-point states arrive as FP64 conservative values plus T derivatives.
//
// f at the interface is eq. (flux): an equilibrium part built on g0 and the left/right parts on
// g_l (u > 0) and g_r (u < 0).  Its time integrals over [0, dt/2] and [0, dt] give the linearised
// f^n and f_t^n, whose moments are F^n, F_t^n (eq. deri-t-f) and Q^n, Q_t^n (eq. deri-t-q).  The
// coefficients of the six time functions are used in closed form (no cancellation).
//
// Precision.  The parts of the flux whose size is that of the pressure are kept in FP64 in either
// form: the conversion of both states to primitives, the split of each side at u = 0 and the
// half-space sums that give the interface equilibrium state W0 and the side fluxes <u psi>, the
// primitives of W0, its Euler flux, and the assembly of F^n, of the interface values and of the
// Prandtl correction.  At low Mach number these are ~1/Ma^2 times larger than the variations that
// drive the flow, so rounding them to FP32 would cost that many digits.  What stays in T are the
// slope and time-derivative products, whose weights (tau, dt) make them small: at the scale of the
// viscous and unsteady parts of the flux, FP32 keeps their relative precision.
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

#include <type_traits>

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

// normal moments by the Gaussian recursion u_k = U u_{k-1} + (k-1) var u_{k-2} (exact on a half
// range bounded at 0 once k >= 2); HALF = 0: the full range; HALF != 0: a half range whose u_0..u_3
// are given (computed in FP64 by the caller)
template <int HALF, class T>
__host__ __device__ __forceinline__ void frame_moments(const Prim<T>& p, T Kdof, FrameMom<T>& m,
                                                       const T* u03 = nullptr) {
  const T var = p.var;
  int k0 = 2;
  if constexpr (HALF == 0) {
    m.u[0] = T(1);
    m.u[1] = p.U;
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) m.u[k] = u03[k];
    k0 = 4;
  }
#pragma unroll
  for (int k = 2; k < 7; ++k)
    if (k >= k0) m.u[k] = p.U * m.u[k - 1] + T(k - 1) * var * m.u[k - 2];
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
// frame moments o' -> lab, stored (SET) or added into L
template <bool SET, class T>
__host__ __device__ __forceinline__ void from_frame(const T o[5], T V, T W, T kv, T L[5]) {
  if constexpr (SET) {
    L[0] = o[0];
    L[1] = o[1];
    L[2] = o[2] + V * o[0];
    L[3] = o[3] + W * o[0];
    L[4] = o[4] + V * o[2] + W * o[3] + kv * o[0];
  } else {
    L[0] = L[0] + o[0];
    L[1] = L[1] + o[1];
    L[2] = L[2] + o[2] + V * o[0];
    L[3] = L[3] + o[3] + W * o[0];
    L[4] = L[4] + o[4] + V * o[2] + W * o[3] + kv * o[0];
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
  SplitSeries split; // series coefficients of the FP64 split at u = 0
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
  f.split = make_split_series();
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

// Values of the FP64 phase that the flux needs again only at its end (G0, SP0 - G0 and the two sides'
// equilibrium interface parts) can be parked outside the registers while the slope products run:
// NoPark keeps them in registers; a kernel may pass a parking place of its own (LDS).
struct NoPark {
  template <class D, class T>
  __host__ __device__ void save(const D*, const T*, const T*, const T*) {}
  template <class D, class T>
  __host__ __device__ void load(D*, T*, T*, T*) {}
};

// conversion between the FP64 type D and the bulk type T (the identity when they are one type)
template <class T, class D>
__host__ __device__ __forceinline__ T bulk(D x) {
  if constexpr (std::is_same<T, D>::value)
    return x;
  else
    return T(x);
}

// Interface flux at one point in the face frame (first axis = face normal).
// Each side's state is Q0 + V: Q0L/Q0R[5] the average of the cell the side belongs to (FP64), VL/VR[5]
// the reconstructed point value relative to it (T); DL/DR[d*5+v]: derivative of variable v along
// face-frame axis d.  Outputs: Fn[5] = F^n (FP64); out[0..4] = F_t; with IFACE also
// out[5..9] = Q^l_n - Q0L, out[10..14] = Q^l_t, out[15..19] = Q^r_n - Q0R, out[20..24] = Q^r_t
// (interface values relative to the own cell's average, which cancels in the closed surface sum of
// the cell's gradient).  Every output is multiplied by qw (a Gauss weight, so that a sum over the
// points of a face needs no scaling; a power of two leaves the results bit for bit those of scaling
// the sum).  D is double (a counting type in the flop counter).
//
// Each Maxwellian (the two sides, then g0) is handled in its own tangentially co-moving frame, where
// the moment products are sparse; the results are shifted back to the lab before they are summed.
// Slopes are solved from the density-weighted derivatives directly (b = rho a), so every piece comes
// out density-weighted without a division.
template <class T, bool IFACE, class D = double, class Park = NoPark>
__host__ __device__ __forceinline__ void gks_flux(const FluxParams& P, double dt, const double* Q0L,
                                                  const T* VL, const T* DL, const double* Q0R,
                                                  const T* VR, const T* DR, D* Fn, T* out,
                                                  Park park = Park(), double qw = 1.0) {
  const T K = T(P.Kdof);
  const T ik3 = T(P.ik3);
  const D gm1 = D(P.gamma - 1.0);
  const D kp2 = D(P.Kdof + 2.0);
  D Ws[2][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Ws[0][v] = data<D>(Q0L[v]) + bulk<D>(VL[v]);
    Ws[1][v] = data<D>(Q0R[v]) + bulk<D>(VR[v]);
  }
  // FP64: primitives of both sides, and their half-space sums W0 = sum_s rho_s <psi>_s and
  // SP0 = sum_s rho_s <u psi>_s (side l over u > 0, side r over u < 0), in the lab frame
  D pres[2], W0[5], SP0[5];
  Prim<T> pr[2];
  T u03[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const D rho = Ws[s][0];
    const D ir = rcp64(rho);
    const D U = Ws[s][1] * ir, V = Ws[s][2] * ir, W = Ws[s][3] * ir;
    const D p = gm1 * (Ws[s][4] - D(0.5) * rho * (U * U + V * V + W * W));
    const D var = p * ir;
    pres[s] = p;
    pr[s].rho = bulk<T>(rho);
    pr[s].U = bulk<T>(U);
    pr[s].V = bulk<T>(V);
    pr[s].W = bulk<T>(W);
    pr[s].var = bulk<T>(var);
    pr[s].lam = T(0.5) * drcp(pr[s].var);
    D pp, pm, tail;
    normal_split(U, var, pp, pm, tail, P.split);
    const D u0 = s == 0 ? pp : pm;
    const D u1 = s == 0 ? U * u0 + tail : U * u0 - tail;
    const D u2 = U * u1 + var * u0;
    const D u3 = U * u2 + D(2) * var * u1;
    u03[s][0] = bulk<T>(u0);
    u03[s][1] = bulk<T>(u1);
    u03[s][2] = bulk<T>(u2);
    u03[s][3] = bulk<T>(u3);
    // <v^2 + w^2 + xi^2> / 2 in the lab
    const D kr = D(0.5) * (V * V + W * W + kp2 * var);
    const D w[5] = {rho * u0, rho * u1, rho * V * u0, rho * W * u0, rho * (D(0.5) * u2 + kr * u0)};
    const D f[5] = {rho * u1, rho * u2, rho * V * u1, rho * W * u1, rho * (D(0.5) * u3 + kr * u1)};
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      W0[v] = s == 0 ? w[v] : W0[v] + w[v];
      SP0[v] = s == 0 ? f[v] : SP0[v] + f[v];
    }
  }
  // relative pressure jump |p_l - p_r| / (p_l + p_r): the difference in FP64, the ratio in T
  const T jump = bulk<T>(fabs(pres[0] - pres[1])) * drcp(bulk<T>(pres[0] + pres[1]));

  // interface equilibrium g0: primitives and Euler flux G0 = rho0 <u psi> in FP64; the difference
  // SP0 - G0 of the two equilibrium fluxes is small where the flow is smooth and goes on in T
  const D ir0 = rcp64(W0[0]);
  const D U0 = W0[1] * ir0, V0 = W0[2] * ir0, Wv0 = W0[3] * ir0;
  const D p064 = gm1 * (W0[4] - D(0.5) * W0[0] * (U0 * U0 + V0 * V0 + Wv0 * Wv0));
  const D G0[5] = {W0[1], W0[1] * U0 + p064, W0[1] * V0, W0[1] * Wv0, U0 * (W0[4] + p064)};
  T dS[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) dS[v] = bulk<T>(SP0[v] - G0[v]);
  Prim<T> p0;
  p0.rho = bulk<T>(W0[0]);
  p0.U = bulk<T>(U0);
  p0.V = bulk<T>(V0);
  p0.W = bulk<T>(Wv0);
  p0.var = bulk<T>(p064 * ir0);
  p0.lam = T(0.5) * drcp(p0.var);
  const T pe = bulk<T>(p064);
  // the equilibrium parts of the two sides' interface values, relative to QL0 / QR0:
  // (1 - w) (W0 - Q0) + w (W^s - Q0), w = e^{-dt/tau0}, tau0 = C jump dt (a zero jump gives w = 0)
  T w = T(0), w1 = T(1), oL[5], oR[5];
  if constexpr (IFACE) {
    w = dexp(-drcp(T(P.tau_c) * jump));
    w1 = T(1) - w;
    const T w1q = T(qw) * w1, wq = T(qw) * w;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      oL[v] = w1q * bulk<T>(W0[v] - data<D>(Q0L[v])) + wq * VL[v];
      oR[v] = w1q * bulk<T>(W0[v] - data<D>(Q0R[v])) + wq * VR[v];
    }
  }
  D G0p[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) G0p[v] = D(qw) * G0[v];
  park.save(G0p, dS, oL, oR);

  // lab sums over the two sides, each piece density-weighted on its half space:
  // dW0[d] = <a_d psi>, SP = {-, <u (a.u) psi>, <u A psi>, -, <(a.u) psi>, <A psi>}
  T dW0[3][5], SP[6][5];
  T eul[2][5];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const Prim<T>& p = pr[s];
    const T* Dd = s ? DR : DL;
    const T V = p.V, W = p.W, kv = T(0.5) * (V * V + W * W);
    FrameMom<T> mh, mf;
    if (s == 0)
      frame_moments<+1>(p, K, mh, u03[0]);
    else
      frame_moments<-1>(p, K, mh, u03[1]);
    frame_moments<0>(p, K, mf);
    SlopeSolver<T> sv;
    sv.init(p, K, ik3);
    // b[d] = rho a_d: <b[d] psi'> = D'[d] over the full range
    T Dp[3][5], b[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      to_frame(Dd + 5 * d, V, W, kv, Dp[d]);
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
    // the side's slope pieces on its half space
    T dw[3][5], s1[5], s2[5], s4[5], s5[5];
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
#pragma unroll
      for (int d = 0; d < 3; ++d) from_frame<true>(dw[d], V, W, kv, dW0[d]);
      from_frame<true>(s1, V, W, kv, SP[1]);
      from_frame<true>(s2, V, W, kv, SP[2]);
      from_frame<true>(s4, V, W, kv, SP[4]);
      from_frame<true>(s5, V, W, kv, SP[5]);
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) from_frame<false>(dw[d], V, W, kv, dW0[d]);
      from_frame<false>(s1, V, W, kv, SP[1]);
      from_frame<false>(s2, V, W, kv, SP[2]);
      from_frame<false>(s4, V, W, kv, SP[4]);
      from_frame<false>(s5, V, W, kv, SP[5]);
    }
    if constexpr (IFACE) {
      from_frame<true>(E, V, W, kv, eul[s]);
#pragma unroll
      for (int v = 0; v < 5; ++v) eul[s][v] = -eul[s][v];
    }
  }

  // G = rho0 x {-, <u (ab.u) psi>, <u Ab psi>, -, <(ab.u) psi>}, in g0's tangential frame;
  // <Ab psi> = -<(ab.u) psi>
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
    T g1[5], g2[5];
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
    from_frame<true>(g1, V, W, kv, G[1]);
    from_frame<true>(g2, V, W, kv, G[2]);
    from_frame<true>(E, V, W, kv, G[4]);
  }

  // collision time (Sec. 4 opening)
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
#pragma unroll
  for (int k = 1; k < 6; ++k) cn[k] = T(qw) * cn[k];
#pragma unroll
  for (int k = 0; k < 6; ++k)
    if (k != 3) ct[k] = T(qw) * ct[k];

  park.load(G0p, dS, oL, oR);
  // F^n = (1 - cn3) G0 + cn3 SP0 + the slope and time-derivative products = G0 (FP64) + dF (T);
  // F_t = ct0 (G0 - SP0) + ...
  T dF[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    dF[v] = cn[3] * dS[v] + cn[1] * G[1][v] + cn[2] * G[2][v] + cn[4] * SP[1][v] + cn[5] * SP[2][v];
    out[v] = ct[1] * G[1][v] + ct[2] * G[2][v] + ct[4] * SP[1][v] + ct[5] * SP[2][v] - ct[0] * dS[v];
  }
  // Q^n = W0 + qs: g0 contributes W0 (<psi>) and (cn1 - cn2) <(ab.u) psi>; the sides their own pieces
  const T cq = cn[1] - cn[2];
  T qs[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) qs[v] = cq * G[4][v] + cn[4] * SP[4][v] + cn[5] * SP[5][v];
  if (P.mu0 > 0.0 && P.prandtl > 0.0 && P.prandtl != 1.0) {
    // heat flux of f^n in the g0 frame, q(F) - U0 e(Q) with q(F) = F_E - U0.F_m + |U0|^2/2 F_rho and
    // e(Q) = Q_E - U0.Q_m + |U0|^2/2 Q_rho; the Euler parts G0 and W0 cancel exactly (q(G0) = U0 e(W0)),
    // which leaves the same form of dF and qs
    const T k2 = T(0.5) * (p0.U * p0.U + p0.V * p0.V + p0.W * p0.W);
    const T qf = dF[4] - (p0.U * dF[1] + p0.V * dF[2] + p0.W * dF[3]) + k2 * dF[0];
    const T qq = qs[4] - (p0.U * qs[1] + p0.V * qs[2] + p0.W * qs[3]) + k2 * qs[0];
    dF[4] = dF[4] + T(1.0 / P.prandtl - 1.0) * (qf - p0.U * qq);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) Fn[v] = G0p[v] + bulk<D>(dF[v]);
  if constexpr (IFACE) {
    const T ctq = ct[1] - ct[2];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T Qt = ctq * G[4][v] + ct[4] * SP[4][v] + ct[5] * SP[5][v];
      out[5 + v] = oL[v] + w1 * qs[v];
      out[10 + v] = w1 * Qt + T(qw) * w * eul[0][v];
      out[15 + v] = oR[v] + w1 * qs[v];
      out[20 + v] = w1 * Qt + T(qw) * w * eul[1][v];
    }
  }
}

}  // namespace cgks
