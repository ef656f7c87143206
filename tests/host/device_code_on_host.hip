// device_code_on_host.hip -- test harness: the library's __host__ __device__ flux and face-evaluation
// templates compiled for the host CPU, behind a small C ABI for the CPU test suite.  Nothing here is
// used by the library itself; it lets the CPU tests compare the device formulation with the oracle.
#include <cstdint>

#include "../../paper_2508_19911_amd/csrc/gks_flux.hpp"
#include "../../paper_2508_19911_amd/csrc/recon.hpp"

using namespace cgks;

extern "C" {

// One interface point in the face frame: wl, wr = conservative value (5) and derivatives (15, d-major)
// of each side; out[30] = F^n, F_t, Q^n / Q_t of the two sides.  precision 0: double, 1: float.
void host_point_flux(int precision, double gamma, double mu0, double tref, double prandtl, double tau_eps,
                     double tau_c, double dt, const double* wl, const double* wr, double* out) {
  const FluxParams fp = make_flux_params(gamma, mu0, tref, prandtl, tau_eps, tau_c);
  // each side's state is its cell average wl / wr plus a zero point value; the interface values
  // come back relative to it and are returned absolute
  if (precision == 0) {
    const double zero[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double dl[15], dr[15], o[25];
    for (int i = 0; i < 15; ++i) {
      dl[i] = wl[5 + i];
      dr[i] = wr[5 + i];
    }
    gks_flux<double, true>(fp, dt, wl, zero, dl, wr, zero, dr, out, o);
    for (int i = 0; i < 25; ++i) out[5 + i] = o[i];
  } else {
    const float zero[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    float dl[15], dr[15], o[25];
    for (int i = 0; i < 15; ++i) {
      dl[i] = (float)wl[5 + i];
      dr[i] = (float)wr[5 + i];
    }
    gks_flux<float, true>(fp, dt, wl, zero, dl, wr, zero, dr, out, o);
    for (int i = 0; i < 25; ++i) out[5 + i] = o[i];
  }
  for (int v = 0; v < 5; ++v) {
    out[10 + v] += wl[v];
    out[20 + v] += wr[v];
  }
}

// The FP64 split of a Maxwellian's normal velocity at u = 0 (mean U, variance var): out = {pp, pm, tail}.
void host_normal_split(double U, double var, double* out) {
  const SplitSeries ss = make_split_series();
  normal_split(U, var, out[0], out[1], out[2], ss);
}

// The 34 coefficients a of one variable evaluated at the 4 Gauss points of the face of axis e on the
// + side (sn = +1) or the - side (sn = -1) by the parity-class routine of the flux kernel:
// val[4], der[4][3] (normalised derivatives).
void host_eval_face(int e, double sn, const double* a, double* val, double* der) {
  double v[4], d[4][3];
  switch (e) {
    case 0: eval_face<1>(a, sn, v, d); break;
    case 1: eval_face<3>(a, sn, v, d); break;
    default: eval_face<5>(a, sn, v, d); break;
  }
  for (int g = 0; g < 4; ++g) {
    val[g] = v[g];
    for (int x = 0; x < 3; ++x) der[g * 3 + x] = d[g][x];
  }
}

}  // extern "C"
