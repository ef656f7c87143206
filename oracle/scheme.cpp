/*
 * scheme.cpp -- oracle: finite-volume assembly, time stepping and diagnostics
 * (arXiv 2508.19911, Sec. 2, 3.1, 3.4 and 4).  TEST INFRASTRUCTURE ONLY.
 *
 *  - L_i = -(1/|Omega|) sum over faces of the 2x2-Gauss face average of F^n (eq. semi with
 *    K = 4 points per face for CGKS-5th, the face midpoint for GKS-2nd); dL/dt likewise with F_t.
 *  - Cell-averaged gradient by Gauss's theorem from the interface values (Sec. 3.1); the cell on
 *    each side of a face takes its own side's value (R10).
 *  - CGKS-5th: two-stage fourth-order update of the averages and the two-stage update of the
 *    interface values (Sec. 3.4); both stages use the same dt.
 *  - GKS-2nd: Q^{n+1} = Q^n + dt L + dt^2/2 dL/dt (Sec. 3.4).
 *  - Time step (Sec. 4 opening), reading R11: dt = min(CFL min_i min_d h_d/(|U_d|+c),
 *    CFL h_min^2/(3 nu_max)), nu = mu(T)/rho, the second term only for viscous flow.
 *  - Diagnostics (Sec. 4.1, 4.2), reading R14: one-point (cell-average) quadrature with the
 *    velocity gradient (grad m - U grad rho)/rho from the cell-averaged gradients.
 */
#include "oracle_internal.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace cgkso {

struct Ctx {
  cgkso_params P;
  long N;
  double h[3];
  std::vector<double> Q, G;  // 5N, 15N
  double t = 0.0;
  long step = 0;
  bool have_state = false;
  std::vector<float> mlp;  // MLP parameters (LEARNED)
  bool have_mlp = false;
  std::vector<unsigned char> flags;
};

static inline long wrap(long i, long n) { return ((i % n) + n) % n; }

static inline long cell_index(const Ctx& c, long i, long j, long k) {
  const cgkso_params& P = c.P;
  return (wrap(k, P.nz) * P.ny + wrap(j, P.ny)) * P.nx + wrap(i, P.nx);
}

// Features of the troubled-cell indicator (reading R17): for rho and rho E, along each axis,
// the values of the cells i-2..i+2 minus the centre value (centre dropped) and h_d dQ/dx_d of
// the same five cells, scaled by s = max|difference| + max|h dQ| + 1e-12 |Q_i| (features 0..53).
// Those are scale-free, but the GENO label compares the variation with the smoothness floor
// h_max^2 S_v, so features 54..58 give, for each conservative variable v, log10 of the largest
// difference or h dQ on the same lines over h_max sqrt(S_v) (clipped below at -12); zero padded.
static void cell_features(const Ctx& c, const double* Q, const double* G, long i, long j, long k,
                          double f[64]) {
  const long N = c.N;
  for (int n = 0; n < 64; ++n) f[n] = 0.0;
  {
    const long c0 = cell_index(c, i, j, k);
    double q5[5];
    for (int v = 0; v < 5; ++v) q5[v] = Q[v * N + c0];
    const double hmax = std::fmax(c.h[0], std::fmax(c.h[1], c.h[2]));
    for (int v = 0; v < 5; ++v) {
      double mx = 0.0;
      for (int d = 0; d < 3; ++d)
        for (int o = -2; o <= 2; ++o) {
          const long ci = cell_index(c, i + (d == 0 ? o : 0), j + (d == 1 ? o : 0), k + (d == 2 ? o : 0));
          mx = std::fmax(mx, std::fabs(Q[v * N + ci] - q5[v]));
          mx = std::fmax(mx, std::fabs(c.h[d] * G[(5 * d + v) * N + ci]));
        }
      f[54 + v] = std::fmax(std::log10(mx / (hmax * std::sqrt(geno_scale(q5, v)))), -12.0);
    }
  }
  const int vars[2] = {0, 4};
  const long c0 = cell_index(c, i, j, k);
  for (int vi = 0; vi < 2; ++vi) {
    const int v = vars[vi];
    double dv[3][4], gv[3][5];
    double mx_d = 0.0, mx_g = 0.0;
    for (int d = 0; d < 3; ++d) {
      int slot = 0;
      for (int o = -2; o <= 2; ++o) {
        const long ii = i + (d == 0 ? o : 0), jj = j + (d == 1 ? o : 0), kk = k + (d == 2 ? o : 0);
        const long ci = cell_index(c, ii, jj, kk);
        if (o != 0) {
          dv[d][slot] = Q[v * N + ci] - Q[v * N + c0];
          mx_d = std::fmax(mx_d, std::fabs(dv[d][slot]));
          ++slot;
        }
        gv[d][o + 2] = c.h[d] * G[(5 * d + v) * N + ci];
        mx_g = std::fmax(mx_g, std::fabs(gv[d][o + 2]));
      }
    }
    const double s = mx_d + mx_g + 1e-12 * std::fabs(Q[v * N + c0]);
    for (int d = 0; d < 3; ++d) {
      double* o = f + vi * 27 + d * 9;
      for (int m = 0; m < 4; ++m) o[m] = dv[d][m] / s;
      for (int m = 0; m < 5; ++m) o[4 + m] = gv[d][m] / s;
    }
  }
}

static void compute_flags(Ctx& c, const double* Q, const double* G) {
  const cgkso_params& P = c.P;
  // flags = the cells on which the nonlinear blend (GENO, or the limiter of GKS-2nd) runs
  c.flags.assign(c.N, P.recon == CGKSO_RECON_LINEAR ? 0 : 1);
  if (P.recon != CGKSO_RECON_LEARNED) return;
  std::vector<float> X(c.N * 64);
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i) {
        double f[64];
        cell_features(c, Q, G, i, j, k, f);
        const long ci = cell_index(c, i, j, k);
        for (int n = 0; n < 64; ++n) X[ci * 64 + n] = static_cast<float>(f[n]);
      }
  std::vector<double> logit(c.N);
  mlp_forward(c.mlp.data(), X.data(), c.N, 1, logit.data());
  for (long n = 0; n < c.N; ++n) c.flags[n] = logit[n] > P.indicator_logit ? 1 : 0;
}

// Permutation taking the global frame to the face frame of axis d (reading R7):
// x-faces (x,y,z), y-faces (y,z,x), z-faces (z,x,y).
static inline int perm(int d, int k) { return (d + k) % 3; }

// Reconstruction of one cell (i, j, k): values and gradients at its 24 face Gauss points,
// rec[((f * 4 + gp) * 5 + v) * 4 + o], o = value, d/dx, d/dy, d/dz.
static void recon_one(const Ctx& c, const double* Q, const double* G, long i, long j, long k,
                      double rec[480]) {
  const cgkso_params& P = c.P;
  const long N = c.N;
  int off[NSTEN][3];
  stencil_offsets(off);
  const long ci = cell_index(c, i, j, k);
  long sc[NSTEN];
  for (int s = 0; s < NSTEN; ++s) sc[s] = cell_index(c, i + off[s][0], j + off[s][1], k + off[s][2]);
  int mode = 0;
  if (P.recon == CGKSO_RECON_NONLINEAR) mode = 1;
  if (P.recon == CGKSO_RECON_LEARNED) mode = c.flags[ci] ? 1 : 0;
  double q5[5];
  for (int v = 0; v < 5; ++v) q5[v] = Q[v * N + ci];
  for (int v = 0; v < 5; ++v) {
    double q[NSTEN], g[NSTEN][3];
    for (int s = 0; s < NSTEN; ++s) {
      q[s] = Q[v * N + sc[s]];
      for (int e = 0; e < 3; ++e) g[s][e] = G[(5 * e + v) * N + sc[s]];
    }
    double out[6][4][4];
    recon_cell(P, q, g, c.h, geno_scale(q5, v), mode, out, nullptr);
    for (int f = 0; f < 6; ++f)
      for (int gp = 0; gp < 4; ++gp)
        for (int o = 0; o < 4; ++o) rec[((f * 4 + gp) * 5 + v) * 4 + o] = out[f][gp][o];
  }
}

// Flux through the face of axis d between the cells with reconstructions recl (low side, its + face)
// and recr (high side, its - face), averaged over the 4 Gauss points: acc[30] = F^n, F_t and the
// interface values Q^n, Q_t of the low and the high side, in the global frame.
static void face_flux(const cgkso_params& P, double dt, int d, const double* recl, const double* recr,
                      double acc[30]) {
  for (int n = 0; n < 30; ++n) acc[n] = 0.0;
  for (int gp = 0; gp < 4; ++gp) {
    double wl[20], wr[20];
    const double* rl = recl + ((2 * d + 1) * 4 + gp) * 20;  // + face of the low cell
    const double* rr = recr + ((2 * d) * 4 + gp) * 20;      // - face of the high cell
    for (int side = 0; side < 2; ++side) {
      const double* r = side ? rr : rl;
      double* w = side ? wr : wl;
      for (int v = 0; v < 5; ++v) {
        // conservative variable v in the face frame: momentum components permuted
        const int vg = (v >= 1 && v <= 3) ? 1 + perm(d, v - 1) : v;
        w[v] = r[vg * 4 + 0];
        for (int dd = 0; dd < 3; ++dd) w[5 + 5 * dd + v] = r[vg * 4 + 1 + perm(d, dd)];
      }
    }
    double o[30];
    point_flux(P, dt, wl, wr, o, nullptr);
    for (int blk = 0; blk < 6; ++blk)
      for (int v = 0; v < 5; ++v) {
        const int vg = (v >= 1 && v <= 3) ? 1 + perm(d, v - 1) : v;
        acc[blk * 5 + vg] += 0.25 * o[blk * 5 + v];
      }
  }
}

// Assembly of one cell from its 3 low faces fm[d] and 3 high faces fp[d]: L, dL/dt and the
// Gauss-theorem sums of the interface values (this cell is the high side of its - face and the low
// side of its + face).  Outputs at out[v * stride], out[(5 d + v) * stride].
static void assemble_one(const Ctx& c, const double* fm[3], const double* fp[3], long stride,
                         double* L, double* Lt, double* sqn, double* sqt) {
  for (int v = 0; v < 5; ++v) {
    double l = 0.0, lt = 0.0;
    for (int d = 0; d < 3; ++d) {
      l -= (fp[d][v] - fm[d][v]) / c.h[d];
      lt -= (fp[d][5 + v] - fm[d][5 + v]) / c.h[d];
      if (sqn) sqn[(5 * d + v) * stride] = (fp[d][10 + v] - fm[d][20 + v]) / c.h[d];
      if (sqt) sqt[(5 * d + v) * stride] = (fp[d][15 + v] - fm[d][25 + v]) / c.h[d];
    }
    if (L) L[v * stride] = l;
    if (Lt) Lt[v * stride] = lt;
  }
}

// One stage of CGKS-5th on (Q, G) with step size dt.  With the learned indicator the flags are
// evaluated on the stage's input when new_flags is set; the second stage of a step keeps those of
// the first (the indicator is evaluated once per time step, on Q^n).
static void stage_cgks5(Ctx& c, const double* Q, const double* G, double dt, double* L, double* Lt,
                        double* sqn, double* sqt, bool new_flags = true) {
  const cgkso_params& P = c.P;
  const long N = c.N;
  if (new_flags) compute_flags(c, Q, G);

  // reconstructed values and gradients at the 24 face Gauss points of every cell
  std::vector<double> rec(N * 480);
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i) recon_one(c, Q, G, i, j, k, &rec[cell_index(c, i, j, k) * 480]);

  // fluxes on the low face of every cell in each direction, averaged over its Gauss points
  std::vector<double> face(3 * N * 30);
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i)
        for (int d = 0; d < 3; ++d) {
          const long cr = cell_index(c, i, j, k);
          const long cl = cell_index(c, i - (d == 0), j - (d == 1), k - (d == 2));
          face_flux(P, dt, d, &rec[cl * 480], &rec[cr * 480], &face[(d * N + cr) * 30]);
        }

  // assembly
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i) {
        const long ci = cell_index(c, i, j, k);
        const double *fm[3], *fp[3];
        for (int d = 0; d < 3; ++d) {
          fm[d] = &face[(d * N + ci) * 30];
          fp[d] = &face[(d * N + cell_index(c, i + (d == 0), j + (d == 1), k + (d == 2))) * 30];
        }
        assemble_one(c, fm, fp, N, L ? L + ci : nullptr, Lt ? Lt + ci : nullptr,
                     sqn ? sqn + ci : nullptr, sqt ? sqt + ci : nullptr);
      }
}

// The same stage at a list of cells only, each from its own neighbourhood: the reconstructions of
// the cell and its 6 face neighbours, the 6 face fluxes, the assembly.  Outputs [5][n], [15][n].
static void stage_cgks5_cells(const Ctx& c, const double* Q, const double* G, double dt,
                              const long* cells, long n, double* L, double* Lt, double* sqn,
                              double* sqt) {
  const cgkso_params& P = c.P;
#pragma omp parallel for
  for (long m = 0; m < n; ++m) {
    const long ci = cells[m];
    const long i = ci % P.nx, j = (ci / P.nx) % P.ny, k = ci / ((long)P.nx * P.ny);
    std::vector<double> rc(480), rn(6 * 480);
    recon_one(c, Q, G, i, j, k, rc.data());
    for (int f = 0; f < 6; ++f) {
      const int d = f / 2, sgn = (f % 2) ? 1 : -1;
      recon_one(c, Q, G, i + (d == 0) * sgn, j + (d == 1) * sgn, k + (d == 2) * sgn, &rn[f * 480]);
    }
    double fmv[3][30], fpv[3][30];
    const double *fm[3], *fp[3];
    for (int d = 0; d < 3; ++d) {
      face_flux(P, dt, d, &rn[(2 * d) * 480], rc.data(), fmv[d]);      // low face: neighbour | cell
      face_flux(P, dt, d, rc.data(), &rn[(2 * d + 1) * 480], fpv[d]);  // high face: cell | neighbour
      fm[d] = fmv[d];
      fp[d] = fpv[d];
    }
    assemble_one(c, fm, fp, n, L ? L + m : nullptr, Lt ? Lt + m : nullptr, sqn ? sqn + m : nullptr,
                 sqt ? sqt + m : nullptr);
  }
}

// One stage of GKS-2nd on Q (face-midpoint fluxes).
static void stage_gks2(Ctx& c, const double* Q, double dt, double* L, double* Lt) {
  const cgkso_params& P = c.P;
  const long N = c.N;
  const int limited = P.recon == CGKSO_RECON_NONLINEAR;
  std::vector<double> rec(N * 120);  // 6 faces x 5 vars x 4
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i) {
        const long ci = cell_index(c, i, j, k);
        const long nb[7] = {ci,
                            cell_index(c, i - 1, j, k), cell_index(c, i + 1, j, k),
                            cell_index(c, i, j - 1, k), cell_index(c, i, j + 1, k),
                            cell_index(c, i, j, k - 1), cell_index(c, i, j, k + 1)};
        for (int v = 0; v < 5; ++v) {
          double q7[7], out[6][4];
          for (int m = 0; m < 7; ++m) q7[m] = Q[v * N + nb[m]];
          recon_cell_gks2(P, q7, c.h, limited, out);
          for (int f = 0; f < 6; ++f)
            for (int o = 0; o < 4; ++o) rec[ci * 120 + (f * 5 + v) * 4 + o] = out[f][o];
        }
      }
  std::vector<double> face(3 * N * 10);
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i)
        for (int d = 0; d < 3; ++d) {
          const long cr = cell_index(c, i, j, k);
          const long cl = cell_index(c, i - (d == 0), j - (d == 1), k - (d == 2));
          double wl[20], wr[20];
          for (int side = 0; side < 2; ++side) {
            const double* r = side ? &rec[cr * 120 + (2 * d) * 20] : &rec[cl * 120 + (2 * d + 1) * 20];
            double* w = side ? wr : wl;
            for (int v = 0; v < 5; ++v) {
              const int vg = (v >= 1 && v <= 3) ? 1 + perm(d, v - 1) : v;
              w[v] = r[vg * 4];
              for (int dd = 0; dd < 3; ++dd) w[5 + 5 * dd + v] = r[vg * 4 + 1 + perm(d, dd)];
            }
          }
          double o[30];
          point_flux(P, dt, wl, wr, o, nullptr);
          for (int blk = 0; blk < 2; ++blk)
            for (int v = 0; v < 5; ++v) {
              const int vg = (v >= 1 && v <= 3) ? 1 + perm(d, v - 1) : v;
              face[(d * N + cr) * 10 + blk * 5 + vg] = o[blk * 5 + v];
            }
        }
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i) {
        const long ci = cell_index(c, i, j, k);
        for (int v = 0; v < 5; ++v) {
          double l = 0.0, lt = 0.0;
          for (int d = 0; d < 3; ++d) {
            const long cp = cell_index(c, i + (d == 0), j + (d == 1), k + (d == 2));
            l -= (face[(d * N + cp) * 10 + v] - face[(d * N + ci) * 10 + v]) / c.h[d];
            lt -= (face[(d * N + cp) * 10 + 5 + v] - face[(d * N + ci) * 10 + 5 + v]) / c.h[d];
          }
          if (L) L[v * N + ci] = l;
          if (Lt) Lt[v * N + ci] = lt;
        }
      }
}

static bool physical(const Ctx& c, const double* Q) {
  for (long n = 0; n < c.N; ++n) {
    double q[5], prim[5], p;
    for (int v = 0; v < 5; ++v) q[v] = Q[v * c.N + n];
    if (!(q[0] > 0.0)) return false;
    cons_to_prim(q, c.P.gamma, prim, &p);
    if (!(p > 0.0) || !std::isfinite(p) || !std::isfinite(q[1]) || !std::isfinite(q[2]) ||
        !std::isfinite(q[3]))
      return false;
  }
  return true;
}

static double compute_dt(const Ctx& c, const double* Q, double cfl) {
  const cgkso_params& P = c.P;
  double dtc = INFINITY, numax = 0.0;
  for (long n = 0; n < c.N; ++n) {
    double q[5], prim[5], p;
    for (int v = 0; v < 5; ++v) q[v] = Q[v * c.N + n];
    cons_to_prim(q, P.gamma, prim, &p);
    const double snd = std::sqrt(P.gamma * p / prim[0]);
    for (int d = 0; d < 3; ++d) dtc = std::fmin(dtc, c.h[d] / (std::fabs(prim[1 + d]) + snd));
    if (P.mu0 > 0.0) numax = std::fmax(numax, viscosity(P, p / prim[0]) / prim[0]);
  }
  double dt = cfl * dtc;
  if (P.mu0 > 0.0) {
    const double hmin = std::fmin(c.h[0], std::fmin(c.h[1], c.h[2]));
    dt = std::fmin(dt, cfl * hmin * hmin / (3.0 * numax));
  }
  return dt;
}

static void advance(Ctx& c, double dt) {
  const long N = c.N;
  if (c.P.scheme == CGKSO_SCHEME_GKS2) {
    std::vector<double> L(5 * N), Lt(5 * N);
    stage_gks2(c, c.Q.data(), dt, L.data(), Lt.data());
    for (long n = 0; n < 5 * N; ++n) c.Q[n] += dt * L[n] + 0.5 * dt * dt * Lt[n];
  } else {
    std::vector<double> L0(5 * N), Lt0(5 * N), sqn0(15 * N), sqt0(15 * N);
    std::vector<double> Lt1(5 * N), sqt1(15 * N);
    stage_cgks5(c, c.Q.data(), c.G.data(), dt, L0.data(), Lt0.data(), sqn0.data(), sqt0.data());
    std::vector<double> Qs(5 * N), Gs(15 * N);
    for (long n = 0; n < 5 * N; ++n) Qs[n] = c.Q[n] + 0.5 * dt * L0[n] + 0.125 * dt * dt * Lt0[n];
    for (long n = 0; n < 15 * N; ++n) Gs[n] = sqn0[n] + 0.5 * dt * sqt0[n];
    stage_cgks5(c, Qs.data(), Gs.data(), dt, nullptr, Lt1.data(), nullptr, sqt1.data(), false);
    for (long n = 0; n < 5 * N; ++n)
      c.Q[n] += dt * L0[n] + dt * dt / 6.0 * (Lt0[n] + 2.0 * Lt1[n]);
    for (long n = 0; n < 15 * N; ++n) c.G[n] = sqn0[n] + dt * sqt1[n];
  }
  c.t += dt;
  c.step += 1;
}

}  // namespace cgkso

using namespace cgkso;

extern "C" {

int cgkso_create(const cgkso_params* p, void** out) {
  if (!p || !out) return CGKSO_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || !(p->gamma > 1.0) || !(p->lx > 0) || !(p->ly > 0) ||
      !(p->lz > 0))
    return CGKSO_EINVAL;
  Ctx* c = new Ctx;
  c->P = *p;
  c->N = static_cast<long>(p->nx) * p->ny * p->nz;
  c->h[0] = p->lx / p->nx;
  c->h[1] = p->ly / p->ny;
  c->h[2] = p->lz / p->nz;
  c->Q.assign(5 * c->N, 0.0);
  c->G.assign(15 * c->N, 0.0);
  c->flags.assign(c->N, p->recon == CGKSO_RECON_LINEAR ? 0 : 1);
  *out = c;
  return CGKSO_OK;
}

void cgkso_destroy(void* ctx) { delete static_cast<Ctx*>(ctx); }

int cgkso_set_state(void* ctx, const double* q, const double* g, double t, long step) {
  Ctx* c = static_cast<Ctx*>(ctx);
  std::memcpy(c->Q.data(), q, sizeof(double) * 5 * c->N);
  if (g)
    std::memcpy(c->G.data(), g, sizeof(double) * 15 * c->N);
  else
    std::fill(c->G.begin(), c->G.end(), 0.0);
  c->t = t;
  c->step = step;
  c->have_state = true;
  return CGKSO_OK;
}

int cgkso_get_state(void* ctx, double* q, double* g, double* t, long* step) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  if (q) std::memcpy(q, c->Q.data(), sizeof(double) * 5 * c->N);
  if (g) std::memcpy(g, c->G.data(), sizeof(double) * 15 * c->N);
  if (t) *t = c->t;
  if (step) *step = c->step;
  return CGKSO_OK;
}

int cgkso_compute_dt(void* ctx, double cfl, double* dt) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  if (!physical(*c, c->Q.data())) return CGKSO_ENONPHYSICAL;
  *dt = compute_dt(*c, c->Q.data(), cfl);
  return CGKSO_OK;
}

int cgkso_stage(void* ctx, double dt, double* L, double* Lt, double* sqn, double* sqt) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  if (c->P.recon == CGKSO_RECON_LEARNED && !c->have_mlp) return CGKSO_ESTATE;
  if (c->P.scheme == CGKSO_SCHEME_GKS2)
    stage_gks2(*c, c->Q.data(), dt, L, Lt);
  else
    stage_cgks5(*c, c->Q.data(), c->G.data(), dt, L, Lt, sqn, sqt);
  return CGKSO_OK;
}

int cgkso_stage_cells(void* ctx, double dt, const long* cells, long n, double* L, double* Lt,
                      double* sqn, double* sqt) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  if (c->P.scheme != CGKSO_SCHEME_CGKS5 || c->P.recon == CGKSO_RECON_LEARNED || !cells || n < 0)
    return CGKSO_EINVAL;
  for (long m = 0; m < n; ++m)
    if (cells[m] < 0 || cells[m] >= c->N) return CGKSO_EINVAL;
  stage_cgks5_cells(*c, c->Q.data(), c->G.data(), dt, cells, n, L, Lt, sqn, sqt);
  return CGKSO_OK;
}

int cgkso_step(void* ctx, int nsteps, double cfl, double t_stop, int* steps_done, double* t_now) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  if (c->P.recon == CGKSO_RECON_LEARNED && !c->have_mlp) return CGKSO_ESTATE;
  if (!(cfl > 0.0) || nsteps < 0) return CGKSO_EINVAL;
  int done = 0;
  int rc = CGKSO_OK;
  for (; done < nsteps; ++done) {
    if (t_stop > 0.0 && c->t >= t_stop) break;
    if (!physical(*c, c->Q.data())) {
      rc = CGKSO_ENONPHYSICAL;
      break;
    }
    double dt = compute_dt(*c, c->Q.data(), cfl);
    if (t_stop > 0.0 && c->t + dt > t_stop) dt = t_stop - c->t;
    advance(*c, dt);
  }
  if (steps_done) *steps_done = done;
  if (t_now) *t_now = c->t;
  return rc;
}

int cgkso_step_fixed(void* ctx, int nsteps, double dt) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  if (c->P.recon == CGKSO_RECON_LEARNED && !c->have_mlp) return CGKSO_ESTATE;
  for (int s = 0; s < nsteps; ++s) {
    if (!physical(*c, c->Q.data())) return CGKSO_ENONPHYSICAL;
    advance(*c, dt);
  }
  return CGKSO_OK;
}

int cgkso_diagnostics(void* ctx, double rho0, double u0, double* out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  const cgkso_params& P = c->P;
  const long N = c->N;
  const double* Q = c->Q.data();
  std::vector<double> Gc;
  const double* G = c->G.data();
  if (P.scheme == CGKSO_SCHEME_GKS2) {
    // GKS-2nd carries no gradient state: central-difference slopes of the averages
    Gc.assign(15 * N, 0.0);
    for (long k = 0; k < P.nz; ++k)
      for (long j = 0; j < P.ny; ++j)
        for (long i = 0; i < P.nx; ++i) {
          const long ci = cell_index(*c, i, j, k);
          for (int d = 0; d < 3; ++d) {
            const long cp = cell_index(*c, i + (d == 0), j + (d == 1), k + (d == 2));
            const long cm = cell_index(*c, i - (d == 0), j - (d == 1), k - (d == 2));
            for (int v = 0; v < 5; ++v)
              Gc[(5 * d + v) * N + ci] = (Q[v * N + cp] - Q[v * N + cm]) / (2.0 * c->h[d]);
          }
        }
    G = Gc.data();
  }
  double ek = 0.0, es = 0.0, ed = 0.0, tot[5] = {0, 0, 0, 0, 0};
  double rmin = INFINITY, pmin = INFINITY;
  long nflag = 0;
  const double vol = c->h[0] * c->h[1] * c->h[2];
  for (long n = 0; n < N; ++n) {
    double q[5], prim[5], p;
    for (int v = 0; v < 5; ++v) {
      q[v] = Q[v * N + n];
      tot[v] += q[v] * vol;
    }
    cons_to_prim(q, P.gamma, prim, &p);
    const double rho = prim[0];
    ek += 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / rho;
    double du[3][3];  // du[i][d] = d U_i / d x_d
    for (int d = 0; d < 3; ++d) {
      const double dr = G[(5 * d + 0) * N + n];
      for (int i = 0; i < 3; ++i) du[i][d] = (G[(5 * d + 1 + i) * N + n] - prim[1 + i] * dr) / rho;
    }
    const double wx = du[2][1] - du[1][2], wy = du[0][2] - du[2][0], wz = du[1][0] - du[0][1];
    const double div = du[0][0] + du[1][1] + du[2][2];
    const double mu = viscosity(P, p / rho);
    es += mu * (wx * wx + wy * wy + wz * wz);
    ed += mu * div * div;
    rmin = std::fmin(rmin, rho);
    pmin = std::fmin(pmin, p);
    nflag += c->flags[n] ? 1 : 0;
  }
  const double norm = 1.0 / (rho0 * u0 * u0 * static_cast<double>(N));
  out[0] = ek * norm;
  out[1] = es * norm;
  out[2] = 4.0 / 3.0 * ed * norm;
  out[3] = out[1] + out[2];
  for (int v = 0; v < 5; ++v) out[4 + v] = tot[v];
  out[9] = rmin;
  out[10] = pmin;
  out[11] = static_cast<double>(nflag) / static_cast<double>(N);
  out[12] = c->t;
  out[13] = static_cast<double>(c->step);
  out[14] = 0.0;
  out[15] = 0.0;
  return CGKSO_OK;
}

// Quadrature form of the diagnostics (Sec. 4.1, 4.2: E_k and the dissipation rates by numerical
// quadrature, velocity derivatives at the quadrature points from the reconstruction).  The rule is the
// tensor 3-point Gauss-Legendre rule on the unit cell (reading: the paper does not name its rule).
int cgkso_diagnostics_quad(void* ctx, double rho0, double u0, double* out) {
  int rc = cgkso_diagnostics(ctx, rho0, u0, out);
  if (rc != CGKSO_OK) return rc;
  Ctx* c = static_cast<Ctx*>(ctx);
  const cgkso_params& P = c->P;
  const long N = c->N;
  const double* Q = c->Q.data();
  const double* G = c->G.data();
  const bool c5 = P.scheme == CGKSO_SCHEME_CGKS5;
  // Gauss-Legendre on [-1/2, 1/2]: 0 and +-sqrt(3/5)/2 with weights 8/18 and 5/18
  const double xa[3] = {-0.5 * std::sqrt(0.6), 0.0, 0.5 * std::sqrt(0.6)};
  const double wa[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  double xq[27][3], wq[27];
  for (int kz = 0; kz < 3; ++kz)
    for (int ky = 0; ky < 3; ++ky)
      for (int kx = 0; kx < 3; ++kx) {
        const int n = (kz * 3 + ky) * 3 + kx;
        xq[n][0] = xa[kx];
        xq[n][1] = xa[ky];
        xq[n][2] = xa[kz];
        wq[n] = wa[kx] * wa[ky] * wa[kz];
      }
  int off[NSTEN][3];
  stencil_offsets(off);
  const int mode = P.recon == CGKSO_RECON_LINEAR ? 0 : 1;
  std::vector<double> cell_sums(3 * N);
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i) {
        const long ci = cell_index(*c, i, j, k);
        double pt[5][27][4];  // [variable][point][value, d/dx, d/dy, d/dz]
        if (c5) {
          double q5[5];
          for (int v = 0; v < 5; ++v) q5[v] = Q[v * N + ci];
          for (int v = 0; v < 5; ++v) {
            double q[NSTEN], g[NSTEN][3];
            for (int s = 0; s < NSTEN; ++s) {
              const long sc = cell_index(*c, i + off[s][0], j + off[s][1], k + off[s][2]);
              q[s] = Q[v * N + sc];
              for (int e = 0; e < 3; ++e) g[s][e] = G[(5 * e + v) * N + sc];
            }
            recon_cell_at(P, q, g, c->h, geno_scale(q5, v), mode, 27, xq, pt[v]);
          }
        } else {
          for (int v = 0; v < 5; ++v) {
            double q7[7];
            q7[0] = Q[v * N + ci];
            for (int d = 0; d < 3; ++d) {
              q7[1 + 2 * d] = Q[v * N + cell_index(*c, i - (d == 0), j - (d == 1), k - (d == 2))];
              q7[2 + 2 * d] = Q[v * N + cell_index(*c, i + (d == 0), j + (d == 1), k + (d == 2))];
            }
            recon_cell_gks2_at(P, q7, c->h, P.recon == CGKSO_RECON_NONLINEAR ? 1 : 0, 27, xq, pt[v]);
          }
        }
        double ek = 0.0, es = 0.0, ed = 0.0;
        for (int n = 0; n < 27; ++n) {
          double q[5], prim[5], p;
          for (int v = 0; v < 5; ++v) q[v] = pt[v][n][0];
          cons_to_prim(q, P.gamma, prim, &p);
          const double rho = prim[0];
          double du[3][3];  // du[a][d] = d U_a / d x_d = (d m_a/dx_d - U_a d rho/dx_d) / rho
          for (int d = 0; d < 3; ++d)
            for (int a = 0; a < 3; ++a) du[a][d] = (pt[1 + a][n][1 + d] - prim[1 + a] * pt[0][n][1 + d]) / rho;
          const double wx = du[2][1] - du[1][2], wy = du[0][2] - du[2][0], wz = du[1][0] - du[0][1];
          const double div = du[0][0] + du[1][1] + du[2][2];
          const double mu = viscosity(P, p / rho);
          ek += wq[n] * 0.5 * rho * (prim[1] * prim[1] + prim[2] * prim[2] + prim[3] * prim[3]);
          es += wq[n] * mu * (wx * wx + wy * wy + wz * wz);
          ed += wq[n] * mu * div * div;
        }
        cell_sums[3 * ci + 0] = ek;
        cell_sums[3 * ci + 1] = es;
        cell_sums[3 * ci + 2] = ed;
      }
  double ek = 0.0, es = 0.0, ed = 0.0;
  for (long n = 0; n < N; ++n) {
    ek += cell_sums[3 * n + 0];
    es += cell_sums[3 * n + 1];
    ed += cell_sums[3 * n + 2];
  }
  const double norm = 1.0 / (rho0 * u0 * u0 * static_cast<double>(N));
  out[0] = ek * norm;
  out[1] = es * norm;
  out[2] = 4.0 / 3.0 * ed * norm;
  out[3] = out[1] + out[2];
  return CGKSO_OK;
}

int cgkso_get_flags(void* ctx, unsigned char* flags) {
  Ctx* c = static_cast<Ctx*>(ctx);
  std::memcpy(flags, c->flags.data(), c->N);
  return CGKSO_OK;
}

int cgkso_indicator_set(void* ctx, const float* params, size_t n, double logit_threshold) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (n != CGKSO_MLP_NPARAM) return CGKSO_EINVAL;
  c->mlp.assign(params, params + n);
  c->P.indicator_logit = logit_threshold;
  c->have_mlp = true;
  return CGKSO_OK;
}

int cgkso_features(void* ctx, float* out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  const cgkso_params& P = c->P;
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i) {
        double f[64];
        cell_features(*c, c->Q.data(), c->G.data(), i, j, k, f);
        const long ci = cell_index(*c, i, j, k);
        for (int n = 0; n < 64; ++n) out[ci * 64 + n] = static_cast<float>(f[n]);
      }
  return CGKSO_OK;
}

int cgkso_chi_deviation(void* ctx, double* dev);

int cgkso_labels(void* ctx, double thr, unsigned char* out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  std::vector<double> dev(c->N);
  const int rc = cgkso_chi_deviation(ctx, dev.data());
  if (rc) return rc;
  for (long n = 0; n < c->N; ++n) out[n] = dev[n] > thr ? 1 : 0;
  return CGKSO_OK;
}

int cgkso_chi_deviation(void* ctx, double* dev) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c->have_state) return CGKSO_ESTATE;
  const cgkso_params& P = c->P;
  const long N = c->N;
  int off[NSTEN][3];
  stencil_offsets(off);
#pragma omp parallel for collapse(2)
  for (long k = 0; k < P.nz; ++k)
    for (long j = 0; j < P.ny; ++j)
      for (long i = 0; i < P.nx; ++i) {
        const long ci = cell_index(*c, i, j, k);
        double worst = 0.0;
        double q5[5];
        for (int v = 0; v < 5; ++v) q5[v] = c->Q[v * N + ci];
        for (int v = 0; v < 5; ++v) {
          double q[NSTEN], g[NSTEN][3], o[6][4][4], info[4];
          for (int s = 0; s < NSTEN; ++s) {
            const long cs = cell_index(*c, i + off[s][0], j + off[s][1], k + off[s][2]);
            q[s] = c->Q[v * N + cs];
            for (int e = 0; e < 3; ++e) g[s][e] = c->G[(5 * e + v) * N + cs];
          }
          recon_cell(P, q, g, c->h, geno_scale(q5, v), 1, o, info);
          worst = std::fmax(worst, std::fabs(1.0 - info[0]));
        }
        dev[ci] = worst;
      }
  return CGKSO_OK;
}

}  // extern "C"
