/*
 * cgks_oracle.h -- FP64 CPU oracle for the CGKS-5th / GKS-2nd stage sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP path in the package.
 *
 * Method: arXiv 2508.19911, "Performance evaluation of high-order compact and
 * second-order gas-kinetic schemes" (Yang, Zhao, Xu).  Every function cites the
 * section / equation it follows.  Points where the paper defers to references
 * that are not available are implemented as explicit readings (R1..R19), listed
 * in the project design notes and in the header comment of each source file.
 *
 * All arithmetic is IEEE double; built with -O2 -ffp-contract=off.
 */
#ifndef CGKS_ORACLE_H
#define CGKS_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CGKSO_OK = 0, CGKSO_EINVAL = -1, CGKSO_ENONPHYSICAL = -4, CGKSO_ESTATE = -5 };
enum { CGKSO_SCHEME_CGKS5 = 0, CGKSO_SCHEME_GKS2 = 1 };
enum { CGKSO_RECON_LINEAR = 0, CGKSO_RECON_NONLINEAR = 1, CGKSO_RECON_LEARNED = 2 };

typedef struct {
  int nx, ny, nz;          /* cells, periodic in every direction; nz == 1 allowed */
  double lx, ly, lz;       /* box lengths, uniform cells h_d = l_d / n_d */
  double gamma;            /* ratio of specific heats; K = (5-3g)/(g-1) internal DOF */
  double mu0;              /* reference dynamic viscosity; 0 => inviscid collision time */
  double prandtl;          /* Prandtl number; 1 (or <= 0) => no heat-flux correction */
  double sutherland_tref;  /* > 0: mu = mu0 * 1.4042 th^1.5/(th+0.4042), th = T/tref; <= 0: mu = mu0 */
  double tau_eps;          /* inviscid collision time factor (paper: 0.05) */
  double tau_c;            /* pressure-jump factor C (paper: 10) */
  double vk_k;             /* Venkatakrishnan K for GKS-2nd nonlinear */
  double geno_dh;          /* GENO high-order linear weight d_H (reading R4a: 0.85) */
  double geno_eps;         /* epsilon in the GENO weights (paper: 1e-15) */
  int scheme;              /* CGKSO_SCHEME_* */
  int recon;               /* CGKSO_RECON_* */
  double indicator_logit;  /* LEARNED: a cell runs GENO iff the MLP logit > this */
} cgkso_params;

/* ---- whole-scheme driver (Sec. 2-3, 4) ---------------------------------- */
int  cgkso_create(const cgkso_params* p, void** ctx);
void cgkso_destroy(void* ctx);
/* q: 5 SoA fields [5][nz][ny][nx]; g: 15 fields, d/dx (5), d/dy (5), d/dz (5). */
int  cgkso_set_state(void* ctx, const double* q, const double* g, double t, long step);
int  cgkso_get_state(void* ctx, double* q, double* g, double* t, long* step);
/* Delta t from the CFL and viscous conditions (Sec. 4 opening). */
int  cgkso_compute_dt(void* ctx, double cfl, double* dt);
/* One stage operator evaluated on the stored state with step size dt:
 * L (5N), dL/dt (5N), Gauss-theorem sums of the interface values Qn (15N) and of their
 * time derivatives Qt (15N).  Any output pointer may be NULL. */
int  cgkso_stage(void* ctx, double dt, double* L, double* Lt, double* sqn, double* sqt);
/* The CGKS-5th stage operator (as cgkso_stage) at the cells cells[0..n) only, each computed from its
 * own neighbourhood (reconstructions of the cell and its 6 face neighbours): L[5][n], Lt[5][n],
 * sqn[15][n], sqt[15][n] (any may be NULL).  LINEAR or NONLINEAR reconstruction; EINVAL otherwise. */
int  cgkso_stage_cells(void* ctx, double dt, const long* cells, long n, double* L, double* Lt,
                       double* sqn, double* sqt);
/* nsteps time steps; the last step is shortened to hit t_stop when t_stop > 0. */
int  cgkso_step(void* ctx, int nsteps, double cfl, double t_stop, int* steps_done, double* t_now);
/* Advance with a prescribed dt (no CFL evaluation). */
int  cgkso_step_fixed(void* ctx, int nsteps, double dt);
/* out[16]: Ek, epsS, epsD, epsT, mass, momx, momy, momz, energy, rho_min, p_min,
 * flagged_fraction, t, step, 0, 0.  rho0, u0 normalise Ek and the dissipation rates. */
int  cgkso_diagnostics(void* ctx, double rho0, double u0, double* out);
/* The same with Ek, epsS, epsD, epsT integrated over each cell by the 3-point Gauss-Legendre rule per
 * axis applied to the cell's reconstruction (values and velocity derivatives at the points from it;
 * CGKS-5th P^4 with GENO for NONLINEAR and LEARNED, GKS-2nd its P^1, limited for NONLINEAR). */
int  cgkso_diagnostics_quad(void* ctx, double rho0, double u0, double* out);
/* Per-cell GENO flag used by the last stage (LEARNED) -- 1 byte per cell. */
int  cgkso_get_flags(void* ctx, unsigned char* flags);

/* ---- building blocks exposed for the pins ------------------------------- */
/* Moments of a normalised Maxwellian (rho, U, V, W, lambda); half = 0 full, +1 u>0, -1 u<0.
 * mu[0..nmax], mv[0..nmax], mw[0..nmax], mxi[0..3] = <(xi^2)^l>. */
void cgkso_moments(const double prim[5], double K, int half, int nmax,
                   double* mu, double* mv, double* mw, double* mxi);
/* Solve <a psi>_g = r for a = (a1..a5), a = a1 + a2 u + a3 v + a4 w + a5 (u^2+v^2+w^2+xi^2)/2. */
void cgkso_micro_slope(const double prim[5], double K, const double r[5], double a[5]);
/* Time integrals c1..c6 of the six time functions of eq. (flux) over [0,T]. */
void cgkso_time_integrals(double T, double tau, double c[6]);
/* Gas-kinetic flux at one Gauss point, in the face frame (first axis = face normal).
 * wl/wr: [0..4] conservative values, [5..9] d/dn, [10..14] d/dt1, [15..19] d/dt2.
 * out[30] = Fn(5), Ft(5), QLn(5), QLt(5), QRn(5), QRt(5).
 * dbg (may be NULL) receives: tau, tau0, W0(5), dW0(15), abar(15), Abar(5), al(15), Al(5), ar(15), Ar(5). */
void cgkso_point_flux(const cgkso_params* p, double dt, const double* wl, const double* wr,
                      double* out, double* dbg);
/* Reconstruction operator: coef[34][75]; columns 0..17 act on Q_k - Q0 of the 18 neighbours
 * (order of cgkso_stencil_offsets), columns 18..74 on h_e (dQ/dx_e) of the 19 cells x 3. */
void cgkso_recon_operator(double* coef);
/* offsets[19][3]: the cell itself, the 6 face neighbours, the 12 edge neighbours. */
void cgkso_stencil_offsets(int* offsets);
/* One cell, one variable: q[19] cell averages, g[19][3] cell-averaged gradients (physical units)
 * on the stencil of cgkso_stencil_offsets; h[3] cell sizes; scale: the variable's magnitude squared
 * (the GENO smoothness floor is eps + h_max^2 scale).  Writes out[6][4][4]: 6 faces
 * (-x,+x,-y,+y,-z,+z), 4 Gauss points, (value, d/dx, d/dy, d/dz), and info[4] = chi, IS_H, IS_L, 0.
 * mode 0 linear, 1 GENO. */
void cgkso_recon_cell(const cgkso_params* p, const double* q, const double* g, const double* h,
                      double scale, int mode, double* out, double* info);
/* GKS-2nd P^1 of one cell and one variable (Sec. 3.3): q7[7] = the cell average, then the averages
 * of the neighbours at -x, +x, -y, +y, -z, +z; h[3] cell sizes; limited != 0 applies the
 * Venkatakrishnan factor (reading R13: eps^2 = (K h)^3 with h the geometric mean cell size, phi the
 * minimum over the six face midpoints).  out[6][4]: faces (-x,+x,-y,+y,-z,+z) x (value at the face
 * midpoint, d/dx, d/dy, d/dz); *phi (may be NULL) receives the limiter factor. */
void cgkso_recon_cell_gks2(const cgkso_params* p, const double* q7, const double* h, int limited,
                           double* out, double* phi);
/* Gauss point tangential offsets on a face (normalised units), gp[4][2]. */
void cgkso_face_gauss_points(double* gp);
/* The GENO scale of variable v (0..4) of the conservative cell average q5[5], the "scale" argument
 * of cgkso_recon_cell: rho^2 for v = 0, 2 rho rhoE for the momenta, (rhoE)^2 for v = 4. */
double cgkso_geno_scale(const double* q5, int v);

/* ---- troubled-cell MLP (BF16 emulated, FP64 arithmetic) ----------------- */
enum { CGKSO_MLP_NIN = 64, CGKSO_MLP_NH = 32, CGKSO_MLP_NPARAM = 4225 };
int  cgkso_indicator_set(void* ctx, const float* params, size_t n, double logit_threshold);
/* Features of every cell of the stored state: out[N][64] (float, unrounded). */
int  cgkso_features(void* ctx, float* out);
/* GENO labels of every cell of the stored state: 1 iff max_v |1 - chi_v| > thr. */
int  cgkso_labels(void* ctx, double thr, unsigned char* out);
/* The quantity the labels threshold: max over the 5 variables of |1 - chi| under full GENO, per cell. */
int  cgkso_chi_deviation(void* ctx, double* dev);
/* Forward pass on n samples x[n][64]: logits[n].  bf16 != 0 rounds inputs, weights and hidden
 * activations to bfloat16 (round to nearest even) as the GPU kernels do. */
void cgkso_mlp_forward(const float* params, const float* x, long n, int bf16, double* logits);
/* Mean binary cross-entropy (with logits) over n samples and its gradient wrt params[4225]. */
double cgkso_mlp_loss_grad(const float* params, const float* x, const float* y, long n, int bf16,
                           double* grad);

#ifdef __cplusplus
}
#endif
#endif
