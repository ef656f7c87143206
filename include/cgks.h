/*
 * cgks.h -- C ABI of the MI355X (gfx950) CGKS-5th / GKS-2nd stage sweep library, libcgks.so.
 *
 * Method: Yang, Zhao, Xu, "Performance evaluation of high-order compact and second-order
 * gas-kinetic schemes in compressible flow simulations", arXiv 2508.19911.  The library advances the
 * compressible Navier-Stokes equations (through the BGK model, Sec. 2) on a uniform, structured,
 * triply periodic box with either
 *   - CGKS-5th (Sec. 3.2): compact P^4 reconstruction from cell averages and cell-averaged
 *     gradients on the 19-cell stencil, optional GENO blend (eq. weno-new), gas-kinetic flux at the
 *     2x2 Gauss points of every face (eq. flux, deri-t-f, deri-t-q), two-stage fourth-order update
 *     of the averages and of the gradients (Sec. 3.4); or
 *   - GKS-2nd (Sec. 3.3): P^1 with an optional Venkatakrishnan limiter, the same flux at the face
 *     midpoints, Q^{n+1} = Q^n + dt L + dt^2/2 dL/dt (Sec. 3.4).
 * The time step follows the CFL and viscous conditions of Sec. 4 (opening).
 *
 * Conventions
 *   - Every call returns int: CGKS_OK (0) or a negative error code; cgks_strerror() gives text.
 *   - Fields are SoA, x fastest: q[v][nz][ny][nx], v = (rho, rho U, rho V, rho W, rho E);
 *     gradients g[15][...] = d/dx of the 5 variables, then d/dy, then d/dz.
 *   - Host arrays are owned by the caller; copies are complete when the call returns.
 *   - The device workspace (cgks_workspace_bytes) and the HIP stream are owned by the caller (for
 *     example a torch uint8 tensor and torch.cuda.current_stream()); the library allocates no device
 *     memory and launches every kernel on that stream.  The workspace must be 256-byte aligned and
 *     outlive the context.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef CGKS_H
#define CGKS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CGKS_OK = 0,
  CGKS_EINVAL = -1,        /* bad size, parameter or enum, or a NULL context */
  CGKS_EWORKSPACE = -2,    /* workspace missing, too small or misaligned */
  CGKS_EDEVICE = -3,       /* a HIP call failed (message kept for cgks_strerror) */
  CGKS_ENONPHYSICAL = -4,  /* rho <= 0, p <= 0 or NaN found at the start of a step */
  CGKS_ESTATE = -5         /* call order: e.g. step before a state was set */
};
enum { CGKS_SCHEME_CGKS5 = 0, CGKS_SCHEME_GKS2 = 1 };
/* CGKS5: LINEAR = P^4 everywhere, NONLINEAR = GENO everywhere, LEARNED = GENO where the troubled-cell
 * network flags the cell (evaluated once per time step on Q^n; both stages use those flags).
 * GKS2: LINEAR = unlimited P^1, NONLINEAR = Venkatakrishnan limiter. */
enum { CGKS_RECON_LINEAR = 0, CGKS_RECON_NONLINEAR = 1, CGKS_RECON_LEARNED = 2 };
/* FP64: every step in double.  FP32_BULK: reconstruction, flux and gradient state in float;
 * cell averages, their stage accumulations, Gauss-point states and cons->prim in double. */
enum { CGKS_PREC_FP64 = 0, CGKS_PREC_FP32_BULK = 1 };
enum { CGKS_IC_VORTEX2D = 0, CGKS_IC_TGV = 1, CGKS_IC_HIT = 2, CGKS_IC_TGV_SUPERSONIC = 3 };

typedef struct {
  int nx, ny, nz;           /* cells per direction (>= 1; nz == 1 runs the 3-D scheme on a 2-D field);
                             nx ny nz < 2^29 (a plane of doubles below 4 GiB) */
  double lx, ly, lz;        /* box lengths; h_d = l_d / n_d */
  double gamma;             /* ratio of specific heats (> 1); internal DOF K = (5 - 3 gamma)/(gamma - 1) */
  double mu0;               /* reference viscosity; 0 selects the inviscid collision time (Sec. 4) */
  double prandtl;           /* Prandtl number (1 or <= 0: no heat-flux correction) */
  double sutherland_tref;   /* > 0: mu = mu0 1.4042 th^1.5/(th + 0.4042), th = T/tref (Sec. 4.2); else mu0 */
  double tau_eps;           /* inviscid collision-time factor (paper: 0.05) */
  double tau_c;             /* pressure-jump factor C of the collision time (paper: 10) */
  double vk_k;              /* Venkatakrishnan constant K, eps^2 = (K h)^3 (GKS2 NONLINEAR) */
  double geno_dh;           /* GENO linear weight of the high-order polynomial (0.85) */
  double geno_eps;          /* GENO epsilon (paper: 1e-15) */
  int scheme;               /* CGKS_SCHEME_* */
  int recon;                /* CGKS_RECON_* */
  int precision;            /* CGKS_PREC_* */
  double indicator_logit;   /* LEARNED: GENO iff the network's logit exceeds this */
} cgks_params;

/* Diagnostics of the current state (Sec. 4.1, 4.2): one-point quadrature of the cell averages;
 * velocity gradients from the cell-averaged gradients ((grad m - U grad rho)/rho; GKS2 uses central
 * differences).  Ek, epsS, epsD, epsT normalised by rho0 u0^2 and the cell count. */
typedef struct {
  double Ek, epsS, epsD, epsT;
  double mass, momx, momy, momz, energy; /* sums of Q |Omega_i| */
  double rho_min, p_min;
  double flagged_fraction;               /* cells that ran the nonlinear blend in the last stage */
  double t;
  double step;
  double reserved[2];
} cgks_diag;

/* Device bytes the caller must provide for these parameters (EINVAL on bad parameters). */
int cgks_workspace_bytes(const cgks_params* p, size_t* bytes);

/* Create a context on the current HIP device.  dev_workspace: device pointer of >= the bytes above,
 * 256-byte aligned; hip_stream: a hipStream_t (NULL = the null stream). */
int cgks_create(const cgks_params* p, void* dev_workspace, size_t bytes, void* hip_stream, void** ctx);
int cgks_destroy(void* ctx);

/* Set the state from host arrays q[5N], g[15N] (g may be NULL: zero gradients; GKS2 ignores g). */
int cgks_set_state(void* ctx, const double* q, const double* g, double t, long step);
/* Initial condition (Sec. 4 test cases); the box is [0, l_x] x [0, l_y] x [0, l_z].
 *   VORTEX2D {strength}, TGV {Ma, rho0, u0} (Sec. 4.1), TGV_SUPERSONIC {Ma} (Sec. 4.2): evaluated on
 *     the device, cell averages by 4x4x4 Gauss-Legendre quadrature and gradients by Gauss's theorem
 *     with 4x4 points per face; seed is ignored.
 *   HIT {Ma_t [, k0 = 8]}: decaying isotropic turbulence generated on the host from seed (see
 *     cgks_ic_host) and copied in.
 * EINVAL for an unknown kind, missing parameters, or a HIT grid that cgks_ic_host rejects. */
int cgks_set_ic(void* ctx, int kind, const double* prm, int nprm, uint64_t seed);
/* Host evaluation of a host-generated initial condition into caller arrays q[5N], g[15N] (the layout
 * of cgks_set_state); no device work and no context.  Only CGKS_IC_HIT: a cubic box (l_x = l_y = l_z,
 * nx = ny = nz a power of two); a seeded solenoidal velocity field with spectrum
 * E(k) ~ k^4 exp(-2 k^2 / k0^2) on the integer wavenumbers 1 <= |k| <= n/2 of the box, exact cell
 * averages and cell-averaged gradients, scaled to u_rms = 1 per component; rho = 1 and uniform
 * p = c^2 / gamma with c = sqrt(3) / Ma_t.  The white noise comes from a counter-based generator
 * (SplitMix64 outputs, Box-Muller normals), so the field is a function of (n, k0, seed) alone.
 * EINVAL for other kinds, a non-cubic or non-power-of-two grid, Ma_t <= 0 or k0 <= 0. */
int cgks_ic_host(const cgks_params* p, int kind, const double* prm, int nprm, uint64_t seed, double* q,
                 double* g);
/* Copy the state to host arrays (double).  Synchronous. */
int cgks_get_state(void* ctx, double* q, double* g, double* t, long* step);

/* The time step the next cgks_step would take at this CFL number. */
int cgks_compute_dt(void* ctx, double cfl, double* dt);
/* Advance nsteps steps at CFL number cfl; when t_stop > 0 the last step is shortened to end at
 * t_stop and stepping stops there.  *steps_done / *t_now report progress (also on error).
 * ENONPHYSICAL leaves the state as it was at the start of the failing step.  dt and the stop are
 * decided on the device; steps are queued in batches (at most 8; before a t_stop, as many as the
 * last time step says are left, plus one) and the host waits once per batch.  A step queued after
 * the stop launches its kernels, which return at once. */
int cgks_step(void* ctx, int nsteps, double cfl, double t_stop, int* steps_done, double* t_now);
/* Advance nsteps steps of the given dt (no CFL evaluation). */
int cgks_step_fixed(void* ctx, int nsteps, double dt);
/* One stage of a time step of size dt (Sec. 3.4), for drivers that exchange sub-domain halos between
 * the two stages.  CGKS-5th: stage 1 builds Q*, grad Q* and the stage-1 sums from the state; stage 2
 * completes the step (t += dt, step += 1).  GKS-2nd: stage 1 is the whole step; stage 2 is EINVAL.
 * EINVAL also for dt <= 0.  The learned indicator runs in stage 1.  Synchronous. */
int cgks_stage_advance(void* ctx, int stage, double dt);
/* Halo copy between two contexts on one device that hold z-neighbouring sub-domains of one periodic
 * box, as a domain decomposition of the sweep needs between its stages (the paper runs its solver on
 * several GPUs by domain decomposition, Sec. 4).  Each context's grid is nx x ny x (nz_i + 2h): nz_i
 * interior z-planes between h ghost planes below and h above, with l_z = (nz_i + 2h) h_z for the common
 * cell size h_z.  The call copies the top h interior planes of `lower` into the bottom ghost planes of
 * `upper` and the bottom h interior planes of `upper` into the top ghost planes of `lower`, for the
 * state the next stage reads: which = 0 the step's state (Q, grad Q), which = 1 the first stage's
 * output (Q*, grad Q*; CGKS-5th only).  A driver of M sub-domains calls it for each pair (i, i+1 mod M)
 * before each stage and before the time-step reduction; the step's dt is the minimum of the
 * sub-domains' cgks_compute_dt.  With h >= 2 (3 with the learned indicator, whose features reach two
 * cells) every interior cell then gets the result of the undivided box bit for bit; the ghost planes'
 * own results are discarded by the next copy.  EINVAL if the grids, precisions or schemes differ, for
 * h < 1, nz_i < h or which outside {0, 1}; ESTATE before both have a state.  Synchronous. */
int cgks_halo_exchange_z(void* lower, void* upper, int h, int which);
/* One stage operator on the current state with step size dt, copied to host arrays (any may be
 * NULL): L[5N], dL/dt[5N] and, for CGKS5, the Gauss-theorem sums sqn[15N], sqt[15N] of the
 * interface values and of their time derivatives.  The state is unchanged. */
int cgks_stage(void* ctx, double dt, double* L, double* Lt, double* sqn, double* sqt);
/* The same stage operator evaluated on the whole grid on the device, returned only at the cells
 * cells[0..n) (host array of cell indices, 0 <= cell < N): L[5][n], Lt[5][n] and, for CGKS5,
 * sqn[15][n], sqt[15][n] (any output may be NULL).  For grids whose full outputs would not fit host
 * memory (512^3: 43 GB).  The face planes of the workspace stage the indices and results, which
 * bounds n by about N/3 (EINVAL beyond, or for a cell out of range).  The state is unchanged. */
int cgks_stage_sampled(void* ctx, double dt, const long* cells, long n, double* L, double* Lt,
                       double* sqn, double* sqt);

int cgks_diagnostics(void* ctx, double rho0, double u0, cgks_diag* out);
/* The same diagnostics with Ek, epsS, epsD, epsT integrated by 3x3x3 Gauss-Legendre quadrature over
 * each cell's reconstruction of the current state (Sec. 4.1, 4.2: values and velocity derivatives at
 * the quadrature points come from the reconstruction): CGKS-5th its P^4 polynomial with the GENO
 * blend (LINEAR: none; NONLINEAR and LEARNED: every cell), GKS-2nd its (limited) P^1.  mu follows
 * the temperature at each point.  The other fields are those of cgks_diagnostics.  Overwrites the
 * workspace's coefficient (slope) planes; the state is unchanged.  Synchronous. */
int cgks_diagnostics_quad(void* ctx, double rho0, double u0, cgks_diag* out);
/* Flags (1 byte per cell): the cells on which the nonlinear blend ran in the last stage (GENO, or
 * the limiter of GKS2): 0 everywhere for LINEAR, 1 for NONLINEAR, the network's decision for LEARNED. */
int cgks_get_flags(void* ctx, unsigned char* flags);

/* ---- troubled-cell network (the learned form of the indicator) -------------------------------------
 * 64 inputs (59 used) -> 32 -> 32 -> 32 -> 1, ReLU, logit output; params[4225] float:
 * W1[32][64], b1[32], W2[32][32], b2[32], W3[32][32], b3[32], w4[32], b4.  Hidden layers run on BF16
 * matrix cores with FP32 accumulation.  Inputs: for rho and rho E, along each axis, the values of the
 * cells i-2..i+2 minus the centre value and h dQ/dx of the same five cells, over
 * s = max|difference| + max|h dQ| + 1e-12 |Q_i| (inputs 0..53); for each of the 5 conservative
 * variables, log10 of the largest such difference or h dQ over h_max sqrt(S_v), S_v = rho^2,
 * 2 rho rhoE (momenta), (rhoE)^2 of the cell (inputs 54..58, clipped below at -12): the variation
 * against the smoothness floor of the GENO weights, which the label depends on. */
int cgks_indicator_set(void* ctx, const float* params, size_t n, double logit_threshold);
int cgks_indicator_get(void* ctx, float* params, size_t n);
/* Features of every cell of the current state (N x 64 float, host). */
int cgks_features(void* ctx, float* out);
/* Logits of the current network for every cell of the current state (host, N floats). */
int cgks_indicator_logits(void* ctx, float* out);
/* Labels of the current state: 1 iff max over the variables of |1 - chi| > thr under full GENO. */
int cgks_labels(void* ctx, double thr, unsigned char* out);
/* Train the network on device samples x[n][64] (bfloat16 bits) and labels y[n] (float 0/1) with
 * mean binary cross-entropy and Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8), minibatch 1024,
 * samples visited in a seeded permutation each epoch.  Weights start from the current parameters.
 * dev_x / dev_y are caller-owned device pointers.  *final_loss: mean loss of the last epoch. */
int cgks_indicator_train(void* ctx, const void* dev_x, const void* dev_y, long n, int epochs,
                         double lr, uint64_t seed, double* final_loss);
/* Loss and gradient of the current parameters on device samples (host output grad[4225]). */
int cgks_indicator_grad(void* ctx, const void* dev_x, const void* dev_y, long n, double* loss,
                        double* grad);

/* ---- no device allocation ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the time step of cgks_compute_dt for a state the caller holds on
 * the device, with no context and no workspace.  q_dev: Q[5][N] (FP64, the layout of cgks_set_state)
 * for the grid and parameters p; dt_dev: caller-owned device output of 2 doubles, dt_dev[0] = the
 * time step at CFL number cfl (CFL and viscous limits), dt_dev[1] = 1.0 if a cell is non-physical
 * (rho <= 0, p <= 0 or NaN; dt_dev[0] is then not meaningful), else 0.0.  The kernels run on
 * hip_stream (NULL: the null stream) and the call returns without waiting for them.  The reduction's
 * block partials live in a static device array of the library (about 48 KiB per device, kept until
 * the process ends), which bounds the reduction to 2048 blocks; any N that cgks_workspace_bytes
 * accepts is handled (threads then fold several cells).  The call allocates nothing.  Every call on a
 * device shares that array: calls that overlap in time on one device race.  EINVAL for bad parameters
 * (as cgks_workspace_bytes), NULL pointers or cfl <= 0; EDEVICE if the array's device address cannot
 * be found or a launch fails. */
int cgks_compute_dt_noalloc(const cgks_params* p, const double* q_dev, void* hip_stream, double cfl,
                            double* dt_dev);

/* ---- kernel timing ---------------------------------------------------------------------------------
 * When enabled, the sweep's kernel launches of the selected classes are bracketed by HIP events on the
 * context's stream.  cgks_timing_read synchronises the stream and returns, per kernel class, the number
 * of launches and their summed duration in ms since the previous read (then resets).  Classes
 * (CGKS_KC_*): 0 time-step reduction, 1 indicator inference, 2 reconstruction coefficients, 3 face
 * flux, 4 stage update.
 * cgks_timing_enable: classes = 0 stops timing; 1 (or any negative value) times every class; otherwise
 * classes = 2 * (bit mask of the timed classes, bit k = class k), e.g. 2 << CGKS_KC_FLUX for the face
 * flux alone.  Enabling creates the events a few hundred launches need up front, so that timed steps
 * create none.  Returns CGKS_EINVAL for a NULL context, CGKS_EDEVICE if an event cannot be created. */
enum { CGKS_KC_DT = 0, CGKS_KC_INFER = 1, CGKS_KC_COEF = 2, CGKS_KC_FLUX = 3, CGKS_KC_UPDATE = 4,
       CGKS_KC_COUNT = 5 };
int cgks_timing_enable(void* ctx, int classes);
int cgks_timing_read(void* ctx, long* count, double* ms, int nclasses);

/* ---- unit-parity hooks (the hot path's device routines on host-supplied inputs) ----------------------
 * Gas-kinetic flux at n points in the face frame (first axis = normal), evaluated by the device
 * routine of the sweep in the context's precision: wl/wr[n][20] = 5 conservative values then the
 * derivatives along the normal and the two tangents (5 each); out[n][30] = F^n, F_t, Q^l_n, Q^l_t,
 * Q^r_n, Q^r_t.  n <= 3 N (the face planes are the scratch).  Host arrays, synchronous. */
int cgks_debug_point_flux(void* ctx, double dt, long n, const double* wl, const double* wr, double* out);
/* The reconstruction coefficients of the current state as the sweep computes them (CGKS5):
 * out[5][34][N] (double), basis order and normalisation of the generated tables (Sec. 3.2). */
int cgks_debug_coefficients(void* ctx, double* out);

const char* cgks_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
