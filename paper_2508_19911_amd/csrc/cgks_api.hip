// cgks_api.hip -- C ABI of libcgks.so (declared in include/cgks.h): context, workspace layout and
// the per-step launch sequence of the CGKS-5th / GKS-2nd sweep on one MI355X.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cgks.h"
#include "kernels.hpp"
#include "hit_ic.hpp"
#include "mlp.hpp"

using namespace cgks;

namespace {

thread_local std::string g_last_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  // F: the FP64 face planes (F^n, 5 per direction); FT: the T face planes (F_t, and for CGKS-5th the
  // interface values: 25 per direction; 5 for GKS-2nd); Fend: the end of both (a scratch region)
  size_t Q, G, Qs, Gs, Acc, GQn, C, F, FT, Fend, flags, red, scal, mlp, total;
};

bool valid(const cgks_params* p) {
  if (!p) return false;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
  // byte offsets and buffer sizes within one plane are 32-bit: a plane of doubles must stay below 4 GiB
  if ((long long)p->nx * p->ny * p->nz >= (1LL << 29)) return false;
  if (!(p->lx > 0) || !(p->ly > 0) || !(p->lz > 0) || !(p->gamma > 1.0)) return false;
  if (p->scheme != CGKS_SCHEME_CGKS5 && p->scheme != CGKS_SCHEME_GKS2) return false;
  if (p->recon < CGKS_RECON_LINEAR || p->recon > CGKS_RECON_LEARNED) return false;
  if (p->scheme == CGKS_SCHEME_GKS2 && p->recon == CGKS_RECON_LEARNED) return false;
  if (p->precision != CGKS_PREC_FP64 && p->precision != CGKS_PREC_FP32_BULK) return false;
  if (p->mu0 < 0.0) return false;
  return true;
}

Grid make_grid(const cgks_params* p) {
  Grid g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.nz = p->nz;
  g.N = (long long)p->nx * p->ny * p->nz;
  g.h[0] = p->lx / p->nx;
  g.h[1] = p->ly / p->ny;
  g.h[2] = p->lz / p->nz;
  for (int d = 0; d < 3; ++d) g.ih[d] = 1.0 / g.h[d];
  return g;
}

Layout layout(const cgks_params* p) {
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  const size_t ts = p->precision == CGKS_PREC_FP64 ? 8 : 4;
  const bool c5 = p->scheme == CGKS_SCHEME_CGKS5;
  const size_t nblk = (N + BLK - 1) / BLK;
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align256(bytes);
    return r;
  };
  L.Q = take(5 * N * 8);
  L.G = take(15 * N * ts);
  L.Qs = take(5 * N * 8);
  L.Gs = take(15 * N * ts);
  L.Acc = take(5 * N * 8);
  L.GQn = take(15 * N * ts);
  // coefficients: P^4 blocks (34 per variable, in 16-byte chunks of 16-cell blocks) or GKS-2nd
  // slope planes (3 per variable); at least 64 floats per cell so the indicator's features fit
  size_t cbytes = c5 ? (ts == 8 ? (size_t)CoefBlock<double>::elements(N) * 8
                                : (size_t)CoefBlock<float>::elements(N) * 4)
                     : 15 * N * ts;
  if (cbytes < 64 * N * 4) cbytes = 64 * N * 4;
  L.C = take(cbytes);
  L.F = take(15 * N * 8);
  L.FT = take((c5 ? 75 : 15) * N * ts);
  L.Fend = o;
  L.flags = take(N);
  L.red = take(nblk * 16 * 8);
  L.scal = take(64 * 8);
  L.mlp = take(mlp::workspace_bytes());
  L.total = o;
  return L;
}

struct Timing {
  bool on = false;
  unsigned mask = 0;  // bit k: class k is timed
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> recs;
};

struct Ctx {
  Timing tm;
  cgks_params p;
  Grid g;
  Layout L;
  char* ws;
  hipStream_t stream;
  FluxParams fp;
  GenoParams gp;
  double vk_eps2;
  double t = 0.0;
  long step = 0;
  double dt_hint = 0.0;  // the last CFL time step read back (sizes the batches before a t_stop)
  bool have_state = false;
  bool have_mlp = false;
  int nblk;
  std::vector<float> mlp_host;
  template <class T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

int dev_error(const char* what, hipError_t e) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return CGKS_EDEVICE;
}

#define HIPCK(call)                                     \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return dev_error(#call, e_);  \
  } while (0)

#define LAUNCHCK(what)                                  \
  do {                                                  \
    hipError_t e_ = hipGetLastError();                  \
    if (e_ != hipSuccess) return dev_error(what, e_);   \
  } while (0)

// ---------------------------------------------------------------------------- kernel timing
hipEvent_t timing_event(Ctx& c) {
  if (c.tm.pool.empty()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = c.tm.pool.back();
  c.tm.pool.pop_back();
  return e;
}

// brackets the launches issued in its scope with events (when timing is on)
struct TimedScope {
  Ctx& c;
  int cls;
  hipEvent_t a = nullptr;
  // a record that fails drops this measurement (timing is diagnostic; the launches are unaffected)
  TimedScope(Ctx& ctx, int k) : c(ctx), cls(k) {
    if (c.tm.on && ((c.tm.mask >> k) & 1u) && (a = timing_event(c)) &&
        hipEventRecord(a, c.stream) != hipSuccess) {
      c.tm.pool.push_back(a);
      a = nullptr;
    }
  }
  ~TimedScope() {
    if (!a) return;
    hipEvent_t b = timing_event(c);
    if (b && hipEventRecord(b, c.stream) == hipSuccess) {
      c.tm.recs.push_back({cls, a, b});
      return;
    }
    c.tm.pool.push_back(a);
    if (b) c.tm.pool.push_back(b);
  }
};

// ---------------------------------------------------------------------------- stage sequences
template <class T>
int run_flags(Ctx& c, const double* Q, const T* G, const double* ctl = nullptr) {
  if (c.p.recon != CGKS_RECON_LEARNED) return CGKS_OK;
  TimedScope ts(c, CGKS_KC_INFER);
  return mlp::launch_infer<T>(c.g, Q, G, c.at<float>(c.L.mlp), c.at<unsigned char>(c.L.flags),
                              nullptr, c.p.indicator_logit, c.at<char>(c.L.mlp), c.stream, ctl);
}

// ctl: the step control; a stopped step skips the launch (nullptr: always run)
template <class T>
int launch_coef(Ctx& c, const double* Q, const T* G, const double* ctl = nullptr) {
  const dim3 grid(coef_blocks(c.g), 5), blk(BLK);  // y: the conservative variable
  T* C = c.at<T>(c.L.C);
  const unsigned char* fl = c.at<unsigned char>(c.L.flags);
  TimedScope ts(c, CGKS_KC_COEF);
  switch (c.p.recon) {
    case CGKS_RECON_LINEAR: k_coef<T, 0><<<grid, blk, 0, c.stream>>>(c.g, Q, G, fl, C, c.gp, ctl); break;
    case CGKS_RECON_NONLINEAR: k_coef<T, 1><<<grid, blk, 0, c.stream>>>(c.g, Q, G, fl, C, c.gp, ctl); break;
    default: k_coef<T, 2><<<grid, blk, 0, c.stream>>>(c.g, Q, G, fl, C, c.gp, ctl); break;
  }
  LAUNCHCK("k_coef");
  return CGKS_OK;
}

// one CGKS-5th stage on (Q, G); STAGE 0 debug, 1 first, 2 second.  The learned indicator runs once
// per time step, on the first stage's input; the second stage keeps its flags.
template <class T, int STAGE>
int stage5(Ctx& c, const double* Q, const T* G, const double* ctl) {
  int rc = STAGE == 2 ? CGKS_OK : run_flags<T>(c, Q, G, ctl);
  if (rc) return rc;
  rc = launch_coef<T>(c, Q, G, ctl);
  if (rc) return rc;
  const dim3 grid(c.nblk), blk(BLK);
  const dim3 fgrid((unsigned)((c.g.N + FLUX_FACES - 1) / FLUX_FACES)), fblk(FLUX_BLK);
  const T* C = c.at<T>(c.L.C);
  double* Fd = c.at<double>(c.L.F);
  T* Fb = c.at<T>(c.L.FT);
  {
    TimedScope t0(c, CGKS_KC_FLUX);
    k_flux5<T, 0><<<fgrid, fblk, 0, c.stream>>>(c.g, Q, C, Fd, Fb, c.fp, ctl);
  }
  {
    TimedScope t1(c, CGKS_KC_FLUX);
    k_flux5<T, 1><<<fgrid, fblk, 0, c.stream>>>(c.g, Q, C, Fd, Fb, c.fp, ctl);
  }
  {
    TimedScope t2(c, CGKS_KC_FLUX);
    k_flux5<T, 2><<<fgrid, fblk, 0, c.stream>>>(c.g, Q, C, Fd, Fb, c.fp, ctl);
  }
  LAUNCHCK("k_flux5");
  Stage5Out o;
  o.Qs = c.at<double>(c.L.Qs);
  o.Acc = c.at<double>(c.L.Acc);
  o.GQn = c.at<T>(c.L.GQn);
  o.Gs = c.at<T>(c.L.Gs);
  o.Q = c.at<double>(c.L.Q);
  o.G = c.at<T>(c.L.G);
  {
    TimedScope tu(c, CGKS_KC_UPDATE);
    k_update5<T, STAGE><<<grid, blk, 0, c.stream>>>(c.g, Fd, Fb, c.at<double>(c.L.Q), o, ctl);
  }
  LAUNCHCK("k_update5");
  return CGKS_OK;
}

template <class T, int DEBUG>
int stage2(Ctx& c, const double* ctl) {
  const dim3 grid(c.nblk), blk(BLK);
  double* Q = c.at<double>(c.L.Q);
  T* S = c.at<T>(c.L.C);
  double* Fd = c.at<double>(c.L.F);
  T* Fb = c.at<T>(c.L.FT);
  {
    TimedScope ts(c, CGKS_KC_COEF);
    if (c.p.recon == CGKS_RECON_NONLINEAR)
      k_slopes2<T, 1><<<grid, blk, 0, c.stream>>>(c.g, Q, S, c.vk_eps2, ctl);
    else
      k_slopes2<T, 0><<<grid, blk, 0, c.stream>>>(c.g, Q, S, c.vk_eps2, ctl);
  }
  {
    TimedScope t0(c, CGKS_KC_FLUX);
    k_flux2<T, 0><<<grid, blk, 0, c.stream>>>(c.g, Q, S, Fd, Fb, c.fp, ctl);
  }
  {
    TimedScope t1(c, CGKS_KC_FLUX);
    k_flux2<T, 1><<<grid, blk, 0, c.stream>>>(c.g, Q, S, Fd, Fb, c.fp, ctl);
  }
  {
    TimedScope t2(c, CGKS_KC_FLUX);
    k_flux2<T, 2><<<grid, blk, 0, c.stream>>>(c.g, Q, S, Fd, Fb, c.fp, ctl);
  }
  {
    TimedScope tu(c, CGKS_KC_UPDATE);
    k_update2<T, DEBUG><<<grid, blk, 0, c.stream>>>(c.g, Fd, Fb, Q, c.at<double>(c.L.Acc),
                                                     c.at<double>(c.L.Qs), ctl);
  }
  LAUNCHCK("gks2 stage");
  return CGKS_OK;
}

template <class T>
int advance(Ctx& c, const double* ctl) {
  int rc;
  if (c.p.scheme == CGKS_SCHEME_GKS2) return stage2<T, 0>(c, ctl);
  rc = stage5<T, 1>(c, c.at<double>(c.L.Q), c.at<T>(c.L.G), ctl);
  if (rc) return rc;
  return stage5<T, 2>(c, c.at<double>(c.L.Qs), c.at<T>(c.L.Gs), ctl);
}

int advance_any(Ctx& c, const double* ctl) {
  return c.p.precision == CGKS_PREC_FP64 ? advance<double>(c, ctl) : advance<float>(c, ctl);
}

// steps queued between two read-backs of the device step control
constexpr int STEP_BATCH = 8;

// the step-control block on the device (after the 11 reduction results in the scalar area)
double* step_ctl(Ctx& c) { return c.at<double>(c.L.scal) + 32; }

// a host-chosen dt for the stage kernels
const double* set_dt(Ctx& c, double dt) {
  double* ctl = step_ctl(c);
  k_ctl_set_dt<<<1, 64, 0, c.stream>>>(ctl, dt);
  return ctl;
}

// dt limits: out[0] = min h/(|U|+c), out[1] = max nu, out[2] = non-physical flag
int dt_limits(Ctx& c, double out[3]) {
  double* part = c.at<double>(c.L.red);
  double* scal = c.at<double>(c.L.scal);
  {
    TimedScope ts(c, CGKS_KC_DT);
    k_dt<<<c.nblk, BLK, 0, c.stream>>>(c.g, c.at<double>(c.L.Q), c.fp, part);
    k_dt_final<<<1, BLK, 0, c.stream>>>(c.nblk, part, scal);
  }
  LAUNCHCK("k_dt");
  HIPCK(hipMemcpyAsync(out, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

double dt_from_limits(const Ctx& c, const double lim[3], double cfl) {
  double dt = cfl * lim[0];
  if (c.p.mu0 > 0.0) {
    const double hmin = std::fmin(c.g.h[0], std::fmin(c.g.h[1], c.g.h[2]));
    dt = std::fmin(dt, cfl * hmin * hmin / (3.0 * lim[1]));
  }
  return dt;
}

}  // namespace

// ============================================================================ C ABI
// quadrature form of Ek, epsS, epsD on the reconstruction of the current state (the coefficient /
// slope planes of the workspace are overwritten; the state is not)
template <class T>
int diag_quad(Ctx& c, double* r) {
  const double* Q = c.at<double>(c.L.Q);
  T* C = c.at<T>(c.L.C);
  double* part = c.at<double>(c.L.red);
  double* scal = c.at<double>(c.L.scal);
  const dim3 grid(c.nblk), blk(BLK);
  if (c.p.scheme == CGKS_SCHEME_CGKS5) {
    const T* G = c.at<T>(c.L.G);
    const unsigned char* fl = c.at<unsigned char>(c.L.flags);
    const dim3 cgrid(coef_blocks(c.g), 5);
    if (c.p.recon == CGKS_RECON_LINEAR)
      k_coef<T, 0><<<cgrid, blk, 0, c.stream>>>(c.g, Q, G, fl, C, c.gp, nullptr);
    else  // GENO everywhere (also for the learned form)
      k_coef<T, 1><<<cgrid, blk, 0, c.stream>>>(c.g, Q, G, fl, C, c.gp, nullptr);
    k_diag_quad5<T><<<grid, blk, 0, c.stream>>>(c.g, Q, C, c.fp, part);
  } else {
    if (c.p.recon == CGKS_RECON_NONLINEAR)
      k_slopes2<T, 1><<<grid, blk, 0, c.stream>>>(c.g, Q, C, c.vk_eps2, nullptr);
    else
      k_slopes2<T, 0><<<grid, blk, 0, c.stream>>>(c.g, Q, C, c.vk_eps2, nullptr);
    k_diag_quad2<T><<<grid, blk, 0, c.stream>>>(c.g, Q, C, c.fp, part);
  }
  k_diag_final<<<1, BLK, 0, c.stream>>>(c.nblk, part, scal);
  LAUNCHCK("k_diag_quad");
  HIPCK(hipMemcpyAsync(r, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

extern "C" {

int cgks_workspace_bytes(const cgks_params* p, size_t* bytes) {
  if (!valid(p) || !bytes) return CGKS_EINVAL;
  *bytes = layout(p).total;
  return CGKS_OK;
}

int cgks_create(const cgks_params* p, void* ws, size_t bytes, void* stream, void** out) {
  if (!valid(p) || !out) return CGKS_EINVAL;
  const Layout L = layout(p);
  if (!ws || bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return CGKS_EWORKSPACE;
  Ctx* c = new Ctx;
  c->p = *p;
  c->L = L;
  c->ws = static_cast<char*>(ws);
  c->stream = static_cast<hipStream_t>(stream);
  c->g = make_grid(p);
  c->fp = make_flux_params(p->gamma, p->mu0, p->sutherland_tref, p->prandtl, p->tau_eps, p->tau_c);
  c->gp.dH = p->geno_dh;
  c->gp.eps = p->geno_eps;
  {
    const double hm = std::fmax(c->g.h[0], std::fmax(c->g.h[1], c->g.h[2]));
    c->gp.hmax2 = hm * hm;
  }
  const double hh = std::cbrt(c->g.h[0] * c->g.h[1] * c->g.h[2]);
  c->vk_eps2 = std::pow(p->vk_k * hh, 3.0);
  c->nblk = (int)((c->g.N + BLK - 1) / BLK);
  // flags = the cells on which the nonlinear blend (GENO, or the GKS-2nd limiter) runs: none for
  // LINEAR, all for NONLINEAR; LEARNED overwrites them before every stage
  hipError_t e = hipMemsetAsync(c->ws + L.flags, p->recon == CGKS_RECON_LINEAR ? 0 : 1, c->g.N, c->stream);
  if (e != hipSuccess) {
    delete c;
    return dev_error("hipMemsetAsync", e);
  }
  *out = c;
  return CGKS_OK;
}

int cgks_destroy(void* ctx) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return CGKS_OK;
  // the caller's workspace must not be released while work of this context is in flight
  const hipError_t sync = hipStreamSynchronize(c->stream);
  for (auto& r : c->tm.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->tm.pool) (void)hipEventDestroy(e);
  delete c;
  return sync == hipSuccess ? CGKS_OK : dev_error("hipStreamSynchronize", sync);
}

int cgks_timing_enable(void* ctx, int classes) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  c.tm.on = classes != 0;
  c.tm.mask = (classes == 1 || classes < 0) ? ~0u : (unsigned)classes >> 1;
  // events for 256 timed launches, created now rather than between timed launches
  constexpr size_t POOL = 512;
  while (c.tm.on && c.tm.pool.size() + 2 * c.tm.recs.size() < POOL) {
    hipEvent_t e;
    HIPCK(hipEventCreate(&e));
    c.tm.pool.push_back(e);
  }
  return CGKS_OK;
}

int cgks_timing_read(void* ctx, long* count, double* ms, int nclasses) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!count || !ms || nclasses < 1) return CGKS_EINVAL;
  for (int k = 0; k < nclasses; ++k) {
    count[k] = 0;
    ms[k] = 0.0;
  }
  HIPCK(hipStreamSynchronize(c.stream));
  for (auto& r : c.tm.recs) {
    float e = 0.0f;
    HIPCK(hipEventElapsedTime(&e, r.a, r.b));
    if (r.cls < nclasses) {
      count[r.cls] += 1;
      ms[r.cls] += e;
    }
    c.tm.pool.push_back(r.a);
    c.tm.pool.push_back(r.b);
  }
  c.tm.recs.clear();
  return CGKS_OK;
}

int cgks_set_state(void* ctx, const double* q, const double* g, double t, long step) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!q) return CGKS_EINVAL;
  const size_t N = c.g.N;
  HIPCK(hipMemcpyAsync(c.ws + c.L.Q, q, 5 * N * 8, hipMemcpyHostToDevice, c.stream));
  if (c.p.precision == CGKS_PREC_FP64) {
    if (g)
      HIPCK(hipMemcpyAsync(c.ws + c.L.G, g, 15 * N * 8, hipMemcpyHostToDevice, c.stream));
    else
      HIPCK(hipMemsetAsync(c.ws + c.L.G, 0, 15 * N * 8, c.stream));
  } else {
    if (g) {
      // stage through the face planes (>= 15 doubles per cell) and convert
      HIPCK(hipMemcpyAsync(c.ws + c.L.F, g, 15 * N * 8, hipMemcpyHostToDevice, c.stream));
      const long long n = 15LL * N;
      k_convert<float><<<(unsigned)((n + BLK - 1) / BLK), BLK, 0, c.stream>>>(
          n, c.at<double>(c.L.F), c.at<float>(c.L.G));
      LAUNCHCK("k_convert");
    } else {
      HIPCK(hipMemsetAsync(c.ws + c.L.G, 0, 15 * N * 4, c.stream));
    }
  }
  HIPCK(hipStreamSynchronize(c.stream));
  c.t = t;
  c.step = step;
  c.dt_hint = 0.0;
  c.have_state = true;
  return CGKS_OK;
}

int cgks_ic_host(const cgks_params* p, int kind, const double* prm, int nprm, uint64_t seed, double* q,
                 double* g) {
  if (!valid(p) || !q || !g) return CGKS_EINVAL;
  if (kind != CGKS_IC_HIT) return CGKS_EINVAL;
  const int n = p->nx;
  if (p->ny != n || p->nz != n || n < 2 || (n & (n - 1)) != 0) return CGKS_EINVAL;
  if (!(p->lx == p->ly && p->ly == p->lz)) return CGKS_EINVAL;
  if (!prm || nprm < 1 || !(prm[0] > 0.0)) return CGKS_EINVAL;
  const double k0 = nprm > 1 ? prm[1] : 8.0;
  if (!(k0 > 0.0)) return CGKS_EINVAL;
  cgks::hit::field(n, p->lx, p->gamma, prm[0], k0, seed, q, g);
  return CGKS_OK;
}

int cgks_set_ic(void* ctx, int kind, const double* prm, int nprm, uint64_t seed) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (kind == CGKS_IC_HIT) {
    // generated on the host, then set like any host state
    const size_t N = c.g.N;
    std::vector<double> q(5 * N), g(15 * N);
    const int rc = cgks_ic_host(&c.p, kind, prm, nprm, seed, q.data(), g.data());
    if (rc) return rc;
    return cgks_set_state(ctx, q.data(), g.data(), 0.0, 0);
  }
  ICParams ip;
  ip.kind = kind == CGKS_IC_TGV_SUPERSONIC ? 2 : kind;
  ip.gamma = c.p.gamma;
  ip.a0 = ip.a1 = ip.a2 = 0.0;
  if (kind == CGKS_IC_VORTEX2D) {
    ip.a0 = (prm && nprm > 0) ? prm[0] : 5.0;
  } else if (kind == CGKS_IC_TGV) {
    if (!prm || nprm < 3) return CGKS_EINVAL;
    ip.a0 = prm[0];
    ip.a1 = prm[1];
    ip.a2 = prm[2];
  } else if (kind == CGKS_IC_TGV_SUPERSONIC) {
    if (!prm || nprm < 1) return CGKS_EINVAL;
    ip.a0 = prm[0];
  } else {
    return CGKS_EINVAL;
  }
  if (c.p.precision == CGKS_PREC_FP64)
    k_ic<double><<<c.nblk, BLK, 0, c.stream>>>(c.g, ip, c.at<double>(c.L.Q), c.at<double>(c.L.G));
  else
    k_ic<float><<<c.nblk, BLK, 0, c.stream>>>(c.g, ip, c.at<double>(c.L.Q), c.at<float>(c.L.G));
  LAUNCHCK("k_ic");
  HIPCK(hipStreamSynchronize(c.stream));
  c.t = 0.0;
  c.step = 0;
  c.dt_hint = 0.0;
  c.have_state = true;
  return CGKS_OK;
}

int cgks_get_state(void* ctx, double* q, double* g, double* t, long* step) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  const size_t N = c.g.N;
  if (q) HIPCK(hipMemcpyAsync(q, c.ws + c.L.Q, 5 * N * 8, hipMemcpyDeviceToHost, c.stream));
  std::vector<float> tmp;
  if (g) {
    if (c.p.precision == CGKS_PREC_FP64) {
      HIPCK(hipMemcpyAsync(g, c.ws + c.L.G, 15 * N * 8, hipMemcpyDeviceToHost, c.stream));
    } else {
      tmp.resize(15 * N);
      HIPCK(hipMemcpyAsync(tmp.data(), c.ws + c.L.G, 15 * N * 4, hipMemcpyDeviceToHost, c.stream));
    }
  }
  HIPCK(hipStreamSynchronize(c.stream));
  if (g && !tmp.empty())
    for (size_t n = 0; n < 15 * N; ++n) g[n] = tmp[n];
  if (t) *t = c.t;
  if (step) *step = c.step;
  return CGKS_OK;
}

int cgks_compute_dt(void* ctx, double cfl, double* dt) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  if (!(cfl > 0.0) || !dt) return CGKS_EINVAL;
  double lim[3];
  int rc = dt_limits(c, lim);
  if (rc) return rc;
  if (lim[2] != 0.0) return CGKS_ENONPHYSICAL;
  *dt = dt_from_limits(c, lim, cfl);
  return CGKS_OK;
}

int cgks_step(void* ctx, int nsteps, double cfl, double t_stop, int* steps_done, double* t_now) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  int done = 0, rc = CGKS_OK;
  if (!c.have_state) rc = CGKS_ESTATE;
  else if (c.p.recon == CGKS_RECON_LEARNED && !c.have_mlp) rc = CGKS_ESTATE;
  else if (!(cfl > 0.0) || nsteps < 0) rc = CGKS_EINVAL;
  if (rc == CGKS_OK && nsteps > 0 && !(t_stop > 0.0 && c.t >= t_stop)) {
    // Steps are queued in batches: dt, the t_stop shortening and the non-physical stop are decided
    // on the device (k_step_control); the host reads t and the step count back once per batch.
    double* ctl = step_ctl(c);
    double* part = c.at<double>(c.L.red);
    double* lim = c.at<double>(c.L.scal);
    const double hmin = std::fmin(c.g.h[0], std::fmin(c.g.h[1], c.g.h[2]));
    const int viscous = c.p.mu0 > 0.0 ? 1 : 0;
    const double t0 = c.t;
    k_ctl_init<<<1, 64, 0, c.stream>>>(ctl, t0);
    int queued = 0;
    double h[5] = {0.0, 0.0, t0, 0.0, c.dt_hint};
    while (rc == CGKS_OK && queued < nsteps) {
      int batch = std::min(STEP_BATCH, nsteps - queued);
      // before a t_stop, queue the steps the last time step says are left and one more: dt drifts
      // slowly, an underestimate costs one more batch, and steps queued past t_stop do no work
      if (t_stop > 0.0 && h[4] > 0.0) {
        const double left = (t_stop - h[2]) / h[4];
        if (left < batch - 1) batch = std::max(1, (int)std::ceil(left) + 1);
      }
      for (int b = 0; b < batch && rc == CGKS_OK; ++b) {
        {
          TimedScope ts(c, CGKS_KC_DT);
          k_dt<<<c.nblk, BLK, 0, c.stream>>>(c.g, c.at<double>(c.L.Q), c.fp, part);
          k_dt_final<<<1, BLK, 0, c.stream>>>(c.nblk, part, lim);
          k_step_control<<<1, 64, 0, c.stream>>>(lim, ctl, cfl, hmin, viscous, t_stop);
        }
        LAUNCHCK("k_dt");
        rc = advance_any(c, ctl);
        if (rc == CGKS_OK) {
          k_step_advance<<<1, 64, 0, c.stream>>>(ctl);
          LAUNCHCK("k_step_advance");
        }
      }
      queued += batch;
      if (rc != CGKS_OK) break;
      {
        hipError_t e = hipMemcpyAsync(h, ctl, 5 * sizeof(double), hipMemcpyDeviceToHost, c.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) {
          rc = dev_error("step control read-back", e);
          break;
        }
      }
      if (h[1] == 2.0) rc = CGKS_ENONPHYSICAL;
      if (h[1] != 0.0) break;
    }
    done = (int)h[3];
    c.t = h[2];
    c.step += done;
    if (h[4] > 0.0) c.dt_hint = h[4];
  }
  if (rc == CGKS_OK) {
    hipError_t e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) rc = dev_error("hipStreamSynchronize", e);
  }
  if (steps_done) *steps_done = done;
  if (t_now) *t_now = c.t;
  return rc;
}

int cgks_step_fixed(void* ctx, int nsteps, double dt) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  if (c.p.recon == CGKS_RECON_LEARNED && !c.have_mlp) return CGKS_ESTATE;
  if (!(dt > 0.0) || nsteps < 0) return CGKS_EINVAL;
  const double* ctl = set_dt(c, dt);
  for (int s = 0; s < nsteps; ++s) {
    int rc = advance_any(c, ctl);
    if (rc) return rc;
    c.t += dt;
    c.step += 1;
  }
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

int cgks_stage_advance(void* ctx, int stage, double dt) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  if (c.p.recon == CGKS_RECON_LEARNED && !c.have_mlp) return CGKS_ESTATE;
  const bool gks2 = c.p.scheme == CGKS_SCHEME_GKS2;
  if (!(dt > 0.0) || stage < 1 || stage > (gks2 ? 1 : 2)) return CGKS_EINVAL;
  const bool f64 = c.p.precision == CGKS_PREC_FP64;
  const double* ctl = set_dt(c, dt);
  int rc;
  if (gks2)
    rc = f64 ? stage2<double, 0>(c, ctl) : stage2<float, 0>(c, ctl);
  else if (stage == 1)
    rc = f64 ? stage5<double, 1>(c, c.at<double>(c.L.Q), c.at<double>(c.L.G), ctl)
             : stage5<float, 1>(c, c.at<double>(c.L.Q), c.at<float>(c.L.G), ctl);
  else
    rc = f64 ? stage5<double, 2>(c, c.at<double>(c.L.Qs), c.at<double>(c.L.Gs), ctl)
             : stage5<float, 2>(c, c.at<double>(c.L.Qs), c.at<float>(c.L.Gs), ctl);
  if (rc) return rc;
  if (gks2 || stage == 2) {
    c.t += dt;
    c.step += 1;
  }
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

int cgks_halo_exchange_z(void* lower, void* upper, int h, int which) {
  if (!lower || !upper || lower == upper) return CGKS_EINVAL;
  Ctx& a = *static_cast<Ctx*>(lower);
  Ctx& b = *static_cast<Ctx*>(upper);
  if (!a.have_state || !b.have_state) return CGKS_ESTATE;
  if (a.g.nx != b.g.nx || a.g.ny != b.g.ny || a.p.precision != b.p.precision || a.p.scheme != b.p.scheme)
    return CGKS_EINVAL;
  if (h < 1 || which < 0 || which > 1 || a.g.nz < 3 * h || b.g.nz < 3 * h) return CGKS_EINVAL;
  if (which == 1 && a.p.scheme == CGKS_SCHEME_GKS2) return CGKS_EINVAL;
  const size_t plane = (size_t)a.g.nx * a.g.ny;
  const size_t ts = a.p.precision == CGKS_PREC_FP64 ? 8 : 4;
  const size_t oq_a = which ? a.L.Qs : a.L.Q, og_a = which ? a.L.Gs : a.L.G;
  const size_t oq_b = which ? b.L.Qs : b.L.Q, og_b = which ? b.L.Gs : b.L.G;
  const int nza = a.g.nz;
  const int ng = a.p.scheme == CGKS_SCHEME_CGKS5 ? 15 : 0;  // GKS-2nd carries no gradients
  // both streams' work so far is complete before the copies; the copies complete before return
  HIPCK(hipStreamSynchronize(b.stream));
  HIPCK(hipStreamSynchronize(a.stream));
  for (int f = 0; f < 5 + ng; ++f) {
    const bool isq = f < 5;
    const size_t es = isq ? 8 : ts;
    const size_t fa = (isq ? oq_a : og_a) + (size_t)(isq ? f : f - 5) * a.g.N * es;
    const size_t fb = (isq ? oq_b : og_b) + (size_t)(isq ? f : f - 5) * b.g.N * es;
    // lower's top interior planes -> upper's bottom ghosts; upper's bottom interior -> lower's top ghosts
    HIPCK(hipMemcpyAsync(b.ws + fb, a.ws + fa + (size_t)(nza - 2 * h) * plane * es, h * plane * es,
                         hipMemcpyDeviceToDevice, a.stream));
    HIPCK(hipMemcpyAsync(a.ws + fa + (size_t)(nza - h) * plane * es, b.ws + fb + (size_t)h * plane * es,
                         h * plane * es, hipMemcpyDeviceToDevice, a.stream));
  }
  HIPCK(hipStreamSynchronize(a.stream));
  return CGKS_OK;
}

int cgks_stage(void* ctx, double dt, double* L, double* Lt, double* sqn, double* sqt) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  if (c.p.recon == CGKS_RECON_LEARNED && !c.have_mlp) return CGKS_ESTATE;
  if (!(dt > 0.0)) return CGKS_EINVAL;
  const bool f64 = c.p.precision == CGKS_PREC_FP64;
  const double* ctl = set_dt(c, dt);
  int rc;
  if (c.p.scheme == CGKS_SCHEME_GKS2)
    rc = f64 ? stage2<double, 1>(c, ctl) : stage2<float, 1>(c, ctl);
  else if (f64)
    rc = stage5<double, 0>(c, c.at<double>(c.L.Q), c.at<double>(c.L.G), ctl);
  else
    rc = stage5<float, 0>(c, c.at<double>(c.L.Q), c.at<float>(c.L.G), ctl);
  if (rc) return rc;
  const size_t N = c.g.N;
  if (L) HIPCK(hipMemcpyAsync(L, c.ws + c.L.Acc, 5 * N * 8, hipMemcpyDeviceToHost, c.stream));
  if (Lt) HIPCK(hipMemcpyAsync(Lt, c.ws + c.L.Qs, 5 * N * 8, hipMemcpyDeviceToHost, c.stream));
  std::vector<float> tn, tt;
  if (c.p.scheme == CGKS_SCHEME_CGKS5) {
    if (f64) {
      if (sqn) HIPCK(hipMemcpyAsync(sqn, c.ws + c.L.GQn, 15 * N * 8, hipMemcpyDeviceToHost, c.stream));
      if (sqt) HIPCK(hipMemcpyAsync(sqt, c.ws + c.L.Gs, 15 * N * 8, hipMemcpyDeviceToHost, c.stream));
    } else {
      if (sqn) {
        tn.resize(15 * N);
        HIPCK(hipMemcpyAsync(tn.data(), c.ws + c.L.GQn, 15 * N * 4, hipMemcpyDeviceToHost, c.stream));
      }
      if (sqt) {
        tt.resize(15 * N);
        HIPCK(hipMemcpyAsync(tt.data(), c.ws + c.L.Gs, 15 * N * 4, hipMemcpyDeviceToHost, c.stream));
      }
    }
  }
  HIPCK(hipStreamSynchronize(c.stream));
  for (size_t n = 0; n < tn.size(); ++n) sqn[n] = tn[n];
  for (size_t n = 0; n < tt.size(); ++n) sqt[n] = tt[n];
  return CGKS_OK;
}

int cgks_stage_sampled(void* ctx, double dt, const long* cells, long n, double* L, double* Lt,
                       double* sqn, double* sqt) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  if (c.p.recon == CGKS_RECON_LEARNED && !c.have_mlp) return CGKS_ESTATE;
  if (!(dt > 0.0) || !cells || n <= 0) return CGKS_EINVAL;
  const bool c5 = c.p.scheme == CGKS_SCHEME_CGKS5;
  if (!c5 && (sqn || sqt)) return CGKS_EINVAL;
  for (long m = 0; m < n; ++m)
    if (cells[m] < 0 || cells[m] >= c.g.N) return CGKS_EINVAL;
  // staging in the face planes, free once the stage has been assembled: indices, then 40 doubles
  // per sampled cell
  const size_t fbytes = c.L.Fend - c.L.F;
  const size_t ibytes = ((size_t)n * 4 + 255) & ~(size_t)255;
  if (ibytes + 40 * (size_t)n * 8 > fbytes) return CGKS_EINVAL;
  const bool f64 = c.p.precision == CGKS_PREC_FP64;
  const double* ctl = set_dt(c, dt);
  int rc;
  if (!c5)
    rc = f64 ? stage2<double, 1>(c, ctl) : stage2<float, 1>(c, ctl);
  else if (f64)
    rc = stage5<double, 0>(c, c.at<double>(c.L.Q), c.at<double>(c.L.G), ctl);
  else
    rc = stage5<float, 0>(c, c.at<double>(c.L.Q), c.at<float>(c.L.G), ctl);
  if (rc) return rc;
  std::vector<uint32_t> idx(cells, cells + n);
  uint32_t* didx = c.at<uint32_t>(c.L.F);
  double* dout = reinterpret_cast<double*>(c.ws + c.L.F + ibytes);
  HIPCK(hipMemcpyAsync(didx, idx.data(), (size_t)n * 4, hipMemcpyHostToDevice, c.stream));
  const long long N = c.g.N;
  const dim3 grid((unsigned)((n + BLK - 1) / BLK)), blk(BLK);
  k_gather_cells<double><<<grid, blk, 0, c.stream>>>(n, didx, c.at<double>(c.L.Acc), 5, N, dout);
  k_gather_cells<double><<<grid, blk, 0, c.stream>>>(n, didx, c.at<double>(c.L.Qs), 5, N, dout + 5 * n);
  if (c5) {
    if (f64) {
      k_gather_cells<double><<<grid, blk, 0, c.stream>>>(n, didx, c.at<double>(c.L.GQn), 15, N, dout + 10 * n);
      k_gather_cells<double><<<grid, blk, 0, c.stream>>>(n, didx, c.at<double>(c.L.Gs), 15, N, dout + 25 * n);
    } else {
      k_gather_cells<float><<<grid, blk, 0, c.stream>>>(n, didx, c.at<float>(c.L.GQn), 15, N, dout + 10 * n);
      k_gather_cells<float><<<grid, blk, 0, c.stream>>>(n, didx, c.at<float>(c.L.Gs), 15, N, dout + 25 * n);
    }
  }
  LAUNCHCK("k_gather_cells");
  std::vector<double> host((size_t)40 * n);
  HIPCK(hipMemcpyAsync(host.data(), dout, (c5 ? 40 : 10) * (size_t)n * 8, hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  if (L) std::copy(host.begin(), host.begin() + 5 * n, L);
  if (Lt) std::copy(host.begin() + 5 * n, host.begin() + 10 * n, Lt);
  if (sqn) std::copy(host.begin() + 10 * n, host.begin() + 25 * n, sqn);
  if (sqt) std::copy(host.begin() + 25 * n, host.begin() + 40 * n, sqt);
  return CGKS_OK;
}

int cgks_diagnostics(void* ctx, double rho0, double u0, cgks_diag* out) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  if (!out) return CGKS_EINVAL;
  double* part = c.at<double>(c.L.red);
  double* scal = c.at<double>(c.L.scal);
  const double vol = c.g.h[0] * c.g.h[1] * c.g.h[2];
  const unsigned char* fl = c.at<unsigned char>(c.L.flags);
  const bool c5 = c.p.scheme == CGKS_SCHEME_CGKS5;
  if (c.p.precision == CGKS_PREC_FP64) {
    if (c5)
      k_diag<double, 0><<<c.nblk, BLK, 0, c.stream>>>(c.g, c.at<double>(c.L.Q), c.at<double>(c.L.G), fl, c.fp, vol, part);
    else
      k_diag<double, 1><<<c.nblk, BLK, 0, c.stream>>>(c.g, c.at<double>(c.L.Q), c.at<double>(c.L.G), fl, c.fp, vol, part);
  } else {
    if (c5)
      k_diag<float, 0><<<c.nblk, BLK, 0, c.stream>>>(c.g, c.at<double>(c.L.Q), c.at<float>(c.L.G), fl, c.fp, vol, part);
    else
      k_diag<float, 1><<<c.nblk, BLK, 0, c.stream>>>(c.g, c.at<double>(c.L.Q), c.at<float>(c.L.G), fl, c.fp, vol, part);
  }
  k_diag_final<<<1, BLK, 0, c.stream>>>(c.nblk, part, scal);
  LAUNCHCK("k_diag");
  double r[11];
  HIPCK(hipMemcpyAsync(r, scal, 11 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  const double norm = 1.0 / (rho0 * u0 * u0 * (double)c.g.N);
  out->Ek = r[0] * norm;
  out->epsS = r[1] * norm;
  out->epsD = 4.0 / 3.0 * r[2] * norm;
  out->epsT = out->epsS + out->epsD;
  out->mass = r[3];
  out->momx = r[4];
  out->momy = r[5];
  out->momz = r[6];
  out->energy = r[7];
  out->flagged_fraction = r[8] / (double)c.g.N;
  out->rho_min = r[9];
  out->p_min = r[10];
  out->t = c.t;
  out->step = (double)c.step;
  out->reserved[0] = out->reserved[1] = 0.0;
  return CGKS_OK;
}

int cgks_diagnostics_quad(void* ctx, double rho0, double u0, cgks_diag* out) {
  if (!ctx) return CGKS_EINVAL;
  int rc = cgks_diagnostics(ctx, rho0, u0, out);
  if (rc) return rc;
  Ctx& c = *static_cast<Ctx*>(ctx);
  double r[3];
  rc = c.p.precision == CGKS_PREC_FP64 ? diag_quad<double>(c, r) : diag_quad<float>(c, r);
  if (rc) return rc;
  const double norm = 1.0 / (rho0 * u0 * u0 * (double)c.g.N);
  out->Ek = r[0] * norm;
  out->epsS = r[1] * norm;
  out->epsD = 4.0 / 3.0 * r[2] * norm;
  out->epsT = out->epsS + out->epsD;
  return CGKS_OK;
}

int cgks_get_flags(void* ctx, unsigned char* flags) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!flags) return CGKS_EINVAL;
  HIPCK(hipMemcpyAsync(flags, c.ws + c.L.flags, c.g.N, hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

// ---------------------------------------------------------------------------- indicator
int cgks_indicator_set(void* ctx, const float* params, size_t n, double logit_threshold) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!params || n != (size_t)mlp::NPARAM) return CGKS_EINVAL;
  c.mlp_host.assign(params, params + n);
  HIPCK(hipMemcpyAsync(c.ws + c.L.mlp, params, n * sizeof(float), hipMemcpyHostToDevice, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  c.p.indicator_logit = logit_threshold;
  c.have_mlp = true;
  return CGKS_OK;
}

int cgks_indicator_get(void* ctx, float* params, size_t n) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!params || n != (size_t)mlp::NPARAM) return CGKS_EINVAL;
  if (!c.have_mlp) return CGKS_ESTATE;
  HIPCK(hipMemcpyAsync(params, c.ws + c.L.mlp, n * sizeof(float), hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

int cgks_features(void* ctx, float* out) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  if (!out || c.p.scheme != CGKS_SCHEME_CGKS5) return CGKS_EINVAL;
  float* buf = c.at<float>(c.L.C);
  int rc;
  if (c.p.precision == CGKS_PREC_FP64)
    rc = mlp::launch_features<double>(c.g, c.at<double>(c.L.Q), c.at<double>(c.L.G), buf, c.stream);
  else
    rc = mlp::launch_features<float>(c.g, c.at<double>(c.L.Q), c.at<float>(c.L.G), buf, c.stream);
  if (rc) return rc;
  HIPCK(hipMemcpyAsync(out, buf, (size_t)c.g.N * 64 * sizeof(float), hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

int cgks_indicator_logits(void* ctx, float* out) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state || !c.have_mlp) return CGKS_ESTATE;
  if (!out || c.p.scheme != CGKS_SCHEME_CGKS5) return CGKS_EINVAL;
  float* logits = c.at<float>(c.L.C);
  int rc;
  if (c.p.precision == CGKS_PREC_FP64)
    rc = mlp::launch_infer<double>(c.g, c.at<double>(c.L.Q), c.at<double>(c.L.G), c.at<float>(c.L.mlp),
                                   c.at<unsigned char>(c.L.flags), logits, c.p.indicator_logit,
                                   c.at<char>(c.L.mlp), c.stream);
  else
    rc = mlp::launch_infer<float>(c.g, c.at<double>(c.L.Q), c.at<float>(c.L.G), c.at<float>(c.L.mlp),
                                  c.at<unsigned char>(c.L.flags), logits, c.p.indicator_logit,
                                  c.at<char>(c.L.mlp), c.stream);
  if (rc) return rc;
  HIPCK(hipMemcpyAsync(out, logits, (size_t)c.g.N * sizeof(float), hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

int cgks_labels(void* ctx, double thr, unsigned char* out) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  if (!out || c.p.scheme != CGKS_SCHEME_CGKS5) return CGKS_EINVAL;
  unsigned char* buf = c.at<unsigned char>(c.L.C);
  int rc;
  if (c.p.precision == CGKS_PREC_FP64)
    rc = mlp::launch_labels<double>(c.g, c.at<double>(c.L.Q), c.at<double>(c.L.G), c.gp, thr, buf, c.stream);
  else
    rc = mlp::launch_labels<float>(c.g, c.at<double>(c.L.Q), c.at<float>(c.L.G), c.gp, thr, buf, c.stream);
  if (rc) return rc;
  HIPCK(hipMemcpyAsync(out, buf, (size_t)c.g.N, hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

int cgks_indicator_train(void* ctx, const void* dev_x, const void* dev_y, long n, int epochs,
                         double lr, uint64_t seed, double* final_loss) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_mlp) return CGKS_ESTATE;
  if (!dev_x || !dev_y || n < 1 || epochs < 0 || !(lr > 0.0)) return CGKS_EINVAL;
  double loss = 0.0;
  int rc = mlp::train(c.at<char>(c.L.mlp), static_cast<const uint16_t*>(dev_x),
                      static_cast<const float*>(dev_y), n, epochs, lr, seed, &loss, c.stream);
  if (rc) return rc;
  HIPCK(hipMemcpyAsync(c.mlp_host.data(), c.ws + c.L.mlp, mlp::NPARAM * sizeof(float),
                       hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  if (final_loss) *final_loss = loss;
  return CGKS_OK;
}

int cgks_indicator_grad(void* ctx, const void* dev_x, const void* dev_y, long n, double* loss,
                        double* grad) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_mlp) return CGKS_ESTATE;
  if (!dev_x || !dev_y || n < 1 || !grad) return CGKS_EINVAL;
  return mlp::loss_grad(c.at<char>(c.L.mlp), static_cast<const uint16_t*>(dev_x),
                        static_cast<const float*>(dev_y), n, loss, grad, c.stream);
}

int cgks_debug_point_flux(void* ctx, double dt, long n, const double* wl, const double* wr, double* out) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (n < 1 || !wl || !wr || !out || !(dt > 0.0)) return CGKS_EINVAL;
  const size_t cap = c.L.Fend - c.L.F;
  if ((size_t)n * 70 * 8 > cap) return CGKS_EINVAL;
  double* d = c.at<double>(c.L.F);
  HIPCK(hipMemcpyAsync(d, wl, n * 20 * 8, hipMemcpyHostToDevice, c.stream));
  HIPCK(hipMemcpyAsync(d + n * 20, wr, n * 20 * 8, hipMemcpyHostToDevice, c.stream));
  const unsigned nb = (unsigned)((n + 63) / 64);
  if (c.p.precision == CGKS_PREC_FP64)
    k_point_flux<double><<<nb, 64, 0, c.stream>>>(n, d, d + n * 20, d + n * 40, c.fp, dt);
  else
    k_point_flux<float><<<nb, 64, 0, c.stream>>>(n, d, d + n * 20, d + n * 40, c.fp, dt);
  LAUNCHCK("k_point_flux");
  HIPCK(hipMemcpyAsync(out, d + n * 40, n * 30 * 8, hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  return CGKS_OK;
}

}  // extern "C"

namespace {
// the coefficient blocks of the device, reordered to out[5][34][N]
template <class T>
int copy_coefficients(Ctx& c, double* out) {
  using CB = CoefBlock<T>;
  std::vector<T> tmp((size_t)CB::elements(c.g.N));
  HIPCK(hipMemcpyAsync(tmp.data(), c.ws + c.L.C, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, c.stream));
  HIPCK(hipStreamSynchronize(c.stream));
  const long long N = c.g.N;
  for (int v = 0; v < 5; ++v)
    for (long long cell = 0; cell < N; ++cell) {
      const long long b = CB::base(cell, v);
      for (int m = 0; m < tab::NB; ++m)
        out[((size_t)v * tab::NB + m) * N + cell] =
            (double)tmp[b + (m / CB::PER) * CB::CHUNK_STRIDE + m % CB::PER];
    }
  return CGKS_OK;
}
}  // namespace

extern "C" {

int cgks_debug_coefficients(void* ctx, double* out) {
  if (!ctx) return CGKS_EINVAL;
  Ctx& c = *static_cast<Ctx*>(ctx);
  if (!c.have_state) return CGKS_ESTATE;
  if (!out || c.p.scheme != CGKS_SCHEME_CGKS5) return CGKS_EINVAL;
  if (c.p.recon == CGKS_RECON_LEARNED && !c.have_mlp) return CGKS_ESTATE;
  int rc;
  if (c.p.precision == CGKS_PREC_FP64) {
    rc = run_flags<double>(c, c.at<double>(c.L.Q), c.at<double>(c.L.G));
    if (!rc) rc = launch_coef<double>(c, c.at<double>(c.L.Q), c.at<double>(c.L.G));
    if (rc) return rc;
    return copy_coefficients<double>(c, out);
  }
  rc = run_flags<float>(c, c.at<double>(c.L.Q), c.at<float>(c.L.G));
  if (!rc) rc = launch_coef<float>(c, c.at<double>(c.L.Q), c.at<float>(c.L.G));
  if (rc) return rc;
  return copy_coefficients<float>(c, out);
}

}  // extern "C"

// ---------------------------------------------------------------------------- no-allocation time step
// The device scratch of cgks_compute_dt_noalloc: the block partials of the time-step reduction (3 per
// block, at most DT_NOALLOC_BLOCKS blocks) and the reduced limits (3 more).  One copy per device, held
// until the process ends and shared by every call on that device.  Host code never uses the array's
// name as an address: the device address comes from hipGetSymbolAddress, once per device.
constexpr int DT_NOALLOC_BLOCKS = 2048;
static __device__ __align__(256) double scratch[3 * DT_NOALLOC_BLOCKS + 3];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;  // the address of `scratch` on device d (nullptr: not looked up yet)

// the device address of `scratch` on the current device
int scratch_address(double** out) {
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* a = nullptr;
    HIPCK(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
    if (!a) return dev_error("hipGetSymbolAddress", hipErrorInvalidSymbol);
    g_scratch_dev[dev] = static_cast<double*>(a);
  }
  *out = g_scratch_dev[dev];
  return CGKS_OK;
}
}  // namespace

extern "C" {

int cgks_compute_dt_noalloc(const cgks_params* p, const double* q_dev, void* hip_stream, double cfl,
                            double* dt_dev) {
  if (!valid(p) || !q_dev || !dt_dev || !(cfl > 0.0)) return CGKS_EINVAL;
  double* part = nullptr;
  const int rc = scratch_address(&part);
  if (rc) return rc;
  double* lim = part + 3 * DT_NOALLOC_BLOCKS;
  const Grid g = make_grid(p);
  const FluxParams fp = make_flux_params(p->gamma, p->mu0, p->sutherland_tref, p->prandtl, p->tau_eps, p->tau_c);
  const int nb = (int)std::min<long long>((g.N + BLK - 1) / BLK, DT_NOALLOC_BLOCKS);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const double hmin = std::fmin(g.h[0], std::fmin(g.h[1], g.h[2]));
  k_dt<<<nb, BLK, 0, st>>>(g, q_dev, fp, part);
  k_dt_final<<<1, BLK, 0, st>>>(nb, part, lim);
  k_dt_value<<<1, 64, 0, st>>>(lim, cfl, hmin, p->mu0 > 0.0 ? 1 : 0, dt_dev);
  LAUNCHCK("cgks_compute_dt_noalloc");
  return CGKS_OK;
}

const char* cgks_strerror(int code) {
  switch (code) {
    case CGKS_OK: return "ok";
    case CGKS_EINVAL: return "invalid argument";
    case CGKS_EWORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case CGKS_EDEVICE: return g_last_error.empty() ? "HIP error" : g_last_error.c_str();
    case CGKS_ENONPHYSICAL: return "non-physical state (rho <= 0, p <= 0 or NaN)";
    case CGKS_ESTATE: return "call order: no state / no indicator set";
    default: return "unknown error";
  }
}

}  // extern "C"
