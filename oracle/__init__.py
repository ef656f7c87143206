"""FP64 CPU oracle for the CGKS-5th / GKS-2nd stage sweep -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  The oracle shares no code with the HIP path; it follows arXiv 2508.19911
(Sec. 2-4) step by step, in plain double precision (see the C++ sources for the citations).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcgks_oracle.so")
_lib = None

SCHEME_CGKS5, SCHEME_GKS2 = 0, 1
RECON_LINEAR, RECON_NONLINEAR, RECON_LEARNED = 0, 1, 2
MLP_NPARAM = 4225


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("gamma", ctypes.c_double), ("mu0", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("sutherland_tref", ctypes.c_double), ("tau_eps", ctypes.c_double), ("tau_c", ctypes.c_double),
        ("vk_k", ctypes.c_double), ("geno_dh", ctypes.c_double), ("geno_eps", ctypes.c_double),
        ("scheme", ctypes.c_int), ("recon", ctypes.c_int), ("indicator_logit", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with the plain host compiler (make)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(["make", "-s", "-C", _HERE, "-B" if force else "libcgks_oracle.so"], check=True)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        D, I, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.cgkso_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(P)]
        L.cgkso_destroy.argtypes = [P]
        L.cgkso_set_state.argtypes = [P, P, P, D, ctypes.c_long]
        L.cgkso_get_state.argtypes = [P, P, P, dp, ctypes.POINTER(ctypes.c_long)]
        L.cgkso_compute_dt.argtypes = [P, D, dp]
        L.cgkso_stage.argtypes = [P, D, P, P, P, P]
        L.cgkso_step.argtypes = [P, I, D, D, ctypes.POINTER(I), dp]
        L.cgkso_step_fixed.argtypes = [P, I, D]
        L.cgkso_diagnostics.argtypes = [P, D, D, P]
        L.cgkso_diagnostics_quad.argtypes = [P, D, D, P]
        L.cgkso_get_flags.argtypes = [P, P]
        L.cgkso_moments.argtypes = [P, D, I, I, P, P, P, P]
        L.cgkso_micro_slope.argtypes = [P, D, P, P]
        L.cgkso_time_integrals.argtypes = [D, D, P]
        L.cgkso_point_flux.argtypes = [ctypes.POINTER(Params), D, P, P, P, P]
        L.cgkso_recon_operator.argtypes = [P]
        L.cgkso_stencil_offsets.argtypes = [P]
        L.cgkso_recon_cell.argtypes = [ctypes.POINTER(Params), P, P, P, D, I, P, P]
        L.cgkso_face_gauss_points.argtypes = [P]
        L.cgkso_recon_cell_gks2.argtypes = [ctypes.POINTER(Params), P, P, I, P, P]
        L.cgkso_chi_deviation.argtypes = [ctypes.c_void_p, P]
        L.cgkso_stage_cells.argtypes = [ctypes.c_void_p, D, P, ctypes.c_long, P, P, P, P]
        L.cgkso_geno_scale.argtypes = [P, I]
        L.cgkso_geno_scale.restype = D
        L.cgkso_indicator_set.argtypes = [P, P, ctypes.c_size_t, D]
        L.cgkso_features.argtypes = [P, P]
        L.cgkso_labels.argtypes = [P, D, P]
        L.cgkso_mlp_forward.argtypes = [P, P, ctypes.c_long, I, P]
        L.cgkso_mlp_loss_grad.argtypes = [P, P, P, ctypes.c_long, I, P]
        L.cgkso_mlp_loss_grad.restype = D
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def make_params(nx, ny, nz, lx, ly, lz, gamma=1.4, mu0=0.0, prandtl=1.0, sutherland_tref=0.0,
                tau_eps=0.05, tau_c=10.0, vk_k=1.0, geno_dh=0.85, geno_eps=1e-15,
                scheme=SCHEME_CGKS5, recon=RECON_LINEAR, indicator_logit=0.0) -> Params:
    return Params(nx, ny, nz, lx, ly, lz, gamma, mu0, prandtl, sutherland_tref, tau_eps, tau_c,
                  vk_k, geno_dh, geno_eps, scheme, recon, indicator_logit)


def params_from_config(cfg) -> Params:
    """Oracle parameters from a :class:`paper_2508_19911_amd.inputs.Case`-like object."""
    return make_params(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, cfg.lz, cfg.gamma, cfg.mu0, cfg.prandtl,
                       cfg.sutherland_tref, cfg.tau_eps, cfg.tau_c, cfg.vk_k, cfg.geno_dh, cfg.geno_eps,
                       cfg.scheme, cfg.recon, 0.0)


class Oracle:
    """Whole-scheme driver over the C oracle (host arrays, FP64)."""

    def __init__(self, params: Params):
        self.p = params
        self.N = params.nx * params.ny * params.nz
        h = ctypes.c_void_p()
        rc = lib().cgkso_create(ctypes.byref(params), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"cgkso_create failed ({rc})")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.cgkso_destroy(self.h)
            self.h = None

    def set_state(self, q, g=None, t=0.0, step=0):
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(5, -1)
        g = None if g is None else np.ascontiguousarray(g, dtype=np.float64).reshape(15, -1)
        lib().cgkso_set_state(self.h, _ptr(q), _ptr(g), float(t), int(step))

    def get_state(self):
        q = np.empty((5, self.N)); g = np.empty((15, self.N))
        t = ctypes.c_double(); s = ctypes.c_long()
        rc = lib().cgkso_get_state(self.h, _ptr(q), _ptr(g), ctypes.byref(t), ctypes.byref(s))
        if rc != 0:
            raise RuntimeError(rc)
        return q, g, t.value, s.value

    def compute_dt(self, cfl):
        dt = ctypes.c_double()
        rc = lib().cgkso_compute_dt(self.h, float(cfl), ctypes.byref(dt))
        if rc != 0:
            raise RuntimeError(rc)
        return dt.value

    def stage(self, dt):
        L = np.empty((5, self.N)); Lt = np.empty((5, self.N))
        sqn = np.empty((15, self.N)); sqt = np.empty((15, self.N))
        rc = lib().cgkso_stage(self.h, float(dt), _ptr(L), _ptr(Lt), _ptr(sqn), _ptr(sqt))
        if rc != 0:
            raise RuntimeError(rc)
        return L, Lt, sqn, sqt

    def stage_cells(self, dt, cells):
        """The stage operator at the given cells only: L[5][n], Lt[5][n], sqn[15][n], sqt[15][n]."""
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        n = cells.size
        L = np.empty((5, n)); Lt = np.empty((5, n)); sqn = np.empty((15, n)); sqt = np.empty((15, n))
        rc = lib().cgkso_stage_cells(self.h, float(dt), _ptr(cells), n, _ptr(L), _ptr(Lt), _ptr(sqn), _ptr(sqt))
        if rc != 0:
            raise RuntimeError(rc)
        return L, Lt, sqn, sqt

    def step(self, nsteps, cfl, t_stop=0.0):
        done = ctypes.c_int(); tn = ctypes.c_double()
        rc = lib().cgkso_step(self.h, int(nsteps), float(cfl), float(t_stop), ctypes.byref(done),
                              ctypes.byref(tn))
        return rc, done.value, tn.value

    def step_fixed(self, nsteps, dt):
        return lib().cgkso_step_fixed(self.h, int(nsteps), float(dt))

    def diagnostics(self, rho0=1.0, u0=1.0, quad=False):
        """One-point diagnostics, or (quad=True) Ek and the dissipation rates by 3x3x3 Gauss quadrature
        of the reconstruction."""
        out = np.zeros(16)
        (lib().cgkso_diagnostics_quad if quad else lib().cgkso_diagnostics)(self.h, float(rho0), float(u0),
                                                                           _ptr(out))
        keys = ["Ek", "epsS", "epsD", "epsT", "mass", "momx", "momy", "momz", "energy", "rho_min",
                "p_min", "flagged_fraction", "t", "step"]
        return dict(zip(keys, out[:14].tolist()))

    def flags(self):
        f = np.empty(self.N, dtype=np.uint8)
        lib().cgkso_get_flags(self.h, _ptr(f))
        return f

    def indicator_set(self, params, logit_threshold):
        params = np.ascontiguousarray(params, dtype=np.float32)
        rc = lib().cgkso_indicator_set(self.h, _ptr(params), params.size, float(logit_threshold))
        if rc != 0:
            raise ValueError(rc)

    def features(self):
        out = np.empty((self.N, 64), dtype=np.float32)
        rc = lib().cgkso_features(self.h, _ptr(out))
        if rc != 0:
            raise RuntimeError(rc)
        return out

    def chi_deviation(self):
        """max over the 5 variables of |1 - chi| under full GENO, per cell (what labels() thresholds)."""
        out = np.empty(self.N)
        rc = lib().cgkso_chi_deviation(self.h, _ptr(out))
        if rc != 0:
            raise RuntimeError(rc)
        return out

    def labels(self, thr=0.01):
        out = np.empty(self.N, dtype=np.uint8)
        rc = lib().cgkso_labels(self.h, float(thr), _ptr(out))
        if rc != 0:
            raise RuntimeError(rc)
        return out


# ---- building blocks ---------------------------------------------------------------------------
def moments(prim, K, half, nmax=8):
    prim = np.ascontiguousarray(prim, dtype=np.float64)
    mu = np.zeros(12); mv = np.zeros(12); mw = np.zeros(12); mxi = np.zeros(4)
    lib().cgkso_moments(_ptr(prim), float(K), int(half), int(nmax), _ptr(mu), _ptr(mv), _ptr(mw), _ptr(mxi))
    return mu[: nmax + 1], mv[: nmax + 1], mw[: nmax + 1], mxi


def micro_slope(prim, K, r):
    prim = np.ascontiguousarray(prim, dtype=np.float64); r = np.ascontiguousarray(r, dtype=np.float64)
    a = np.zeros(5)
    lib().cgkso_micro_slope(_ptr(prim), float(K), _ptr(r), _ptr(a))
    return a


def time_integrals(T, tau):
    c = np.zeros(6)
    lib().cgkso_time_integrals(float(T), float(tau), _ptr(c))
    return c


def point_flux(params: Params, dt, wl, wr, debug=False):
    wl = np.ascontiguousarray(wl, dtype=np.float64); wr = np.ascontiguousarray(wr, dtype=np.float64)
    out = np.zeros(30); dbg = np.zeros(2 + 5 + 15 + 15 + 5 + 20 + 20)
    lib().cgkso_point_flux(ctypes.byref(params), float(dt), _ptr(wl), _ptr(wr), _ptr(out), _ptr(dbg))
    if not debug:
        return out
    names = {}
    o = 0
    for key, n in [("tau", 1), ("tau0", 1), ("W0", 5), ("dW0", 15), ("abar", 15), ("Abar", 5),
                   ("al", 15), ("Al", 5), ("ar", 15), ("Ar", 5)]:
        names[key] = dbg[o:o + n].copy() if n > 1 else float(dbg[o])
        o += n
    for key in ("dW0", "abar", "al", "ar"):
        names[key] = names[key].reshape(3, 5)
    return out, names


def recon_operator():
    c = np.zeros((34, 75))
    lib().cgkso_recon_operator(_ptr(c))
    return c


def stencil_offsets():
    o = np.zeros((19, 3), dtype=np.int32)
    lib().cgkso_stencil_offsets(_ptr(o))
    return o


def face_gauss_points():
    g = np.zeros((4, 2))
    lib().cgkso_face_gauss_points(_ptr(g))
    return g


def recon_cell(params: Params, q, g, h, mode, scale=1.0):
    """scale: the variable's magnitude squared (GENO smoothness floor eps + h_max^2 scale)."""
    q = np.ascontiguousarray(q, dtype=np.float64); g = np.ascontiguousarray(g, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.zeros((6, 4, 4)); info = np.zeros(4)
    lib().cgkso_recon_cell(ctypes.byref(params), _ptr(q), _ptr(g), _ptr(h), float(scale), int(mode),
                           _ptr(out), _ptr(info))
    return out, info


def recon_cell_gks2(params: Params, q7, h, limited):
    """GKS-2nd P^1 of one variable: q7 = (cell, -x, +x, -y, +y, -z, +z) averages.  Returns
    out[6][4] (face-midpoint value and the three derivatives per face) and the limiter factor."""
    q7 = np.ascontiguousarray(q7, dtype=np.float64); h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.zeros((6, 4)); phi = np.zeros(1)
    lib().cgkso_recon_cell_gks2(ctypes.byref(params), _ptr(q7), _ptr(h), int(limited), _ptr(out), _ptr(phi))
    return out, float(phi[0])


def geno_scale(q5, v):
    q5 = np.ascontiguousarray(q5, dtype=np.float64)
    return lib().cgkso_geno_scale(_ptr(q5), int(v))


def mlp_forward(params, x, bf16=True):
    params = np.ascontiguousarray(params, dtype=np.float32); x = np.ascontiguousarray(x, dtype=np.float32)
    n = x.shape[0]
    z = np.zeros(n)
    lib().cgkso_mlp_forward(_ptr(params), _ptr(x), n, int(bf16), _ptr(z))
    return z


def mlp_loss_grad(params, x, y, bf16=True):
    params = np.ascontiguousarray(params, dtype=np.float32); x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    g = np.zeros(MLP_NPARAM)
    loss = lib().cgkso_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(y), x.shape[0], int(bf16), _ptr(g))
    return loss, g
