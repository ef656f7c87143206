"""Thin Python binding over libcgks.so (the C ABI of include/cgks.h).

Argument marshalling only: every step of the sweep runs in the library's HIP kernels.  PyTorch
provides the device workspace (a uint8 tensor) and the stream (torch.cuda.current_stream()).
Loading fails loudly when the library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcgks.so")

SCHEME_CGKS5, SCHEME_GKS2 = 0, 1
RECON_LINEAR, RECON_NONLINEAR, RECON_LEARNED = 0, 1, 2
PREC_FP64, PREC_FP32_BULK = 0, 1
IC_VORTEX2D, IC_TGV, IC_HIT, IC_TGV_SUPERSONIC = 0, 1, 2, 3
MLP_NPARAM = 4225
ERRORS = {0: "ok", -1: "EINVAL", -2: "EWORKSPACE", -3: "EDEVICE", -4: "ENONPHYSICAL", -5: "ESTATE"}

# every entry point declared in include/cgks.h
SYMBOLS = [
    "cgks_workspace_bytes", "cgks_create", "cgks_destroy", "cgks_set_state", "cgks_set_ic", "cgks_ic_host",
    "cgks_get_state", "cgks_compute_dt", "cgks_step", "cgks_step_fixed", "cgks_stage", "cgks_stage_sampled",
    "cgks_stage_advance", "cgks_halo_exchange_z", "cgks_compute_dt_noalloc",
    "cgks_diagnostics", "cgks_diagnostics_quad", "cgks_get_flags", "cgks_indicator_set", "cgks_indicator_get",
    "cgks_features", "cgks_indicator_logits", "cgks_labels", "cgks_indicator_train",
    "cgks_indicator_grad", "cgks_timing_enable", "cgks_timing_read", "cgks_debug_point_flux",
    "cgks_debug_coefficients", "cgks_strerror",
]
KERNEL_CLASSES = ["dt", "infer", "coef", "flux", "update"]


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("gamma", ctypes.c_double), ("mu0", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("sutherland_tref", ctypes.c_double), ("tau_eps", ctypes.c_double), ("tau_c", ctypes.c_double),
        ("vk_k", ctypes.c_double), ("geno_dh", ctypes.c_double), ("geno_eps", ctypes.c_double),
        ("scheme", ctypes.c_int), ("recon", ctypes.c_int), ("precision", ctypes.c_int),
        ("indicator_logit", ctypes.c_double),
    ]


class Diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ["Ek", "epsS", "epsD", "epsT", "mass", "momx", "momy", "momz", "energy", "rho_min",
                 "p_min", "flagged_fraction", "t", "step", "r0", "r1"]]


class CgksError(RuntimeError):
    def __init__(self, what, code):
        msg = load().cgks_strerror(code).decode()
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({msg})")
        self.code = code


_lib = None


def load():
    """Load libcgks.so (built by ``python -m paper_2508_19911_amd.build``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_19911_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded, the one that owns the
    # streams and the device memory it is handed (loaded the other way round, a second runtime comes
    # up that does not see the device)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    pp = ctypes.POINTER(Params)
    L.cgks_workspace_bytes.argtypes = [pp, ctypes.POINTER(Z)]
    L.cgks_create.argtypes = [pp, P, Z, P, ctypes.POINTER(P)]
    L.cgks_destroy.argtypes = [P]
    L.cgks_set_state.argtypes = [P, P, P, D, ctypes.c_long]
    L.cgks_set_ic.argtypes = [P, I, P, I, ctypes.c_uint64]
    L.cgks_ic_host.argtypes = [pp, I, P, I, ctypes.c_uint64, P, P]
    L.cgks_stage_advance.argtypes = [P, I, D]
    L.cgks_compute_dt_noalloc.argtypes = [pp, P, P, D, P]
    L.cgks_halo_exchange_z.argtypes = [P, P, I, I]
    L.cgks_get_state.argtypes = [P, P, P, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_long)]
    L.cgks_compute_dt.argtypes = [P, D, ctypes.POINTER(D)]
    L.cgks_step.argtypes = [P, I, D, D, ctypes.POINTER(I), ctypes.POINTER(D)]
    L.cgks_step_fixed.argtypes = [P, I, D]
    L.cgks_stage.argtypes = [P, D, P, P, P, P]
    L.cgks_stage_sampled.argtypes = [P, D, P, ctypes.c_long, P, P, P, P]
    L.cgks_diagnostics.argtypes = [P, D, D, ctypes.POINTER(Diag)]
    L.cgks_diagnostics_quad.argtypes = [P, D, D, ctypes.POINTER(Diag)]
    L.cgks_get_flags.argtypes = [P, P]
    L.cgks_indicator_set.argtypes = [P, P, Z, D]
    L.cgks_indicator_get.argtypes = [P, P, Z]
    L.cgks_features.argtypes = [P, P]
    L.cgks_indicator_logits.argtypes = [P, P]
    L.cgks_labels.argtypes = [P, D, P]
    L.cgks_indicator_train.argtypes = [P, P, P, ctypes.c_long, I, D, ctypes.c_uint64, ctypes.POINTER(D)]
    L.cgks_indicator_grad.argtypes = [P, P, P, ctypes.c_long, ctypes.POINTER(D), P]
    L.cgks_timing_enable.argtypes = [P, I]
    L.cgks_timing_read.argtypes = [P, P, P, I]
    L.cgks_debug_point_flux.argtypes = [P, D, ctypes.c_long, P, P, P]
    L.cgks_debug_coefficients.argtypes = [P, P]
    L.cgks_strerror.argtypes = [I]
    L.cgks_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(what, rc):
    if rc != 0:
        raise CgksError(what, rc)


def ic_host(case, kind, prm=(), seed=0):
    """cgks_ic_host: a host-generated initial condition (q[5][N], g[15][N]) for the grid of case."""
    p = params_from_case(case)
    a = np.ascontiguousarray(prm, dtype=np.float64)
    q = np.empty((5, case.N)); g = np.empty((15, case.N))
    _check("cgks_ic_host", load().cgks_ic_host(ctypes.byref(p), int(kind), _p(a) if a.size else None, a.size,
                                               int(seed), _p(q), _p(g)))
    return q, g


def params_from_case(case, precision=PREC_FP64, indicator_logit=0.0) -> Params:
    return Params(case.nx, case.ny, case.nz, case.lx, case.ly, case.lz, case.gamma, case.mu0,
                  case.prandtl, case.sutherland_tref, case.tau_eps, case.tau_c, case.vk_k, case.geno_dh,
                  case.geno_eps, case.scheme, case.recon, precision, indicator_logit)


class Solver:
    """One context of the library on one GPU, with a torch-owned workspace and stream."""

    def __init__(self, case, precision=PREC_FP64, device="cuda:0", indicator_logit=0.0):
        import torch

        L = load()
        self.case = case
        self.N = case.N
        self.p = params_from_case(case, precision, indicator_logit)
        nbytes = ctypes.c_size_t()
        _check("cgks_workspace_bytes", L.cgks_workspace_bytes(ctypes.byref(self.p), ctypes.byref(nbytes)))
        self.device = torch.device(device)
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check("cgks_create", L.cgks_create(ctypes.byref(self.p), ctypes.c_void_p(aligned), nbytes.value,
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None:
            load().cgks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state ---------------------------------------------------------------------------------------
    def set_state(self, q, g=None, t=0.0, step=0):
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(5, -1)
        g = None if g is None else np.ascontiguousarray(g, dtype=np.float64).reshape(15, -1)
        _check("cgks_set_state", load().cgks_set_state(self.h, _p(q), _p(g), float(t), int(step)))

    def set_ic(self, kind, prm=(), seed=0):
        a = np.ascontiguousarray(prm, dtype=np.float64)
        _check("cgks_set_ic", load().cgks_set_ic(self.h, int(kind), _p(a) if a.size else None, a.size,
                                                 int(seed)))

    def get_state(self):
        q = np.empty((5, self.N)); g = np.empty((15, self.N))
        t = ctypes.c_double(); s = ctypes.c_long()
        _check("cgks_get_state", load().cgks_get_state(self.h, _p(q), _p(g), ctypes.byref(t), ctypes.byref(s)))
        return q, g, t.value, s.value

    # ---- stepping ----------------------------------------------------------------------------------
    def compute_dt(self, cfl):
        dt = ctypes.c_double()
        _check("cgks_compute_dt", load().cgks_compute_dt(self.h, float(cfl), ctypes.byref(dt)))
        return dt.value

    def step(self, nsteps, cfl, t_stop=0.0, check=True):
        done = ctypes.c_int(); tn = ctypes.c_double()
        rc = load().cgks_step(self.h, int(nsteps), float(cfl), float(t_stop), ctypes.byref(done), ctypes.byref(tn))
        if check:
            _check("cgks_step", rc)
        return rc, done.value, tn.value

    def stage_advance(self, stage, dt):
        _check("cgks_stage_advance", load().cgks_stage_advance(self.h, int(stage), float(dt)))

    def halo_exchange_z(self, upper, h, which):
        """cgks_halo_exchange_z(self = the lower sub-domain, upper, h, which)"""
        _check("cgks_halo_exchange_z", load().cgks_halo_exchange_z(self.h, upper.h, int(h), int(which)))

    def step_fixed(self, nsteps, dt):
        _check("cgks_step_fixed", load().cgks_step_fixed(self.h, int(nsteps), float(dt)))

    def stage(self, dt):
        L = np.empty((5, self.N)); Lt = np.empty((5, self.N))
        sqn = np.empty((15, self.N)); sqt = np.empty((15, self.N))
        _check("cgks_stage", load().cgks_stage(self.h, float(dt), _p(L), _p(Lt), _p(sqn), _p(sqt)))
        return L, Lt, sqn, sqt

    def stage_sampled(self, dt, cells):
        """The stage operator computed on the device for the whole grid, returned at the given cells:
        L[5][n], Lt[5][n], sqn[15][n], sqt[15][n] (the last two None for GKS-2nd)."""
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        n = cells.size
        L = np.empty((5, n)); Lt = np.empty((5, n))
        c5 = self.case.scheme == SCHEME_CGKS5
        sqn = np.empty((15, n)) if c5 else None
        sqt = np.empty((15, n)) if c5 else None
        _check("cgks_stage_sampled", load().cgks_stage_sampled(
            self.h, float(dt), _p(cells), n, _p(L), _p(Lt), _p(sqn) if c5 else None, _p(sqt) if c5 else None))
        return L, Lt, sqn, sqt

    def diagnostics(self, rho0=1.0, u0=1.0, quad=False):
        """One-point diagnostics of the cell averages, or (quad=True) Ek and the dissipation rates by
        3x3x3 Gauss quadrature of the reconstruction."""
        d = Diag()
        name = "cgks_diagnostics_quad" if quad else "cgks_diagnostics"
        _check(name, getattr(load(), name)(self.h, float(rho0), float(u0), ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in Diag._fields_[:14]}

    def flags(self):
        f = np.empty(self.N, dtype=np.uint8)
        _check("cgks_get_flags", load().cgks_get_flags(self.h, _p(f)))
        return f

    # ---- indicator ---------------------------------------------------------------------------------
    def indicator_set(self, params, logit_threshold):
        params = np.ascontiguousarray(params, dtype=np.float32)
        _check("cgks_indicator_set", load().cgks_indicator_set(self.h, _p(params), params.size, float(logit_threshold)))

    def indicator_get(self):
        out = np.empty(MLP_NPARAM, dtype=np.float32)
        _check("cgks_indicator_get", load().cgks_indicator_get(self.h, _p(out), out.size))
        return out

    def features(self):
        out = np.empty((self.N, 64), dtype=np.float32)
        _check("cgks_features", load().cgks_features(self.h, _p(out)))
        return out

    def logits(self):
        out = np.empty(self.N, dtype=np.float32)
        _check("cgks_indicator_logits", load().cgks_indicator_logits(self.h, _p(out)))
        return out

    def labels(self, thr=0.01):
        out = np.empty(self.N, dtype=np.uint8)
        _check("cgks_labels", load().cgks_labels(self.h, float(thr), _p(out)))
        return out

    def indicator_train(self, x_dev, y_dev, epochs, lr, seed=0):
        """x_dev: torch uint16/int16 tensor [n, 64] of bfloat16 bits; y_dev: float32 [n] on the device."""
        n = int(y_dev.numel())
        loss = ctypes.c_double()
        _check("cgks_indicator_train", load().cgks_indicator_train(
            self.h, ctypes.c_void_p(x_dev.data_ptr()), ctypes.c_void_p(y_dev.data_ptr()), n, int(epochs),
            float(lr), int(seed), ctypes.byref(loss)))
        return loss.value

    def timing(self, on=True, classes=None):
        """Time the sweep's launches with HIP events: every class, or only `classes` (names from
        KERNEL_CLASSES); on=False stops."""
        code = 0 if not on else (1 if classes is None else
                                 2 * sum(1 << KERNEL_CLASSES.index(k) for k in set(classes)))
        _check("cgks_timing_enable", load().cgks_timing_enable(self.h, code))

    def timing_read(self):
        """{class: (launches, summed ms)} since the previous read."""
        n = len(KERNEL_CLASSES)
        cnt = np.zeros(n, dtype=np.int64); ms = np.zeros(n)
        _check("cgks_timing_read", load().cgks_timing_read(self.h, _p(cnt), _p(ms), n))
        return {k: (int(cnt[i]), float(ms[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def point_flux(self, dt, wl, wr):
        wl = np.ascontiguousarray(wl, dtype=np.float64).reshape(-1, 20)
        wr = np.ascontiguousarray(wr, dtype=np.float64).reshape(-1, 20)
        out = np.empty((wl.shape[0], 30))
        _check("cgks_debug_point_flux", load().cgks_debug_point_flux(self.h, float(dt), wl.shape[0], _p(wl), _p(wr), _p(out)))
        return out

    def coefficients(self):
        out = np.empty((5, 34, self.N))
        _check("cgks_debug_coefficients", load().cgks_debug_coefficients(self.h, _p(out)))
        return out

    def indicator_grad(self, x_dev, y_dev):
        n = int(y_dev.numel())
        loss = ctypes.c_double()
        g = np.zeros(MLP_NPARAM)
        _check("cgks_indicator_grad", load().cgks_indicator_grad(
            self.h, ctypes.c_void_p(x_dev.data_ptr()), ctypes.c_void_p(y_dev.data_ptr()), n, ctypes.byref(loss), _p(g)))
        return loss.value, g


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (round to nearest even), as uint16."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    special = (u & 0x7F800000) == 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    r = np.where(special, (u >> 16) & 0xFFFF, r)
    return r.astype(np.uint16)
