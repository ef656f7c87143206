"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded inputs.

FP64 bar: <= 1e-12 relative, element by element against the natural scale of each conservative
field (rho, the momenta and rho E separately; see scales(): the size of the field's state, flux and
their rates, whose 1e-16 is the rounding floor of any FP64 implementation), and field by field in L2
with a floor at 1e-6 of the largest field (so identically-zero fields, rho W in 2-D, compare roundoff
at the largest field's scale).  Grids span several blocks with ragged tails.  The FP32-bulk form is checked
against the same oracle with a bar of O(100) float roundings at the same scales.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2508_19911_amd import inputs

pytestmark = pytest.mark.gpu


def cg():
    from paper_2508_19911_amd import cgks
    return cgks


def scales(case, q):
    """Natural scales of the stage outputs, per conservative field (rho; the three momenta; rho E),
    from the state q: with a = |U|_max + c the signal speed of a cell,
      Q:   rho, rho a (a momentum's interface values and half-space sums carry rho sqrt(p/rho)), rho E;
      L:   the size of the field's flux over h: rho a, rho a^2 (the pressure), (rho E + p) a;
      Lt:  L a / h;  sqn: Q / h;  sqt: Q a / h^2.
    The rounding floor of any FP64 implementation is ~1e-16 of these.  Each is a vector of 5 (one
    per field); a row r of a compared array belongs to field r mod 5."""
    rho = q[0]; U = q[1:4] / rho
    p = (case.gamma - 1) * (q[4] - 0.5 * rho * (U ** 2).sum(0))
    a = np.abs(U).max(0) + np.sqrt(case.gamma * p / rho)
    h = min(case.h)
    sq = np.array([rho.max()] + [(rho * a).max()] * 3 + [np.abs(q[4]).max()])
    sf = np.array([(rho * a).max()] + [(rho * a * a).max()] * 3 + [((np.abs(q[4]) + p) * a).max()])
    vmax = float(a.max())
    return {"L": sf / h, "Lt": sf * vmax / h ** 2, "sqn": sq / h, "sqt": sq * vmax / h ** 2, "Q": sq}


def scaled_err(a, b, scale):
    """max over elements of |a - b| / scale, element by element against the scale of its own
    conservative field (arrays are [rows][cells], row r of field r mod 5; scale: 5 values)"""
    a, b = np.asarray(a), np.asarray(b)
    rows = a.shape[0]
    sc = np.asarray(scale, dtype=float)[np.arange(rows) % 5].reshape((rows,) + (1,) * (a.ndim - 1))
    return float((np.abs(a - b) / sc).max())


def field_err(a, b):
    """max over fields of ||a_f - b_f||_2 / max(||b_f||_2, 1e-6 max_f ||b_f||_2): relative per field,
    with fields far below the largest (identically zero ones, such as rho W in 2-D) compared at the
    largest field's scale"""
    a = np.asarray(a).reshape(a.shape[0], -1); b = np.asarray(b).reshape(b.shape[0], -1)
    nb = np.sqrt((b ** 2).sum(axis=1))
    floor = 1e-6 * max(nb.max(), 1e-300)
    return float((np.sqrt(((a - b) ** 2).sum(axis=1)) / np.maximum(nb, floor)).max())


def pair(case, state, precision=0, learned_params=None, logit_thr=0.0):
    q, g = state
    o = oracle.Oracle(oracle.params_from_config(case))
    s = cg().Solver(case, precision=precision, indicator_logit=logit_thr)
    if learned_params is not None:
        o.indicator_set(learned_params, logit_thr)
        s.indicator_set(learned_params, logit_thr)
    o.set_state(q, g)
    s.set_state(q, g)
    return o, s


CASES = {
    "vortex16": lambda: (inputs.vortex_case(16), None),
    "tgv8": lambda: (inputs.tgv_case(8), None),
    "ragged_viscous": lambda: (inputs.tgv_case(8, ma=0.3).with_(nx=13, ny=7, nz=5, lx=3.1, ly=1.9, lz=1.3), 11),
    "ragged_inviscid": lambda: (inputs.vortex_case(8).with_(nx=11, ny=9, nz=3, lz=2.0), 12),
    # rows a multiple of the flux block (16 cells) long, ny != nz: no ragged flux block
    "rows16_viscous": lambda: (inputs.tgv_case(8, ma=0.3).with_(nx=32, ny=6, nz=10, lx=3.3, ly=1.1, lz=1.7), 14),
}


def make_state(name):
    case, seed = CASES[name]()
    if seed is None:
        return case, inputs.initial_state(case)
    return case, inputs.seeded_smooth_state(case, seed=seed, amp=0.15)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("recon", [0, 1])
def test_stage_fp64(name, recon):
    case, st = make_state(name)
    case = case.with_(recon=recon)
    o, s = pair(case, st)
    dt = o.compute_dt(0.5)
    assert abs(s.compute_dt(0.5) - dt) <= 1e-15 * dt
    ro = o.stage(dt)
    rg = s.stage(dt)
    sc = scales(case, st[0])
    for k, (a, b) in enumerate(zip(rg, ro)):
        key = ["L", "Lt", "sqn", "sqt"][k]
        e = scaled_err(a, b, sc[key])
        assert e <= 1e-12, (name, recon, key, e)


@pytest.mark.parametrize("name,recon,nsteps", [("vortex16", 0, 20), ("vortex16", 1, 6), ("tgv8", 1, 4),
                                               ("ragged_viscous", 1, 3), ("ragged_inviscid", 0, 3)])
def test_steps_fp64(name, recon, nsteps):
    case, st = make_state(name)
    case = case.with_(recon=recon)
    o, s = pair(case, st)
    rc, done, t = o.step(nsteps, 0.5)
    assert rc == 0
    _, done_g, t_g = s.step(nsteps, 0.5)
    assert done_g == done and abs(t_g - t) <= 1e-13 * t
    qo, go, _, _ = o.get_state()
    qg, gg, _, _ = s.get_state()
    sc = scales(case, st[0])
    # rounding differences accumulate at most linearly over the steps of a stable scheme
    bar = 1e-12 * nsteps
    assert scaled_err(qg, qo, sc["Q"]) <= bar
    assert field_err(qg, qo) <= bar
    assert scaled_err(gg, go, sc["sqn"]) <= bar


@pytest.mark.parametrize("recon", [0, 1])
def test_gks2_fp64(recon):
    case, st = make_state("ragged_viscous")
    case = case.with_(scheme=1, recon=recon)
    o, s = pair(case, st)
    dt = o.compute_dt(0.5)
    Lo, Lto, _, _ = o.stage(dt)
    Lg, Ltg, _, _ = s.stage(dt)
    sc = scales(case, st[0])
    assert scaled_err(Lg, Lo, sc["L"]) <= 1e-12 and scaled_err(Ltg, Lto, sc["Lt"]) <= 1e-12
    o.step(5, 0.5); s.step(5, 0.5)
    assert scaled_err(s.get_state()[0], o.get_state()[0], sc["Q"]) <= 1e-12
    assert field_err(s.get_state()[0], o.get_state()[0]) <= 1e-12


@pytest.mark.parametrize("recon", [0, 1])
def test_gks2_fp32_bulk(recon):
    """GKS-2nd in the FP32-bulk form: slopes and flux in float, accumulation in FP64; the bar of the
    FP32 form (O(100) float roundings at the natural scales)."""
    case, st = make_state("ragged_viscous")
    case = case.with_(scheme=1, recon=recon)
    o, s = pair(case, st, precision=1)
    dt = o.compute_dt(0.5)
    Lo, Lto, _, _ = o.stage(dt)
    Lg, Ltg, _, _ = s.stage(dt)
    sc = scales(case, st[0])
    eps32 = 2.0 ** -24
    assert scaled_err(Lg, Lo, sc["L"]) <= 100 * eps32 and scaled_err(Ltg, Lto, sc["Lt"]) <= 100 * eps32
    o.step(5, 0.5); s.step(5, 0.5)
    assert scaled_err(s.get_state()[0], o.get_state()[0], sc["Q"]) <= 10 * eps32


def test_diagnostics_fp64():
    case, st = make_state("tgv8")
    case = case.with_(recon=1)
    o, s = pair(case, st)
    o.step(2, 0.5); s.step(2, 0.5)
    do = o.diagnostics(1.0, 1.0); dg = s.diagnostics(1.0, 1.0)
    for k in ["Ek", "epsS", "epsD", "epsT", "mass", "energy", "rho_min", "p_min"]:
        assert abs(dg[k] - do[k]) <= 1e-12 * max(abs(do[k]), 1e-30), (k, dg[k], do[k])
    for k in ["momx", "momy", "momz"]:
        assert abs(dg[k] - do[k]) <= 1e-12 * do["mass"]


@pytest.mark.parametrize("scheme,recon", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("precision", [0, 1])
def test_diagnostics_quadrature(scheme, recon, precision):
    """cgks_diagnostics_quad against the oracle's quadrature diagnostics on a seeded state of a ragged
    13x7x5 grid (two blocks of the reduction): FP64 to 1e-12 relative; the FP32-bulk form (FP32
    gradients and coefficients) to 1e-6 for E_k and 2e-5 for the dissipation rates."""
    case, st = make_state("ragged_viscous")
    case = case.with_(scheme=scheme, recon=recon)
    o, s = pair(case, st, precision=precision)
    do = o.diagnostics(1.0, 1.0, quad=True)
    dg = s.diagnostics(1.0, 1.0, quad=True)
    d1 = s.diagnostics(1.0, 1.0)
    bars = {"Ek": 1e-12, "epsS": 1e-12, "epsD": 1e-12, "epsT": 1e-12} if precision == 0 else \
        {"Ek": 1e-6, "epsS": 2e-5, "epsD": 2e-5, "epsT": 2e-5}
    for k, bar in bars.items():
        assert abs(dg[k] - do[k]) <= bar * abs(do[k]), (k, dg[k], do[k])
    assert dg["Ek"] != d1["Ek"] and dg["mass"] == d1["mass"]
    # the state is unchanged: a second call gives the same numbers
    assert s.diagnostics(1.0, 1.0, quad=True) == dg


def test_fp32_bulk_against_oracle():
    """FP32-bulk: float rounding of the flux (~2^-24 of the largest flux component) divided by h sets
    the error of one stage operator; after a few steps the state error stays at that level."""
    case, st = make_state("tgv8")
    case = case.with_(recon=1)
    o, s = pair(case, st, precision=1)
    dt = o.compute_dt(0.5)
    Lo, Lto, sno, sto = o.stage(dt)
    Lg, Ltg, sng, stg = s.stage(dt)
    sc = scales(case, st[0])
    eps32 = 2.0 ** -24
    # float rounding of O(100) flux terms: bar 100 eps32 at each quantity's natural scale
    for key, a, b in [("L", Lg, Lo), ("Lt", Ltg, Lto), ("sqn", sng, sno), ("sqt", stg, sto)]:
        e = scaled_err(a, b, sc[key])
        assert e <= 100 * eps32, (key, e)
    o.step(3, 0.5); s.step(3, 0.5)
    e = scaled_err(s.get_state()[0], o.get_state()[0], sc["Q"])
    assert e <= 10 * eps32, e


def test_device_initial_condition_matches_inputs():
    case = inputs.tgv_case(12, ma=0.1)
    q, g = inputs.tgv_state(case)
    s = cg().Solver(case)
    s.set_ic(cg().IC_TGV, [case.ma, case.rho0, case.u0])
    qg, gg, _, _ = s.get_state()
    assert np.abs(qg - q).max() <= 1e-12 * np.abs(q).max()
    assert np.abs(gg - g).max() <= 1e-11 * max(np.abs(g).max(), 1.0)
    cs = inputs.tgv_case(10, ma=2.0, supersonic=True)
    qs, gs = inputs.tgv_state(cs)
    ss = cg().Solver(cs)
    ss.set_ic(cg().IC_TGV_SUPERSONIC, [2.0])
    qg, gg, _, _ = ss.get_state()
    assert np.abs(qg - qs).max() <= 1e-12 * np.abs(qs).max()
    assert np.abs(gg - gs).max() <= 1e-11 * max(np.abs(gs).max(), 1.0)
    ch = inputs.hit_case(16, ma_t=1.0, seed=77)
    qh, gh = inputs.hit_state(ch)
    for prec in (0, 1):
        sh = cg().Solver(ch, precision=prec)
        sh.set_ic(cg().IC_HIT, [ch.ma, 8.0], seed=ch.seed)
        qg, gg, t, step = sh.get_state()
        assert t == 0.0 and step == 0
        assert np.abs(qg - qh).max() <= 1e-12 * np.abs(qh).max()
        # FP32-bulk keeps the gradients in float
        assert np.abs(gg - gh).max() <= (1e-12 if prec == 0 else 1e-6) * np.abs(gh).max()
        sh.close()
    cv = inputs.vortex_case(16)
    qv, gv = inputs.vortex_state(cv)
    sv = cg().Solver(cv)
    sv.set_ic(cg().IC_VORTEX2D, [5.0])
    qg, gg, _, _ = sv.get_state()
    assert np.abs(qg - qv).max() <= 1e-12 * np.abs(qv).max()
    assert np.abs(gg - gv).max() <= 1e-11


def test_free_stream_bitwise_and_determinism():
    case = inputs.tgv_case(9).with_(recon=1, nx=9, ny=6, nz=5, ly=1.1, lz=0.7)
    q, g = inputs.uniform_state(case, rho=1.1, u=(0.2, -0.3, 0.4), p=0.9)
    s = cg().Solver(case)
    s.set_state(q, g)
    s.step(3, 0.5)
    q1, g1, _, _ = s.get_state()
    assert np.array_equal(q1, q) and not np.any(g1)
    case2, st = make_state("ragged_viscous")
    case2 = case2.with_(recon=1)
    outs = []
    for _ in range(2):
        s = cg().Solver(case2)
        s.set_state(*st)
        s.step(3, 0.5)
        outs.append(s.get_state())
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_nonphysical_reported_and_state_kept():
    case = inputs.tgv_case(6, ma=0.3)
    q, g = inputs.uniform_state(case)
    q[4, 7] = -1.0
    s = cg().Solver(case)
    s.set_state(q, g)
    rc, done, _ = s.step(2, 0.5, check=False)
    assert rc == -4 and done == 0
    assert np.array_equal(s.get_state()[0], q)


def test_step_batches_and_t_stop():
    """cgks_step queues its steps in batches with dt and the t_stop shortening decided on the device:
    a t_stop reached inside the second batch gives the oracle's step count, time and state; a further
    call at t_stop takes no step."""
    case, st = make_state("tgv8")
    case = case.with_(recon=1)
    o, s = pair(case, st)
    dt0 = o.compute_dt(0.5)
    t_stop = 10.5 * dt0  # about 11 steps: inside the second batch, the last one shortened
    rc, done, t = o.step(10 ** 6, 0.5, t_stop=t_stop)
    assert rc == 0 and 9 <= done <= 16
    rc_g, done_g, t_g = s.step(10 ** 6, 0.5, t_stop=t_stop)
    assert rc_g == 0 and done_g == done and abs(t_g - t) <= 1e-13 * t and abs(t_g - t_stop) <= 1e-13 * t_stop
    qo = o.get_state()[0]
    qg = s.get_state()[0]
    assert scaled_err(qg, qo, scales(case, st[0])["Q"]) <= 1e-12 * done
    rc_g, done_g, t_g2 = s.step(5, 0.5, t_stop=t_stop)
    assert rc_g == 0 and done_g == 0 and t_g2 == t_g


@pytest.mark.parametrize("nsteps", [1, 8, 9, 17])
def test_batched_steps_equal_single_steps(nsteps):
    """nsteps steps in one call (queued in batches of up to 8) leave the same state, time and step
    count, bit for bit, as nsteps calls of one step; a call of zero steps changes nothing."""
    case, st = make_state("tgv8")
    case = case.with_(recon=1)
    a = cg().Solver(case, precision=1)
    b = cg().Solver(case, precision=1)
    a.set_state(*st)
    b.set_state(*st)
    rc, done, t = a.step(nsteps, 0.5)
    assert rc == 0 and done == nsteps
    for _ in range(nsteps):
        assert b.step(1, 0.5)[1] == 1
    qa, ga, ta, na = a.get_state()
    qb, gb, tb, nb = b.get_state()
    assert ta == tb == t and na == nb == nsteps
    assert np.array_equal(qa, qb) and np.array_equal(ga, gb)
    rc, done, t0 = a.step(0, 0.5)
    assert rc == 0 and done == 0 and t0 == ta and np.array_equal(a.get_state()[0], qa)
    a.close()
    b.close()


@pytest.mark.parametrize("scheme", [0, 1])
def test_repeated_t_stop_calls(scheme):
    """Output-interval loop: successive calls each run to the next t_stop (a few steps each, the
    batches then sized from the last time step).  Step counts, times and the state follow the oracle
    making the same calls."""
    case, st = make_state("tgv8")
    case = case.with_(scheme=scheme, recon=1)
    o, s = pair(case, st)
    dt0 = o.compute_dt(0.5)
    total = 0
    for k in range(1, 6):
        t_stop = 2.7 * k * dt0
        rc, done, t = o.step(10 ** 6, 0.5, t_stop=t_stop)
        rc_g, done_g, t_g = s.step(10 ** 6, 0.5, t_stop=t_stop)
        assert rc == rc_g == 0 and done_g == done and abs(t_g - t) <= 1e-13 * t, (k, done, done_g, t, t_g)
        total += done
    assert total >= 13
    assert scaled_err(s.get_state()[0], o.get_state()[0], scales(case, st[0])["Q"]) <= 1e-12 * total


@pytest.mark.parametrize("recon", [1, 2])
def test_kernel_timing_classes(recon):
    """Timing every class counts each step's launches (one time-step reduction, per stage one
    coefficient launch, three face-flux launches and one update; the indicator once per step); timing
    the face flux alone records only its launches; timed steps give the untimed state bitwise."""
    cgks = cg()
    case = inputs.tgv_case(12, ma=0.3).with_(recon=recon)
    st = inputs.tgv_state(case)
    states = []
    for classes in (None, ["flux"], "off"):
        s = cgks.Solver(case, precision=1)
        if recon == 2:
            s.indicator_set(np.zeros(cgks.MLP_NPARAM, dtype=np.float32), 0.0)
        s.set_state(*st)
        if classes != "off":
            s.timing(True, classes=classes)
        _, done, _ = s.step(3, 0.5)
        assert done == 3
        kt = s.timing_read()
        if classes is None:
            assert kt["dt"][0] == 3 and kt["coef"][0] == 6 and kt["flux"][0] == 18 and kt["update"][0] == 6
            assert kt["infer"][0] == (3 if recon == 2 else 0)
            assert all(ms > 0.0 for c, ms in kt.values() if c)
        elif classes == ["flux"]:
            assert kt["flux"][0] == 18 and kt["flux"][1] > 0.0
            assert all(kt[k] == (0, 0.0) for k in ("dt", "infer", "coef", "update"))
        else:
            assert all(v == (0, 0.0) for v in kt.values())
        states.append(s.get_state()[0])
        s.close()
    assert np.array_equal(states[0], states[2]) and np.array_equal(states[1], states[2])


def test_conservation_fp32_bulk():
    case, st = make_state("ragged_viscous")
    case = case.with_(recon=1)
    s = cg().Solver(case, precision=1)
    s.set_state(*st)
    d0 = s.diagnostics()
    s.step(5, 0.5)
    d1 = s.diagnostics()
    for k in ["mass", "momx", "momy", "momz", "energy"]:
        assert abs(d1[k] - d0[k]) <= 1e-12 * abs(d0["energy"]), (k, d1[k] - d0[k])


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 1), (3, 2, 1), (1, 5, 1)])
@pytest.mark.parametrize("recon", [0, 1])
def test_degenerate_grids(dims, recon):
    """Grids of one to six cells: every stencil neighbour wraps onto the cell itself or its twin, and
    the 16-cell blocks of the coefficients and faces are almost empty. Stage operator and two steps
    against the oracle at the FP64 bar."""
    case = inputs.tgv_case(4, ma=0.3).with_(nx=dims[0], ny=dims[1], nz=dims[2], lx=1.3, ly=1.1, lz=0.7,
                                            recon=recon)
    st = inputs.seeded_smooth_state(case, seed=13, amp=0.1)
    o, s = pair(case, st)
    dt = o.compute_dt(0.3)
    sc = scales(case, st[0])
    for key, a, b in zip(["L", "Lt", "sqn", "sqt"], s.stage(dt), o.stage(dt)):
        assert scaled_err(a, b, sc[key]) <= 1e-12, key
    o.step_fixed(2, dt); s.step_fixed(2, dt)
    assert scaled_err(s.get_state()[0], o.get_state()[0], sc["Q"]) <= 2e-12


def test_sampled_stage_rejects_bad_cell_lists():
    case = inputs.tgv_case(6, ma=0.3)
    s = cg().Solver(case)
    s.set_state(*inputs.seeded_smooth_state(case, seed=2, amp=0.1))
    dt = s.compute_dt(0.3)
    for cells in ([], [case.N], [-1], [0, case.N + 5]):
        with pytest.raises(cg().CgksError) as e:
            s.stage_sampled(dt, np.array(cells, dtype=np.int64))
        assert e.value.code == -1
    with pytest.raises(cg().CgksError):
        s.stage_sampled(-1.0, np.array([0]))
    s.close()


@pytest.fixture(scope="module")
def tgv32_oracle_20_steps():
    """The oracle's 20 steps of the 32^3 Taylor-Green vortex (about 2 minutes of host time), shared."""
    case = inputs.tgv_case(32).with_(recon=1)
    st = inputs.tgv_state(case)
    o = oracle.Oracle(oracle.params_from_config(case))
    o.set_state(*st)
    rc, done, _ = o.step(20, case.cfl)
    assert rc == 0 and done == 20
    return case, st, o.get_state()[0]


@pytest.mark.parametrize("precision", [0, 1])
def test_tgv32_twenty_steps(precision, tgv32_oracle_20_steps):
    """The Taylor-Green vortex on 32^3 (GENO), 20 steps at the 3-D CFL, against the oracle: FP64 at
    1e-12 per field (L2) and at the natural scale; the FP32-bulk form within 1e-5 per field."""
    case, st, qo = tgv32_oracle_20_steps
    s = cg().Solver(case, precision=precision)
    s.set_state(*st)
    _, done_g, _ = s.step(20, case.cfl)
    assert done_g == 20
    qg = s.get_state()[0]
    if precision == 0:
        assert field_err(qg, qo) <= 1e-12
        assert scaled_err(qg, qo, scales(case, st[0])["Q"]) <= 1e-12
    else:
        # density and energy per field; momentum as a vector (its z component is 100x smaller than
        # the others at this time, while its error sits at the same float floor of the pressure)
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        e_rho, e_E, e_m = rel(qg[0], qo[0]), rel(qg[4], qo[4]), rel(qg[1:4], qo[1:4])
        per_field = [rel(qg[v], qo[v]) for v in range(5)]
        print("FP32-bulk after 20 steps, relative L2 per field:", np.array2string(np.array(per_field), precision=2))
        assert max(e_rho, e_E, e_m) <= 1e-5, (e_rho, e_E, e_m)


@pytest.mark.parametrize("precision", [0, 1])
def test_supersonic_tgv_geno_steps(precision):
    """The supersonic Taylor-Green vortex (Ma 2, Re 1600, Pr 0.7, Sutherland; Sec. 4.2) on 16^3 with
    GENO everywhere: the device runs to t = 3, where shocklets have formed and the blend departs from
    P^4 in most cells; from that state 8 more steps against the oracle.  FP64 at the FP64 bars per field;
    the FP32-bulk form within 1e-6 per field (L2)."""
    cgks = cg()
    case = inputs.tgv_case(16, ma=2.0, supersonic=True).with_(recon=1)
    s = cgks.Solver(case, precision=precision)
    s.set_ic(cgks.IC_TGV_SUPERSONIC, [2.0])
    _, done, t = s.step(10 ** 6, case.cfl, t_stop=3.0)
    assert abs(t - 3.0) <= 1e-12 and done > 20
    assert s.labels(0.01).mean() > 0.3  # the nonlinear blend is active
    q, g, _, _ = s.get_state()
    o = oracle.Oracle(oracle.params_from_config(case))
    o.set_state(q, g)
    rc, done_o, t_o = o.step(8, case.cfl)
    assert rc == 0 and done_o == 8
    _, done_g, t_g = s.step(8, case.cfl)
    # the FP32-bulk state differs from the oracle's by float rounding, and so do its time steps
    assert done_g == 8 and abs((t_g - 3.0) - t_o) <= (1e-12 if precision == 0 else 1e-7 * t_o)
    qo, go, _, _ = o.get_state()
    qg, gg, _, _ = s.get_state()
    s.close()
    if precision == 0:
        sc = scales(case, q)
        assert field_err(qg, qo) <= 1e-12 * 8
        assert scaled_err(qg, qo, sc["Q"]) <= 1e-12 * 8
        assert scaled_err(gg, go, sc["sqn"]) <= 1e-12 * 8
    else:
        rel = [float(np.linalg.norm(qg[v] - qo[v]) / np.linalg.norm(qo[v] - qo[v].mean() + 1e-300))
               for v in range(5)]
        assert max(rel) <= 1e-6, rel
