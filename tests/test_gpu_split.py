"""Domain decomposition of the sweep in one process: the periodic box split into two z-slabs, each a
context of its own with ghost planes, stepped stage by stage with explicit halo copies between the
stages (cgks_halo_exchange_z) and the minimum of the two sub-domains' time steps.  The interior cells
must equal the undivided run bit for bit: every cell's stage result depends only on the data of its
stencil, which the copies reproduce.  This is the one-device part of the multi-GPU layout (the paper
runs on several GPUs by domain decomposition, Sec. 4); the copies stand where the exchange between
devices would be."""
import numpy as np
import pytest

from paper_2508_19911_amd import inputs

pytestmark = pytest.mark.gpu


def cg():
    from paper_2508_19911_amd import cgks
    return cgks


def sub_case(case, nz_i, h):
    """The sub-domain grid nx x ny x (nz_i + 2h) with the box length that gives the same h_z bit for bit."""
    hz = case.lz / case.nz
    nze = nz_i + 2 * h
    lz = hz * nze
    while lz / nze != hz:
        lz = np.nextafter(lz, np.inf if lz / nze < hz else -np.inf)
    return case.with_(nz=nze, lz=float(lz))


def slab(a, k0, nze, nz):
    """planes (k0 + k) mod nz, k = 0..nze-1, of a [f][nz*ny*nx] array"""
    f = a.shape[0]
    a3 = a.reshape(f, nz, -1)
    return a3[:, [(k0 + k) % nz for k in range(nze)], :].reshape(f, -1)


def interior(a, h, nz_i):
    f = a.shape[0]
    return a.reshape(f, nz_i + 2 * h, -1)[:, h:h + nz_i, :].reshape(f, -1)


@pytest.mark.parametrize("scheme,recon,precision", [(0, 1, 0), (0, 1, 1), (0, 0, 1), (0, 2, 1), (1, 1, 0),
                                                    (1, 0, 1)])
def test_two_slabs_equal_the_undivided_run(scheme, recon, precision):
    cgks = cg()
    case = inputs.tgv_case(12, ma=0.3).with_(nx=12, ny=10, nz=16, lz=2 * np.pi * 16 / 12, scheme=scheme,
                                             recon=recon)
    q, g = inputs.seeded_smooth_state(case, seed=21, amp=0.12)
    nz_i = case.nz // 2
    h = 3 if recon == cgks.RECON_LEARNED else 2
    params, thr = None, 0.0
    if recon == cgks.RECON_LEARNED:
        # random weights, thresholded at the median logit of the state: half the cells flagged
        rng = np.random.default_rng(5)
        params = (0.3 * rng.standard_normal(cgks.MLP_NPARAM)).astype(np.float32)
        probe = cgks.Solver(case, precision=precision)
        probe.indicator_set(params, 0.0)
        probe.set_state(q, g)
        thr = float(np.median(probe.logits()))
        probe.close()
    def solver(c):
        s = cgks.Solver(c, precision=precision, indicator_logit=thr)
        if params is not None:
            s.indicator_set(params, thr)
        return s
    whole = solver(case)
    whole.set_state(q, g)
    sc = sub_case(case, nz_i, h)
    subs = [solver(sc), solver(sc)]
    for i, s in enumerate(subs):
        s.set_state(slab(q, i * nz_i - h, nz_i + 2 * h, case.nz), slab(g, i * nz_i - h, nz_i + 2 * h, case.nz))
    if params is not None:
        flagged = whole.logits() > thr
        assert 0.1 < flagged.mean() < 0.9  # both branches of the learned switch are taken
    for step in range(3):
        for i in range(2):
            subs[i].halo_exchange_z(subs[(i + 1) % 2], h, 0)
        dt = min(s.compute_dt(case.cfl) for s in subs)
        assert dt == whole.compute_dt(case.cfl)
        _, done, _ = whole.step(1, case.cfl)
        assert done == 1
        for s in subs:
            s.stage_advance(1, dt)
        if scheme == cgks.SCHEME_CGKS5:
            for i in range(2):
                subs[i].halo_exchange_z(subs[(i + 1) % 2], h, 1)
            for s in subs:
                s.stage_advance(2, dt)
        qw, gw, tw, nw = whole.get_state()
        for i, s in enumerate(subs):
            qs, gs, ts, ns = s.get_state()
            assert ts == tw and ns == nw
            assert np.array_equal(interior(qs, h, nz_i), slab(qw, i * nz_i, nz_i, case.nz)), (step, i)
            if scheme == cgks.SCHEME_CGKS5:
                assert np.array_equal(interior(gs, h, nz_i), slab(gw, i * nz_i, nz_i, case.nz)), (step, i)
    for s in subs + [whole]:
        s.close()


def test_halo_exchange_rejects_mismatched_contexts():
    cgks = cg()
    case = inputs.tgv_case(8, ma=0.3)
    a = cgks.Solver(case.with_(nz=8))
    b = cgks.Solver(case.with_(nx=6, nz=8))
    c = cgks.Solver(case.with_(nz=8), precision=1)
    d = cgks.Solver(case.with_(nz=8))
    with pytest.raises(cgks.CgksError) as e:
        a.halo_exchange_z(d, 2, 0)
    assert e.value.code == -5  # no state yet
    for s in (a, b, c, d):
        s.set_state(*inputs.uniform_state(s.case))
    for other, hh, which in ((b, 2, 0), (c, 2, 0), (d, 3, 0), (d, 2, 2), (d, 0, 0), (a, 2, 0)):
        with pytest.raises(cgks.CgksError) as e:
            a.halo_exchange_z(other, hh, which)
        assert e.value.code == -1
    a.halo_exchange_z(d, 2, 0)
    for s in (a, b, c, d):
        s.close()
