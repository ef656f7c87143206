"""GPU parity of the troubled-cell network (the learned form of the GENO switch) against the oracle.

* features: the scaled stencil data in FP64 on both sides, rounded to float once (2 float ulps); the
  five log10 variation ratios with an FP32 logarithm on the device (2e-6 in log10 units);
* logits: BF16 matrix cores with FP32 accumulation vs the oracle's FP64 arithmetic on bf16-rounded
  inputs, weights and hidden activations: a hidden activation may round to the neighbouring bf16
  value (FP32 vs FP64 accumulation), so the bar is a few bf16 half-ulps propagated: 1e-2 x logit scale;
* gradients of the mean BCE: FP32 matrix cores for the backward pass vs FP64 backpropagation through
  the same bf16-rounded forward: 1e-3 relative on the gradient vector;
* GENO labels: the same chi (FP64) on both sides: identical;
* LEARNED stage: flags identical where no logit is within 1e-3 of the threshold, stage operator at the
  FP64 bar.
"""
import numpy as np
import pytest

import oracle
from paper_2508_19911_amd import inputs

pytestmark = pytest.mark.gpu


def cg():
    from paper_2508_19911_amd import cgks
    return cgks


def rand_params(seed, scale=0.25):
    rng = np.random.default_rng(seed)
    p = (rng.normal(size=oracle.MLP_NPARAM) * scale).astype(np.float32)
    p[2048:2080] = np.abs(p[2048:2080])  # positive first-layer biases: active ReLUs
    return p


def state(n=10, seed=4, amp=0.3):
    case = inputs.tgv_case(n, ma=0.3).with_(nx=n, ny=n - 2, nz=n - 3, lx=2.0, ly=1.6, lz=1.4)
    return case, inputs.seeded_smooth_state(case, seed=seed, amp=amp)


def test_features_match_oracle():
    case, st = state()
    o = oracle.Oracle(oracle.params_from_config(case)); o.set_state(*st)
    s = cg().Solver(case); s.set_state(*st)
    fo = o.features(); fg = s.features()
    assert fg.shape == fo.shape
    # scaled stencil data: FP64 on both sides (a product by 1/s on the device), one float rounding
    assert np.all(np.abs(fg[:, :54] - fo[:, :54]) <= 2.4e-7 * np.maximum(np.abs(fo[:, :54]), 1e-30))
    # log10 of the variation ratio: FP32 logarithm on the device, a few float ulps of the log
    assert np.all(np.abs(fg[:, 54:] - fo[:, 54:]) <= 2e-6)


def test_logits_match_oracle_bf16():
    case, st = state()
    s = cg().Solver(case); s.set_state(*st)
    p = rand_params(1)
    s.indicator_set(p, 0.0)
    zg = s.logits()
    x = s.features()
    zo = oracle.mlp_forward(p, x, bf16=True)
    scale = max(np.abs(zo).max(), 1.0)
    assert np.abs(zg - zo).max() <= 1e-2 * scale, np.abs(zg - zo).max()
    assert np.median(np.abs(zg - zo)) <= 1e-4 * scale


@pytest.mark.parametrize("dims", [(70, 5, 3), (64, 2, 2), (9, 7, 6)])
def test_fp32_inference_ragged_matches_oracle(dims):
    """FP32-bulk inference (FP64 averages, FP32 gradients): its logits against the oracle's BF16
    emulation on the per-cell features of the same state, on grids whose rows are not multiples of the
    256-cell block and on a grid smaller than one block, at the bar of the FP64 form's test."""
    nx, ny, nz = dims
    case = inputs.tgv_case(8, ma=0.3).with_(nx=nx, ny=ny, nz=nz, lx=0.05 * nx, ly=0.3 * ny, lz=0.4 * nz)
    st = inputs.seeded_smooth_state(case, seed=7, amp=0.3)
    s = cg().Solver(case, precision=1); s.set_state(*st)
    p = rand_params(3)
    s.indicator_set(p, 0.0)
    zg = s.logits()
    zo = oracle.mlp_forward(p, s.features(), bf16=True)
    scale = max(np.abs(zo).max(), 1.0)
    assert np.abs(zg - zo).max() <= 1e-2 * scale, np.abs(zg - zo).max()
    assert np.median(np.abs(zg - zo)) <= 1e-4 * scale
    s.close()


def test_gradient_matches_oracle():
    import torch
    cgks = cg()
    rng = np.random.default_rng(3)
    n = 2500  # several minibatches with a ragged tail
    x = rng.normal(size=(n, 64)).astype(np.float32)
    x[:, 54:] = 0
    y = (rng.uniform(size=n) < 0.3).astype(np.float32)
    xb = cgks.to_bf16_bits(x)
    p = rand_params(2)
    case, _ = state()
    s = cgks.Solver(case)
    s.indicator_set(p, 0.0)
    xd = torch.from_numpy(xb.view(np.int16)).cuda()
    yd = torch.from_numpy(y).cuda()
    loss_g, grad_g = s.indicator_grad(xd, yd)
    x_r = (xb.astype(np.uint32) << 16).view(np.float32)  # the bf16 values the device sees
    loss_o, grad_o = oracle.mlp_loss_grad(p, x_r, y, bf16=True)
    assert abs(loss_g - loss_o) <= 1e-5 * abs(loss_o)
    assert np.linalg.norm(grad_g - grad_o) <= 1e-3 * np.linalg.norm(grad_o), np.linalg.norm(grad_g - grad_o) / np.linalg.norm(grad_o)


def test_training_reduces_loss():
    import torch
    cgks = cg()
    rng = np.random.default_rng(5)
    n = 8192
    x = rng.normal(size=(n, 64)).astype(np.float32)
    x[:, 54:] = 0
    y = ((x[:, 0] + 0.5 * x[:, 3] - 0.3 * x[:, 10]) > 0.2).astype(np.float32)
    p = rand_params(6, scale=0.1)
    case, _ = state()
    s = cgks.Solver(case)
    s.indicator_set(p, 0.0)
    xd = torch.from_numpy(cgks.to_bf16_bits(x).view(np.int16)).cuda()
    yd = torch.from_numpy(y).cuda()
    l0, _ = s.indicator_grad(xd, yd)
    lf = s.indicator_train(xd, yd, epochs=20, lr=3e-3, seed=1)
    l1, _ = s.indicator_grad(xd, yd)
    assert l1 < 0.3 * l0 and lf < 0.5 * l0, (l0, lf, l1)
    # the trained weights drive the device inference: accuracy on the training set
    pt = s.indicator_get()
    z = oracle.mlp_forward(pt, (cgks.to_bf16_bits(x).astype(np.uint32) << 16).view(np.float32), bf16=True)
    assert np.mean((z > 0) == (y > 0.5)) > 0.95


@pytest.mark.parametrize("precision", [0, 1])
def test_labels_match_oracle(precision):
    case, st = state(n=16, seed=9, amp=0.05)
    # a density and energy jump over the lower third of the box so some cells are labelled
    q, g = st
    q = q.copy(); q[0, : case.N // 3] *= 1.3; q[4, : case.N // 3] *= 1.3
    o = oracle.Oracle(oracle.params_from_config(case)); o.set_state(q, g)
    s = cg().Solver(case, precision=precision); s.set_state(q, g)
    lo = o.labels(0.01); lg = s.labels(0.01)
    assert 0 < lo.sum() < case.N
    if precision == 0:
        assert np.array_equal(lo, lg)  # the same FP64 chi on both sides
    else:
        # the device decides in FP32: identical wherever the FP64 deviation |1 - chi| is farther from
        # the threshold than float rounding of chi can move it
        dev = o.chi_deviation()
        clear = np.abs(dev - 0.01) > 1e-4
        assert clear.mean() > 0.9
        assert np.array_equal(lo[clear], lg[clear])


def test_learned_stage_matches_oracle():
    case, st = state(n=12, seed=9, amp=0.2)
    case = case.with_(recon=2)
    p = rand_params(11)
    o = oracle.Oracle(oracle.params_from_config(case)); o.set_state(*st)
    s = cg().Solver(case, indicator_logit=0.0); s.set_state(*st)
    x = s.features()
    z = oracle.mlp_forward(p, x, bf16=True)
    thr = float(np.median(z))  # half the cells flagged
    gap = np.abs(z - thr).min()
    if gap < 1e-3 * max(1.0, np.abs(z).max()):
        thr += 0.5 * np.sort(np.abs(z - thr))[1]
    o.indicator_set(p, thr); s.indicator_set(p, thr)
    dt = o.compute_dt(0.5)
    Lo, Lto, _, _ = o.stage(dt)
    Lg, Ltg, _, _ = s.stage(dt)
    fo = o.flags(); fg = s.flags()
    assert 0.2 < fo.mean() < 0.8
    assert np.array_equal(fo, fg)
    rho = st[0][0]; U = st[0][1:4] / rho
    vmax = float((np.abs(U).max(0) + np.sqrt(1.4 * 0.4 * (st[0][4] - 0.5 * rho * (U ** 2).sum(0)) / rho)).max())
    scale = np.abs(st[0]).max() * vmax / min(case.h)
    assert np.abs(Lg - Lo).max() <= 1e-12 * scale


def test_learned_steps_match_oracle():
    """Two LEARNED steps: the flags are evaluated once per step on Q^n and serve both stages, on both
    sides; the threshold sits in the widest gap of the logits near their median so no decision is
    within rounding of it, and the states agree at the FP64 bar."""
    case, st = state(n=12, seed=9, amp=0.2)
    case = case.with_(recon=2)
    p = rand_params(11)
    s = cg().Solver(case, indicator_logit=0.0); s.set_state(*st)
    z = np.sort(oracle.mlp_forward(p, s.features(), bf16=True))
    mid = len(z) // 2
    lo, hi = mid - len(z) // 5, mid + len(z) // 5
    k = lo + int(np.argmax(np.diff(z[lo:hi])))
    thr = 0.5 * (z[k] + z[k + 1])
    o = oracle.Oracle(oracle.params_from_config(case)); o.set_state(*st)
    o.indicator_set(p, thr); s.indicator_set(p, thr)
    dt = 0.5 * o.compute_dt(0.5)
    for _ in range(2):
        o.step_fixed(1, dt); s.step_fixed(1, dt)
        assert np.array_equal(o.flags(), s.flags())
    assert 0.2 < o.flags().mean() < 0.8
    qo, go, _, _ = o.get_state()
    qg, gg, _, _ = s.get_state()
    assert np.abs(qg - qo).max() <= 2e-12 * np.abs(qo).max()
    assert np.abs(gg - go).max() <= 2e-11 * np.abs(go).max()
