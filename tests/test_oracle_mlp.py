"""Pins of the oracle's troubled-cell network (the learned indicator form, reading R17).

* backpropagated gradient of the mean binary cross-entropy vs central finite differences (FP64);
* bfloat16 round-to-nearest-even emulation on values with known roundings;
* a hand-built network with a closed-form logit;
* features: a smooth field gives bounded, scale-free features; a uniform field gives zeros.
"""
import numpy as np
import pytest

import oracle
from paper_2508_19911_amd import inputs


def rand_params(rng, scale=0.3):
    return (rng.normal(size=oracle.MLP_NPARAM) * scale).astype(np.float32)


def test_gradient_vs_finite_differences():
    rng = np.random.default_rng(0)
    p = rand_params(rng)
    x = rng.normal(size=(12, 64)).astype(np.float32)
    y = (rng.uniform(size=12) > 0.5).astype(np.float32)
    loss, g = oracle.mlp_loss_grad(p, x, y, bf16=False)
    # the parameter vector is float32: use steps representable around each value and compare a sample
    idx = np.concatenate([rng.choice(2048, 20, replace=False), 2048 + np.arange(32),
                          rng.choice(np.arange(2080, 4192), 20, replace=False), np.arange(4192, 4225)])
    for i in idx:
        e = 1e-6
        pp = p.astype(np.float64)
        lp = _loss64(pp, i, +e, x, y)
        lm = _loss64(pp, i, -e, x, y)
        fd = (lp - lm) / (2 * e)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-7, (i, fd, g[i])


def _loss64(p, i, e, x, y):
    """Loss with parameter i moved by e, evaluated by a plain numpy forward pass in float64."""
    q = p.copy(); q[i] += e
    W1 = q[:2048].reshape(32, 64); b1 = q[2048:2080]
    W2 = q[2080:3104].reshape(32, 32); b2 = q[3104:3136]
    W3 = q[3136:4160].reshape(32, 32); b3 = q[4160:4192]
    w4 = q[4192:4224]; b4 = q[4224]
    h = np.maximum(x.astype(np.float64) @ W1.T + b1, 0)
    h = np.maximum(h @ W2.T + b2, 0)
    h = np.maximum(h @ W3.T + b3, 0)
    z = h @ w4 + b4
    return np.mean(np.maximum(z, 0) - y * z + np.log1p(np.exp(-np.abs(z))))


def test_forward_matches_numpy_fp64():
    rng = np.random.default_rng(1)
    p = rand_params(rng)
    x = rng.normal(size=(50, 64)).astype(np.float32)
    z = oracle.mlp_forward(p, x, bf16=False)
    W1 = p[:2048].reshape(32, 64).astype(np.float64)
    h = np.maximum(x @ W1.T + p[2048:2080], 0)
    h = np.maximum(h @ p[2080:3104].reshape(32, 32).T.astype(np.float64) + p[3104:3136], 0)
    h = np.maximum(h @ p[3136:4160].reshape(32, 32).T.astype(np.float64) + p[4160:4192], 0)
    ref = h @ p[4192:4224].astype(np.float64) + p[4224]
    assert np.allclose(z, ref, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_emulation():
    # a network that passes x[0] through: h = relu(x0) on every layer with unit weights
    p = np.zeros(oracle.MLP_NPARAM, dtype=np.float32)
    p[0] = 1.0          # W1[0][0]
    p[2080] = 1.0       # W2[0][0]
    p[3136] = 1.0       # W3[0][0]
    p[4192] = 1.0       # w4[0]
    cases = {
        1.0: 1.0,
        1.0 + 2.0 ** -8: 1.0,                      # tie -> even (mantissa ...0)
        1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,      # tie -> even (mantissa ...10)
        1.0 + 2.0 ** -8 + 2.0 ** -12: 1.0 + 2.0 ** -7,  # above the tie -> up
        3.14159: 3.140625,
    }
    x = np.zeros((len(cases), 64), dtype=np.float32)
    x[:, 0] = list(cases.keys())
    z = oracle.mlp_forward(p, x, bf16=True)
    assert np.allclose(z, list(cases.values()), rtol=0, atol=0), z
    z64 = oracle.mlp_forward(p, x, bf16=False)
    assert np.allclose(z64, x[:, 0].astype(np.float64), rtol=0, atol=0)


def test_features_uniform_and_smooth():
    case = inputs.tgv_case(8, ma=0.3)
    o = oracle.Oracle(oracle.params_from_config(case))
    q, g = inputs.uniform_state(case)
    o.set_state(q, g)
    f = o.features()
    assert f.shape == (case.N, 64) and np.all(f[:, :54] == 0) and np.all(f[:, 59:] == 0)
    assert np.all(f[:, 54:59] == -12.0)  # no variation at all: the clip
    q, g = inputs.tgv_state(case)
    o.set_state(q, g)
    f = o.features()
    assert np.all(np.abs(f[:, :54]) <= 1.0 + 1e-6)
    assert np.all(f[:, 59:] == 0)
    assert np.abs(f[:, :54]).max() > 0.1
    # every feature is unchanged when the whole state is scaled (rho, rho U, rho E all by 3)
    o.set_state(3.0 * q, 3.0 * g)
    f3 = o.features()
    assert np.allclose(f3, f, rtol=0, atol=2e-6)


def test_scale_features_single_cell_bump():
    """A density bump delta in one cell of a uniform gas at rest (pressure uniform, zero gradients):
    only the density scale feature moves, and only for the cells whose 5-cell axis lines reach the
    bump: log10(delta / (h_max rho_i)); every other cell and variable sits at the clip, -12."""
    n = 8
    case = inputs.tgv_case(n, ma=0.3).with_(nx=n, ny=n, nz=n, lx=1.6, ly=1.2, lz=0.8)
    q, g = inputs.uniform_state(case, rho=1.0, u=(0.0, 0.0, 0.0), p=0.7)
    delta = 0.05
    bump = (3 * n + 4) * n + 5  # (i, j, k) = (5, 4, 3)
    q[0, bump] += delta
    o = oracle.Oracle(oracle.params_from_config(case))
    o.set_state(q, g)
    f = o.features()
    hmax = 1.6 / n
    for c in range(case.N):
        i, j, k = c % n, (c // n) % n, c // (n * n)
        d = [abs(i - 5), abs(j - 4), abs(k - 3)]
        on_line = sorted(d)[:2] == [0, 0] and max(d) <= 2
        rho = 1.0 + (delta if c == bump else 0.0)
        want = np.log10(delta / (hmax * rho)) if on_line else -12.0
        assert abs(f[c, 54] - want) <= 1e-6 * abs(want), (c, f[c, 54], want)
        assert np.all(f[c, 55:59] == -12.0)
