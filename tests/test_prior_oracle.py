"""Pins of the learned-prior oracle (CPU): back-propagation against central
finite differences, the forward pass against torch's float64 layers, the
bfloat16 rounding against torch's conversion, and the edge features against
properties their definition fixes."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import prior
from paper_1605_02669_amd import inputs


def _problem(rows=40, seed=0):
    g = np.random.default_rng(seed)
    X = g.normal(size=(rows, 4)).astype(np.float32)
    y = g.uniform(size=rows)
    p = prior.init_params(seed)
    for k in ("b1", "b2", "b3"):
        p[k] = g.normal(scale=0.1, size=p[k].shape).astype(np.float32)
    return p, X, y


def test_backprop_matches_finite_differences():
    p, X, y = _problem()
    g = prior.grads(p, X, y)
    h = 1e-6
    rng = np.random.default_rng(1)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            q = {k: v.astype(np.float64) for k, v in p.items()}
            q[name] = q[name].copy().reshape(-1)
            base = q[name][idx]
            q[name][idx] = base + h
            q[name] = q[name].reshape(p[name].shape)
            lp = _loss64(q, X, y)
            q[name] = q[name].reshape(-1)
            q[name][idx] = base - h
            q[name] = q[name].reshape(p[name].shape)
            lm = _loss64(q, X, y)
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (name, idx, fd, an)


def _loss64(q, X, y):
    x = X.astype(np.float64)
    h1 = np.maximum(x @ q["W1"] + q["b1"], 0)
    h2 = np.maximum(h1 @ q["W2"] + q["b2"], 0)
    z = (h2 @ q["W3"] + q["b3"])[:, 0]
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def test_forward_matches_torch_layers():
    import torch
    p, X, y = _problem(rows=64, seed=3)
    z, _ = prior.forward(p, X)
    t = torch.tensor(X, dtype=torch.float64)
    W = {k: torch.tensor(v, dtype=torch.float64) for k, v in p.items()}
    h = torch.relu(torch.nn.functional.linear(t, W["W1"].T, W["b1"]))
    h = torch.relu(torch.nn.functional.linear(h, W["W2"].T, W["b2"]))
    zt = torch.nn.functional.linear(h, W["W3"].T, W["b3"])[:, 0]
    assert np.allclose(z, zt.numpy(), rtol=0, atol=1e-12)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(zt, torch.tensor(y)).item()
    assert abs(prior.loss(p, X, y) - lt) < 1e-12


def test_bf16_rounding_matches_torch():
    import torch
    g = np.random.default_rng(5)
    x = np.concatenate([g.normal(size=5000) * 10.0 ** g.integers(-8, 8, size=5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0]]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(prior.bf16(x), ref)


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_feature_definition_properties(kind):
    n = 120
    xy = inputs.uniform(n, 3) if kind == "uniform" else inputs.clustered(n, 3)
    o = oracle.Oracle(xy, cl=16)
    d, cand = o.dist(), o.cand()
    F = prior.features(xy, cand, d).reshape(n, 16, 4)
    # rank feature, normalised distance within [0, 1] and 1 at the 16th
    assert np.allclose(F[:, :, 3], np.arange(16) / 15.0)
    assert np.all(F[:, :, 2] <= 1.0 + 1e-7) and np.all(F[:, :, 2] >= 0)
    assert np.allclose(F[:, 15, 2], 1.0)
    # (dx, dy) has the length the integer distance rounds, within 1/2 / s_i
    s = np.array([max(d[i, cand[i, 15]], 1) for i in range(n)], dtype=np.float64)
    eu = np.hypot(F[:, :, 0].astype(np.float64), F[:, :, 1].astype(np.float64))
    assert np.all(np.abs(eu - F[:, :, 2]) <= 0.5 / s[:, None] + 1e-5)
    # invariant under translation of the instance
    F2 = prior.features(xy + 1234.5, cand, d).reshape(n, 16, 4)
    assert np.allclose(F, F2, atol=1e-4)


def test_adam_step_matches_torch_optimizer():
    """The oracle's Adam against torch.optim.Adam (an independent
    implementation of the same published update), float64, five steps."""
    import torch
    rng = np.random.default_rng(3)
    p = prior.init_params(4)
    p = {k: v.astype(np.float64) for k, v in p.items()}
    tp = {k: torch.tensor(v.copy(), dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=3e-3, betas=(0.8, 0.99), eps=1e-7)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    for step in range(1, 6):
        g = {k: rng.normal(size=val.shape) * (10.0 ** -step) for k, val in p.items()}
        prior.adam_step(p, g, m, v, step, lr=3e-3, beta1=0.8, beta2=0.99, eps=1e-7)
        for k in tp:
            tp[k].grad = torch.tensor(g[k], dtype=torch.float64)
        opt.step()
        for k in p:
            np.testing.assert_allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)
