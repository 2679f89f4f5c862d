"""Pins of the FP64 reference network used to check the GPU training kernels:
its manual backward pass against central finite differences of its own loss,
and the pinball loss against its definition."""
from __future__ import annotations

import numpy as np

from oracle import mlp


def _setup(seed=0, B=64):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, mlp.NPARAMS)
    X = rng.normal(0, 1, (B, mlp.NIN))
    Y = rng.normal(0, 1, (B, mlp.NOUT))
    u = rng.uniform(0, 1, B)
    return p, X, Y, u


def test_backward_matches_finite_differences():
    p, X, Y, u = _setup()
    _, g = mlp.loss_and_grad(p, X, Y, u)
    rng = np.random.default_rng(1)
    idx = rng.choice(mlp.NPARAMS, 200, replace=False)
    h = 1e-6
    fd = []
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd.append((mlp.loss_and_grad(pp, X, Y, u)[0] - mlp.loss_and_grad(pm, X, Y, u)[0]) / (2 * h))
    fd = np.array(fd)
    assert np.allclose(g[idx], fd, rtol=1e-5, atol=1e-9)


def test_pinball_quantile_property():
    """The minimiser of the mean pinball loss at level u is the u-quantile."""
    rng = np.random.default_rng(2)
    y = rng.exponential(1.0, 20001)
    for u in (0.1, 0.5, 0.9):
        grid = np.linspace(0, 5, 2001)
        L = [np.mean((y - q) * (u - (y < q))) for q in grid]
        assert abs(grid[int(np.argmin(L))] - np.quantile(y, u)) < 0.01


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.14159], dtype=np.float64)
    r = mlp.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert abs(r[3] + 3.14159) < 2 ** -6
