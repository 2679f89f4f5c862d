"""Pins of the FP64 reference network used to check the GPU training kernels:
its manual backward pass against central finite differences of its own loss
(with masked one-sided outputs and the side label), and each loss against the
statistic it must estimate (quantile, log of the mean, logit)."""
from __future__ import annotations

import numpy as np

from oracle import mlp


def _setup(seed=0, B=64):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, mlp.NPARAMS)
    X = rng.normal(0, 1, (B, mlp.NIN))
    Y = rng.normal(0, 1, (B, mlp.NOUT))
    u = rng.uniform(0, 1, B)
    # side label and one-sided masks as the records give them
    pos = rng.uniform(0, 1, B) < 0.5
    Y[:, mlp.O_LOGIT] = pos
    Y[~pos, mlp.O_XPOS] = np.nan
    Y[pos, mlp.O_XNEG] = np.nan
    return p, X, Y, u


def test_backward_matches_finite_differences():
    p, X, Y, u = _setup()
    Y[:3, mlp.N_OUT] += 3.0  # some samples beyond the deviance clamp (s4 d > 4)
    s4 = 1.7
    _, g = mlp.loss_and_grad(p, X, Y, u, s4=s4)
    rng = np.random.default_rng(1)
    idx = rng.choice(mlp.NPARAMS, 200, replace=False)
    h = 1e-6
    fd = []
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd.append((mlp.loss_and_grad(pp, X, Y, u, s4=s4)[0] - mlp.loss_and_grad(pm, X, Y, u, s4=s4)[0]) / (2 * h))
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


def test_deviance_minimiser_is_log_mean():
    """The minimiser m of the mean log-deviance E f(y - m) over samples y = ln N
    is ln E[N] (not the mean or a quantile of ln N), for a skewed N."""
    rng = np.random.default_rng(4)
    N = 1.0 + rng.exponential(50.0, 200001)
    y = np.log(N)
    grid = np.linspace(2.0, 6.0, 4001)
    L = [np.mean(mlp.deviance(y - m)[0]) for m in grid]
    m = grid[int(np.argmin(L))]
    assert abs(m - np.log(N.mean())) < 2e-3
    assert abs(m - y.mean()) > 0.3


def test_logistic_minimiser_is_logit():
    """The minimiser of the mean logistic loss over labels b ~ Bernoulli(q) is logit(q)."""
    rng = np.random.default_rng(5)
    b = (rng.uniform(0, 1, 100001) < 0.3).astype(float)
    grid = np.linspace(-3, 3, 6001)
    L = [np.mean(np.logaddexp(0.0, o) - b * o) for o in grid]
    o = grid[int(np.argmin(L))]
    assert abs(o - np.log(b.mean() / (1 - b.mean()))) < 2e-3


def test_raw_targets_masks():
    rec = np.zeros((3, 10))
    rec[:, 3] = [1.5, -2.0, 0.0]
    rec[:, 4:9] = np.arange(15).reshape(3, 5)
    y = mlp.raw_targets(rec)
    assert y[0, mlp.O_XPOS] == 1.5 and np.isnan(y[0, mlp.O_XNEG]) and y[0, mlp.O_LOGIT] == 1
    assert np.isnan(y[1, mlp.O_XPOS]) and y[1, mlp.O_XNEG] == 2.0 and y[1, mlp.O_LOGIT] == 0
    assert y[2, mlp.O_XPOS] == 0.0 and y[2, mlp.O_LOGIT] == 1
    assert np.all(y[:, 1:6] == rec[:, 4:9])


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.14159], dtype=np.float64)
    r = mlp.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert abs(r[3] + 3.14159) < 2 ** -6
