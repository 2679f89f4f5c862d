"""Pins of the FP64 reference network used to check the GPU training kernels:
its manual backward pass against central finite differences of its own loss
(marginal and conditional rows, per-output quantile levels, masked one-sided
outputs and the side label), and each loss against the statistic it must
estimate (quantile, log of the mean, logit)."""
from __future__ import annotations

import numpy as np

from oracle import mlp


def _setup(seed=0, B=64):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, mlp.NPARAMS)
    cond = rng.uniform(0, 1, B) < 0.3
    ua, ub, uc = rng.uniform(0, 1, (3, B))
    rec = rng.normal(0, 1, (B, 11))
    rec[:, 9] = 1.0
    X = mlp.inputs(rng.normal(3, 1, B), rng.uniform(-4, -2, B), rng.normal(0, 2, B), ua, ub, uc,
                   rng.uniform(0, 1.4, B), cond)
    Y = mlp.raw_targets(rec, cond)
    U = mlp.levels(ua, ub, uc, cond)
    return p, X, Y, U, cond


def test_backward_matches_finite_differences():
    p, X, Y, U, cond = _setup()
    assert cond.any() and (~cond).any()
    m = np.flatnonzero(~cond)[:3]
    Y[m, mlp.O_LOGN] += 3.0  # some samples beyond the deviance clamp (s4 d > 4)
    s4 = 1.7
    _, g = mlp.loss_and_grad(p, X, Y, U, s4=s4)
    rng = np.random.default_rng(1)
    idx = rng.choice(mlp.NPARAMS, 200, replace=False)
    h = 1e-6
    fd = []
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd.append((mlp.loss_and_grad(pp, X, Y, U, s4=s4)[0] - mlp.loss_and_grad(pm, X, Y, U, s4=s4)[0]) / (2 * h))
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
    rec = np.zeros((4, 11))
    rec[:, 3] = [1.5, -2.0, 0.0, 0.7]
    rec[:, 4:9] = np.arange(20).reshape(4, 5)
    rec[:, 10] = [0.1, 0.2, 0.3, 0.4]
    cond = np.array([False, False, False, True])
    y = mlp.raw_targets(rec, cond)
    assert y[0, mlp.O_XPOS] == 1.5 and np.isnan(y[0, mlp.O_XNEG]) and y[0, mlp.O_LOGIT] == 1
    assert np.isnan(y[1, mlp.O_XPOS]) and y[1, mlp.O_XNEG] == 2.0 and y[1, mlp.O_LOGIT] == 0
    assert y[2, mlp.O_XPOS] == 0.0 and y[2, mlp.O_LOGIT] == 1
    assert np.all(y[:3, [mlp.O_S, mlp.O_T, mlp.O_LOGN, mlp.O_LOGX2]] == rec[:3][:, [4, 5, 7, 8]])
    # marginal rows carry no direction targets, conditional rows only those
    assert np.all(np.isnan(y[:3, [mlp.O_MU, mlp.O_ALPHA, mlp.O_SPARE]]))
    assert y[3, mlp.O_MU] == rec[3, 6] and y[3, mlp.O_ALPHA] == 0.4
    assert np.all(np.isnan(np.delete(y[3], [mlp.O_MU, mlp.O_ALPHA])))


def test_levels_and_inputs_by_row_kind():
    cond = np.array([False, True])
    U = mlp.levels(np.array([0.1, 0.2]), np.array([0.3, 0.4]), np.array([0.5, 0.6]), cond)
    assert U[0, mlp.O_XPOS] == U[0, mlp.O_XNEG] == U[0, mlp.O_LOGX2] == 0.1
    assert U[0, mlp.O_S] == 0.3 and U[0, mlp.O_T] == 0.5 and np.isnan(U[0, mlp.O_MU])
    assert U[1, mlp.O_MU] == 0.2 and U[1, mlp.O_ALPHA] == 0.4 and np.isnan(U[1, mlp.O_S])
    e = 1.0 / (1.0 + np.exp(-4.0))  # level whose encoding is 1
    X = mlp.inputs([3.5, 3.5], [-3, -3], [4, 4], [0.5, 0.5], [e, e], [1 - e, -2.0], [0.3, np.sqrt(2)], cond)
    assert np.allclose(X[0], [0, 0, 1, 0, 1, -1, 0, 0])
    assert np.allclose(X[1], [0, 0, 1, 0, 1, -0.5, 1, 1])
    # extreme levels stay distinct: 0.999 and 0.9999 differ by about 0.58
    assert mlp.level_in(0.9999) - mlp.level_in(0.999) > 0.5


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.14159], dtype=np.float64)
    r = mlp.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert abs(r[3] + 3.14159) < 2 ** -6
