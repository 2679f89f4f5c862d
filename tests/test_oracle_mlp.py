"""Pins of the FP64 reference network used to check the GPU training kernels:
its manual backward pass against central finite differences of its own loss
(marginal and conditional rows, per-output quantile levels, masked one-sided
outputs, the face and side labels), each loss against the statistic it must
estimate (quantile, log of the mean, logit, log-probabilities), and the
reduction of oracle records to the network's frame against the cube's own
symmetry."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import mlp


def _records(rng, B):
    rec = np.zeros((B, 20))
    rec[:, mlp.R_LT] = rng.uniform(1.5, 5, B)
    rec[:, mlp.R_LA] = rng.uniform(-4, -2, B)
    rec[:, mlp.R_X] = rng.uniform(0, 2, B)
    q = np.sort(rng.uniform(0, 1, (B, 3)), axis=1)
    rec[:, mlp.R_Q0:mlp.R_Q2 + 1] = q
    rec[:, mlp.R_LD] = rec[:, mlp.R_LT] + np.log10(1 - q[:, 2])
    v = rng.normal(size=(B, 3))
    rec[:, mlp.R_N0:mlp.R_N2 + 1] = v / np.linalg.norm(v, axis=1)[:, None]
    rec[:, mlp.R_FACE] = rng.integers(0, 6, B)
    rec[:, mlp.R_YS:mlp.R_ALPHA + 1] = rng.normal(0, 1, (B, 4))
    rec[:, mlp.R_XOUT] = rng.normal(0, 3, B)
    rec[:, mlp.R_LOGN] = rng.normal(3, 1, B)
    rec[:, mlp.R_LOGX2] = rng.normal(0, 1, B)
    rec[:, mlp.R_VALID] = 1.0
    return rec


def _setup(seed=0, B=64):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, mlp.NPARAMS)
    cond = rng.uniform(0, 1, B) < 0.3
    u = rng.uniform(0, 1, (B, 4))
    rec = _records(rng, B)
    X = mlp.inputs(rec, u, cond)
    Y = mlp.raw_targets(rec, cond)
    U = mlp.levels(u, cond)
    return p, X, Y, U, cond


def test_backward_matches_finite_differences():
    p, X, Y, U, cond = _setup()
    assert cond.any() and (~cond).any()
    m = np.flatnonzero(~cond)[:3]
    Y[m, mlp.O_LOGN] += 3.0  # some samples beyond the deviance clamp (s9 d > 4)
    s9 = 1.7
    _, g = mlp.loss_and_grad(p, X, Y, U, s9=s9)
    rng = np.random.default_rng(1)
    used = np.array(sorted(mlp.MARGINAL + mlp.CONDITIONAL))
    idx = np.concatenate([rng.choice(mlp.NPARAMS, 200, replace=False),
                          mlp.NPARAMS - mlp.NOUT + used])  # every used output's bias
    h = 1e-6  # a pinball kink inside a difference shifts it by a few 1e-5 (relative)
    fd = []
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd.append((mlp.loss_and_grad(pp, X, Y, U, s9=s9)[0] - mlp.loss_and_grad(pm, X, Y, U, s9=s9)[0]) / (2 * h))
    fd = np.array(fd)
    assert np.allclose(g[idx], fd, rtol=1e-4, atol=1e-9)


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


def test_softmax_minimiser_is_log_probabilities():
    """Gradient descent on the mean face cross-entropy over labels drawn with
    probabilities P drives softmax(o) to P (the logits to log P + const)."""
    rng = np.random.default_rng(6)
    P = np.array([0.05, 0.1, 0.15, 0.2, 0.1, 0.4])
    F = rng.choice(6, 200000, p=P)
    emp = np.bincount(F, minlength=6) / F.size
    o = np.zeros(6)
    for _ in range(3000):
        out = np.zeros((6, mlp.NOUT))
        out[:, :6] = o
        Yb = np.full((6, mlp.NOUT), np.nan)
        Yb[:, 0] = np.arange(6)
        _, d = mlp.losses(out, Yb, np.full((6, mlp.NOUT), np.nan))
        o -= 5.0 * (d[:, :6] * emp[:, None] * 6).sum(axis=0)
    sm = np.exp(o - o.max())
    sm /= sm.sum()
    assert np.allclose(sm, emp, atol=2e-3), (sm, emp)


def test_raw_targets_masks():
    rng = np.random.default_rng(7)
    rec = _records(rng, 4)
    rec[:, mlp.R_XOUT] = [1.5, -2.0, 0.0, 0.7]
    rec[:, mlp.R_FACE] = [3, 0, 5, 2]
    rec[3, mlp.R_YS:mlp.R_ALPHA + 1] = [-2.0, 0.5, 0.6, 1.2]
    cond = np.array([False, False, False, True])
    y = mlp.raw_targets(rec, cond)
    # |x_out| only in the exit face's column, the side label from its sign
    for i, (f, ax, b) in enumerate(((3, 1.5, 1), (0, 2.0, 0), (5, 0.0, 1))):
        xa = y[i, list(mlp.XABS)]
        assert xa[f] == ax and np.isnan(np.delete(xa, f)).all() and y[i, mlp.O_SIDE] == b
    assert np.all(y[:3, 0] == rec[:3, mlp.R_FACE])
    assert np.all(y[:3, [mlp.O_LOGN, mlp.O_LOGX2]] == rec[:3][:, [mlp.R_LOGN, mlp.R_LOGX2]])
    # marginal rows carry no conditional targets, conditional rows only those;
    # unused outputs none
    assert np.all(np.isnan(y[:3, list(mlp.CONDITIONAL) + list(mlp.UNUSED)]))
    assert np.allclose(y[3, list(mlp.CONDITIONAL)], [np.arcsinh(-2.0), np.arcsinh(0.5), 0.36, 1.2])
    assert np.all(np.isnan(np.delete(y[3], list(mlp.CONDITIONAL))))
    assert len(mlp.UNUSED) == mlp.NOUT - 6 - 3 - 6 - 4


def test_levels_and_inputs_by_row_kind():
    rng = np.random.default_rng(8)
    rec = _records(rng, 2)
    rec[:, mlp.R_LT] = 3.0
    rec[:, mlp.R_LD] = 2.0
    rec[:, mlp.R_X] = 1.0
    rec[1, mlp.R_FACE] = 4
    rec[1, mlp.R_XOUT] = -2.0
    cond = np.array([False, True])
    u = np.array([[0.1, 0.2, 0.3, 0.4], [0.5, 0.6, 0.7, 0.8]])
    U = mlp.levels(u, cond)
    assert np.all(U[0, list(mlp.XABS)] == 0.1) and U[0, mlp.O_LOGX2] == 0.2
    assert np.isnan(U[0, mlp.O_YS]) and np.isnan(U[1, list(mlp.XABS)]).all()
    assert (U[1, mlp.O_YS], U[1, mlp.O_YT], U[1, mlp.O_MU2], U[1, mlp.O_ALPHA]) == (0.5, 0.6, 0.7, 0.8)
    X = mlp.inputs(rec, u, cond)
    assert np.allclose(X[:, [0, 2, 6]], 0.0)
    assert np.all(X[0, 14:] == 0.0)
    assert X[1, 14] == 1.0 and X[1, 15] == -0.5 and X[1, 20] == 1.0 and X[1, 16:22].sum() == 1.0
    # extreme levels stay distinct: 0.999 and 0.9999 differ by about 0.58
    assert mlp.level_in(0.9999) - mlp.level_in(0.999) > 0.5


def test_reduction_to_the_network_frame():
    """Walks from a start point and from its image under a symmetry of the cube
    (axis permutation and reflections, x_in sign reversed) reduce to the same
    conditions and to samples of the same exit distribution (two-sample KS of
    every reduced output and equal face frequencies)."""
    from scipy import stats
    q = np.array([0.2, -0.6, 0.35])
    n = 6000
    a = mlp.reduce_records(oracle.cell_escape_record(n, 20.0, 1e-3, 0.7, q, n_in=[0.6, 0.0, 0.8], seed=11,
                                                     threads=4))
    qi = np.array([-0.6, 0.35, -0.2])  # new axes (y, z, -x) of the old frame
    b = mlp.reduce_records(oracle.cell_escape_record(n, 20.0, 1e-3, -0.7, qi, n_in=[0.0, 0.8, -0.6], seed=12,
                                                     threads=4))
    assert np.allclose(a[0, :10], b[0, :10]) and np.allclose(a[0, mlp.R_Q0:mlp.R_Q2 + 1], [0.2, 0.35, 0.6])
    fa = np.bincount(a[:, mlp.R_FACE].astype(int), minlength=6)
    fb = np.bincount(b[:, mlp.R_FACE].astype(int), minlength=6)
    m = (fa + fb) > 40
    z = (fa[m] - fb[m]) / np.sqrt(fa[m] + fb[m])
    assert np.max(np.abs(z)) < 4.5, (fa, fb)
    for face in (4, 5):
        ma, mb = a[:, mlp.R_FACE] == face, b[:, mlp.R_FACE] == face
        for col in (mlp.R_YS, mlp.R_YT, mlp.R_MU, mlp.R_ALPHA, mlp.R_XOUT, mlp.R_LOGN):
            assert stats.ks_2samp(a[ma, col], b[mb, col]).pvalue > 1e-3, (face, col)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.14159], dtype=np.float64)
    r = mlp.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert abs(r[3] + 3.14159) < 2 ** -6
