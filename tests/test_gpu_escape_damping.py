"""The learned escape over a range of damping values: one network trained on
single-cell escapes recorded at a = 1e-4, 1e-3 and 1e-2 (log10 a is one of its
inputs) against held-out plain escapes at the two ends of the range and at an
interpolated a = 3e-3, and the damping range it may be used on.  Runs after
test_gpu_escape.py (the context holds one network)."""
from __future__ import annotations

import numpy as np
import pytest
from scipy import stats

from oracle import mlp
from paper_2608_09340_amd import workloads as W

pytestmark = pytest.mark.gpu
A_TRAIN = (1e-4, 1e-3, 1e-2)


@pytest.fixture(scope="module")
def trained_range(gpu_ctx):
    from paper_2608_09340_amd.escape import train_escape
    gpu_ctx.krt_tables_build([(a, 0) for a in A_TRAIN] + [(3e-3, 0)])
    return train_escape(gpu_ctx, lines=[0, 1, 2], n_records=9_000_000, seed=2, log10_tau=(1.0, 5.0))


def test_fitted_damping_range(gpu_ctx, trained_range):
    import torch
    from paper_2608_09340_amd import krt
    w = torch.zeros(krt.ESC_NPARAMS + krt.ESC_NNORM, dtype=torch.float32, device="cuda")
    gpu_ctx.krt_escape_get_weights(w)
    o = krt.ESC_NPARAMS + 2 * krt.ESC_NOUT + krt.ESC_NCAL
    lo, hi = w[o:o + 2].cpu().numpy()
    assert abs(lo + 4.0) < 1e-5 and abs(hi + 2.0) < 1e-5, (lo, hi)


@pytest.mark.parametrize("line,a", [(0, 1e-4), (2, 1e-2), (3, 3e-3)])
@pytest.mark.parametrize("tau,xin", [(3e2, 0.0), (3e3, 1.0)])
def test_samples_vs_plain_across_damping(gpu_ctx, trained_range, line, a, tau, xin):
    """At fixed (tau_R, a, x_in), samples drawn as the transport draws them vs
    held-out plain escapes: KS of exit frequency, exit point, cosine and
    alignment angle below 0.05, ln E[N_s] within 0.08."""
    import torch
    from paper_2608_09340_amd import krt
    n = 20000
    out = torch.zeros((n, krt.ESC_NREC), dtype=torch.float32, device="cuda")
    lt = np.log10(tau)
    gpu_ctx.krt_escape_record(line, n, 99, 1 << 40, lt, lt, out, x_fixed=xin)
    plain = out.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(17)
    la = np.log10(a)
    raw = np.stack([np.full(n, lt), np.full(n, la), np.full(n, xin), rng.uniform(0, 1, n), rng.uniform(0, 1, n),
                    rng.uniform(0, 1, n), np.zeros(n), np.zeros(n)], 1)
    pred = torch.zeros((n, krt.ESC_NOUT), dtype=torch.float32, device="cuda")
    gpu_ctx.krt_escape_forward(torch.from_numpy(raw.astype(np.float32)).cuda(), pred)
    m = pred.cpu().numpy().astype(np.float64)
    pos = rng.uniform(0, 1, n) < 1.0 / (1.0 + np.exp(-m[:, mlp.O_LOGIT]))
    xo = np.where(pos, np.maximum(m[:, mlp.O_XPOS], 0.0), -np.maximum(m[:, mlp.O_XNEG], 0.0))
    s_l, t_l = np.clip(m[:, mlp.O_S], -1, 1), np.clip(m[:, mlp.O_T], -1, 1)
    raw2 = np.stack([np.full(n, lt), np.full(n, la), np.full(n, xin), rng.uniform(0, 1, n), rng.uniform(0, 1, n),
                     xo, np.hypot(s_l, t_l), np.ones(n)], 1)
    gpu_ctx.krt_escape_forward(torch.from_numpy(raw2.astype(np.float32)).cuda(), pred)
    m2 = pred.cpu().numpy().astype(np.float64)
    ks = {"x_out": stats.ks_2samp(xo, plain[:, 3]).statistic, "s": stats.ks_2samp(s_l, plain[:, 4]).statistic,
          "mu": stats.ks_2samp(np.clip(m2[:, mlp.O_MU], 1e-3, 1), plain[:, 6]).statistic,
          "alpha": stats.ks_2samp(np.clip(m2[:, mlp.O_ALPHA], 0, np.pi), plain[:, 10]).statistic}
    ln_mean = np.log(np.mean(np.exp(plain[:, 7])))
    print(f"a={a:g} tau={tau:g} x_in={xin}: KS " + " ".join(f"{k} {v:.4f}" for k, v in ks.items()) +
          f"; ln E[N_s] learned {m[:, 4].mean():.4f} plain {ln_mean:.4f}")
    assert max(ks.values()) < 0.05, ks
    assert abs(m[:, 4].mean() - ln_mean) < 0.08


def test_damping_outside_range_refused(gpu_ctx, trained_range):
    """A line with a = 2e-2 lies beyond the API's range and the fitted one."""
    from paper_2608_09340_amd import krt
    T = krt.Transport(W.cube(n=4, tau0=1e3, a=2e-2), ctx=gpu_ctx)
    with pytest.raises(Exception):
        T.run(1000, seed=0, escape_mode=1)
