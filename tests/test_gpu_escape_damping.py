"""The learned whole-cell escape over a range of damping values: one network
trained on whole-cell walks recorded at a = 1e-4, 1e-3 and 1e-2 (log10 a is one
of its inputs) against held-out plain walks at the two ends of the range and
at an interpolated a = 3e-3, and the damping range it may be used on.  Runs
after test_gpu_escape.py (the context holds one network)."""
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
    return train_escape(gpu_ctx, lines=[0, 1, 2], n_records=9_000_000, seed=2)


def test_fitted_damping_range(gpu_ctx, trained_range):
    import torch
    from paper_2608_09340_amd import krt
    w = torch.zeros(krt.ESC_NPARAMS + krt.ESC_NNORM, dtype=torch.float32, device="cuda")
    gpu_ctx.krt_escape_get_weights(w)
    o = krt.ESC_NPARAMS + 2 * krt.ESC_NOUT + krt.ESC_NCAL
    lo, hi = w[o:o + 2].cpu().numpy()
    assert abs(lo + 4.0) < 1e-5 and abs(hi + 2.0) < 1e-5, (lo, hi)


@pytest.mark.parametrize("line,a", [(0, 1e-4), (2, 1e-2), (3, 3e-3)])
@pytest.mark.parametrize("tau,xin,q", [(3e2, 0.0, (0.2, 0.4, 0.9)), (3e3, 1.0, (0.1, 0.5, 0.998))])
def test_samples_vs_plain_across_damping(gpu_ctx, trained_range, line, a, tau, xin, q):
    """At a fixed condition (isotropic incoming directions), samples drawn as
    the transport draws them vs held-out plain walks at that damping: exit-face
    total variation below 0.04, KS of the exit frequency and, on the most
    frequent face, of the offsets, cosine and alpha below 0.06; ln E[N_s]
    within 0.06."""
    import torch
    from paper_2608_09340_amd import krt
    n = 20000
    lt = np.log10(tau)
    out = torch.zeros((n, krt.ESC_NREC), dtype=torch.float32, device="cuda")
    gpu_ctx.krt_escape_record(line, n, 99, 1 << 40, lt, lt, out, x_in=xin, q=q)
    plain = out.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(17)
    cond = np.zeros((n, 20))
    cond[:, mlp.R_LT] = lt
    cond[:, mlp.R_LA] = np.log10(a)
    cond[:, mlp.R_X] = xin
    cond[:, mlp.R_Q0:mlp.R_Q2 + 1] = q
    cond[:, mlp.R_LD] = lt + np.log10(1 - q[2])
    v = rng.normal(size=(n, 3))
    cond[:, mlp.R_N0:mlp.R_N2 + 1] = v / np.linalg.norm(v, axis=1)[:, None]

    def fwd(c, flag):
        raw = np.concatenate([c[:, :10], rng.uniform(0, 1, (n, 4)), np.full((n, 1), flag),
                              c[:, [mlp.R_XOUT]], c[:, [mlp.R_FACE]]], axis=1)
        pred = torch.zeros((n, krt.ESC_NOUT), dtype=torch.float32, device="cuda")
        gpu_ctx.krt_escape_forward(torch.from_numpy(raw.astype(np.float32)).cuda(), pred)
        return pred.cpu().numpy().astype(np.float64)

    m = fwd(cond, 0.0)
    pf = np.exp(m[:, :6] - m[:, :6].max(axis=1, keepdims=True))
    pf /= pf.sum(axis=1, keepdims=True)
    face = (rng.uniform(0, 1, n)[:, None] > np.cumsum(pf, axis=1)).sum(axis=1).clip(0, 5)
    pos = rng.uniform(0, 1, n) < 1.0 / (1.0 + np.exp(-m[:, mlp.O_SIDE]))
    mag = np.maximum(m[np.arange(n), mlp.O_XABS + face], 0.0)
    xo = np.where(pos, mag, -mag)
    cond[:, mlp.R_FACE] = face
    cond[:, mlp.R_XOUT] = xo
    m2 = fwd(cond, 1.0)
    fp = np.bincount(plain[:, mlp.R_FACE].astype(int), minlength=6) / n
    tv = 0.5 * np.abs(fp - np.bincount(face, minlength=6) / n).sum()
    top = int(np.argmax(fp))
    mp, ml_ = plain[:, mlp.R_FACE] == top, face == top
    ks = {"x_out": stats.ks_2samp(xo, plain[:, mlp.R_XOUT]).statistic}
    back = {"ys": np.sinh(m2[:, mlp.O_YS]), "yt": np.sinh(m2[:, mlp.O_YT]),
            "mu": np.sqrt(np.clip(m2[:, mlp.O_MU2], 1e-6, 1.0)), "alpha": m2[:, mlp.O_ALPHA]}
    for name, col in (("ys", mlp.R_YS), ("yt", mlp.R_YT), ("mu", mlp.R_MU), ("alpha", mlp.R_ALPHA)):
        ks[name] = stats.ks_2samp(back[name][ml_], plain[mp, col]).statistic
    ln_mean = np.log(np.mean(np.exp(plain[:, mlp.R_LOGN])))
    print(f"a={a:g} tau_c={tau:g} x_in={xin}: face TV {tv:.4f} KS " + " ".join(f"{k} {v:.4f}" for k, v in ks.items())
          + f"; ln E[N_s] learned {m[:, mlp.O_LOGN].mean():.4f} plain {ln_mean:.4f}")
    assert tv < 0.04, tv
    assert max(ks.values()) < 0.06, ks
    assert abs(m[:, mlp.O_LOGN].mean() - ln_mean) < 0.06


def test_damping_outside_range_refused(gpu_ctx, trained_range):
    """A line with a = 2e-2 lies beyond the API's range and the fitted one."""
    from paper_2608_09340_amd import krt
    T = krt.Transport(W.cube(n=4, tau0=1e3, a=2e-2), ctx=gpu_ctx)
    with pytest.raises(Exception):
        T.run(1000, seed=0, escape_mode=1)
