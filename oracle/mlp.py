"""FP64 CPU reference of the escape network -- TEST INFRASTRUCTURE.

Same parameter layout as the GPU (one flat vector): W1[8][128], b1[128],
W2[128][128], b2, W3[128][128], b3, W4[128][10], b4[10]; activations SiLU.

Inputs (8), normalised as ((log10 tau - 3.5)/1.5, log10 a + 3, x_in / 4,
L(u_a), L(u_b), w, r_in, flag) with L(u) = logit(u) / 4 the encoding of a
quantile level (extreme levels get distinct inputs, so the far wing of the
exit frequency is not flattened).  A row is either *marginal* (flag 0,
w = L(u_c), r_in 0) or *conditional* (flag 1, w = x_out / 4 and
r_in = sqrt(2) r - 1 with x_out the exit frequency and r the exit point's
distance from the face centre): the network is evaluated once at three
independent quantile levels for the exit frequency, exit point and count,
then once more at the sampled exit frequency and point for the exit
direction, which depends on both (photons leaving near an edge travel away
from the face centre; wing photons leave closer to the normal).

Outputs (index: meaning, loss, level), for a record with exit frequency x:
  marginal rows
  0: quantile of x given x >= 0                 pinball at u_a, records with x >= 0
  1: quantile of s (exit point, first axis)      pinball at u_b
  2: quantile of t (exit point, second axis)     pinball at u_c
  4: ln E[N_s | condition]                       weighted log-deviance (below)
  5: quantile of ln <x^2> over the scatterings   pinball at u_a
  6: logit P(x >= 0 | condition)                 logistic (Bernoulli) loss
  7: quantile of -x given x < 0                  pinball at u_a, records with x < 0
  conditional rows (given r and x_out)
  3: quantile of mu (exit cosine to the normal)  pinball at u_a
  8: quantile of alpha (angle between the exit   pinball at u_b
     direction's tangential part and the exit point's offset (s, t))
  9: unused (keeps the parameter block an even number of floats)
The exit frequency is bimodal (blue and red peaks with an empty core between
them), so one smooth quantile function of the signed x would fill the gap;
the two one-sided quantiles and the side probability form a two-component
mixture whose components are each unimodal.

Pinball loss: rho_u(y - o) = (y - o)(u - 1{y < o}).  Output 4 uses the scaled
log-deviance w f(d) / s4 with w = 1/4, d = s4 (y4 - o4) and
f(d) = e^d - 1 - d (continued linearly beyond d = 4, so a rare very long
escape cannot dominate a batch); its minimiser satisfies E[e^(y - m)] = 1,
i.e. e^m = E[N_s].  Output 6 uses softplus(o) - b o with b = 1{x >= 0}, whose
minimiser is the logit of P(x >= 0).  Every loss is averaged over the whole
batch (masked samples contribute zero) and the outputs' losses are summed.
The manual backward pass is pinned by finite differences
(tests/test_oracle_mlp.py).  ``bf16=True`` rounds weights and activations to
bfloat16 (round to nearest even) where the GPU kernels do, to separate the
arithmetic error of the kernels from the storage format.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 8, 128, 10
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (NH, NOUT)), ("b4", (NOUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
NNORM = 2 * NOUT
O_XPOS, O_S, O_T, O_MU, O_LOGN, O_LOGX2, O_LOGIT, O_XNEG, O_ALPHA, O_SPARE = range(NOUT)
MARGINAL = (O_XPOS, O_S, O_T, O_LOGN, O_LOGX2, O_LOGIT, O_XNEG)
CONDITIONAL = (O_MU, O_ALPHA)
N_OUT = O_LOGN
DEV_CLAMP = 4.0
LEVEL_MIN = 1e-4
DEV_WEIGHT = 0.25


def unpack(p):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(a):
    """Round to bfloat16 (nearest even) and back to float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def inputs(lt, la, xin, ua, ub, w, r, cond):
    """Normalised inputs; w is u_c on marginal rows and the exit frequency x_out
    on conditional rows; r (exit point radius) is ignored on marginal rows."""
    cond = np.asarray(cond, dtype=bool)
    lt, la, xin, ua, ub, w, r = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64)
                                                      for v in (lt, la, xin, ua, ub, w, r)))
    wl = np.where(cond, 0.5, w)  # the level slot of a marginal row
    return np.stack([(lt - 3.5) / 1.5, la + 3.0, xin / 4.0, level_in(ua), level_in(ub),
                     np.where(cond, w / 4.0, level_in(wl)), np.where(cond, np.sqrt(2.0) * r - 1.0, 0.0),
                     cond.astype(np.float64)], axis=-1)


def level_in(u):
    """Network input of a quantile level u: logit(u) / 4, u clamped to the
    trained levels [1e-4, 1 - 1e-4] (beyond them a network would extrapolate)."""
    u = np.clip(np.asarray(u, dtype=np.float64), LEVEL_MIN, 1.0 - LEVEL_MIN)
    return 0.25 * (np.log(u) - np.log1p(-u))


def levels(ua, ub, uc, cond):
    """Quantile level of each output per row [B, NOUT] (NaN for the outputs
    that are not quantiles or not trained on that kind of row)."""
    cond = np.asarray(cond, dtype=bool)
    U = np.full((cond.shape[0], NOUT), np.nan)
    for k in (O_XPOS, O_XNEG, O_LOGX2):
        U[:, k] = np.where(cond, np.nan, ua)
    U[:, O_S] = np.where(cond, np.nan, ub)
    U[:, O_T] = np.where(cond, np.nan, uc)
    U[:, O_MU] = np.where(cond, ua, np.nan)
    U[:, O_ALPHA] = np.where(cond, ub, np.nan)
    return U


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, X, bf=False):
    P = unpack(p)
    r = bf16 if bf else (lambda a: a)
    W = {k: (r(v) if k.startswith("W") else v) for k, v in P.items()}
    cache = {"X": X}
    h = r(X)
    for i in (1, 2, 3):
        z = h @ W[f"W{i}"] + W[f"b{i}"]
        cache[f"z{i}"] = z
        cache[f"h{i - 1}"] = h
        h = r(silu(z))
    cache["h3"] = h
    out = h @ W["W4"] + W["b4"]
    return out, cache, W


def deviance(d):
    """f(d) = e^d - 1 - d for d <= 4, its tangent continuation beyond; and f'(d)."""
    d = np.asarray(d, dtype=np.float64)
    dc = np.minimum(d, DEV_CLAMP)
    f = np.exp(dc) - 1.0 - dc + (np.exp(DEV_CLAMP) - 1.0) * np.maximum(d - DEV_CLAMP, 0.0)
    return f, np.exp(dc) - 1.0


def losses(out, Y, U, s4=1.0):
    """Mean over the batch of the summed per-output losses, and dL/dout.
    Y: normalised targets (NaN where an output is masked for that sample);
    Y[:, 6] is the side label b in {0, 1}; U: per-output quantile levels."""
    B = out.shape[0]
    live = ~np.isnan(Y)
    Yz = np.where(live, Y, 0.0)
    Uz = np.where(np.isnan(U), 0.0, U)
    ind = (Yz < out).astype(np.float64)
    lk = (Yz - out) * (Uz - ind)
    dout = (ind - Uz) / B
    f, fp = deviance(s4 * (Yz[:, O_LOGN] - out[:, O_LOGN]))
    lk[:, O_LOGN] = DEV_WEIGHT * f / s4
    dout[:, O_LOGN] = -DEV_WEIGHT * fp / B
    o6, b = out[:, O_LOGIT], Yz[:, O_LOGIT]
    lk[:, O_LOGIT] = np.logaddexp(0.0, o6) - b * o6
    dout[:, O_LOGIT] = (1.0 / (1.0 + np.exp(-o6)) - b) / B
    lk = np.where(live, lk, 0.0)
    dout = np.where(live, dout, 0.0)
    return float(np.sum(lk) / B), dout


def loss_and_grad(p, X, Y, U, bf=False, s4=1.0):
    """s4: the target scale of output 4 (norm[NOUT + 4])."""
    out, c, W = forward(p, X, bf)
    loss, d = losses(out, Y, U, s4)
    g = {"W4": c["h3"].T @ d, "b4": d.sum(0)}
    dh = d @ W["W4"].T
    for i in (3, 2, 1):
        dz = dh * dsilu(c[f"z{i}"])
        g[f"W{i}"] = c[f"h{i - 1}"].T @ dz
        g[f"b{i}"] = dz.sum(0)
        dh = dz @ W[f"W{i}"].T
    return loss, pack(g)


def raw_targets(rec, cond=None):
    """Records [.., x_out, s, t, mu, lnNs, lnx2, valid, alpha] -> per-output
    physical targets [B, NOUT] (NaN where masked; column 6 is the side label).
    cond marks conditional rows (default: none)."""
    B = rec.shape[0]
    cond = np.zeros(B, dtype=bool) if cond is None else np.asarray(cond, dtype=bool)
    x = rec[:, 3].astype(np.float64)
    pos = x >= 0.0
    y = np.full((B, NOUT), np.nan)
    y[:, O_XPOS] = np.where(pos, x, np.nan)
    y[:, O_S] = rec[:, 4]
    y[:, O_T] = rec[:, 5]
    y[:, O_MU] = rec[:, 6]
    y[:, O_LOGN] = rec[:, 7]
    y[:, O_LOGX2] = rec[:, 8]
    y[:, O_LOGIT] = pos.astype(np.float64)
    y[:, O_XNEG] = np.where(pos, np.nan, -x)
    y[:, O_ALPHA] = rec[:, 10]
    y[cond[:, None] & np.isin(np.arange(NOUT), MARGINAL)[None, :]] = np.nan
    y[~cond[:, None] & np.isin(np.arange(NOUT), CONDITIONAL)[None, :]] = np.nan
    y[:, O_SPARE] = np.nan
    return y


def targets_normalised(rec, norm, cond=None):
    """Normalised targets: (raw - mean) / scale; the side label stays 0/1
    (its normalisation is fixed at mean 0, scale 1)."""
    return (raw_targets(rec, cond) - norm[:NOUT]) / norm[NOUT:2 * NOUT]
