"""FP64 CPU reference of the escape network -- TEST INFRASTRUCTURE.

Same parameter layout as the GPU (one flat vector): W1[4][128], b1[128],
W2[128][128], b2, W3[128][128], b3, W4[128][6], b4[6]; activations SiLU;
outputs 0-3 and 5 are conditional quantiles trained with the pinball loss
rho_u(y - o) = (y - o)(u - 1{y < o}); output 4 is ln E[N_s | condition],
trained with the weighted, scaled log-deviance w f(d) / s4 (w = 1/4),
d = s4 (y4 - o4), where
f(d) = e^d - 1 - d (continued linearly beyond d = 4, so a rare very long
escape cannot dominate a batch), whose minimiser satisfies E[e^(y - m)] = 1,
i.e. e^m = E[N_s].  Losses are averaged over the batch and summed over the
outputs.  Inputs are normalised as ((log10 tau - 3.5)/1.5, log10 a + 3,
x_in / 4, 2u - 1).  The manual backward pass is pinned by finite differences
(tests/test_oracle_mlp.py).  ``bf16=True`` rounds weights and activations to
bfloat16 (round to nearest even) where the GPU kernels do, to separate the
arithmetic error of the kernels from the storage format.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 4, 128, 6
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (NH, NOUT)), ("b4", (NOUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


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


def inputs(lt, la, xin, u):
    return np.stack([(np.asarray(lt) - 3.5) / 1.5, np.asarray(la) + 3.0, np.asarray(xin) / 4.0,
                     2.0 * np.asarray(u) - 1.0], axis=-1).astype(np.float64)


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


DEV_CLAMP = 4.0
DEV_WEIGHT = 0.25
N_OUT = 4  # index of the ln E[N_s] output


def deviance(d):
    """f(d) = e^d - 1 - d for d <= 4, its tangent continuation beyond; and f'(d)."""
    d = np.asarray(d, dtype=np.float64)
    dc = np.minimum(d, DEV_CLAMP)
    f = np.exp(dc) - 1.0 - dc + (np.exp(DEV_CLAMP) - 1.0) * np.maximum(d - DEV_CLAMP, 0.0)
    return f, np.exp(dc) - 1.0


def pinball(out, Y, u, s4=1.0):
    """Mean over the batch of the summed per-output losses, and dL/dout.
    Outputs other than 4: pinball at level u.  Output 4: w f(s4 (y - o)) / s4."""
    B = out.shape[0]
    ind = (Y < out).astype(np.float64)
    lk = (Y - out) * (u[:, None] - ind)
    dout = (ind - u[:, None]) / B
    f, fp = deviance(s4 * (Y[:, N_OUT] - out[:, N_OUT]))
    lk[:, N_OUT] = DEV_WEIGHT * f / s4
    dout[:, N_OUT] = -DEV_WEIGHT * fp / B
    return float(np.sum(lk) / B), dout


def loss_and_grad(p, X, Y, u, bf=False, s4=1.0):
    """s4: the target scale of output 4 (norm[6 + 4])."""
    out, c, W = forward(p, X, bf)
    loss, d = pinball(out, Y, u, s4)
    g = {"W4": c["h3"].T @ d, "b4": d.sum(0)}
    dh = d @ W["W4"].T
    for i in (3, 2, 1):
        dz = dh * dsilu(c[f"z{i}"])
        g[f"W{i}"] = c[f"h{i - 1}"].T @ dz
        g[f"b{i}"] = dz.sum(0)
        dh = dz @ W[f"W{i}"].T
    return loss, pack(g)


def targets_normalised(rec, norm):
    """Records [.., x_out, s, t, mu, lnNs, lnx2, valid] -> normalised targets."""
    y = rec[:, 3:9].astype(np.float64)
    return (y - norm[:NOUT]) / norm[NOUT:]
