"""FP64 CPU reference of the whole-cell escape network -- TEST INFRASTRUCTURE.

Same parameter layout as the GPU (one flat vector): W1[24][128], b1[128],
W2[128][128], b2, W3[128][128], b3, W4[128][32], b4[32]; hidden activations
leaky ReLU max(z, z/16).

The network describes how a photon that scatters inside a homogeneous static
cubic cell leaves it (the plain walk of Sec. 2.1-2.3 confined to one cell; the
paper itself has no learned part).  Conditions are given in the cell's
reduced frame: the start point's absolute coordinates sorted ascending,
q0 <= q1 <= q2 (in half-widths; axis 2 is the nearest face), the incoming
direction in the same frame and |x_in| (the exit frequency's sign follows
x_in's).  Inputs (24):

  0  (log10 tau_c - 3) / 1.2      tau_c: line-centre depth centre to face
  1  log10 a + 3
  2  |x_in| - 1
  3-5 2 q - 1
  6  (log10 depth - 2) / 1.2      depth = tau_c (1 - q2), to the nearest face
  7-9 incoming direction (reduced frame)
  10-13 L(u_a), L(u_b), L(u_c), L(u_d)  quantile levels, L(u) = logit(u) / 4
  14 flag: 0 marginal row, 1 conditional row
  15 conditional: x_out / 4 (reduced sign), else 0
  16-21 conditional: one-hot exit face F = 2 axis + (normal along +axis), else 0
  22, 23 zero

Outputs (index: meaning, loss, level):
  marginal rows
  0-5   logits of the exit face                      softmax cross-entropy
  6     logit P(x_out >= 0)                          logistic
  7     ln E[N_s | condition]                        weighted log-deviance
  8     quantile of ln <x^2> over the scatterings    pinball at u_b
  16-21 quantile of |x_out| given exit face F        pinball at u_a, records
        (output 16 + F)                              leaving through F
  conditional rows (given the exit face and x_out)
  9     quantile of asinh(ys)                        pinball at u_a
  10    quantile of asinh(yt)                        pinball at u_b
  11    quantile of mu^2 (mu the exit cosine)        pinball at u_c
  12    quantile of alpha (tangential direction vs   pinball at u_d
        the exit offset)
  13-15, 22-31 unused
ys, yt are the exit point's offsets from the start point's projection onto
the exit face (along the two axes following the exit axis cyclically) over
the start point's distance to that face's plane.  The offsets' heavy tails
(the plane distance can be tiny) are compressed by asinh and the cosine is
learned as mu^2, whose quantile function near mu = 0 is smooth (the exit
cosine of an optically thick medium has a density vanishing linearly at 0);
both maps are monotone, so quantiles transform with them.  The exit
frequency's magnitude depends strongly on the exit face (photons leaving
through the near face need a shorter wing excursion), so it has one quantile
output per face; its sign is nearly independent of the face.

Pinball loss rho_u(y - o) = (y - o)(u - 1{y < o}); output 7 uses the scaled
log-deviance w f(d) / s7 with w = 1/4, d = s7 (y7 - o7), f(d) = e^d - 1 - d
continued linearly beyond d = 4, whose minimiser is ln E[N_s]; the face
logits use -log softmax(o)_F, whose minimiser is the log-probabilities (up to
a constant); output 6 uses softplus(o) - b o, b = 1{x_out >= 0}.  Losses are
averaged over the batch and summed over outputs.  The manual backward pass is
pinned by finite differences (tests/test_oracle_mlp.py).  ``bf=True`` rounds
weights and activations to bfloat16 where the GPU kernels do, and adds the
quantile levels' rounding residuals (rounded again) through their own layer-1
weights, as the GPU's extra operand slots do.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 24, 128, 32
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (NH, NOUT)), ("b4", (NOUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
NCAL = 256
NNORM = 2 * NOUT + NCAL + 8
O_FACE = 0
O_SIDE, O_LOGN, O_LOGX2, O_YS, O_YT, O_MU2, O_ALPHA = range(6, 13)
O_XABS = 16
FACES = tuple(range(6))
XABS = tuple(O_XABS + f for f in FACES)
MARGINAL = FACES + (O_SIDE, O_LOGN, O_LOGX2) + XABS
CONDITIONAL = (O_YS, O_YT, O_MU2, O_ALPHA)
UNUSED = tuple(k for k in range(NOUT) if k not in MARGINAL + CONDITIONAL)
DEV_CLAMP = 4.0
LEVEL_MIN = 1e-4
DEV_WEIGHT = 0.25
# record columns (oracle.cell_escape_record and the GPU records share them)
(R_LT, R_LA, R_X, R_Q0, R_Q1, R_Q2, R_LD, R_N0, R_N1, R_N2, R_FACE, R_YS, R_YT, R_MU, R_ALPHA, R_XOUT,
 R_LOGN, R_LOGX2, R_VALID) = range(19)


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


def level_in(u):
    """Network input of a quantile level u: logit(u) / 4, u clamped to the
    trained levels [1e-4, 1 - 1e-4] (beyond them a network would extrapolate)."""
    u = np.clip(np.asarray(u, dtype=np.float64), LEVEL_MIN, 1.0 - LEVEL_MIN)
    return 0.25 * (np.log(u) - np.log1p(-u))


def inputs(rec, u, cond):
    """Normalised inputs [B, NIN] of records in the reduced frame (columns R_*;
    x_in >= 0) at quantile levels u [B, 4]; conditional rows take the record's
    exit face and exit frequency."""
    rec = np.asarray(rec, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64).reshape(-1, 4)
    cond = np.asarray(cond, dtype=bool)
    B = rec.shape[0]
    X = np.zeros((B, NIN))
    X[:, 0] = (rec[:, R_LT] - 3.0) / 1.2
    X[:, 1] = rec[:, R_LA] + 3.0
    X[:, 2] = rec[:, R_X] - 1.0
    X[:, 3:6] = 2.0 * rec[:, R_Q0:R_Q2 + 1] - 1.0
    X[:, 6] = (rec[:, R_LD] - 2.0) / 1.2
    X[:, 7:10] = rec[:, R_N0:R_N2 + 1]
    X[:, 10:14] = level_in(u)
    X[:, 14] = cond
    X[:, 15] = np.where(cond, rec[:, R_XOUT] / 4.0, 0.0)
    face = rec[:, R_FACE].astype(np.int64)
    X[np.arange(B), 16 + face] = np.where(cond, 1.0, 0.0)
    return X


def levels(u, cond):
    """Quantile level of each output per row [B, NOUT] (NaN for outputs that
    are not quantiles or not trained on that kind of row)."""
    u = np.asarray(u, dtype=np.float64).reshape(-1, 4)
    cond = np.asarray(cond, dtype=bool)
    U = np.full((cond.shape[0], NOUT), np.nan)
    for k in XABS:
        U[:, k] = np.where(cond, np.nan, u[:, 0])
    U[:, O_LOGX2] = np.where(cond, np.nan, u[:, 1])
    for k, j in ((O_YS, 0), (O_YT, 1), (O_MU2, 2), (O_ALPHA, 3)):
        U[:, k] = np.where(cond, u[:, j], np.nan)
    return U


LEAK = 0.0625


def act(z):
    """Hidden activation: leaky ReLU max(z, z / 16)."""
    return np.maximum(z, LEAK * z)


def dact(z):
    return np.where(z > 0.0, 1.0, LEAK)


def forward(p, X, bf=False):
    P = unpack(p)
    r = bf16 if bf else (lambda a: a)
    W = {k: (r(v) if k.startswith("W") else v) for k, v in P.items()}
    cache = {"X": X}
    h = r(X)
    for i in (1, 2, 3):
        z = h @ W[f"W{i}"] + W[f"b{i}"]
        if i == 1 and bf:
            # the GPU adds the bfloat16 rounding residuals of the four quantile
            # levels through extra operand slots tied to their weights
            z = z + r(X[:, 10:14] - h[:, 10:14]) @ W["W1"][10:14]
        cache[f"z{i}"] = z
        cache[f"h{i - 1}"] = h
        h = r(act(z))
    cache["h3"] = h
    out = h @ W["W4"] + W["b4"]
    return out, cache, W


def deviance(d):
    """f(d) = e^d - 1 - d for d <= 4, its tangent continuation beyond; and f'(d)."""
    d = np.asarray(d, dtype=np.float64)
    dc = np.minimum(d, DEV_CLAMP)
    f = np.exp(dc) - 1.0 - dc + (np.exp(DEV_CLAMP) - 1.0) * np.maximum(d - DEV_CLAMP, 0.0)
    return f, np.exp(dc) - 1.0


def losses(out, Y, U, s9=1.0):
    """Mean over the batch of the summed per-output losses, and dL/dout.
    Y: normalised targets (NaN where an output is masked for that sample);
    Y[:, 0] holds the exit face label F on marginal rows (columns 1-5 unused),
    Y[:, 6] the side label b in {0, 1}; U: per-output quantile levels."""
    B = out.shape[0]
    live = ~np.isnan(Y)
    Yz = np.where(live, Y, 0.0)
    Uz = np.where(np.isnan(U), 0.0, U)
    ind = (Yz < out).astype(np.float64)
    lk = (Yz - out) * (Uz - ind)
    dout = (ind - Uz) / B
    # ln E[N_s]: log-deviance
    f, fp = deviance(s9 * (Yz[:, O_LOGN] - out[:, O_LOGN]))
    lk[:, O_LOGN] = DEV_WEIGHT * f / s9
    dout[:, O_LOGN] = -DEV_WEIGHT * fp / B
    # side: logistic
    o6, b = out[:, O_SIDE], Yz[:, O_SIDE]
    lk[:, O_SIDE] = np.logaddexp(0.0, o6) - b * o6
    dout[:, O_SIDE] = (1.0 / (1.0 + np.exp(-o6)) - b) / B
    # exit face: softmax cross-entropy, counted in column 0
    lf = out[:, :6]
    mx = lf.max(axis=1, keepdims=True)
    e = np.exp(lf - mx)
    sm = e / e.sum(axis=1, keepdims=True)
    F = Yz[:, 0].astype(np.int64)
    rows = np.arange(B)
    lk[:, 0] = (mx[:, 0] + np.log(e.sum(axis=1))) - lf[rows, F]
    lk[:, 1:6] = 0.0
    onehot = np.zeros_like(sm)
    onehot[rows, F] = 1.0
    dout[:, :6] = (sm - onehot) / B
    fl = live[:, 0]
    lk[:, :6] = np.where(fl[:, None], lk[:, :6], 0.0)
    dout[:, :6] = np.where(fl[:, None], dout[:, :6], 0.0)
    live[:, 1:6] = fl[:, None]
    lk = np.where(live, lk, 0.0)
    dout = np.where(live, dout, 0.0)
    return float(np.sum(lk) / B), dout


def loss_and_grad(p, X, Y, U, bf=False, s9=1.0):
    """s9: the target scale of the ln E[N_s] output (norm[NOUT + O_LOGN])."""
    out, c, W = forward(p, X, bf)
    loss, d = losses(out, Y, U, s9)
    g = {"W4": c["h3"].T @ d, "b4": d.sum(0)}
    dh = d @ W["W4"].T
    for i in (3, 2, 1):
        dz = dh * dact(c[f"z{i}"])
        g[f"W{i}"] = c[f"h{i - 1}"].T @ dz
        g[f"b{i}"] = dz.sum(0)
        dh = dz @ W[f"W{i}"].T
    return loss, pack(g)


def raw_targets(rec, cond=None):
    """Records (columns R_*, reduced frame) -> per-output physical targets
    [B, NOUT] (NaN where masked; column 0 holds the face label, column 6 the
    side label; the exit-frequency magnitude only in its exit face's column;
    the offsets as asinh, the cosine squared).  cond marks conditional rows
    (default: none)."""
    rec = np.asarray(rec, dtype=np.float64)
    B = rec.shape[0]
    cond = np.zeros(B, dtype=bool) if cond is None else np.asarray(cond, dtype=bool)
    x = rec[:, R_XOUT]
    F = rec[:, R_FACE].astype(np.int64)
    y = np.full((B, NOUT), np.nan)
    y[:, 0] = rec[:, R_FACE]
    y[:, O_SIDE] = (x >= 0.0).astype(np.float64)
    y[np.arange(B), O_XABS + F] = np.abs(x)
    y[:, O_LOGN] = rec[:, R_LOGN]
    y[:, O_LOGX2] = rec[:, R_LOGX2]
    y[:, O_YS] = np.arcsinh(rec[:, R_YS])
    y[:, O_YT] = np.arcsinh(rec[:, R_YT])
    y[:, O_MU2] = rec[:, R_MU] ** 2
    y[:, O_ALPHA] = rec[:, R_ALPHA]
    y[cond[:, None] & np.isin(np.arange(NOUT), MARGINAL)[None, :]] = np.nan
    y[~cond[:, None] & np.isin(np.arange(NOUT), CONDITIONAL)[None, :]] = np.nan
    y[:, list(UNUSED)] = np.nan
    return y


def targets_normalised(rec, norm, cond=None):
    """Normalised targets (raw - mean) / scale; the face and side labels keep
    their values (their normalisation is fixed at mean 0, scale 1)."""
    return (raw_targets(rec, cond) - norm[:NOUT]) / norm[NOUT:2 * NOUT]


def reduce_records(rec):
    """Oracle records in any frame -> the network's reduced frame: start point
    coordinates |q| sorted ascending (axis 2 nearest the start), directions,
    exit face and exit offsets permuted and reflected alike, x_in >= 0 (the
    sign of x_out flipped with it).  mu and alpha are invariant."""
    rec = np.array(rec, dtype=np.float64, copy=True)
    B = rec.shape[0]
    r = np.arange(B)
    q = rec[:, R_Q0:R_Q2 + 1].copy()
    sg = np.where(q < 0, -1.0, 1.0)
    order = np.argsort(np.abs(q), axis=1, kind="stable")   # new axis j <- old axis order[j]
    inv = np.argsort(order, axis=1)                         # old axis o -> new axis inv[o]
    rec[:, R_Q0:R_Q2 + 1] = np.abs(q)[r[:, None], order]
    n = rec[:, R_N0:R_N2 + 1] * sg
    rec[:, R_N0:R_N2 + 1] = n[r[:, None], order]
    F = rec[:, R_FACE].astype(np.int64)
    ax, side = F // 2, np.where(F % 2 == 1, 1.0, -1.0)
    off_old = np.zeros((B, 3))
    off_old[r, (ax + 1) % 3] = rec[:, R_YS]
    off_old[r, (ax + 2) % 3] = rec[:, R_YT]
    off_new = (off_old * sg)[r[:, None], order]
    nax = inv[r, ax]
    rec[:, R_FACE] = 2 * nax + (side * sg[r, ax] > 0)
    rec[:, R_YS] = off_new[r, (nax + 1) % 3]
    rec[:, R_YT] = off_new[r, (nax + 2) % 3]
    sx = np.where(rec[:, R_X] < 0, -1.0, 1.0)
    rec[:, R_X] *= sx
    rec[:, R_XOUT] *= sx
    return rec
