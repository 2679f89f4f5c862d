"""FP64 CPU reference of the ray-tracing imaging pass -- TEST INFRASTRUCTURE.

Formal solution of the line transfer equation along lines of sight toward a
camera on one of the six grid axes (Sec. 2.2.2, eq. imaging-formal and
eq. imaging-alphas), cell by cell from the far side of the grid to the camera:

    I_out,k = I_in,k exp(-dtau_k) + S_k (1 - exp(-dtau_k)),
    dtau_k  = alpha_k dl,  alpha_k = k0 H(a, x_k) + kappa_abs,  S_k = j_k / alpha_k + S_emis,k,

with x_k the centre of channel k (lab frame) moved to the cell's gas frame,
x_k - n_cam . v (the sign convention of the transport), dl the cell width
along the ray and kappa_abs an optional grey absorption coefficient per cell
(the Monte Carlo pass scatters only; absorption enters here).  For
alpha_k dl -> 0 the scattering term is
j_k dl (the limit of j (1 - e^{-dtau}) / alpha).  H(a, x) is the oracle's
Faddeeva-based Voigt function.  Pixels are the grid cells of the plane
normal to the axis, ordered with the lower remaining axis fastest; the output
is [pixel][channel].
"""
from __future__ import annotations

import numpy as np

from . import voigt_H

AXES = {0: (0, 1), 1: (1, 1), 2: (2, 1), 3: (0, -1), 4: (1, -1), 5: (2, -1)}


def image(n, lo, hi, k0, vel, a, emis, ch_lo, ch_hi, axis, src=None, kabs=None):
    """n[3], lo[3], hi[3]; k0 [ncell]; vel [3][ncell] or None; emis [ncell][nch];
    axis 0..5 = +x, +y, +z, -x, -y, -z (the camera direction); src [ncell][nch]
    emission source function or None; kabs [ncell] absorption coefficient or
    None.  Returns I [npix][nch] (FP64)."""
    n = [int(v) for v in n]
    nx, ny, nz = n
    nch = emis.shape[1]
    d, sgn = AXES[int(axis)]
    dl = (hi[d] - lo[d]) / n[d]
    k0 = np.asarray(k0, dtype=np.float64).reshape(nz, ny, nx)
    ka = np.zeros((nz, ny, nx)) if kabs is None else np.asarray(kabs, dtype=np.float64).reshape(nz, ny, nx)
    E = np.asarray(emis, dtype=np.float64).reshape(nz, ny, nx, nch)
    S0 = None if src is None else np.asarray(src, dtype=np.float64).reshape(nz, ny, nx, nch)
    ncam = np.zeros(3)
    ncam[d] = sgn
    vdot = np.zeros((nz, ny, nx))
    if vel is not None:
        v = np.asarray(vel, dtype=np.float64).reshape(3, nz, ny, nx)
        vdot = ncam[0] * v[0] + ncam[1] * v[1] + ncam[2] * v[2]
    xk = ch_lo + (np.arange(nch) + 0.5) * (ch_hi - ch_lo) / nch
    # move the ray axis last: arrays [p1][p0][along][...] with pixel = p1 * n_p0 + p0
    if d == 0:
        perm = (0, 1, 2)   # (z, y, x): pixels (k, j), j fastest
    elif d == 1:
        perm = (0, 2, 1)   # (z, x, y): pixels (k, i), i fastest
    else:
        perm = (1, 2, 0)   # (y, x, z): pixels (j, i), i fastest
    k0p = np.transpose(k0, perm)
    kap = np.transpose(ka, perm)
    vp = np.transpose(vdot, perm)
    Ep = np.transpose(E, perm + (3,))
    Sp = None if S0 is None else np.transpose(S0, perm + (3,))
    n1, n0, nl = k0p.shape
    I = np.zeros((n1, n0, nch))
    order = range(nl) if sgn > 0 else range(nl - 1, -1, -1)
    for s in order:  # from the far side toward the camera
        xg = xk[None, None, :] - vp[:, :, s][:, :, None]
        H = voigt_H(a, xg.reshape(-1)).reshape(xg.shape)
        alpha = k0p[:, :, s][:, :, None] * H + kap[:, :, s][:, :, None]
        dtau = alpha * dl
        att = np.exp(-dtau)
        # j (1 - e^{-dtau}) / alpha written as j dl (1 - e^{-dtau}) / dtau, finite at dtau -> 0
        frac = np.where(dtau > 1e-12, -np.expm1(-dtau) / np.where(dtau > 1e-12, dtau, 1.0), 1.0 - 0.5 * dtau)
        I = I * att + Ep[:, :, s, :] * dl * frac
        if Sp is not None:
            I = I + Sp[:, :, s, :] * (-np.expm1(-dtau))
    return I.reshape(n1 * n0, nch)
