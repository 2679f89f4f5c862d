"""Seeded synthetic inputs for the line-transfer pass (plain data, no method).

Each builder returns a problem dict of numpy arrays and scalars:

    grid   : n[3], lo[3], hi[3], bc[3] (0 vacuum, 1 periodic), k0[ncell] (line-centre
             opacity per unit length, n_l*sigma_0), vel[3, ncell] (bulk velocity in
             Doppler units) or None, eps[ncell] or None, emis[ncell] or None,
             kabs[ncell] (grey absorption coefficient, units of k0) or None
    line   : a (damping), phase (0 isotropic, 1 dipole)
    source : kind (0 point, 1 plane z=pos[2], 2 volume, 3 beam), pos[3], dir[3],
             profile (0 delta at x0, 1 Voigt, 2 Gaussian), x0
    tally  : spec_nbins, spec_lo, spec_hi, emis_nch, ch_lo, ch_hi, n_cam[3], jbar

Cells are ordered x fastest: cell = (k*ny + j)*nx + i.  Fields are binary32,
as the GPU consumes them; the oracle widens the same arrays to FP64.  This
module holds no part of the transport arithmetic: it only lays out the
media of the paper's validation problems and of the benchmark workloads.
"""
from __future__ import annotations

import numpy as np

VACUUM, PERIODIC = 0, 1
SRC_POINT, SRC_PLANE, SRC_VOLUME, SRC_BEAM = 0, 1, 2, 3
PROF_DELTA, PROF_VOIGT, PROF_GAUSS = 0, 1, 2
PHASE_ISO, PHASE_DIPOLE = 0, 1


def _cell_centres(n, lo, hi):
    axes = [lo[d] + (np.arange(n[d]) + 0.5) * (hi[d] - lo[d]) / n[d] for d in range(3)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def _problem(n, lo, hi, bc, k0, a, *, vel=None, eps=None, emis=None, kabs=None, phase=PHASE_ISO,
             source=None, tally=None, max_events=1 << 40):
    return {
        "grid": {"n": list(n), "lo": list(lo), "hi": list(hi), "bc": list(bc),
                 "k0": np.ascontiguousarray(k0, dtype=np.float32).reshape(-1),
                 "vel": None if vel is None else np.ascontiguousarray(vel, dtype=np.float32).reshape(3, -1),
                 "eps": None if eps is None else np.ascontiguousarray(eps, dtype=np.float32).reshape(-1),
                 "emis": None if emis is None else np.ascontiguousarray(emis, dtype=np.float32).reshape(-1),
                 "kabs": None if kabs is None else np.ascontiguousarray(kabs, dtype=np.float32).reshape(-1)},
        "line": {"a": float(a), "phase": int(phase)},
        "source": source,
        "tally": tally,
        "max_events": int(max_events),
    }


def slab(tau0=1e3, a=1e-2, nz=32, *, spec=(200, -30.0, 30.0), phase=PHASE_ISO, nxy=1):
    """Static homogeneous slab |z| <= 1, periodic in x and y, plane source at z = 0
    emitting x = 0 isotropically; tau0 is the line-centre depth midplane-to-face."""
    n = (nxy, nxy, nz)
    k0 = np.full(n[0] * n[1] * n[2], tau0 / 1.0)
    return _problem(n, (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0), (PERIODIC, PERIODIC, VACUUM), k0, a,
                    phase=phase,
                    source={"kind": SRC_PLANE, "pos": (0.0, 0.0, 0.0), "profile": PROF_DELTA, "x0": 0.0},
                    tally={"spec_nbins": spec[0], "spec_lo": spec[1], "spec_hi": spec[2]})


def dusty_slab(tau0=1e5, a=0.015, tau_a=0.03, nz=64, nxy=1, spec=(200, -60.0, 60.0)):
    """Static slab |z| <= 1, periodic in x and y, grey (dust) absorption depth
    tau_a from midplane to face, plane source at z = 0 emitting x = 0 photons
    isotropically (the dusty-slab setup of Sec. 3.2).  tau0 is the depth in the
    convention of the analytic escape fraction (Neufeld's), the mean depth
    sqrt(pi) k0 of the normalised profile, as for the paper's other slab
    depths in Sec. 3; the line-centre opacity is k0 = tau0 / sqrt(pi)."""
    p = slab(tau0 / np.sqrt(np.pi), a, nz, spec=spec, nxy=nxy)
    p["grid"]["kabs"] = np.full(nxy * nxy * nz, tau_a, dtype=np.float32)
    return p


def slab_c0():
    """1x1x32 slab, tau0 = 1e3, a = 1e-2, isotropic phase, 200 bins over [-30, 30]."""
    return slab(1e3, 1e-2, 32)


def sphere(n=64, tau0=1e6, a=4.7e-4, *, phase=PHASE_DIPOLE, spec=(256, -80.0, 80.0),
           emis=(32, -24.0, 24.0), vmax=0.0, source="point", jbar=False):
    """Uniform sphere of radius 1 in [-1, 1]^3 (cells with centre radius <= 1),
    line-centre radial depth tau0; optional homologous velocity v = vmax * r."""
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    nn = (n, n, n)
    x, y, z = _cell_centres(nn, lo, hi)
    r = np.sqrt(x * x + y * y + z * z)
    inside = r <= 1.0
    k0 = np.where(inside, tau0 / 1.0, 0.0)
    vel = None
    if vmax != 0.0:
        vel = np.stack([vmax * x, vmax * y, vmax * z]) * inside[None, :]
    if source == "point":
        src = {"kind": SRC_POINT, "pos": (0.0, 0.0, 0.0), "profile": PROF_DELTA, "x0": 0.0}
        em = None
    else:
        src = {"kind": SRC_VOLUME, "pos": (0.0, 0.0, 0.0), "profile": PROF_VOIGT, "x0": 0.0}
        em = inside.astype(np.float32)
    tally = {"spec_nbins": spec[0], "spec_lo": spec[1], "spec_hi": spec[2],
             "jbar": int(jbar)}
    if emis is not None:
        tally.update({"emis_nch": emis[0], "ch_lo": emis[1], "ch_hi": emis[2], "n_cam": (1.0, 0.0, 0.0)})
    return _problem(nn, lo, hi, (VACUUM,) * 3, k0, a, vel=vel, emis=em, phase=phase,
                    source=src, tally=tally)


def sphere_c1():
    """64^3 static sphere, tau0 = 1e6, a = 4.7e-4, dipole phase, central point source;
    spectrum 256 bins over [-80, 80]; emissivity 32 channels over [-24, 24], camera +x."""
    return sphere(64, 1e6, 4.7e-4)


def expanding_sphere_c2():
    """128^3 homologously expanding sphere, v = 20 r (Doppler units), tau0 = 1e5,
    a = 1e-3, isotropic R_IIA, uniform volume emission with a Voigt profile;
    spectrum 512 bins over [-64, 64]; emissivity 64 channels over [-40, 40]."""
    return sphere(128, 1e5, 1e-3, phase=PHASE_ISO, spec=(512, -64.0, 64.0), emis=(64, -40.0, 40.0),
                  vmax=20.0, source="volume")


def cube(n=32, tau0=1e3, a=4.73e-3, spec=(200, -20.0, 20.0)):
    """Uniform cube [-1, 1]^3, line-centre depth tau0 centre-to-face, uniform volume
    source with a thermal Gaussian profile (the code-comparison benchmark setup)."""
    nn = (n, n, n)
    k0 = np.full(n ** 3, tau0)
    return _problem(nn, (-1.0,) * 3, (1.0,) * 3, (VACUUM,) * 3, k0, a,
                    emis=np.ones(n ** 3, dtype=np.float32),
                    source={"kind": SRC_VOLUME, "pos": (0.0, 0.0, 0.0), "profile": PROF_GAUSS, "x0": 0.0},
                    tally={"spec_nbins": spec[0], "spec_lo": spec[1], "spec_hi": spec[2]})


def thin_moving_slab(tau=0.01, a=0.01, vz=1.0, nch=32, nx=4):
    """Optically thin slab moving at v_z along +z, lit by a beam of line-centre
    photons along +x entering at the x = -1 face; camera along +z (g = 0).
    tau is the line-centre depth of the 2-unit beam path."""
    n = (nx, 1, 1)
    ncell = nx
    k0 = np.full(ncell, tau / 2.0)
    vel = np.zeros((3, ncell))
    vel[2, :] = vz
    return _problem(n, (-1.0,) * 3, (1.0,) * 3, (VACUUM,) * 3, k0, a, vel=vel,
                    source={"kind": SRC_BEAM, "pos": (-1.0, 0.0, 0.0), "dir": (1.0, 0.0, 0.0),
                            "profile": PROF_DELTA, "x0": 0.0},
                    tally={"spec_nbins": 64, "spec_lo": -8.0, "spec_hi": 8.0,
                           "emis_nch": nch, "ch_lo": -5.0, "ch_hi": 5.0, "n_cam": (0.0, 0.0, 1.0)})


def uniform_thin_sphere(n=32, k0=1e-3, a=1e-2):
    """Optically thin uniformly emitting sphere of radius 1 (mean-intensity pin)."""
    p = sphere(n, k0, a, phase=PHASE_ISO, emis=None, source="volume", jbar=True)
    return p


# ---------------------------------------------------------------- clouds ---
def gaussian_random_field(n, slope=-4.0, seed=2, ncomp=1, solenoidal=False):
    """Periodic Gaussian random field(s) on n^3 with power spectrum P(k) ~ k^slope
    (k = 0 removed), from PCG64 white noise; solenoidal projection for vectors.
    Returns [ncomp, n, n, n] float64 with zero mean."""
    rng = np.random.default_rng(seed)
    k = np.fft.fftfreq(n) * n
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros_like(kk)
    amp[kk > 0] = kk[kk > 0] ** (slope / 2.0)
    comps = []
    for _ in range(ncomp):
        w = rng.standard_normal((n, n, n))
        comps.append(np.fft.fftn(w) * amp)
    if solenoidal and ncomp == 3:
        with np.errstate(invalid="ignore", divide="ignore"):
            kh = [np.where(kk > 0, c / kk, 0.0) for c in (kx, ky, kz)]
        dot = kh[0] * comps[0] + kh[1] * comps[1] + kh[2] * comps[2]
        comps = [comps[i] - kh[i] * dot for i in range(3)]
    out = np.stack([np.real(np.fft.ifftn(c)) for c in comps])
    return out - out.mean(axis=(1, 2, 3), keepdims=True)


def cloud_fields(n=128, sigma_lnrho=1.5, vrms3d=3.0, seed_rho=2, seed_v=3):
    """Lognormal density (GRF, P ~ k^-4, sigma of ln rho = 1.5, mean rho = 1) and a
    solenoidal GRF velocity (P ~ k^-4, 3-D rms 3 in thermal units), x fastest."""
    g = gaussian_random_field(n, -4.0, seed_rho, 1)[0]
    g = g / g.std() * sigma_lnrho
    rho = np.exp(g)
    rho /= rho.mean()
    v = gaussian_random_field(n, -4.0, seed_v, 3, solenoidal=True)
    v *= vrms3d / np.sqrt(np.mean(np.sum(v * v, axis=0)))
    # arrays are [z][y][x] -> flatten with x fastest
    return rho.reshape(-1), v.reshape(3, -1)


def rotor(n_levels=5, a0=1e-3, theta=0.5, seed=4):
    """Synthetic linear rotor: levels J = 0..L-1, g = 2J+1, E_J/kT = theta J(J+1)/2,
    lines J+1 -> J with A = (J+1)^3 (units of A_10), frequencies ~ (J+1), so the
    damping a_l = a0 (l+1)^2 and sigma0_l ~ g_u/g_l; downward collision rate
    coefficients log-uniform over two decades around A_10 (per unit collider
    density), upward by detailed balance inside the solver."""
    rng = np.random.default_rng(seed)
    J = np.arange(n_levels)
    g = 2.0 * J + 1.0
    E = theta * J * (J + 1) / 2.0
    A = np.zeros((n_levels, n_levels))
    for u in range(1, n_levels):
        A[u, u - 1] = float(u) ** 3
    Cd = np.tril(10.0 ** rng.uniform(-1.0, 1.0, (n_levels, n_levels)), -1)
    sigma0 = np.array([(2 * l + 3) / (2 * l + 1) for l in range(n_levels - 1)], dtype=np.float64)
    a = np.array([a0 * (l + 1) ** 2 for l in range(n_levels - 1)], dtype=np.float64)
    return {"E": E, "g": g, "A": A, "Cd": Cd, "sigma0": sigma0, "a": a}


def cloud_c3(n=128, packets_per_line=10_000_000):
    """Turbulent molecular cloud on [0,1]^3 (vacuum faces for packets): density
    and velocity fields, the rotor, collider density = rho, species density
    n_tot = rho * n_scale with n_scale set so that the mean line-0 cell depth
    at collisional equilibrium is 1.  Level populations, opacities and emission
    weights are produced by the level solver itself (krt_levels_update)."""
    rho, v = cloud_fields(n)
    rot = rotor()
    return {"n": [n, n, n], "lo": [0.0, 0.0, 0.0], "hi": [1.0, 1.0, 1.0], "bc": [VACUUM] * 3,
            "rho": rho.astype(np.float64), "vel": v.astype(np.float32), "rotor": rot,
            "ncoll": rho.astype(np.float64), "dx": 1.0 / n, "packets_per_line": packets_per_line}


def cloud_c4(n=128, a=1e-3, tau_p70=1e2, spec=(512, -64.0, 64.0), emis=(32, -16.0, 16.0)):
    """The turbulent cloud rescaled for the learned escape: one line, a = 1e-3,
    eps = 0, density scaled so the 70th percentile of the line-centre cell depth
    k0 dx is 1e2 (30% of cells in [1e2, ~1e5]); Voigt volume emission ~ rho."""
    rho, v = cloud_fields(n)
    dx = 1.0 / n
    k0 = rho * (tau_p70 / np.percentile(rho, 70.0)) / dx
    return _problem((n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (VACUUM,) * 3, k0, a, vel=v,
                    emis=rho.astype(np.float32), phase=PHASE_ISO,
                    source={"kind": SRC_VOLUME, "pos": (0.0, 0.0, 0.0), "profile": PROF_VOIGT, "x0": 0.0},
                    tally={"spec_nbins": spec[0], "spec_lo": spec[1], "spec_hi": spec[2],
                           "emis_nch": emis[0], "ch_lo": emis[1], "ch_hi": emis[2], "n_cam": (1.0, 0.0, 0.0)})
