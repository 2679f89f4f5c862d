"""The seeded synthetic inputs have the structure their recipes state: the
Gaussian random fields' power-law spectra and solenoidal velocity, the
turbulent cloud's lognormal density and velocity normalisation, the learned-
escape cloud's depth percentile, the synthetic rotor's constants and the
uniform sphere's radial depth.  CPU only; small grids."""
from __future__ import annotations

import numpy as np

from paper_2608_09340_amd import workloads as W


def _shell_power(f):
    n = f.shape[0]
    P = np.abs(np.fft.fftn(f)) ** 2
    k = np.fft.fftfreq(n) * n
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    shell = np.rint(np.sqrt(kx * kx + ky * ky + kz * kz)).astype(int)
    ks = np.arange(2, n // 3)
    return ks, np.array([P[shell == s].mean() for s in ks])


def test_grf_power_law_slope_and_zero_mean():
    f = W.gaussian_random_field(48, slope=-4.0, seed=5, ncomp=1)[0]
    assert abs(f.mean()) < 1e-12 * f.std()
    ks, P = _shell_power(f)
    slope = np.polyfit(np.log(ks), np.log(P), 1)[0]
    assert abs(slope + 4.0) < 0.3, slope
    g = W.gaussian_random_field(48, slope=-2.0, seed=5, ncomp=1)[0]
    ks, P = _shell_power(g)
    assert abs(np.polyfit(np.log(ks), np.log(P), 1)[0] + 2.0) < 0.3


def test_solenoidal_velocity_is_divergence_free():
    """k . v(k) = 0 on every mode off the Nyquist planes (there the real part
    of the inverse transform cannot keep the projection)."""
    n = 16
    v = W.gaussian_random_field(n, slope=-4.0, seed=3, ncomp=3, solenoidal=True)
    V = [np.fft.fftn(c) for c in v]
    k = np.fft.fftfreq(n) * n
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    div = kx * V[0] + ky * V[1] + kz * V[2]
    norm = np.sqrt(kx * kx + ky * ky + kz * kz) * np.sqrt(sum(np.abs(c) ** 2 for c in V))
    ok = (np.abs(kx) < n // 2) & (np.abs(ky) < n // 2) & (np.abs(kz) < n // 2) & (norm > 0)
    assert np.max(np.abs(div[ok]) / norm[ok]) < 1e-10
    # and the field is not trivially zero
    assert np.sqrt(np.mean(np.sum(v * v, axis=0))) > 0


def test_cloud_fields_normalisation():
    rho, v = W.cloud_fields(n=32)
    assert rho.shape == (32 ** 3,) and v.shape == (3, 32 ** 3)
    assert np.all(rho > 0)
    assert abs(rho.mean() - 1.0) < 1e-12
    assert abs(np.log(rho).std() - 1.5) < 1e-9          # dividing by the mean only shifts ln rho
    assert abs(np.sqrt(np.mean(np.sum(v * v, axis=0))) - 3.0) < 1e-9


def test_learned_escape_cloud_depth_percentile():
    p = W.cloud_c4(n=32)
    n = p["grid"]["n"][0]
    dx = 1.0 / n
    tau = p["grid"]["k0"].astype(np.float64) * dx
    assert abs(np.percentile(tau, 70.0) / 1e2 - 1.0) < 1e-5
    assert p["line"]["a"] == 1e-3 and p["grid"]["eps"] is None
    rho, _ = W.cloud_fields(n=32)
    # volume emission follows the density, opacity too
    assert np.allclose(p["grid"]["emis"], rho.astype(np.float32))
    assert np.allclose(tau / rho, tau[0] / rho[0], rtol=1e-5)


def test_rotor_constants():
    r = W.rotor(n_levels=5, a0=1e-3, theta=0.5)
    J = np.arange(5)
    assert np.array_equal(r["g"], 2 * J + 1)
    assert np.allclose(r["E"], 0.5 * J * (J + 1) / 2)
    A = r["A"]
    for u in range(5):
        for l in range(5):
            assert A[u, l] == (float(u) ** 3 if l == u - 1 else 0.0)
    Cd = r["Cd"]
    assert np.all(np.triu(Cd) == 0.0)
    low = Cd[np.tril_indices(5, -1)]
    assert np.all((low >= 0.1) & (low <= 10.0))
    assert np.allclose(r["a"], 1e-3 * (np.arange(4) + 1) ** 2)
    assert np.allclose(r["sigma0"], r["g"][1:] / r["g"][:-1])


def test_uniform_sphere_radial_depth():
    n, tau0 = 32, 1e3
    p = W.sphere(n, tau0, 1e-3)
    k0 = p["grid"]["k0"].reshape(n, n, n).astype(np.float64)   # [z][y][x]
    assert set(np.unique(k0)) == {0.0, tau0}
    dx = 2.0 / n
    inside = (k0 > 0).sum() * dx ** 3
    assert abs(inside / (4.0 / 3.0 * np.pi) - 1.0) < 0.03
    # along +x from the centre (the row next to the centre point): tau0 within one cell
    row = k0[n // 2, n // 2, n // 2:]
    assert abs(row.sum() * dx - tau0) <= tau0 * dx
