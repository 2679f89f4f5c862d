"""Lambda iteration on a turbulent cloud (multi-level rotor, 4 lines): the
GPU's mean-intensity tally against the oracle (batch means on aggregated
blocks), the GPU level solve against the oracle's solve of the same system,
and the invariants of the iteration."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2608_09340_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lam(gpu_ctx):
    from paper_2608_09340_amd.lambda_iter import LambdaIteration
    cloud = W.cloud_c3(n=32)
    return LambdaIteration(cloud, gpu_ctx)


def _blocks(v, n, b=4):
    f = n // b
    return v.reshape(b, f, b, f, b, f).sum(axis=(1, 3, 5)).reshape(-1)


def test_jbar_line0_vs_oracle(lam):
    """First formal solution of line 0 (collisional-equilibrium opacities, frozen
    emission, destruction eps): per-packet J-bar sums in 4^3 blocks, GPU vs oracle."""
    nc = lam.ncell
    prob = {"grid": {"n": lam.cloud["n"], "lo": lam.cloud["lo"], "hi": lam.cloud["hi"], "bc": lam.cloud["bc"],
                     "k0": lam.k0[:nc].cpu().numpy(), "vel": lam.vel.cpu().numpy(),
                     "eps": lam.eps[:nc].cpu().numpy(), "emis": lam.emis[:nc].cpu().numpy()},
            "line": {"a": float(lam.rot["a"][0]), "phase": 0},
            "source": {"kind": 2, "profile": 1},
            "tally": {"spec_nbins": 64, "spec_lo": -16.0, "spec_hi": 16.0, "jbar": 1}}
    B, Ng, No = 16, 50000, 2500
    jg, jo = [], []
    for b in range(B):
        lam.transport_line(0, Ng, seed=21, packet_offset=b * Ng)
        jg.append(_blocks(lam.jraw.cpu().numpy() * 2.0 ** -36, 32) / Ng)
        r = oracle.mc_run(prob, No, seed=21, packet_offset=(1 << 30) + b * No)
        jo.append(_blocks(r["jbar"], 32) / No)
    jg, jo = np.array(jg), np.array(jo)
    z = (jg.mean(0) - jo.mean(0)) / np.sqrt(jg.var(0, ddof=1) / B + jo.var(0, ddof=1) / B + 1e-300)
    m = jo.mean(0) > 1e-3 * jo.mean(0).max()
    assert np.max(np.abs(z[m])) < 4.5, np.max(np.abs(z[m]))


def test_lambda_iteration_levels(lam):
    """Three cycles: populations positive and summing to n_tot; the GPU FP64
    level solve equals the oracle's solve of the same rate equations with the
    GPU's mean intensities (1e-9 relative)."""
    hist = lam.iterate(3, 200_000, seed=5)
    assert all(rc == 0 for h in hist for rc in h["rc"]), hist
    nc, nl = lam.ncell, lam.nl
    P = lam.pops.cpu().numpy().reshape(nc, nl)
    nt = lam.ntot.cpu().numpy()
    assert np.all(P > 0)
    assert np.allclose(P.sum(1), nt, rtol=1e-10)
    jb = lam.jbar.cpu().numpy().reshape(nl - 1, nc).astype(np.float64)
    s0 = lam.rot["sigma0"]
    gamma = 4 * np.pi * np.sqrt(np.pi) * s0[:, None] * jb
    ref = oracle.levels_solve(lam.rot["E"], lam.rot["g"], lam.rot["A"], lam.rot["Cd"],
                              lam.ncoll.cpu().numpy(), nt, gamma=gamma)
    assert np.max(np.abs(P - ref) / np.abs(ref)) < 1e-9
    k0 = lam.k0.cpu().numpy().reshape(nl - 1, nc)
    assert np.allclose(k0, (P[:, :nl - 1] * s0[None, :]).T, rtol=1e-6)
    assert hist[-1]["max_rel_change"] < hist[0]["max_rel_change"] * 1.5


@pytest.mark.parametrize("nl", [2, 3, 4, 5, 6, 7, 8])
def test_level_solve_every_level_count(gpu_ctx, nl):
    """The level solve at every level count the library accepts (a kernel
    instance per count, its matrices in registers), on 3000 cells with
    collision rates over six decades and mean intensities over four: the
    populations equal the oracle's solve of the same rate equations, sum to
    n_tot, and give k0 = n_l sigma0.  The two eliminations round in different
    orders; their difference is of order the machine epsilon times the
    largest entries (so times n_tot) in absolute terms, which at eight levels
    is up to 2e-8 of the smallest populations (4e-9 of n_tot): the bound is
    1e-9 relative plus 1e-13 n_tot absolute."""
    import torch
    from paper_2608_09340_amd import krt
    rng = np.random.default_rng(100 + nl)
    nc = 3000
    j = np.arange(nl, dtype=np.float64)
    E = 0.4 * j * (j + 1)                     # rotor ladder in units of kT
    g = 2 * j + 1
    A = np.zeros((nl, nl))
    Cd = np.zeros((nl, nl))
    for u in range(1, nl):
        A[u, u - 1] = 1e-2 * u ** 3
        for l in range(u):
            Cd[u, l] = 3e-3 / (u - l)
    s0 = rng.uniform(0.5, 2.0, nl - 1)
    ncoll = 10.0 ** rng.uniform(-2, 4, nc)
    ntot = rng.uniform(0.5, 2.0, nc)
    jbar = (10.0 ** rng.uniform(-3, 1, (nl - 1, nc))).astype(np.float32)
    keep = [np.ascontiguousarray(v, dtype=np.float64).reshape(-1) for v in (E, g, A, Cd, s0)]
    nc_d = torch.from_numpy(ncoll).cuda()
    nt_d = torch.from_numpy(ntot).cuda()
    jb_d = torch.from_numpy(jbar).cuda()
    pops = torch.zeros(nc * nl, dtype=torch.float64, device="cuda")
    k0 = torch.zeros((nl - 1) * nc, dtype=torch.float32, device="cuda")
    eps = torch.zeros((nl - 1) * nc, dtype=torch.float32, device="cuda")
    d = krt.krt_levels_desc()
    d.n_levels, d.ncell = nl, nc
    d.E, d.g, d.A, d.Cd, d.sigma0 = [k.ctypes.data for k in keep]
    d.ncoll_dev, d.ntot_dev, d.pops_dev = nc_d.data_ptr(), nt_d.data_ptr(), pops.data_ptr()
    d.k0_out_dev, d.eps_out_dev = k0.data_ptr(), eps.data_ptr()
    gpu_ctx.krt_levels_update(d, jb_d)
    P = pops.cpu().numpy().reshape(nc, nl)
    gamma = 4 * np.pi * np.sqrt(np.pi) * s0[:, None] * jbar.astype(np.float64)
    ref = oracle.levels_solve(E, g, A, Cd, ncoll, ntot, gamma=gamma)
    assert np.all(P > 0)
    assert np.allclose(P.sum(1), ntot, rtol=1e-10)
    assert np.all(np.abs(P - ref) <= 1e-9 * np.abs(ref) + 1e-13 * ntot[:, None]), np.max(np.abs(P - ref) / np.abs(ref))
    e = eps.cpu().numpy()
    assert np.allclose(k0.cpu().numpy().reshape(nl - 1, nc), (P[:, :nl - 1] * s0[None, :]).T, rtol=1e-6)
    assert np.all((e > 0) & (e < 1))


def test_frozen_source_and_line_powers(lam):
    """krt_levels_update's emission output is n_u A_ul of its own populations
    (binary32 rounding), and its line powers equal the cell volume times the
    FP64 sum of n_u A_ul over the oracle's collisional-equilibrium solve of
    the same cells (1e-9 relative): the Lambda iteration's frozen source
    (Sec. 2.1.3) comes from the library, not from host arithmetic."""
    nc, nl = lam.ncell, lam.nl
    P0 = lam.pops0.cpu().numpy().reshape(nc, nl)
    A = lam.rot["A"]
    em = lam.emis.cpu().numpy().reshape(nl - 1, nc)
    for l in range(nl - 1):
        want = (P0[:, l + 1] * A[l + 1, l]).astype(np.float32)
        assert np.array_equal(em[l], want), l
    ref = oracle.levels_solve(lam.rot["E"], lam.rot["g"], A, lam.rot["Cd"], lam.ncoll.cpu().numpy(),
                              lam.ntot.cpu().numpy())
    for l in range(nl - 1):
        lum = lam.vcell * np.sum(ref[:, l + 1] * A[l + 1, l])
        assert abs(lam.lum[l] / lum - 1) < 1e-9, (l, lam.lum[l], lum)
