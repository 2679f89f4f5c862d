"""Per-cell temperature on the GPU (frequencies in units of the local Doppler
width, Sec. 2.1), as classes and as a continuum (Sec. 2.2.1's two-dimensional
Voigt table over log-spaced damping values): exact identities, the Voigt
interpolation against its bound, and moving grids against the FP64 oracle
(which takes the per-cell width directly)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2608_09340_amd import workloads as W
from stats_util import chi2_two_sample

pytestmark = pytest.mark.gpu


def _cube(a, scale, tclass=None, bratio=None, vel=0.0, n=6, tau=40.0, cell_bratio=None):
    c = (np.arange(n) + 0.5) / n * 2 - 1
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    v = None if vel == 0.0 else vel * np.stack([X, Y, Z]).reshape(3, -1)
    p = W._problem((n, n, n), (-1.0,) * 3, (1.0,) * 3, (0, 0, 0), np.full(n ** 3, tau), a, vel=v,
                   emis=np.ones(n ** 3, dtype=np.float32),
                   source={"kind": W.SRC_VOLUME, "pos": (0.0, 0.0, 0.0), "profile": W.PROF_VOIGT, "x0": 0.0},
                   tally={"spec_nbins": 64, "spec_lo": -10.0 * scale, "spec_hi": 10.0 * scale, "emis_nch": 16,
                          "ch_lo": -8.0 * scale, "ch_hi": 8.0 * scale, "n_cam": (1.0, 0.0, 0.0)})
    if tclass is not None:
        p["grid"]["tclass"] = np.asarray(tclass, dtype=np.uint8).reshape(-1)
        p["grid"]["tclass_bratio"] = list(bratio)
    if cell_bratio is not None:
        p["grid"]["bratio"] = np.asarray(cell_bratio, dtype=np.float32).reshape(-1)
    return p


def test_temperature_scaling_bit_identical(gpu_ctx):
    """Every cell at twice the reference Doppler width with damping 2e-3 at the
    reference is the reference-width medium at damping 1e-3 with every
    frequency doubled: the class tables equal the line tables of a = 1e-3 and
    every scaling is by 2 (exact), so spectrum and emissivity (over doubled
    ranges) and the counters are bit-identical."""
    from paper_2608_09340_amd import krt
    n = 6
    TA = krt.Transport(_cube(2e-3, 2.0, tclass=np.zeros(n ** 3), bratio=[2.0]), ctx=gpu_ctx)
    ra = TA.run(300_000, seed=7)
    TB = krt.Transport(_cube(1e-3, 1.0), ctx=gpu_ctx)
    rb = TB.run(300_000, seed=7)
    assert ra["rc"] == 0 and rb["rc"] == 0
    assert np.array_equal(ra["spec_raw"], rb["spec_raw"])
    assert np.array_equal(ra["emis_raw"], rb["emis_raw"])
    assert ra["counters"] == rb["counters"]


def test_three_temperatures_vs_oracle(gpu_ctx):
    """Expanding 6^3 cube (v = 1.5 r) with a cold core (0.5 b_ref), a reference
    shell and a hot rim (2.5 b_ref), Voigt volume source: the GPU's escaped
    spectrum against the oracle's (two-sample chi^2/dof < 1.5, every |z| <
    4.5), and the emissivity per (temperature class, channel) by batch means
    (a packet scatters many times, so emissivity bins are not Poisson): every
    |z| < 4.5 and mean z^2 < 1.6; mean scatterings per packet within 3%."""
    from paper_2608_09340_amd import krt
    n = 6
    c = (np.arange(n) + 0.5) / n * 2 - 1
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2).reshape(-1)
    tcl = np.where(r < 0.6, 0, np.where(r < 1.2, 1, 2))
    p = _cube(2e-3, 1.0, tclass=tcl, bratio=[0.5, 1.0, 2.5], vel=1.5, tau=200.0)
    T = krt.Transport(p, ctx=gpu_ctx)
    g = T.run(1_000_000, seed=0)
    assert g["rc"] == 0 and g["counters"]["status"] == 0
    o = oracle.mc_run(p, 40_000, seed=0, packet_offset=1 << 32)
    chi2, dof, zmax = chi2_two_sample(g["spec_raw"], o["spec"])
    print(f"spectrum chi2/dof {chi2 / dof:.3f} zmax {zmax:.2f}")
    assert chi2 / dof < 1.5 and zmax < 4.5, (chi2, dof, zmax)

    def agg(em):
        em = np.asarray(em, dtype=np.float64).reshape(n ** 3, 16)
        return np.concatenate([em[tcl == k].sum(axis=0) for k in range(3)])

    def batches(run, B):
        v = np.stack([run(b) for b in range(B)])
        return v.mean(axis=0), v.var(axis=0, ddof=1) / B

    Ng, No, B = 50_000, 2_000, 20
    mg, vg = batches(lambda b: agg(T.run(Ng, seed=2, packet_offset=b * Ng)["emis_raw"] * 2.0 ** -20) / Ng, B)
    mo, vo = batches(lambda b: agg(oracle.mc_run(p, No, seed=2, packet_offset=(1 << 30) + b * No)["emis"]) / No, B)
    m = mo > 0.02 * mo.max()
    z = (mg[m] - mo[m]) / np.sqrt(vg[m] + vo[m])
    print(f"emissivity batch means: max|z| {np.max(np.abs(z)):.2f}, mean z^2 {np.mean(z ** 2):.2f} over {m.sum()} bins")
    assert np.max(np.abs(z)) < 4.5 and np.mean(z ** 2) < 1.6
    mgs = g["counters"]["scatterings"] / 1_000_000
    mos = o["counters"]["scatterings"] / 40_000
    assert abs(mgs / mos - 1) < 0.03, (mgs, mos)


def test_classes_refused_with_learned_or_profile_modes(gpu_ctx):
    from paper_2608_09340_amd import krt
    T = krt.Transport(_cube(2e-3, 1.0, tclass=np.zeros(216), bratio=[1.0]), ctx=gpu_ctx)
    with pytest.raises(Exception, match="temperature classes"):
        T.run(1000, seed=0, profile_mode=1)


def test_class_index_out_of_range_refused_at_upload(gpu_ctx):
    """A class index naming no class is refused when the grid is uploaded,
    before any kernel could index the class tables with it."""
    from paper_2608_09340_amd import krt
    tcl = np.zeros(216, dtype=np.uint8)
    tcl[17] = 2
    with pytest.raises(Exception, match="class index"):
        krt.Transport(_cube(2e-3, 1.0, tclass=tcl, bratio=[1.0, 2.0]), ctx=gpu_ctx)


def test_unit_ratio_class_reproduces_plain_walk(gpu_ctx):
    """Every cell in one class of Doppler width b_ref: the class tables equal
    the line tables and every frequency scale is 1, so on a static grid the
    temperature-class transport (its own kernel instance, tables in global
    memory) reproduces the plain walk's tallies bit for bit.  (In a moving
    medium the two instances may contract the frequency update and the n.v
    shift into different fused multiply-adds, so they agree to rounding only;
    the oracle comparison above covers that case.)"""
    from paper_2608_09340_amd import krt
    n = 6
    TA = krt.Transport(_cube(2e-3, 1.0, tclass=np.zeros(n ** 3), bratio=[1.0], tau=200.0), ctx=gpu_ctx)
    ra = TA.run(200_000, seed=11)
    TB = krt.Transport(_cube(2e-3, 1.0, tau=200.0), ctx=gpu_ctx)
    rb = TB.run(200_000, seed=11)
    assert ra["rc"] == 0 and rb["rc"] == 0
    assert np.array_equal(ra["spec_raw"], rb["spec_raw"])
    assert np.array_equal(ra["emis_raw"], rb["emis_raw"])
    assert ra["counters"] == rb["counters"]


def _radius(n=6):
    c = (np.arange(n) + 0.5) / n * 2 - 1
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return np.sqrt(X ** 2 + Y ** 2 + Z ** 2).reshape(-1)


def test_continuum_unit_width_reproduces_plain_walk(gpu_ctx):
    """Every cell at the reference width as a continuum: one Voigt table and
    one sampler table, both the line's own, every frequency scale 1 and the
    upper interpolation weight 0, so on a static grid the continuum kernel
    reproduces the plain walk's tallies bit for bit."""
    from paper_2608_09340_amd import krt
    n = 6
    TA = krt.Transport(_cube(2e-3, 1.0, tau=200.0, cell_bratio=np.ones(n ** 3)), ctx=gpu_ctx)
    ra = TA.run(200_000, seed=11)
    TB = krt.Transport(_cube(2e-3, 1.0, tau=200.0), ctx=gpu_ctx)
    rb = TB.run(200_000, seed=11)
    assert ra["rc"] == 0 and rb["rc"] == 0
    assert np.array_equal(ra["spec_raw"], rb["spec_raw"])
    assert np.array_equal(ra["emis_raw"], rb["emis_raw"])
    assert ra["counters"] == rb["counters"]


def test_continuum_voigt_within_interpolation_bound(gpu_ctx):
    """The opacity of a cell of width r b_ref is H(a / r, x) interpolated
    linearly in ln a between the two of 64 log-spaced damping nodes around it.
    H is a Gaussian core plus a damping part proportional to a, so with node
    spacing D in ln a the interpolation error is at most D^2 / 8 of H (the
    second derivative of e^s over e^s); against the oracle's Faddeeva H at the
    cell's exact damping, widths 0.5..2.5 (D = ln 5 / 63), the error stays
    under that bound plus the tables' own 3e-6, and it is not vacuous: at the
    worst point it exceeds a tenth of the bound."""
    import torch
    from paper_2608_09340_amd import krt
    a = 2e-3
    rng = np.random.default_rng(3)
    br = np.linspace(0.5, 2.5, 216)
    T = krt.Transport(_cube(a, 1.0, cell_bratio=br), ctx=gpu_ctx)
    T._ensure_bound()
    m = 200_000
    r = np.exp(rng.uniform(np.log(0.5), np.log(2.5), m)).astype(np.float32)
    x = np.concatenate([rng.uniform(0.0, 8.0, m // 2), np.exp(rng.uniform(np.log(8.0), np.log(3000.0), m - m // 2))])
    x = x.astype(np.float32)
    out = torch.empty(m, dtype=torch.float32, device="cuda")
    gpu_ctx.krt_debug_voigt_cont(0, torch.from_numpy(r).cuda(), torch.from_numpy(x).cuda(), out)
    got = out.cpu().numpy().astype(np.float64)
    k = 40_000  # the oracle's Faddeeva H at each point's own damping
    ref = np.array([oracle.voigt_H(a / float(ri), float(xi))[0] for ri, xi in zip(r[:k], x[:k])])
    rel = np.abs(got[:k] - ref) / ref
    D = np.log(5.0) / 63
    bound = D * D / 8 + 3e-6
    print(f"continuum Voigt: max rel err {rel.max():.3e} (bound {bound:.3e}) at r {r[np.argmax(rel)]:.4f} "
          f"x {x[np.argmax(rel)]:.3f}")
    assert rel.max() < bound, rel.max()
    assert rel.max() > 0.1 * D * D / 8


def test_continuum_temperature_vs_oracle(gpu_ctx):
    """Expanding 6^3 cube (v = 1.5 r) whose Doppler width rises smoothly from
    0.45 b_ref at the centre to 2.6 b_ref at the corners (every cell its own
    width), Voigt volume source: the GPU's escaped spectrum against the
    oracle's, which takes each cell's exact width (two-sample chi^2/dof < 1.5,
    every |z| < 4.5), and the emissivity per (radial shell, channel) by batch
    means: every |z| < 4.5 and mean z^2 < 1.6; mean scatterings per packet
    within 3%."""
    from paper_2608_09340_amd import krt
    n = 6
    rad = _radius(n)
    br = 0.45 + 2.15 * (rad / rad.max()) ** 1.5
    p = _cube(2e-3, 1.0, vel=1.5, tau=200.0, cell_bratio=br)
    T = krt.Transport(p, ctx=gpu_ctx)
    g = T.run(1_000_000, seed=0)
    assert g["rc"] == 0 and g["counters"]["status"] == 0
    o = oracle.mc_run(p, 40_000, seed=0, packet_offset=1 << 32)
    chi2, dof, zmax = chi2_two_sample(g["spec_raw"], o["spec"])
    print(f"continuum spectrum chi2/dof {chi2 / dof:.3f} zmax {zmax:.2f}")
    assert chi2 / dof < 1.5 and zmax < 4.5, (chi2, dof, zmax)
    shell = np.digitize(rad, [0.6, 1.0, 1.4])

    def agg(em):
        em = np.asarray(em, dtype=np.float64).reshape(n ** 3, 16)
        return np.concatenate([em[shell == k].sum(axis=0) for k in range(4)])

    def batches(run, B):
        v = np.stack([run(b) for b in range(B)])
        return v.mean(axis=0), v.var(axis=0, ddof=1) / B

    Ng, No, B = 50_000, 2_000, 20
    mg, vg = batches(lambda b: agg(T.run(Ng, seed=2, packet_offset=b * Ng)["emis_raw"] * 2.0 ** -20) / Ng, B)
    mo, vo = batches(lambda b: agg(oracle.mc_run(p, No, seed=2, packet_offset=(1 << 30) + b * No)["emis"]) / No, B)
    msk = mo > 0.02 * mo.max()
    z = (mg[msk] - mo[msk]) / np.sqrt(vg[msk] + vo[msk])
    print(f"continuum emissivity batch means: max|z| {np.max(np.abs(z)):.2f}, mean z^2 {np.mean(z ** 2):.2f} "
          f"over {msk.sum()} bins")
    assert np.max(np.abs(z)) < 4.5 and np.mean(z ** 2) < 1.6
    mgs = g["counters"]["scatterings"] / 1_000_000
    mos = o["counters"]["scatterings"] / 40_000
    assert abs(mgs / mos - 1) < 0.03, (mgs, mos)


def test_continuum_refusals(gpu_ctx):
    """Per-cell widths with classes, outside [0.05, 20], with the learned
    escape or a profile mode, or through the no-allocation entry point are
    refused with a message, before any kernel runs."""
    from paper_2608_09340_amd import krt
    with pytest.raises(Exception, match="exclusive"):
        krt.Transport(_cube(2e-3, 1.0, tclass=np.zeros(216), bratio=[1.0], cell_bratio=np.ones(216)), ctx=gpu_ctx)
    bad = np.ones(216)
    bad[5] = 25.0
    with pytest.raises(Exception, match="bratio"):
        krt.Transport(_cube(2e-3, 1.0, cell_bratio=bad), ctx=gpu_ctx)
    T = krt.Transport(_cube(2e-3, 1.0, cell_bratio=np.linspace(0.8, 1.2, 216)), ctx=gpu_ctx)
    with pytest.raises(Exception, match="bratio"):
        T.run(1000, seed=0, profile_mode=1)
    with pytest.raises(Exception, match="noalloc"):
        T.run(1000, seed=0, noalloc=True)
