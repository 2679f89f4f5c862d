"""Benchmark of the Monte Carlo line-transfer pass on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--packets N] [--budget-s S]
                    [--legs c0,c1,c2,c3,profile,cube]

Headline workload: the turbulent cloud (128^3, lognormal density with
sigma_ln rho = 1.5 from a P(k) ~ k^-4 Gaussian random field, solenoidal
P(k) ~ k^-4 velocity of 3-D rms 3 v_th), density scaled so 30% of cells have a
line-centre depth k0 dx in [1e2, ~1e5], one line a = 1e-3, Voigt volume source
proportional to density, escaped spectrum 512 bins on [-64, 64), emissivity
128^3 x 32 channels on [-16, 16) toward +x, 1e8 packets per step.

Before the timed region (not counted): the escape network is trained on the
GPU from single-cell escapes the plain walk records, and the same workload is
run twice with the plain random walk (packet ranges [0, N) and [2^40, 2^40+N))
for the reference tallies, the plain throughput and the plain-vs-plain noise
floor.  A step is one krt_mc_run of N packets with the learned escape
(emission, flights, resonant scatterings, network calls in thick cells, int64
tallies, FP32 finalise), inputs resident in HBM; step s runs packets
[2^41 + s N, 2^41 + (s+1) N).  `value` is scatterings-equivalent per second:
the plain walk's scatterings for N packets of this workload per learned step
time.  The tallies stay in HBM during the timed steps; those of the last one
are read back afterwards and compared with the plain ones (spectrum and
emissivity L1, emissivity total).

The timed loop stops starting steps once the next one would end past
--budget-s (warmup likewise past --warmup-budget-s): `steps` and `warmup` in
the JSON line are the steps actually run.

Prints one JSON line as soon as the headline is done: roofline of the learned
transport kernel (HIP-event duration from the library), and the FP64 CPU oracle
timed on a bounded sample of the same workload with the plain walk.  Optional
legs (--legs) run after that line and print a second JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue slots per scattering of the plain transport, from the step list of
# the method (one flight segment ending in an interaction, one resonant
# scattering, its tallies).  Quarter-rate instructions (32x32->64 integer
# multiply, transcendental) cost 4 slots; the terms of each item are listed
# beside it.
LEDGER = {
    "philox_2_blocks": 2 * 10 * (2 * 4 + 4),     # 2 wide multiplies + 4 xor/add per round
    "uniform_maps_8": 8 * 3,
    "flight": 3 + 2 + 7 + 1 + 3 * (4 + 3) + 4 + 2 + (4 + 1) + 3 * 4,  # gas frame, Voigt, DDA, step, move
    "tau_log": 4 + 1,
    "upar_sampler": 12 + 15 + 8 + (4 + 4 + 4 + 3) + 4,  # pieces, row/node, bilinear, tan, sqrt map
    "box_muller": 4 + 4 + 4 + 4 + 2,
    "direction": 2 + 8 + 12 + 12 + (6 + 4),         # g, sincos psi, basis, rotate, renormalise
    "frequency_update": 6 + 3,
    "counters": 3,
}
LEDGER_DIPOLE = 4 * 4 + 6          # log, sqrt, exp, rcp of the dipole inversion + FMAs
LEDGER_EMIS = 6 + 5 + 8 + 3 + 2 + 8  # camera projection, x_cam, channel, phase weight, fixed point, cache
# VALU issue slots of one network call of the learned escape for its asking
# lane (the matrix products run on the matrix cores and count as FLOP):
LEDGER_CALL = {
    "philox_2_blocks": 2 * 10 * (2 * 4 + 4),                 # the call's draws
    "frame_condition": 20 + 2 * 4 + 10,                      # sorted |offsets|, two log10, reduced direction
    "inputs_2_evals": 2 * (24 * 2 + 4 * (4 + 4) + 14),       # normalise, logit levels (log, rcp), bf16 + residuals
    "hidden_epilogues_2_evals": 2 * 3 * 128 * 5 // 2,        # leaky ReLU (mul, median) + bf16 pair per value
    "outputs": 23 * 2,                                       # de-normalise the outputs read
    "face_side_xabs": 6 * (4 + 2) + 4 * 2 + 6,               # softmax, face and side choices, |x| of the face
    "exit_geometry": 2 * (4 + 4 + 2) + 4 + 2 * 4 + 40,       # sinh x2, sqrt, sincos alpha, back to the cell frame
    "deposit": 6 * (2 * 4 + 10 + 12 + 4) + 2 * 4 + 2 * 26,   # ~6 channels within 3 sd: erf (rcp, exp, poly), int64,
                                                             # atomic; two more erf for the coverage
}
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12  # 39.32 T lane-slots/s (non-packed 32-bit VALU)
PEAK_MFMA_BF16_TFLOPS = 2500.0            # dense BF16 matrix cores


def ledger_per_scatter(dipole: bool, emis: bool) -> int:
    return sum(LEDGER.values()) + (LEDGER_DIPOLE if dipole else 0) + (LEDGER_EMIS if emis else 0)


# Sources compiled into the transport kernels; HBM traffic measured by the
# profiler is reported only while these are byte-identical to the ones the
# counters were taken on.
KERNEL_SOURCES = ["krt_transport.hip", "krt_device.h", "krt_kernels.h", "krt_mlp.h", "krt_internal.h"]
PROFILES = os.path.join(ROOT, "profiles")
PROFILE_SUMMARY = os.path.join(PROFILES, "mc_transport_sphere64.md")
PROFILE_SUMMARY_LEARNED = os.path.join(PROFILES, "mc_transport_learned_cloud128.md")


def kernel_source_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_09340_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_traffic(path=None, packets=None):
    """HBM bytes per launch from a committed counter summary, or None when the
    kernel sources changed since it was taken.  A summary taken at fewer
    packets than the timed launch gives bytes per packet (the transport's
    traffic is per packet: its tallies and field gathers), scaled to `packets`."""
    path = path or PROFILE_SUMMARY
    try:
        kv = {}
        for line in open(path):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
        if kv.get("kernel_source_sha256") != kernel_source_sha256():
            return None
        if packets is not None and "hbm_bytes_per_packet" in kv:
            return float(kv["hbm_bytes_per_packet"]) * packets
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_info():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(prob, seconds_target=20.0, workload=""):
    """The FP64 oracle as it stands, on the host's cores (at most 16 threads,
    one GPU's share of a shared host), on a bounded sample of the same workload with the plain walk:
    consecutive batches of packets, each sized from the rate so far, until
    about `seconds_target` seconds of oracle work have run."""
    import oracle
    model, ncpu = cpu_info()
    threads = max(1, min(ncpu, 16))
    n_done, sc, dt = 0, 0, 0.0
    n = 4 * threads  # first batch: a few packets per thread to measure the rate
    while dt < 0.75 * seconds_target:
        t = time.perf_counter()
        r = oracle.mc_run(prob, n, seed=0, packet_offset=(1 << 42) + n_done, threads=threads)
        dt += time.perf_counter() - t
        sc += r["counters"]["scatterings"]
        n_done += n
        rate = n_done / max(dt, 1e-3)
        n = int(max(threads, min(4096 * threads, rate * (seconds_target - dt))))
    log(f"cpu baseline: {n_done} packets in {dt:.1f} s")
    return {"value": sc / dt, "unit": "scatterings/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_done} packets (ids from 2^42, seed 0) of {workload}, plain walk, {sc} scatterings, "
                      f"{dt:.1f} s on {threads} threads of {model}",
            "packets_per_s": n_done / dt}


def _agg_blocks(em, n, b=8):
    nch = em.shape[1]
    f = n // b
    return em.reshape(b, f, b, f, b, f, nch).sum(axis=(1, 3, 5)).reshape(-1)


def _l1(u, v):
    import numpy as np
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    return float(np.abs(u - v).sum() / u.sum())


C4_WORKLOAD = ("turbulent cloud 128^3 (lognormal density sigma_ln rho = 1.5 from a P(k)~k^-4 random field, "
               "solenoidal P(k)~k^-4 velocity rms 3 v_th), density scaled so 30% of cells have line-centre "
               "depth k0 dx in [1e2, ~1e5]; a = 1e-3, isotropic phase, Voigt volume source ~ density; "
               "spectrum 512 bins [-64, 64), emissivity 128^3 x 32 channels [-16, 16) toward +x")


def headline_c4(ctx, args):
    """Plain vs learned escape on the cloud: training and plain references
    before the timed region, then timed learned steps."""
    import numpy as np
    import torch
    from paper_2608_09340_amd import krt, workloads as W
    from paper_2608_09340_amd.escape import train_escape, DEFAULT_RUN, DEFAULT_LOG10_TAU, DEFAULT_STAGES
    N = args.packets
    prob = W.cloud_c4(n=128)
    t0 = time.perf_counter()
    krt.Transport(W.slab(10.0, 1e-3, 4), ctx=ctx)  # line tables for a = 1e-3
    stages = tuple((max(1, int(round(st * args.train_scale))), b, lr) for st, b, lr in DEFAULT_STAGES)
    tr = train_escape(ctx, 0, seed=1, log10_tau=DEFAULT_LOG10_TAU, stages=stages)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    hist = tr["hist"]
    del tr
    log(f"escape network trained in {t_train:.1f} s")
    T = krt.Transport(prob, ctx=ctx)
    pa = T.run(N, seed=0)
    ms_plain = ctx.krt_last_transport_ms()
    log(f"plain reference: {ms_plain:.0f} ms")
    pb = T.run(N, seed=0, packet_offset=1 << 40)
    ms_plain2 = ctx.krt_last_transport_ms()
    log(f"plain repeat: {ms_plain2:.0f} ms")
    if pa["rc"] or pb["rc"]:
        raise RuntimeError("plain reference runs failed")
    ea, eb = (_agg_blocks(r["emis_raw"].astype(np.float64), 128) for r in (pa, pb))
    scat_plain = pa["counters"]["scatterings"]
    run_kw = dict(DEFAULT_RUN)

    # the tallies stay on the device during the timed steps; the last step's are
    # read back after the timed region for the comparison with the plain walk
    def step(s):
        r = T.run(N, seed=0, packet_offset=(1 << 41) + s * N, escape_mode=1, host=False, **run_kw)
        if r["rc"]:
            raise RuntimeError(f"learned step failed rc={r['rc']} counters={r['counters']}")
        return r, ctx.krt_last_transport_ms()

    warm = 0
    tw = time.perf_counter()
    while warm < args.warmup:
        step(-1 - warm)
        warm += 1
        if time.perf_counter() - tw > args.warmup_budget_s:
            break
    torch.cuda.synchronize()
    runs, kms = [], []
    t_start = time.perf_counter()
    while len(runs) < args.steps:
        r, ms = step(len(runs))
        runs.append(r)
        kms.append(ms)
        log(f"timed step {len(runs) - 1}: learned {ms:.0f} ms")
        el = time.perf_counter() - t_start
        if el + el / len(runs) > args.budget_s:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    K = len(runs)
    c = runs[-1]["counters"]
    spec_last = T.spec_raw.cpu().numpy()
    em = _agg_blocks(T.emis_raw.cpu().numpy().reshape(T.ncell, T.nch).astype(np.float64), 128)
    km = sum(kms) / K
    # roofline of the learned transport kernel: the scatterings it still walks
    # and its network calls on the VALU ledgers, network products on the BF16
    # matrix cores
    calls = sum(r["counters"]["mlp_calls"] for r in runs) / K
    scat_l = sum(r["counters"]["scatterings"] for r in runs) / K
    ops_call = sum(LEDGER_CALL.values())
    valu = (scat_l * ledger_per_scatter(False, True) + calls * ops_call) / (km * 1e-3) / 1e12
    mfma = calls * 2 * MLP_FLOP_PER_EVAL / (km * 1e-3) / 1e12
    return {
        "value": scat_plain * K / wall, "K": K, "W": warm, "wall": wall,
        "kernel_ms": km,
        "roofline": {"bound": "alu", "achieved": valu, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                     "frac": valu / PEAK_VALU_TOPS, "traffic": profiled_traffic(PROFILE_SUMMARY_LEARNED, N),
                     "kernel": "mc_transport_kernel<1, 512> (learned escape, fused)",
                     "ops_per_scattering": ledger_per_scatter(False, True), "ops_per_call": ops_call,
                     "mfma": {"achieved": mfma, "peak": PEAK_MFMA_BF16_TFLOPS, "unit": "TFLOP/s",
                              "frac": mfma / PEAK_MFMA_BF16_TFLOPS,
                              "flop_per_call": 2 * MLP_FLOP_PER_EVAL}},
        "learned": {
            "plain_kernel_ms": ms_plain, "plain_kernel_ms_repeat": ms_plain2,
            "plain_scatterings": scat_plain, "plain_scatterings_per_s": scat_plain / (ms_plain * 1e-3),
            "learned_kernel_ms": km, "learned_kernel_ms_steps": kms,
            "speedup_kernel": ms_plain / km,
            "scatterings_equivalent_per_s_kernel": scat_plain / (km * 1e-3),
            "learned_scatterings_run": c["scatterings"], "network_calls": c["mlp_calls"],
            "skipped_scatterings": c["skipped_scatterings"],
            "spectrum_L1": _l1(pa["spec_raw"], spec_last),
            "spectrum_L1_floor": _l1(pa["spec_raw"], pb["spec_raw"]),
            "emissivity_L1": _l1(ea, em), "emissivity_L1_floor": _l1(ea, eb),
            "emissivity_total_ratio": float(em.sum() / ea.sum()),
            "L1_definition": "sum |x - plain| / sum plain over the 514 spectrum bins and over 8^3 blocks x 32 "
                             "channels of emissivity; the last timed learned step (packets 2^41 + (K - 1) N + [0, N)) "
                             "against plain (packets [0, N)); floor = plain [0, N) against plain 2^40 + [0, N)",
            "train_s": t_train, "train_loss_first_last": [float(hist[:5].mean()), float(hist[-200:].mean())],
            "run_options": run_kw,
        },
        "prob": prob,
    }


MLP_FLOP_PER_EVAL = 2 * (24 * 128 + 128 * 128 + 128 * 128 + 128 * 32)  # one sample through 24->3x128->32


def sphere_c1_leg(ctx, packets=1_000_000):
    """64^3 static sphere (tau0 = 1e6, a = 4.7e-4, dipole, central point source,
    256-bin spectrum, 64^3 x 32-channel emissivity): one plain transport of
    `packets` packets with its VALU roofline, then the imaging pass."""
    from paper_2608_09340_amd import krt, workloads as W
    prob = W.sphere_c1()
    T = krt.Transport(prob, ctx=ctx)
    r = T.run(packets, seed=0)
    ms = ctx.krt_last_transport_ms()
    if r["rc"]:
        raise RuntimeError("sphere leg failed")
    c = r["counters"]
    lps = ledger_per_scatter(True, True)
    ach = c["scatterings"] * lps / (ms * 1e-3) / 1e12
    log(f"static sphere: {ms:.0f} ms")
    T.image(axis=0)
    im = []
    for _ in range(5):
        T.image(axis=0)
        im.append(ctx.krt_last_image_ms())
    nx, ny, nz = T.n
    nb = T.ncell * T.nch * 4 + T.ncell * 4 + ny * nz * T.nch * 4  # emissivity, k0 (static), image
    t_im = min(im) * 1e-3
    return {"workload": "static uniform sphere 64^3, radial line-centre tau0=1e6, a=4.7e-4, dipole phase, "
                        "central point source x=0, spectrum 256 bins [-80,80), emissivity 64^3 x 32 channels "
                        f"[-24,24) toward +x, plain random walk, {packets} packets",
            "kernel_ms": ms, "scatterings": c["scatterings"], "scatterings_per_s": c["scatterings"] / (ms * 1e-3),
            "packets_per_s": packets / (ms * 1e-3),
            "mean_scatterings_per_packet": c["scatterings"] / packets,
            "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                         "frac": ach / PEAK_VALU_TOPS, "traffic": profiled_traffic(PROFILE_SUMMARY),
                         "ops_per_scattering": lps},
            "imaging": {"what": f"image toward +x, {ny}x{nz} pixels x {T.nch} channels", "kernel_ms": min(im),
                        "roofline": {"bound": "hbm", "achieved": nb / t_im / 1e9, "peak": 8000.0, "unit": "GB/s",
                                     "frac": nb / t_im / 8e12, "bytes_per_launch": nb}}}


def slab_c0_leg(ctx, packets=10_000):
    """1x1x32 static slab, tau0 = 1e3, a = 1e-2, plane source at x = 0, 200 bins."""
    from paper_2608_09340_amd import krt, workloads as W
    T = krt.Transport(W.slab_c0(), ctx=ctx)
    T.run(packets, seed=0, packet_offset=1 << 40)
    r = T.run(packets, seed=0)
    ms = ctx.krt_last_transport_ms()
    if r["rc"]:
        raise RuntimeError("slab leg failed")
    c = r["counters"]
    return {"workload": f"static slab 1x1x32, tau0=1e3, a=1e-2, isotropic, plane source x=0, {packets} packets",
            "kernel_ms": ms, "scatterings": c["scatterings"], "mean_scatterings_per_packet": c["scatterings"] / packets,
            "scatterings_per_s": c["scatterings"] / (ms * 1e-3), "packets_per_s": packets / (ms * 1e-3)}


def expanding_sphere_leg(ctx, packets=10_000_000):
    """128^3 homologously expanding sphere (v = 20 r, tau0 = 1e5, a = 1e-3, isotropic
    R_IIA, Voigt volume source; 512-bin spectrum, 128^3 x 64-channel emissivity)."""
    from paper_2608_09340_amd import krt, workloads as W
    T = krt.Transport(W.expanding_sphere_c2(), ctx=ctx)
    r = T.run(packets, seed=0)
    ms = ctx.krt_last_transport_ms()
    if r["rc"]:
        raise RuntimeError("expanding-sphere leg failed")
    c = r["counters"]
    log(f"expanding sphere: {ms:.0f} ms")
    T.image(axis=0)
    im = []
    for _ in range(3):
        T.image(axis=0)
        im.append(ctx.krt_last_image_ms())
    nb = T.ncell * T.nch * 4 + T.ncell * 8 + T.n[1] * T.n[2] * T.nch * 4  # emissivity, k0 + v_x, image
    t_im = min(im) * 1e-3
    lps = ledger_per_scatter(False, True)
    ach = c["scatterings"] * lps / (ms * 1e-3) / 1e12
    return {"workload": "expanding sphere 128^3, v = 20 r, tau0=1e5, a=1e-3, isotropic R_IIA, Voigt volume "
                        f"source, spectrum 512 bins, emissivity 128^3 x 64 channels, {packets} packets",
            "kernel_ms": ms, "scatterings": c["scatterings"], "scatterings_per_s": c["scatterings"] / (ms * 1e-3),
            "packets_per_s": packets / (ms * 1e-3), "crossings": c["crossings"],
            "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                         "frac": ach / PEAK_VALU_TOPS, "ops_per_scattering": lps},
            "imaging": {"what": "image toward +x, 128x128 pixels x 64 channels", "kernel_ms": min(im),
                        "roofline": {"bound": "hbm", "achieved": nb / t_im / 1e9, "peak": 8000.0, "unit": "GB/s",
                                     "frac": nb / t_im / 8e12, "bytes_per_launch": nb}}}


def profile_mode_leg(ctx, packets=10_000_000):
    """The paper's opacity-profile modes as an A/B on the expanding sphere:
    tables in LDS (production), the same tables read from global memory
    (identical tallies; the cost of the table placement), and the analytic
    blended profile (the exact redistribution with an inconsistent opacity:
    its spectrum L1 against the tabulated profile)."""
    import numpy as np
    from paper_2608_09340_amd import krt, workloads as W
    T = krt.Transport(W.expanding_sphere_c2(), ctx=ctx)
    res, spec = {}, {}
    for name, mode in (("lds_tables", 0), ("global_tables", 1), ("analytic_profile", 2)):
        r = T.run(packets, seed=0, profile_mode=mode)
        if r["rc"]:
            raise RuntimeError(f"profile mode {mode} failed")
        res[name] = {"kernel_ms": ctx.krt_last_transport_ms(), "scatterings": r["counters"]["scatterings"]}
        spec[name] = r["spec_raw"].astype(np.float64)
        log(f"profile mode {mode}: {res[name]['kernel_ms']:.0f} ms")
    s0 = spec["lds_tables"]
    res["global_tables"]["identical_spectrum"] = bool(np.array_equal(s0, spec["global_tables"]))
    res["analytic_profile"]["spectrum_L1_vs_tables"] = float(np.abs(spec["analytic_profile"] - s0).sum() / s0.sum())
    res["workload"] = f"expanding sphere 128^3 (as above), {packets} packets, seed 0"
    return res


def lambda_leg(ctx, n=128, packets=10_000_000, iterations=10):
    """Lambda iteration on the 128^3 turbulent cloud with the 5-level rotor:
    `iterations` cycles of transport of each of the 4 lines with the
    mean-intensity tally, then the FP64 level solve of every cell."""
    import torch
    from paper_2608_09340_amd import workloads as W
    from paper_2608_09340_amd.lambda_iter import LambdaIteration
    lam = LambdaIteration(W.cloud_c3(n=n), ctx)
    torch.cuda.synchronize()
    t = time.perf_counter()
    hist = lam.iterate(iterations, packets, seed=0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    if any(any(h["rc"]) for h in hist):
        raise RuntimeError("lambda leg failed")
    log(f"lambda iteration: {iterations} cycles in {wall:.1f} s")
    return {"workload": f"turbulent cloud {n}^3, 5-level rotor, 4 lines, {packets} packets per line per cycle, "
                        f"{iterations} cycles of transport + FP64 level solve",
            "wall_s": wall, "transport_kernel_ms_per_cycle": [h["kernel_ms"] for h in hist],
            "level_solve_ms_per_cycle": [h.get("levels_ms") for h in hist],
            "max_rel_change_per_cycle": [h["max_rel_change"] for h in hist],
            "scatterings_per_cycle": [h["scatterings"] for h in hist], "cells": lam.ncell}


def cube_context_leg(ctx, packets=(1_000, 10_000, 100_000, 1_000_000, 10_000_000)):
    """The paper's code-comparison cube (32^3, line-centre tau0 = 1e3 centre to
    face, a = 4.73e-3, uniform volume source with a thermal Gaussian profile):
    kernel time and scatterings per packet at the paper's packet counts, so
    its packets/s can be turned into scatterings/s (context only)."""
    from paper_2608_09340_amd import krt, workloads as W
    T = krt.Transport(W.cube(), ctx=ctx)
    out = []
    for n in packets:
        r = T.run(n, seed=0)
        ms = ctx.krt_last_transport_ms()
        if r["rc"]:
            raise RuntimeError("cube leg failed")
        c = r["counters"]
        out.append({"packets": n, "kernel_ms": ms, "scatterings": c["scatterings"],
                    "mean_scatterings_per_packet": c["scatterings"] / n,
                    "packets_per_s": n / (ms * 1e-3), "scatterings_per_s": c["scatterings"] / (ms * 1e-3)})
        log(f"cube {n} packets: {ms:.1f} ms")
    return {"workload": "uniform cube 32^3, tau0=1e3, a=4.73e-3, volume source, Gaussian profile, plain walk",
            "runs": out}


LEGS = {"c0": slab_c0_leg, "c1": sphere_c1_leg, "c2": expanding_sphere_leg, "c3": lambda_leg,
        "profile": profile_mode_leg, "cube": cube_context_leg}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed learned steps (at most; see --budget-s)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=100_000_000)
    ap.add_argument("--budget-s", type=float, default=60.0,
                    help="no timed step is started that would end past this many seconds of timed work")
    ap.add_argument("--warmup-budget-s", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--train-scale", type=float, default=1.0,
                    help="scales the training steps (counter-collection runs, where every dispatch is slow)")
    ap.add_argument("--legs", default="", help="comma-separated extra legs run after the headline line: "
                                               + ",".join(LEGS))
    ap.add_argument("--legs-only", action="store_true",
                    help="run only the --legs (no headline line; counter runs of one leg)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (calibrates FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (packet ranges would "
              "shard across GPUs, joined by one int64 all-reduce of the tallies)", file=sys.stderr)
        sys.exit(2)
    legs = [s for s in args.legs.split(",") if s]
    bad = [s for s in legs if s not in LEGS]
    if bad:
        print(f"unknown legs {bad}; choose from {sorted(LEGS)}", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_09340_amd import krt

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4}), flush=True)
        return

    ctx = krt.Context(0)
    if args.legs_only:
        print(json.dumps({"legs": {name: LEGS[name](ctx) for name in legs}}), flush=True)
        return
    h = headline_c4(ctx, args)
    out = {
        "metric": "scatterings/s on 1 MI355X, plain vs MLP-escape at spectrum L1<=2% vs oracle",
        "value": h["value"],
        "unit": "scatterings/s",
        "n_gpus": 1,
        "steps": h["K"],
        "warmup": h["W"],
        "ms_per_step": h["wall"] * 1e3 / h["K"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": C4_WORKLOAD + f", {args.packets} packets per step, learned escape "
                                             "(plain walk below threshold); value = plain-walk scatterings "
                                             "for the same packets per learned step time",
                   "packets_per_step": args.packets, "grid": [128, 128, 128], "seed": 0,
                   "network": "BF16 weights and activations, FP32 accumulation on MFMA",
                   "steps_requested": args.steps, "warmup_requested": args.warmup,
                   "train_scale": args.train_scale,
                   "budget_s": args.budget_s},
        "packets_per_s": args.packets * h["K"] / h["wall"],
        "transport_kernel_ms": h["kernel_ms"],
        "roofline": h["roofline"],
        "learned_vs_plain": h["learned"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(h["prob"], workload="the same cloud")
    print(json.dumps(out), flush=True)
    if legs:
        extra = {}
        for name in legs:
            extra[name] = LEGS[name](ctx)
        print(json.dumps({"legs": extra}), flush=True)


if __name__ == "__main__":
    main()
