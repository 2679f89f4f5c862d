"""Benchmark of the Monte Carlo line-transfer pass on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--packets N] [--workload sphere64]

A step is one krt_mc_run over a batch of packets of the static-sphere workload
(64^3 grid, radial line-centre depth 1e6, a = 4.7e-4, dipole phase, central
point source, escaped spectrum 256 bins on [-80, 80), emissivity 64^3 x 32
channels on [-24, 24) toward +x): emission, flights, resonant scatterings,
int64 tallies and the FP32 finalise, with grid and tables already resident in
HBM.  The default batch is the full 1e6 packets of that workload.  Warmup steps
are full-size batches from a disjoint packet range.

Prints one JSON line: whole-job scatterings/s, the ALU roofline of the
transport kernel (HIP-event duration of that kernel, from the library), and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
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
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12  # 39.32 T lane-slots/s (non-packed 32-bit VALU)


def ledger_per_scatter(dipole: bool, emis: bool) -> int:
    return sum(LEDGER.values()) + (LEDGER_DIPOLE if dipole else 0) + (LEDGER_EMIS if emis else 0)


# Sources compiled into the transport kernel; the HBM traffic measured by the
# profiler (profiles/mc_transport_sphere64.md) is reported only while these are
# byte-identical to the ones it was measured on.
KERNEL_SOURCES = ["krt_transport.hip", "krt_device.h", "krt_kernels.h", "krt_mlp.h", "krt_internal.h"]
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "mc_transport_sphere64.md")


def kernel_source_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_09340_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_traffic():
    """HBM bytes per transport launch from the committed counter summary, or
    None when the kernel sources changed since it was taken."""
    try:
        kv = {}
        for line in open(PROFILE_SUMMARY):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
        if kv.get("kernel_source_sha256") != kernel_source_sha256():
            return None
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


def cpu_baseline(prob, seconds_target=40.0):
    """The FP64 oracle as it stands, on all host cores, on a bounded sample."""
    import oracle
    model, ncpu = cpu_info()
    threads = ncpu
    n = threads  # first: one packet per thread to size the sample
    t = time.perf_counter()
    r = oracle.mc_run(prob, n, seed=0, packet_offset=1 << 40, threads=threads)
    dt = time.perf_counter() - t
    if dt < seconds_target / 4:
        n2 = int(max(n, min(64 * threads, n * seconds_target / max(dt, 1e-3) * 0.8)))
        t = time.perf_counter()
        r = oracle.mc_run(prob, n2, seed=0, packet_offset=1 << 40, threads=threads)
        dt = time.perf_counter() - t
        n = n2
    sc = r["counters"]["scatterings"]
    log(f"cpu baseline: {n} packets in {dt:.1f} s")
    return {"value": sc / dt, "unit": "scatterings/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} packets (ids from 2^40, seed 0) of the same workload, {sc} scatterings, "
                      f"{dt:.1f} s on {threads} threads of {model}",
            "packets_per_s": n / dt}


def _agg_blocks(em, n, b=8):
    nch = em.shape[1]
    f = n // b
    return em.reshape(b, f, b, f, b, f, nch).sum(axis=(1, 3, 5)).reshape(-1)


def learned_escape_leg(ctx, n=128, packets=10_000_000, settings=((50.0, 16), (30.0, 16), (100.0, 8))):
    """Turbulent cloud rescaled for the learned escape (n^3, 30% of cells with
    line-centre depth >= 1e2): train the escape network on GPU-recorded
    single-cell escapes, then run the same packets with the plain random walk
    (twice, for the noise floor) and with the learned escape at each
    (tau_R threshold, lanes a wave needs to call) setting.  Reports kernel
    times, the speedup in scatterings-equivalent per second and the spectrum
    and emissivity L1 of each learned run against the plain one; the first
    setting is the headline."""
    import numpy as np
    import torch
    from paper_2608_09340_amd import krt, workloads as W
    from paper_2608_09340_amd.escape import train_escape
    t0 = time.perf_counter()
    krt.Transport(W.slab(10.0, 1e-3, 4), ctx=ctx)  # line tables for a = 1e-3
    tr = train_escape(ctx, 0, seed=1, log10_tau=(1.0, 5.0))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    hist = tr["hist"]
    del tr
    log(f"learned escape: trained in {t_train:.1f} s")
    T = krt.Transport(W.cloud_c4(n=n), ctx=ctx)
    pa = T.run(packets, seed=0)
    ms_plain = ctx.krt_last_transport_ms()
    pb = T.run(packets, seed=0, packet_offset=1 << 40)
    ms_plain2 = ctx.krt_last_transport_ms()
    if pa["rc"] or pb["rc"]:
        raise RuntimeError("learned-escape leg: plain runs failed")

    def l1(u, v):
        u = np.asarray(u, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        return float(np.abs(u - v).sum() / u.sum())

    ea, eb = (_agg_blocks(r["emis_raw"].astype(np.float64), n) for r in (pa, pb))
    sa = pa["counters"]["scatterings"]
    runs = []
    for tau_min, lanes in settings:
        ml = T.run(packets, seed=0, escape_mode=1, esc_tau_min=tau_min, esc_min_lanes=lanes)
        ms_mlp = ctx.krt_last_transport_ms()
        if ml["rc"]:
            raise RuntimeError("learned-escape leg: learned run failed")
        em = _agg_blocks(ml["emis_raw"].astype(np.float64), n)
        c = ml["counters"]
        log(f"learned escape tau_R >= {tau_min:g}, {lanes} lanes: plain {ms_plain:.0f} ms, learned {ms_mlp:.0f} ms")
        runs.append({"esc_tau_min": tau_min, "esc_min_lanes": lanes, "learned_kernel_ms": ms_mlp,
                     "speedup": ms_plain / ms_mlp, "scatterings_equivalent_per_s": sa / (ms_mlp * 1e-3),
                     "scatterings": c["scatterings"], "network_calls": c["mlp_calls"],
                     "skipped_scatterings": c["skipped_scatterings"],
                     "spectrum_L1": l1(pa["spec_raw"], ml["spec_raw"]), "emissivity_L1": l1(ea, em),
                     "emissivity_total_ratio": float(em.sum() / ea.sum())})
    head = runs[0]
    return {
        "workload": f"turbulent cloud {n}^3 (lognormal density sigma_ln=1.5, P(k)~k^-4 velocity rms 3, "
                    f"70th-percentile cell depth 1e2), a=1e-3, Voigt volume source, {packets} packets",
        "train_s": t_train, "train_loss_first_last": [float(hist[:5].mean()), float(hist[-200:].mean())],
        "plain_kernel_ms": ms_plain, "plain_kernel_ms_repeat": ms_plain2, "learned_kernel_ms": head["learned_kernel_ms"],
        "speedup": head["speedup"],
        "plain_scatterings_per_s": sa / (ms_plain * 1e-3),
        "scatterings_equivalent_per_s": head["scatterings_equivalent_per_s"],
        "spectrum_L1": head["spectrum_L1"], "spectrum_L1_floor": l1(pa["spec_raw"], pb["spec_raw"]),
        "emissivity_L1": head["emissivity_L1"], "emissivity_L1_floor": l1(ea, eb),
        "emissivity_total_ratio": head["emissivity_total_ratio"],
        "settings": runs,
        "L1_definition": "sum |learned - plain| / sum plain; emissivity aggregated to 8^3 blocks x channels",
    }


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
    return {"workload": "expanding sphere 128^3, v = 20 r, tau0=1e5, a=1e-3, isotropic R_IIA, Voigt volume "
                        f"source, spectrum 512 bins, emissivity 128^3 x 64 channels, {packets} packets",
            "kernel_ms": ms, "scatterings": c["scatterings"], "scatterings_per_s": c["scatterings"] / (ms * 1e-3),
            "packets_per_s": packets / (ms * 1e-3), "crossings": c["crossings"],
            # the same VALU ledger as the headline (isotropic, emissivity tally): this
            # workload has no long-packet tail, so it shows the transport's bulk rate
            "roofline": {"bound": "alu", "achieved": c["scatterings"] * ledger_per_scatter(False, True) / (ms * 1e-3) / 1e12,
                         "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                         "frac": c["scatterings"] * ledger_per_scatter(False, True) / (ms * 1e-3) / 1e12 / PEAK_VALU_TOPS,
                         "ops_per_scattering": ledger_per_scatter(False, True)},
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


def lambda_leg(ctx, n=128, packets=10_000_000):
    """One Lambda-iteration cycle on the 128^3 turbulent cloud with the 5-level
    rotor: transport of each of the 4 lines with the mean-intensity tally, then
    the FP64 level solve of every cell."""
    import torch
    from paper_2608_09340_amd import workloads as W
    from paper_2608_09340_amd.lambda_iter import LambdaIteration
    lam = LambdaIteration(W.cloud_c3(n=n), ctx)
    runs = [lam.transport_line(l, packets, seed=l) for l in range(lam.nlines)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    lam._levels(lam.jbar)
    torch.cuda.synchronize()
    t_lev = time.perf_counter() - t
    if any(r["rc"] for r in runs):
        raise RuntimeError("lambda leg failed")
    log(f"lambda iteration: {sum(r['kernel_ms'] for r in runs):.0f} ms transport")
    return {"workload": f"turbulent cloud {n}^3, 5-level rotor, 4 lines, {packets} packets per line, "
                        "one transport + level-solve cycle",
            "transport_kernel_ms_per_line": [r["kernel_ms"] for r in runs],
            "scatterings_per_line": [r["counters"]["scatterings"] for r in runs],
            "destroyed_per_line": [r["counters"]["destroyed"] for r in runs],
            "level_solve_ms": t_lev * 1e3, "cells": lam.ncell}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-escape", action="store_true", help="skip the learned-escape comparison leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the expanding-sphere and Lambda-iteration legs")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (calibrates FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (packet ranges would "
              "shard across GPUs, joined by one int64 all-reduce of the tallies)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_09340_amd import krt, workloads as W

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4}), flush=True)
        return

    prob = W.sphere_c1()
    ctx = krt.Context(0)
    T = krt.Transport(prob, ctx=ctx)
    dipole = prob["line"]["phase"] == 1
    emis = prob["tally"].get("emis_nch", 0) > 0

    for w in range(args.warmup):
        T.run(args.packets, seed=args.seed, packet_offset=(1 << 36) + w * args.packets)
        log(f"warmup step {w} done: {ctx.krt_last_transport_ms():.0f} ms")
    torch.cuda.synchronize()

    scat = 0
    kern_ms = []
    emitted = 0
    t0 = time.perf_counter()
    for s in range(args.steps):
        r = T.run(args.packets, seed=args.seed, packet_offset=s * args.packets)
        if r["rc"] != 0:
            raise RuntimeError(f"krt_mc_run rc={r['rc']} counters={r['counters']}")
        scat += r["counters"]["scatterings"]
        emitted += r["counters"]["emitted"]
        kern_ms.append(ctx.krt_last_transport_ms())
        log(f"timed step {s} done: {kern_ms[-1]:.0f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # imaging pass over the step's emissivity toward the camera (+x)
    T.image(axis=0)
    img_ms = []
    for _ in range(5):
        T.image(axis=0)
        img_ms.append(ctx.krt_last_image_ms())
    nx, ny, nz = T.n
    ncell, nch = T.ncell, T.nch
    img_bytes = ncell * nch * 4 + ncell * 4 + ny * nz * nch * 4  # emissivity, k0 (static medium), image
    img_t = min(img_ms) * 1e-3
    log(f"imaging: {min(img_ms):.3f} ms")

    lps = ledger_per_scatter(dipole, emis)
    kms = sum(kern_ms) / len(kern_ms)
    achieved = (scat / args.steps) * lps / (kms * 1e-3) / 1e12
    out = {
        "metric": "scatterings/s on 1 MI355X, plain vs MLP-escape at spectrum L1<=2% vs oracle",
        "value": scat / wall,
        "unit": "scatterings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "static uniform sphere 64^3, radial line-centre tau0=1e6, a=4.7e-4, "
                               "dipole phase, central point source x=0, spectrum 256 bins [-80,80), "
                               "emissivity 64^3 x 32 channels [-24,24) toward +x, plain random walk",
                   "packets_per_step": args.packets, "grid": [64, 64, 64], "seed": args.seed,
                   "mean_scatterings_per_packet": scat / max(emitted, 1)},
        "packets_per_s": emitted / wall,
        "transport_kernel_ms": kms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                     "frac": achieved / PEAK_VALU_TOPS, "traffic": profiled_traffic(),
                     "ops_per_scattering": lps},
    }
    out["imaging"] = {
        "what": f"ray-traced image toward +x of the step's emissivity, {ny}x{nz} pixels x {nch} channels",
        "kernel_ms": min(img_ms),
        "roofline": {"bound": "hbm", "achieved": img_bytes / img_t / 1e9, "peak": 8000.0, "unit": "GB/s",
                     "frac": img_bytes / img_t / 8e12, "bytes_per_launch": img_bytes},
    }
    if not args.no_extra:
        out["expanding_sphere"] = expanding_sphere_leg(ctx)
        out["profile_modes"] = profile_mode_leg(ctx)
        out["lambda_iteration"] = lambda_leg(ctx)
    if not args.no_escape:
        out["learned_escape"] = learned_escape_leg(ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
