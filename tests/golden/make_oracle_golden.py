"""Write oracle reference tallies used by the GPU parity tests.

Calls only the FP64 oracle (``oracle/``) on the seeded synthetic workloads.
Outputs are plain text: one integer per line for spectra, preceded by a
header comment with the workload, packet range and seed.

    python tests/golden/make_oracle_golden.py c0|sphere4|c1|c2 [threads]

Emissivity references are written as batch sums aggregated over radial shells
of cell-centre radius (16 shells over [0, 1]) x channels, one row per batch of
consecutive packet ids, so the tests can form batch means.
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2608_09340_amd import workloads as W  # noqa: E402


def write_spec(path, spec, header):
    with open(path, "w") as f:
        for h in header:
            f.write(f"# {h}\n")
        for v in spec:
            f.write(f"{int(v)}\n")


def c0(threads):
    # static slab 1x1x32, tau0 = 1e3, a = 1e-2: 1e6 packets, seed 0, ids [1e6, 2e6)
    # (disjoint from the ids the GPU runs, so the two samples are independent)
    prob = W.slab_c0()
    t = time.time()
    r = oracle.mc_run(prob, 1_000_000, seed=0, packet_offset=1_000_000, threads=threads)
    dt = time.time() - t
    c = r["counters"]
    write_spec(os.path.join(HERE, "c0_slab_oracle_spec_1e6.txt"), r["spec"],
               ["FP64 oracle escaped spectrum, static slab 1x1x32 |z|<=1, tau0=1e3 (line centre, midplane to face),",
                "a=1e-2, isotropic phase, plane source z=0 at x=0; 200 bins on [-30,30) + under/overflow;",
                "packets [1000000, 2000000), Philox seed 0; written by tests/golden/make_oracle_golden.py",
                f"scatterings={c['scatterings']} escaped={c['escaped']} wall={dt:.1f}s threads={threads}"])
    print("c0 done", dt, c)


def shell_index(n, nshell=16):
    """Radial shell of every cell of an n^3 grid on [-1, 1]^3 (cell-centre
    radius r, shell floor(r nshell) for r <= 1, -1 outside)."""
    c = -1 + (np.arange(n) + 0.5) * 2.0 / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z).reshape(-1)
    s = np.minimum((r * nshell).astype(np.int64), nshell - 1)
    return np.where(r <= 1.0, s, -1)


def shell_sum(em, shells, nshell=16):
    out = np.zeros((nshell, em.shape[1]))
    m = shells >= 0
    np.add.at(out, shells[m], em[m])
    return out


def batched(prob, name, n_total, n_batch, offset, threads, header, nshell=16):
    """Oracle run of n_total packets from `offset` in batches of n_batch
    consecutive ids; writes <name>_spec.txt (total escaped counts) and
    <name>_emis_shells.txt (per batch: nshell x nch emissivity weights)."""
    shells = shell_index(prob["grid"]["n"][0], nshell)
    spec = None
    rows = []
    scat = 0
    t = time.time()
    for b in range(n_total // n_batch):
        r = oracle.mc_run(prob, n_batch, seed=0, packet_offset=offset + b * n_batch, threads=threads)
        spec = r["spec"] if spec is None else spec + r["spec"]
        rows.append(shell_sum(r["emis"], shells, nshell).reshape(-1))
        scat += r["counters"]["scatterings"]
        print(f"{name} batch {b} done {time.time() - t:.0f}s", flush=True)
    dt = time.time() - t
    nch = prob["tally"]["emis_nch"]
    hdr = header + [f"packets [{offset}, {offset + n_total}) in batches of {n_batch}, Philox seed 0; "
                    "written by tests/golden/make_oracle_golden.py",
                    f"scatterings={scat} wall={dt:.1f}s threads={threads}"]
    write_spec(os.path.join(HERE, f"{name}_spec.txt"), spec, hdr)
    np.savetxt(os.path.join(HERE, f"{name}_emis_shells.txt"), np.asarray(rows), fmt="%.10e",
               header="\n".join(hdr + [f"rows: batches; columns: shell * {nch} + channel ({nshell} radial shells "
                                       "of cell-centre radius over [0, 1]); FP64 emissivity weights (phase weight "
                                       "per scattering toward the camera)"]))
    print(name, "done", dt, scat, flush=True)


def sphere4(threads):
    # the static sphere's physics at a cheaper depth: 64^3, tau0 = 1e4, a = 4.7e-4,
    # dipole, central x = 0 point source; 256 bins on [-16, 16), 32 channels on [-8, 8)
    batched(W.sphere(64, 1e4, 4.7e-4, spec=(256, -16.0, 16.0), emis=(32, -8.0, 8.0)), "sphere4",
            1_000_000, 50_000, 1 << 32, threads,
            ["FP64 oracle, static sphere 64^3 radius 1, tau0=1e4 (line centre, centre to edge), a=4.7e-4,",
             "dipole phase, point source at the centre x=0; spectrum 256 bins on [-16,16) + under/overflow;",
             "emissivity 32 channels on [-8,8) toward +x"])


def c1(threads):
    # the static sphere benchmark: 64^3, tau0 = 1e6, a = 4.7e-4, dipole
    batched(W.sphere_c1(), "c1", 10_000, 500, 1 << 32, threads,
            ["FP64 oracle, static sphere 64^3 radius 1, tau0=1e6, a=4.7e-4, dipole, central point source x=0;",
             "spectrum 256 bins on [-80,80) + under/overflow; emissivity 32 channels on [-24,24) toward +x"])


def c2(threads):
    # the expanding sphere benchmark: 128^3, v = 20 r, tau0 = 1e5, a = 1e-3, Voigt volume source
    batched(W.expanding_sphere_c2(), "c2", 100_000, 5_000, 1 << 32, threads,
            ["FP64 oracle, homologously expanding sphere 128^3, v=20 r (thermal units), tau0=1e5, a=1e-3,",
             "isotropic phase, uniform volume source with the Voigt profile; spectrum 512 bins on [-64,64)",
             "+ under/overflow; emissivity 64 channels on [-40,40) toward +x"])


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c0"
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    {"c0": c0, "sphere4": sphere4, "c1": c1, "c2": c2}[which](threads)
