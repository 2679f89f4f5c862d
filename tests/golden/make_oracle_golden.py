"""Write oracle reference tallies used by the GPU parity tests.

Calls only the FP64 oracle (``oracle/``) on the seeded synthetic workloads.
Outputs are plain text: one integer per line for spectra, preceded by a
header comment with the workload, packet range and seed.

    python tests/golden/make_oracle_golden.py c0 [threads]
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


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c0"
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    {"c0": c0}[which](threads)
