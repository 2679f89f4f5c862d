"""Training recipe of the learned whole-cell escape: record whole-cell walks
with the plain transport arithmetic on the GPU (krt_escape_record), fit the
output normalisation, then run the BF16-MFMA training kernels
(krt_escape_train) in stages of decreasing learning rate and growing batch,
then calibrate the mean scattering count (krt_escape_calibrate).  Only the
order of the library calls lives here; records, gradients and Adam updates
are computed by libkrt.
"""
from __future__ import annotations

import numpy as np

from . import krt

# (steps, batch, learning rate): Adam, learning rate halved per stage, batch
# doubled up to 32768; 180000 steps, about 420 passes over 8e6 records (six
# times the first recipe; on the 128^3 cloud at 1e7 packets the emissivity
# error against the plain walk falls from L1 0.0125 at half as many steps to
# 0.010, for 17 s of training instead of 10; four times as many steps gain
# nothing more)
DEFAULT_STAGES = ((36000, 4096, 2e-3), (36000, 8192, 1e-3), (36000, 16384, 5e-4), (36000, 32768, 2.5e-4),
                  (36000, 32768, 1.25e-4))


# Run options of the learned escape on the benchmark cloud: network calls in
# cells at least 50 line-centre mean free paths deep (raised to the training
# records' smallest tau_c, 10^1.5 from centre to face), at scattering points at
# least 3 below the nearest face, in batches of whole 16-sample blocks, a
# qualifying scattering held for at most 32 iterations (fused schedule).
DEFAULT_RUN = {"esc_cell_tau_min": 50.0, "esc_tau_min": 3.0, "esc_min_lanes": 16, "esc_wait": 32}
# log10 tau_c (centre to face) range of the training records for that setting
DEFAULT_LOG10_TAU = (1.5, 5.0)


def train_escape(ctx: "krt.Context", line: int = 0, n_records: int = 8_000_000, seed: int = 1,
                 log10_tau=DEFAULT_LOG10_TAU, stages=DEFAULT_STAGES, record_offset: int = 0, lines=None,
                 depth_lo: float = 0.3) -> dict:
    """Record `n_records` whole-cell walks from cells with log10 tau_c uniform
    in `log10_tau` and start points whose log10 depth below the nearest face
    is uniform from `depth_lo` up (line `line`, or split evenly over `lines`
    to cover several damping values, whose tables must be built), initialise
    the network from `seed`, fit the normalisation (and the ranges the network
    may then be used on), train, and calibrate the predicted mean scattering
    count per (log10 tau_c, log10 depth, |x_in|) bin on the records.  Returns
    the record buffer and the per-step loss history (all stages,
    concatenated)."""
    import torch
    dev = torch.device("cuda", ctx.device)
    lines = [line] if lines is None else [int(v) for v in lines]
    rec = torch.zeros((n_records, krt.ESC_NREC), dtype=torch.float32, device=dev)
    bounds = np.linspace(0, n_records, len(lines) + 1).astype(np.int64)
    for k, ln in enumerate(lines):
        b0, b1 = int(bounds[k]), int(bounds[k + 1])
        # disjoint packet ranges, so records of different lines are independent
        ctx.krt_escape_record(ln, b1 - b0, seed, record_offset + b0, log10_tau[0], log10_tau[1], rec[b0:b1],
                              depth_lo=depth_lo)
    ctx.krt_escape_init(seed)
    ctx.krt_escape_fit_norm(rec, n_records)
    hist = []
    for k, (steps, batch, lr) in enumerate(stages):
        h = torch.zeros(steps, dtype=torch.float32, device=dev)
        ctx.krt_escape_train(rec, n_records, steps, batch, lr, seed * 1000 + 11 + k, h)
        hist.append(h.cpu().numpy())
    ctx.krt_escape_calibrate(rec, n_records)
    return {"rec": rec, "hist": np.concatenate(hist), "log10_tau": tuple(log10_tau)}
