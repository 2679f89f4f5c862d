"""Lambda iteration of the line-transfer pass with multi-level populations
(Sec. 2.1.3): alternate the Monte Carlo formal solution for each line
(krt_mc_run with the mean-intensity tally) with the per-cell statistical-
equilibrium update (krt_levels_update), starting from collisional
equilibrium.  The initial emission (n_u A_ul of the collisional-equilibrium
populations) is frozen across cycles; only the line opacities follow the
populations (the paper's prescription).

This module only orders the library calls and marshals buffers; the transport,
the tallies and the FP64 level solves all run in libkrt's kernels.
"""
from __future__ import annotations

import time

import numpy as np

from . import krt


class LambdaIteration:
    def __init__(self, cloud: dict, ctx: "krt.Context", tau_mean_line0: float = 1.0):
        import torch
        self.torch = torch
        self.ctx = ctx
        dev = torch.device("cuda", ctx.device)
        self.dev = dev
        self.cloud = cloud
        n = cloud["n"]
        self.ncell = n[0] * n[1] * n[2]
        rot = cloud["rotor"]
        self.rot = rot
        self.nl = len(rot["E"])
        self.nlines = self.nl - 1
        self.dx = (cloud["hi"][0] - cloud["lo"][0]) / n[0]
        self.vcell = self.dx ** 3
        nc = self.ncell
        self.ncoll = torch.from_numpy(np.asarray(cloud["ncoll"], dtype=np.float64)).to(dev)
        rho = np.asarray(cloud["rho"], dtype=np.float64)
        self.pops = torch.zeros(nc * self.nl, dtype=torch.float64, device=dev)
        self.k0 = torch.zeros(self.nlines * nc, dtype=torch.float32, device=dev)
        self.eps = torch.zeros(self.nlines * nc, dtype=torch.float32, device=dev)
        self._keep = [np.ascontiguousarray(rot[k], dtype=np.float64) for k in ("E", "g", "A", "Cd", "sigma0")]
        # species density scaled so that the mean line-0 cell depth at collisional equilibrium is tau_mean_line0
        self.ntot = torch.from_numpy(rho).to(dev)
        self._levels(None)
        k0_0 = self.k0[:nc].double().mean().item()
        scale = tau_mean_line0 / (k0_0 * self.dx)
        self.ntot = torch.from_numpy(rho * scale).to(dev)
        self._levels(None)
        # frozen emission per line, n_u A_ul per unit volume, and the line powers
        # (cell volume x sum over cells), from the library's level solve at
        # collisional equilibrium
        self.emis = torch.zeros(self.nlines * nc, dtype=torch.float32, device=dev)
        self.lum = self._levels(None, emis_out=self.emis)
        self.pops0 = self.pops.clone()
        vel = np.asarray(cloud["vel"], dtype=np.float32).reshape(3, nc)
        self.vel = torch.from_numpy(vel).to(dev)
        ctx.krt_grid_upload(n, cloud["lo"], cloud["hi"], cloud["bc"], self.k0, self.vel, self.eps, self.emis,
                            n_lines=self.nlines)
        ctx.krt_tables_build([(float(a), 0) for a in rot["a"]])
        self.jbar = torch.zeros(self.nlines * nc, dtype=torch.float32, device=dev)
        self.jraw = torch.zeros(nc, dtype=torch.int64, device=dev)
        self.spec_raw = torch.zeros(66, dtype=torch.int64, device=dev)
        self.counters = torch.zeros(krt.KRT_NCOUNTERS, dtype=torch.int64, device=dev)

    def _levels(self, jbar, emis_out=None):
        """krt_levels_update over all cells; with emis_out, also the emission
        n_u A_ul per cell and the line powers (returned, one per line)."""
        d = krt.krt_levels_desc()
        d.n_levels = self.nl
        d.ncell = self.ncell
        d.E, d.g, d.A, d.Cd, d.sigma0 = [k.ctypes.data for k in self._keep]
        d.ncoll_dev, d.ntot_dev, d.pops_dev = self.ncoll.data_ptr(), self.ntot.data_ptr(), self.pops.data_ptr()
        d.k0_out_dev, d.eps_out_dev = self.k0.data_ptr(), self.eps.data_ptr()
        lum = None
        if emis_out is not None:
            lum = np.zeros(self.nlines, dtype=np.float64)
            d.emis_out_dev = emis_out.data_ptr()
            d.cell_volume = self.vcell
            d.lum_out = lum.ctypes.data
        self.ctx.krt_levels_update(d, jbar)
        return None if lum is None else lum.tolist()

    def transport_line(self, line: int, n_packets: int, seed: int, packet_offset: int = 0) -> dict:
        nc = self.ncell
        prob = {"source": {"kind": 2, "profile": 1}, "tally": {"spec_nbins": 64, "spec_lo": -16.0,
                                                                "spec_hi": 16.0, "jbar": 1}}
        o = krt.make_opts(prob, line=line, packet_offset=packet_offset, luminosity=self.lum[line])
        t = krt.krt_tallies()
        t.spec_raw_dev = self.spec_raw.data_ptr()
        t.counters_dev = self.counters.data_ptr()
        t.jbar_raw_dev = self.jraw.data_ptr()
        t.jbar_dev = self.jbar.data_ptr() + 4 * line * nc
        rc = self.ctx.krt_mc_run(n_packets, seed, o, t)
        c = dict(zip(krt.COUNTER_NAMES, self.counters.cpu().numpy()[:len(krt.COUNTER_NAMES)].tolist()))
        return {"rc": rc, "counters": c, "kernel_ms": self.ctx.krt_last_transport_ms()}

    def iterate(self, n_iter: int, n_packets: int, seed: int = 0) -> list:
        hist = []
        nc = self.ncell
        for it in range(n_iter):
            old = self.pops.clone()
            runs = [self.transport_line(l, n_packets, seed + it * 16 + l) for l in range(self.nlines)]
            self.torch.cuda.synchronize()
            t0 = time.perf_counter()
            self._levels(self.jbar)
            t_lev = (time.perf_counter() - t0) * 1e3
            P, Q = self.pops.view(nc, self.nl), old.view(nc, self.nl)
            dmax = float(((P - Q).abs() / Q.abs().clamp_min(1e-300)).max().item())
            hist.append({"iteration": it, "max_rel_change": dmax,
                         "scatterings": sum(r["counters"]["scatterings"] for r in runs),
                         "kernel_ms": sum(r["kernel_ms"] for r in runs), "levels_ms": t_lev,
                         "rc": [r["rc"] for r in runs]})
        return hist
