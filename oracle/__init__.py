"""FP64 CPU oracle for the Monte Carlo line-transfer pass -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2608_09340_amd``): the two meet only through the plain input arrays
made by ``paper_2608_09340_amd.workloads``.

The C core (``krt_oracle.c``) states each step with its citation of the paper;
this module only marshals arguments.  Functions without a pin say so in their
docstring ("parity unpinned").
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "krt_oracle.c")
_LIB = os.path.join(_HERE, "libkrt_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-Wall",
               "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class OrcProblem(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("bc", C.c_int32 * 3),
        ("k0", C.c_void_p), ("vel", C.c_void_p), ("eps", C.c_void_p), ("emis", C.c_void_p), ("bratio", C.c_void_p),
        ("kabs", C.c_void_p),
        ("a", C.c_double), ("phase", C.c_int32), ("source", C.c_int32), ("src_pos", C.c_double * 3),
        ("src_dir", C.c_double * 3),
        ("src_profile", C.c_int32), ("src_x0", C.c_double),
        ("spec_nbins", C.c_int32), ("spec_lo", C.c_double), ("spec_hi", C.c_double),
        ("emis_nch", C.c_int32), ("ch_lo", C.c_double), ("ch_hi", C.c_double), ("n_cam", C.c_double * 3),
        ("jbar", C.c_int32), ("max_events", C.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        p = C.c_void_p
        L.orc_philox_batch.argtypes = [C.c_int64, p, p, p]
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_voigt_H.argtypes = [C.c_double, C.c_double]
        L.orc_voigt_H.restype = C.c_double
        L.orc_voigt_batch.argtypes = [C.c_int64, C.c_double, p, p]
        L.orc_sample_upar_batch.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_uint64,
                                            C.c_uint64, C.c_uint32, p, p]
        L.orc_bin_batch.argtypes = [C.c_int64, p, C.c_int, C.c_double, C.c_double, p]
        L.orc_mc_run.argtypes = [C.POINTER(OrcProblem), C.c_uint64, C.c_uint64, C.c_uint64, C.c_int,
                                 p, p, p, p, p]
        L.orc_mc_run.restype = C.c_int
        L.orc_levels_solve.argtypes = [C.c_int, C.c_int64, p, p, p, p, p, p, p, p]
        L.orc_levels_solve.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------- primitives
def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Philox4x32-10 blocks: ctr [n,4] uint32, key [n,2] uint32 -> [n,4] uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def u01(w: int) -> float:
    return lib().orc_u01(int(w))


def voigt_H(a: float, x) -> np.ndarray:
    x = np.ascontiguousarray(np.atleast_1d(x), dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_voigt_batch(x.size, float(a), _ptr(x), _ptr(out))
    return out


def sample_upar(n: int, x: float, a: float, seed: int = 0, packet: int = 0, ev0: int = 1):
    """n exact draws of u_par | x (one per event index); returns (draws, mean trials)."""
    out = np.empty(n, dtype=np.float64)
    tt = np.zeros(1, dtype=np.int64)
    lib().orc_sample_upar_batch(n, float(x), float(a), int(seed), int(packet), int(ev0),
                                _ptr(out), _ptr(tt))
    return out, tt[0] / max(n, 1)


def bin_index(x: np.ndarray, nb: int, lo: float, hi: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.int32)
    lib().orc_bin_batch(x.size, _ptr(x), int(nb), float(lo), float(hi), _ptr(out))
    return out


# ---------------------------------------------------------------- transport
COUNTER_NAMES = ["emitted", "escaped", "destroyed", "scatterings", "crossings", "stuck",
                 "trials", "status"]


def mc_run(prob: dict, n_packets: int, seed: int = 0, packet_offset: int = 0,
           threads: int | None = None, packet_log: bool = False) -> dict:
    """Run the FP64 oracle Monte Carlo on the problem dict (see workloads).

    Returns spectrum counts (nb+2, under/overflow at the ends), emissivity
    weights [ncell, nch] (FP64), jbar sums [ncell] (FP64, sum dl*H/sqrt(pi)),
    counters and optionally the per-packet log [n, 8] = (x_lab, n_scat,
    outcome, n_x, n_y, n_z, cell, last event).
    """
    g = prob["grid"]
    n = [int(v) for v in g["n"]]
    ncell = n[0] * n[1] * n[2]
    k0 = np.ascontiguousarray(g["k0"], dtype=np.float32).reshape(-1)
    assert k0.size == ncell
    vel = g.get("vel")
    vel = None if vel is None else np.ascontiguousarray(vel, dtype=np.float32).reshape(3, ncell)
    eps = g.get("eps")
    eps = None if eps is None else np.ascontiguousarray(eps, dtype=np.float32).reshape(-1)
    kabs = g.get("kabs")
    kabs = None if kabs is None else np.ascontiguousarray(kabs, dtype=np.float32).reshape(-1)
    emis = g.get("emis")
    emis = None if emis is None else np.ascontiguousarray(emis, dtype=np.float32).reshape(-1)
    P = OrcProblem()
    P.n[:] = n
    P.lo[:] = [float(v) for v in g["lo"]]
    P.hi[:] = [float(v) for v in g["hi"]]
    P.bc[:] = [int(v) for v in g["bc"]]
    P.k0 = k0.ctypes.data
    P.vel = None if vel is None else vel.ctypes.data
    P.eps = None if eps is None else eps.ctypes.data
    P.kabs = None if kabs is None else kabs.ctypes.data
    P.emis = None if emis is None else emis.ctypes.data
    # per-cell Doppler width b_cell / b_ref: an explicit per-cell array, or
    # temperature classes (class index per cell and the ratio of each class)
    br = g.get("bratio")
    if br is None and g.get("tclass") is not None:
        br = np.asarray(g["tclass_bratio"], dtype=np.float32)[np.asarray(g["tclass"]).reshape(-1)]
    br = None if br is None else np.ascontiguousarray(br, dtype=np.float32).reshape(-1)
    assert br is None or br.size == ncell
    P.bratio = None if br is None else br.ctypes.data
    ln = prob["line"]
    P.a = float(ln["a"])
    P.phase = int(ln.get("phase", 0))
    src = prob["source"]
    P.source = int(src["kind"])
    P.src_pos[:] = [float(v) for v in src.get("pos", (0.0, 0.0, 0.0))]
    P.src_dir[:] = [float(v) for v in src.get("dir", (0.0, 0.0, 1.0))]
    P.src_profile = int(src.get("profile", 0))
    P.src_x0 = float(src.get("x0", 0.0))
    t = prob["tally"]
    P.spec_nbins = int(t["spec_nbins"])
    P.spec_lo = float(t["spec_lo"])
    P.spec_hi = float(t["spec_hi"])
    P.emis_nch = int(t.get("emis_nch", 0))
    P.ch_lo = float(t.get("ch_lo", 0.0))
    P.ch_hi = float(t.get("ch_hi", 1.0))
    P.n_cam[:] = [float(v) for v in t.get("n_cam", (1.0, 0.0, 0.0))]
    P.jbar = int(t.get("jbar", 0))
    P.max_events = int(prob.get("max_events", 1 << 40))
    spec = np.zeros(P.spec_nbins + 2, dtype=np.int64)
    em = np.zeros((ncell, P.emis_nch), dtype=np.float64) if P.emis_nch > 0 else None
    jb = np.zeros(ncell, dtype=np.float64) if P.jbar else None
    cnt = np.zeros(8, dtype=np.int64)
    plog = np.zeros((n_packets, 8), dtype=np.float64) if packet_log else None
    if threads is None:
        threads = os.cpu_count() or 1
    rc = lib().orc_mc_run(C.byref(P), int(n_packets), int(packet_offset), int(seed), int(threads),
                          _ptr(spec), _ptr(em), _ptr(jb), _ptr(cnt), _ptr(plog))
    if rc != 0:
        raise RuntimeError(f"orc_mc_run failed: {rc}")
    out = {"spec": spec, "counters": dict(zip(COUNTER_NAMES, cnt.tolist()))}
    if em is not None:
        out["emis"] = em
    if jb is not None:
        out["jbar"] = jb
    if plog is not None:
        out["packet_log"] = plog
    return out


# ---------------------------------------------------------------- levels
def levels_solve(E, g, A, Cd, ncoll, ntot, gamma=None) -> np.ndarray:
    """Per-cell statistical equilibrium (FP64); returns pops [ncell, nl]."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    Cd = np.ascontiguousarray(Cd, dtype=np.float64)
    ncoll = np.ascontiguousarray(ncoll, dtype=np.float64).reshape(-1)
    ntot = np.ascontiguousarray(ntot, dtype=np.float64).reshape(-1)
    nl = E.size
    ncell = ncoll.size
    gm = None if gamma is None else np.ascontiguousarray(gamma, dtype=np.float64).reshape(nl - 1, ncell)
    pops = np.empty((ncell, nl), dtype=np.float64)
    rc = lib().orc_levels_solve(nl, ncell, _ptr(E), _ptr(g), _ptr(A), _ptr(Cd), _ptr(ncoll),
                                _ptr(ntot), _ptr(gm), _ptr(pops))
    if rc != 0:
        raise RuntimeError(f"orc_levels_solve failed: {rc}")
    return pops


# ---------------------------------------------------------- whole-cell escape
CELL_REC = 20
(R_LT, R_LA, R_X, R_Q0, R_Q1, R_Q2, R_LD, R_N0, R_N1, R_N2, R_FACE, R_YS, R_YT, R_MU, R_ALPHA, R_XOUT,
 R_LOGN, R_LOGX2, R_VALID) = range(19)


def cell_escape_record(n: int, tau_c: float, a: float, x_in: float, q, n_in=None, seed: int = 0,
                       offset: int = 0, threads: int | None = None) -> np.ndarray:
    """Plain FP64 whole-cell escapes (reference for the learned escape): the
    photon scatters at q inside the cube [-1, 1]^3 of line-centre depth tau_c
    from centre to face and walks until it leaves.  Returns [n, 20] records
    (columns R_*): the condition (log10 tau_c, log10 a, x_in, q, log10 depth,
    n_in), the exit face 2 axis + (normal along +axis), the exit point's
    offsets from q's projection over q's distance to the face plane, the exit
    cosine mu, the angle alpha between the tangential direction and that
    offset, x_out, ln N_s, ln <x^2> and a valid flag."""
    L = lib()
    if not hasattr(L, "_cell_set"):
        L.orc_cell_escape_record.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                             C.c_void_p, C.c_uint64, C.c_uint64, C.c_int, C.c_void_p]
        L.orc_cell_escape_record.restype = C.c_int
        L._cell_set = True
    qq = np.ascontiguousarray(q, dtype=np.float64).reshape(3)
    nn = None if n_in is None else np.ascontiguousarray(n_in, dtype=np.float64).reshape(3)
    out = np.zeros((n, CELL_REC), dtype=np.float64)
    rc = L.orc_cell_escape_record(int(n), float(tau_c), float(a), float(x_in), _ptr(qq), _ptr(nn), int(seed),
                                  int(offset), int(threads or os.cpu_count() or 1), _ptr(out))
    if rc != 0:
        raise ValueError("cell_escape_record needs |q_k| < 1")
    return out


# ---------------------------------------------------------------- finalise
FOUR_PI = 4.0 * np.pi


def finalize(spec=None, emis=None, jbar=None, *, n_packets, luminosity=1.0, spec_bins=None, channels=None,
             cell_volume=None, emis_frac_bits=0, jbar_frac_bits=0):
    """Step O7, the FP64 normalisation of the tallies (Sec. 2.3: the reductions
    are FP64; Sec. 2.2.1 eq. scat-line: the emissivity is the scattered power
    per unit volume, solid angle and frequency), as the plain definitions:

      spectrum   L * count / (N dx_bin)                         per unit x
      emissivity L * w 2^-F / (4 pi N V_cell dx_ch)             per volume, steradian, unit x
      J-bar      L * s 2^-Fj / (4 pi N V_cell)                  s = sum dl H(a, x)/sqrt(pi)

    N packets carry total luminosity L, so one packet carries L/N.  Raw tallies
    may be FP64 weights (the oracle's own, F = 0) or fixed-point integers of
    F fraction bits (values times 2^F); they are converted to FP64 before
    scaling.  spec_bins = (nb, lo, hi), channels = (nch, lo, hi).  Returns a
    dict of FP64 arrays for the tallies given."""
    N = float(n_packets)
    L = float(luminosity)
    out = {}
    if spec is not None:
        nb, lo, hi = spec_bins
        dxb = (float(hi) - float(lo)) / float(nb)
        out["spec"] = np.asarray(spec, dtype=np.float64) * (L / (N * dxb))
    if emis is not None:
        nch, lo, hi = channels
        dxc = (float(hi) - float(lo)) / float(nch)
        w = np.asarray(emis, dtype=np.float64) * 2.0 ** (-int(emis_frac_bits))
        out["emis"] = w * (L / (FOUR_PI * N * float(cell_volume) * dxc))
    if jbar is not None:
        s = np.asarray(jbar, dtype=np.float64) * 2.0 ** (-int(jbar_frac_bits))
        out["jbar"] = s * (L / (FOUR_PI * N * float(cell_volume)))
    return out
