"""Thin ctypes binding of libkrt (include/krt.h), same names, argument marshalling only.

Every step of the pass runs in the HIP library; torch supplies device memory
and the stream.  Importing this module on a machine without the built library
raises immediately: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkrt.so")

KRT_OK, KRT_EINVAL, KRT_EHIP, KRT_EDEVICE, KRT_ESTATE = 0, -1, -2, -3, -4
KRT_NCOUNTERS = 16
COUNTER_NAMES = ["emitted", "escaped", "destroyed", "scatterings", "crossings", "stuck",
                 "mlp_calls", "status", "emis_dropped", "skipped_scatterings"]


class krt_grid_desc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("bc", C.c_int32 * 3), ("n_lines", C.c_int32),
                ("k0_dev", C.c_void_p), ("vel_dev", C.c_void_p), ("eps_dev", C.c_void_p),
                ("emis_dev", C.c_void_p), ("kabs_dev", C.c_void_p), ("tclass_dev", C.c_void_p),
                ("n_tclass", C.c_int32),
                ("tclass_bratio", C.c_double * 8), ("bratio_dev", C.c_void_p)]


class krt_line_desc(C.Structure):
    _fields_ = [("a", C.c_double), ("phase", C.c_int32), ("reserved", C.c_int32)]


class krt_run_opts(C.Structure):
    _fields_ = [("line", C.c_int32), ("source", C.c_int32), ("src_pos", C.c_double * 3),
                ("src_dir", C.c_double * 3), ("src_profile", C.c_int32), ("src_x0", C.c_double),
                ("spec_nbins", C.c_int32), ("spec_lo", C.c_double), ("spec_hi", C.c_double),
                ("emis_nch", C.c_int32), ("ch_lo", C.c_double), ("ch_hi", C.c_double),
                ("n_cam", C.c_double * 3), ("jbar", C.c_int32), ("accumulate", C.c_int32),
                ("packet_offset", C.c_uint64), ("max_events", C.c_uint64),
                ("escape_mode", C.c_int32), ("wg_size", C.c_int32), ("wg_per_cu", C.c_int32),
                ("emis_frac_bits", C.c_int32), ("jbar_frac_bits", C.c_int32),
                ("norm_packets", C.c_uint64), ("luminosity", C.c_double),
                ("esc_tau_min", C.c_double), ("esc_cell_tau_min", C.c_double), ("esc_min_lanes", C.c_int32),
                ("esc_tail_lanes", C.c_int32), ("tail_lanes", C.c_int32), ("profile_mode", C.c_int32),
                ("esc_park", C.c_int32), ("esc_park_cap", C.c_uint32), ("esc_park_tail", C.c_uint32),
                ("esc_park_budget", C.c_uint32), ("esc_wait", C.c_int32)]


class krt_escape_cond(C.Structure):
    _fields_ = [("log10_tau_lo", C.c_double), ("log10_tau_hi", C.c_double), ("log10_depth_lo", C.c_double),
                ("fixed", C.c_int32), ("iso_dir", C.c_int32), ("x_in", C.c_double), ("q", C.c_double * 3),
                ("n_in", C.c_double * 3)]


class krt_tallies(C.Structure):
    _fields_ = [("spec_raw_dev", C.c_void_p), ("emis_raw_dev", C.c_void_p),
                ("jbar_raw_dev", C.c_void_p), ("counters_dev", C.c_void_p),
                ("packet_log_dev", C.c_void_p), ("spec_dev", C.c_void_p),
                ("emis_dev", C.c_void_p), ("jbar_dev", C.c_void_p)]


class krt_levels_desc(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("ncell", C.c_int64), ("E", C.c_void_p), ("g", C.c_void_p), ("A", C.c_void_p),
                ("Cd", C.c_void_p), ("sigma0", C.c_void_p), ("ncoll_dev", C.c_void_p),
                ("ntot_dev", C.c_void_p), ("pops_dev", C.c_void_p), ("k0_out_dev", C.c_void_p),
                ("eps_out_dev", C.c_void_p), ("emis_out_dev", C.c_void_p), ("cell_volume", C.c_double),
                ("lum_out", C.c_void_p)]


class krt_image_desc(C.Structure):
    _fields_ = [("line", C.c_int32), ("axis", C.c_int32), ("nch", C.c_int32), ("ch_lo", C.c_double),
                ("ch_hi", C.c_double), ("emis_dev", C.c_void_p), ("src_dev", C.c_void_p),
                ("image_dev", C.c_void_p), ("kabs_dev", C.c_void_p)]


EXPORTS = ["krt_create", "krt_destroy", "krt_last_error", "krt_device_cus", "krt_last_transport_ms",
           "krt_last_network_ms", "krt_last_rounds",
           "krt_grid_upload",
           "krt_tables_build", "krt_mc_run", "krt_mc_run_noalloc", "krt_levels_update", "krt_debug_philox",
           "krt_debug_bins", "krt_debug_voigt", "krt_debug_voigt_analytic", "krt_debug_voigt_cont", "krt_debug_upar",
           "krt_escape_init", "krt_escape_record", "krt_escape_fit_norm", "krt_escape_calibrate", "krt_escape_grad",
           "krt_escape_train", "krt_escape_get_weights", "krt_escape_put_weights", "krt_escape_forward",
           "krt_image", "krt_last_image_ms"]
ESC_NPARAMS, ESC_NNORM, ESC_NIN, ESC_NOUT, ESC_NCAL, ESC_NREC = 40352, 328, 17, 32, 256, 20

_lib = None


def load(path: str = LIB_PATH):
    """Load libkrt.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libkrt.so not built at {path}: run python -m paper_2608_09340_amd.build")
    L = C.CDLL(path)
    p, i32, i64, u64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_uint32
    L.krt_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, p]
    L.krt_create.restype = C.c_int
    L.krt_destroy.argtypes = [p]
    L.krt_destroy.restype = None
    L.krt_last_error.argtypes = [p]
    L.krt_last_error.restype = C.c_char_p
    L.krt_device_cus.argtypes = [p]
    L.krt_device_cus.restype = C.c_int
    L.krt_last_transport_ms.argtypes = [p]
    L.krt_last_transport_ms.restype = C.c_double
    L.krt_last_network_ms.argtypes = [p]
    L.krt_last_network_ms.restype = C.c_double
    L.krt_last_rounds.argtypes = [p]
    L.krt_last_rounds.restype = C.c_int64
    L.krt_grid_upload.argtypes = [p, C.POINTER(krt_grid_desc)]
    L.krt_tables_build.argtypes = [p, C.POINTER(krt_line_desc), C.c_int]
    L.krt_mc_run.argtypes = [p, u64, u64, C.POINTER(krt_run_opts), C.POINTER(krt_tallies)]
    L.krt_mc_run_noalloc.argtypes = [p, u64, u64, C.POINTER(krt_run_opts), C.POINTER(krt_tallies)]
    L.krt_levels_update.argtypes = [p, C.POINTER(krt_levels_desc), p]
    L.krt_debug_philox.argtypes = [p, p, p, p, i64]
    L.krt_debug_bins.argtypes = [p, p, i64, i32, C.c_double, C.c_double, p]
    L.krt_debug_voigt.argtypes = [p, i32, p, i64, p]
    L.krt_debug_voigt_analytic.argtypes = [p, C.c_double, p, i64, p]
    L.krt_debug_voigt_cont.argtypes = [p, i32, p, p, i64, p]
    L.krt_debug_upar.argtypes = [p, i32, C.c_float, u64, u64, u32, i64, p]
    L.krt_escape_init.argtypes = [p, u64]
    L.krt_escape_record.argtypes = [p, i32, u64, u64, u64, C.POINTER(krt_escape_cond), p]
    L.krt_escape_fit_norm.argtypes = [p, p, u64]
    L.krt_escape_calibrate.argtypes = [p, p, u64]
    L.krt_escape_grad.argtypes = [p, p, p, p, i32, p, p]
    L.krt_escape_train.argtypes = [p, p, u64, i32, i32, C.c_double, u64, p]
    L.krt_escape_get_weights.argtypes = [p, p, u64]
    L.krt_escape_put_weights.argtypes = [p, p, u64]
    L.krt_escape_forward.argtypes = [p, p, i64, p]
    L.krt_image.argtypes = [p, C.POINTER(krt_image_desc)]
    L.krt_last_image_ms.argtypes = [p]
    L.krt_last_image_ms.restype = C.c_float
    for name in ["krt_grid_upload", "krt_tables_build", "krt_mc_run", "krt_mc_run_noalloc", "krt_levels_update",
                 "krt_debug_philox", "krt_debug_bins", "krt_debug_voigt", "krt_debug_voigt_analytic",
                 "krt_debug_voigt_cont", "krt_debug_upar", "krt_escape_init", "krt_escape_record", "krt_escape_fit_norm", "krt_escape_calibrate",
                 "krt_escape_grad",
                 "krt_escape_train", "krt_escape_get_weights", "krt_escape_put_weights",
                 "krt_escape_forward", "krt_image"]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


class KrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"krt error {code}: {msg}")
        self.code = code


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """Owns one krt_ctx on the current torch device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.L = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        rc = self.L.krt_create(C.byref(h), int(device), C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise KrtError(rc, "krt_create failed")
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            self.L.krt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise KrtError(rc, self.L.krt_last_error(self.h).decode())

    @property
    def cus(self) -> int:
        return self.L.krt_device_cus(self.h)

    def krt_last_transport_ms(self) -> float:
        return self.L.krt_last_transport_ms(self.h)

    def krt_last_network_ms(self) -> float:
        return self.L.krt_last_network_ms(self.h)

    def krt_last_rounds(self) -> int:
        return int(self.L.krt_last_rounds(self.h))

    # ------------------------------------------------------------- calls
    def krt_grid_upload(self, n, lo, hi, bc, k0, vel=None, eps=None, emis=None, n_lines=1, tclass=None,
                        tclass_bratio=None, kabs=None, bratio=None):
        """tclass: device uint8 [ncell] temperature class per cell (or None);
        tclass_bratio: the Doppler width of each class over the reference;
        kabs: device FP32 [ncell] grey absorption coefficient (or None);
        bratio: device FP32 [ncell] Doppler width of each cell over the
        reference (a continuum of temperatures; or None)."""
        d = krt_grid_desc()
        d.n[:] = [int(v) for v in n]
        d.lo[:] = [float(v) for v in lo]
        d.hi[:] = [float(v) for v in hi]
        d.bc[:] = [int(v) for v in bc]
        d.n_lines = int(n_lines)
        d.k0_dev = k0.data_ptr()
        d.vel_dev = None if vel is None else vel.data_ptr()
        d.eps_dev = None if eps is None else eps.data_ptr()
        d.emis_dev = None if emis is None else emis.data_ptr()
        d.kabs_dev = None if kabs is None else kabs.data_ptr()
        if tclass is not None:
            br = [float(v) for v in tclass_bratio]
            d.tclass_dev = tclass.data_ptr()
            d.n_tclass = len(br)
            d.tclass_bratio[:len(br)] = br
        d.bratio_dev = None if bratio is None else bratio.data_ptr()
        self._keep["grid"] = (k0, vel, eps, emis, tclass, kabs, bratio)  # borrowed by the library
        self.bound = None  # no Transport owns the context's grid until it binds
        self._check(self.L.krt_grid_upload(self.h, C.byref(d)))

    def krt_tables_build(self, lines):
        arr = (krt_line_desc * len(lines))()
        for i, (a, phase) in enumerate(lines):
            arr[i].a = float(a)
            arr[i].phase = int(phase)
        self.bound = None
        self._check(self.L.krt_tables_build(self.h, arr, len(lines)))

    def krt_mc_run(self, n_packets, seed, opts: krt_run_opts, tallies: krt_tallies) -> int:
        rc = self.L.krt_mc_run(self.h, int(n_packets), int(seed), C.byref(opts), C.byref(tallies))
        if rc not in (0, KRT_EDEVICE):
            self._check(rc)
        return rc

    def krt_mc_run_noalloc(self, n_packets, seed, opts: krt_run_opts, tallies: krt_tallies) -> int:
        rc = self.L.krt_mc_run_noalloc(self.h, int(n_packets), int(seed), C.byref(opts), C.byref(tallies))
        if rc not in (0, KRT_EDEVICE):
            self._check(rc)
        return rc

    def krt_levels_update(self, desc: krt_levels_desc, jbar=None):
        self._check(self.L.krt_levels_update(self.h, C.byref(desc), _ptr(jbar)))

    # learned escape
    def krt_escape_init(self, seed):
        self._check(self.L.krt_escape_init(self.h, int(seed)))

    def krt_escape_record(self, line, n, seed, offset, lt_lo, lt_hi, out, depth_lo=0.3, x_in=None, q=None,
                          n_in=None):
        """Whole-cell walks: log10 tau_c uniform in [lt_lo, lt_hi]; with x_in and
        q given (reduced frame) every walk starts there, from direction n_in or
        isotropic directions (n_in None); otherwise the training distribution
        with log10 depth from depth_lo up."""
        c = krt_escape_cond()
        c.log10_tau_lo, c.log10_tau_hi, c.log10_depth_lo = float(lt_lo), float(lt_hi), float(depth_lo)
        if x_in is not None:
            c.fixed = 1
            c.x_in = float(x_in)
            c.q[:] = [float(v) for v in q]
            if n_in is None:
                c.iso_dir = 1
            else:
                c.n_in[:] = [float(v) for v in n_in]
        self._check(self.L.krt_escape_record(self.h, int(line), int(n), int(seed), int(offset), C.byref(c),
                                             _ptr(out)))

    def krt_escape_fit_norm(self, rec, n):
        self._check(self.L.krt_escape_fit_norm(self.h, _ptr(rec), int(n)))

    def krt_escape_calibrate(self, rec, n):
        self._check(self.L.krt_escape_calibrate(self.h, _ptr(rec), int(n)))

    def krt_escape_grad(self, rec, idx, u, grad_out, loss_out=None):
        """u: [batch][5] = (u_a, u_b, u_c, u_d, 1 for a conditional row else 0)."""
        if tuple(u.shape) != (idx.numel(), 5):
            raise ValueError(f"u must be [{idx.numel()}][5], got {tuple(u.shape)}")
        self._check(self.L.krt_escape_grad(self.h, _ptr(rec), _ptr(idx), _ptr(u), int(idx.numel()),
                                           _ptr(grad_out), _ptr(loss_out)))

    def krt_escape_train(self, rec, n, steps, batch, lr, seed, loss_hist=None):
        self._check(self.L.krt_escape_train(self.h, _ptr(rec), int(n), int(steps), int(batch), float(lr),
                                            int(seed), _ptr(loss_hist)))

    def krt_escape_get_weights(self, out):
        self._check(self.L.krt_escape_get_weights(self.h, _ptr(out), out.numel()))

    def krt_escape_put_weights(self, w):
        self._check(self.L.krt_escape_put_weights(self.h, _ptr(w), w.numel()))

    def krt_escape_forward(self, inp, out):
        """inp: [n][17] raw (log10 tau_c, log10 a, |x_in|, q0, q1, q2, log10 depth, n_in (3), u_a, u_b,
        u_c, u_d, flag, x_out, face); out: [n][32]."""
        if inp.dim() != 2 or inp.shape[1] != ESC_NIN or tuple(out.shape) != (inp.shape[0], ESC_NOUT):
            raise ValueError(f"inp must be [n][{ESC_NIN}] and out [n][{ESC_NOUT}]")
        self._check(self.L.krt_escape_forward(self.h, _ptr(inp), inp.shape[0], _ptr(out)))

    def krt_image(self, desc: krt_image_desc):
        self._check(self.L.krt_image(self.h, C.byref(desc)))

    def krt_last_image_ms(self) -> float:
        return float(self.L.krt_last_image_ms(self.h))

    def krt_debug_philox(self, ctr, key, out):
        self._check(self.L.krt_debug_philox(self.h, _ptr(ctr), _ptr(key), _ptr(out), ctr.shape[0]))

    def krt_debug_bins(self, x, nb, lo, hi, out):
        self._check(self.L.krt_debug_bins(self.h, _ptr(x), x.numel(), int(nb), float(lo), float(hi), _ptr(out)))

    def krt_debug_voigt_analytic(self, a, x, out):
        self._check(self.L.krt_debug_voigt_analytic(self.h, float(a), _ptr(x), x.numel(), _ptr(out)))

    def krt_debug_voigt_cont(self, line, r, x, out):
        self._check(self.L.krt_debug_voigt_cont(self.h, int(line), _ptr(r), _ptr(x), x.numel(), _ptr(out)))

    def krt_debug_voigt(self, line, x, out):
        self._check(self.L.krt_debug_voigt(self.h, int(line), _ptr(x), x.numel(), _ptr(out)))

    def krt_debug_upar(self, line, x, seed, packet, ev0, out):
        self._check(self.L.krt_debug_upar(self.h, int(line), float(x), int(seed), int(packet), int(ev0),
                                          out.numel(), _ptr(out)))


def make_opts(prob: dict, *, line=0, packet_offset=0, accumulate=False, max_events=0,
              wg_size=0, wg_per_cu=0, emis_frac_bits=0, jbar_frac_bits=0, norm_packets=0, escape_mode=0,
              luminosity=0.0, esc_tau_min=0.0, esc_cell_tau_min=0.0, esc_min_lanes=0, esc_tail_lanes=0,
              tail_lanes=0, profile_mode=0, esc_park=0, esc_park_cap=0, esc_park_tail=0,
              esc_park_budget=0, esc_wait=0) -> krt_run_opts:
    """krt_run_opts from a workload problem dict (paper_2608_09340_amd.workloads)."""
    o = krt_run_opts()
    src, t = prob["source"], prob["tally"]
    o.line = int(line)
    o.source = int(src["kind"])
    o.src_pos[:] = [float(v) for v in src.get("pos", (0.0, 0.0, 0.0))]
    o.src_dir[:] = [float(v) for v in src.get("dir", (0.0, 0.0, 1.0))]
    o.src_profile = int(src.get("profile", 0))
    o.src_x0 = float(src.get("x0", 0.0))
    o.spec_nbins = int(t["spec_nbins"])
    o.spec_lo = float(t["spec_lo"])
    o.spec_hi = float(t["spec_hi"])
    o.emis_nch = int(t.get("emis_nch", 0))
    o.ch_lo = float(t.get("ch_lo", 0.0))
    o.ch_hi = float(t.get("ch_hi", 1.0))
    o.n_cam[:] = [float(v) for v in t.get("n_cam", (1.0, 0.0, 0.0))]
    o.jbar = int(t.get("jbar", 0))
    o.accumulate = int(bool(accumulate))
    o.packet_offset = int(packet_offset)
    mx = max_events or prob.get("max_events", 0)
    o.max_events = int(min(mx, 0xFFFFFFFE)) if mx else 0
    o.escape_mode = int(escape_mode)
    o.wg_size = int(wg_size)
    o.wg_per_cu = int(wg_per_cu)
    o.emis_frac_bits = int(emis_frac_bits)
    o.jbar_frac_bits = int(jbar_frac_bits)
    o.norm_packets = int(norm_packets)
    o.luminosity = float(luminosity)
    o.esc_tau_min = float(esc_tau_min)
    o.esc_cell_tau_min = float(esc_cell_tau_min)
    o.esc_min_lanes = int(esc_min_lanes)
    o.esc_tail_lanes = int(esc_tail_lanes)
    o.esc_park = int(esc_park)
    o.esc_park_cap = int(esc_park_cap)
    o.esc_park_tail = int(esc_park_tail)
    o.esc_park_budget = int(esc_park_budget)
    o.esc_wait = int(esc_wait)
    o.profile_mode = int(profile_mode)
    o.tail_lanes = int(tail_lanes)
    return o


class Transport:
    """Grid + tables + tally buffers for one workload dict, on torch device memory."""

    def __init__(self, prob: dict, device: int = 0, ctx: Context | None = None, lines=None):
        import torch
        self.torch = torch
        self.prob = prob
        self.ctx = ctx or Context(device)
        dev = torch.device("cuda", device)
        self.dev = dev
        g = prob["grid"]
        self.n = [int(v) for v in g["n"]]
        self.ncell = self.n[0] * self.n[1] * self.n[2]
        self.n_lines = int(np.asarray(g["k0"]).size // self.ncell)
        f32 = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
        self.k0 = f32(g["k0"])
        self.vel = f32(g.get("vel"))
        self.eps = f32(g.get("eps"))
        self.emis_w = f32(g.get("emis"))
        self.kabs = f32(g.get("kabs"))
        tcl = g.get("tclass")
        self.tclass = None if tcl is None else torch.from_numpy(
            np.ascontiguousarray(tcl, dtype=np.uint8).reshape(-1)).to(dev)
        self.bratio = f32(g.get("bratio"))
        ln = prob["line"]
        self.lines = [(ln["a"], ln.get("phase", 0))] if lines is None else lines
        self._bind()
        t = prob["tally"]
        self.nsb = int(t["spec_nbins"]) + 2
        self.nch = int(t.get("emis_nch", 0))
        i64 = lambda n: torch.zeros(n, dtype=torch.int64, device=dev)
        self.spec_raw = i64(self.nsb)
        self.counters = i64(KRT_NCOUNTERS)
        self.emis_raw = i64(self.ncell * self.nch) if self.nch > 0 else None
        self.jbar_raw = i64(self.ncell) if t.get("jbar", 0) else None
        self.spec = torch.zeros(self.nsb, dtype=torch.float32, device=dev)
        self.emis = torch.zeros(self.ncell * self.nch, dtype=torch.float32, device=dev) if self.nch > 0 else None
        self.jbar = torch.zeros(self.ncell, dtype=torch.float32, device=dev) if self.jbar_raw is not None else None

    def _bind(self):
        """Upload this workload's grid (borrowed device fields) and build its
        line tables in the context; a context holds one grid at a time, so a
        Transport whose context has since taken another grid binds again
        before its next call."""
        g = self.prob["grid"]
        self.ctx.krt_grid_upload(self.n, g["lo"], g["hi"], g["bc"], self.k0, self.vel, self.eps, self.emis_w,
                                 n_lines=self.n_lines, tclass=self.tclass, tclass_bratio=g.get("tclass_bratio"),
                                 kabs=self.kabs, bratio=self.bratio)
        self.ctx.krt_tables_build(self.lines)
        self.ctx.bound = self

    def _ensure_bound(self):
        if getattr(self.ctx, "bound", None) is not self:
            self._bind()

    def tallies(self, packet_log=None) -> krt_tallies:
        t = krt_tallies()
        t.spec_raw_dev = self.spec_raw.data_ptr()
        t.counters_dev = self.counters.data_ptr()
        t.emis_raw_dev = None if self.emis_raw is None else self.emis_raw.data_ptr()
        t.jbar_raw_dev = None if self.jbar_raw is None else self.jbar_raw.data_ptr()
        t.packet_log_dev = None if packet_log is None else packet_log.data_ptr()
        t.spec_dev = self.spec.data_ptr()
        t.emis_dev = None if self.emis is None else self.emis.data_ptr()
        t.jbar_dev = None if self.jbar is None else self.jbar.data_ptr()
        return t

    def image(self, axis: int = 0, line: int = 0, src=None, kabs=None):
        """Ray-traced image toward the camera axis from the emissivity of the last run
        (its FP32 finalised form), with an optional emission source function
        src [ncell][nch] and grey absorption coefficient kabs [ncell] (device
        FP32); returns a [npix][nch] device tensor."""
        self._ensure_bound()
        t = self.prob["tally"]
        nx, ny, nz = self.n
        npix = {0: ny * nz, 1: nx * nz, 2: nx * ny}[axis % 3]
        out = self.torch.zeros((npix, self.nch), dtype=self.torch.float32, device=self.dev)
        d = krt_image_desc()
        d.line, d.axis, d.nch = int(line), int(axis), int(self.nch)
        d.ch_lo, d.ch_hi = float(t["ch_lo"]), float(t["ch_hi"])
        d.emis_dev = self.emis.data_ptr()
        d.src_dev = None if src is None else src.data_ptr()
        d.kabs_dev = None if kabs is None else kabs.data_ptr()
        d.image_dev = out.data_ptr()
        self.ctx.krt_image(d)
        return out

    def run(self, n_packets: int, seed: int = 0, packet_log: bool = False, noalloc: bool = False,
            host: bool = True, **kw) -> dict:
        """One krt_mc_run (or krt_mc_run_noalloc) over this workload; returns the
        raw tallies and counters on the host (host=False: the counters only, the
        tallies stay in this object's device tensors until the next run)."""
        self._ensure_bound()
        opts = make_opts(self.prob, **kw)
        plog = None
        if packet_log:
            plog = self.torch.zeros((n_packets, 8), dtype=self.torch.float32, device=self.dev)
        call = self.ctx.krt_mc_run_noalloc if noalloc else self.ctx.krt_mc_run
        rc = call(n_packets, seed, opts, self.tallies(plog))
        out = {"rc": rc, "counters": dict(zip(COUNTER_NAMES, self.counters.cpu().numpy()[:len(COUNTER_NAMES)].tolist()))}
        if not host:
            return out
        out["spec_raw"] = self.spec_raw.cpu().numpy().copy()
        if self.emis_raw is not None:
            out["emis_raw"] = self.emis_raw.cpu().numpy().reshape(self.ncell, self.nch).copy()
        if self.jbar_raw is not None:
            out["jbar_raw"] = self.jbar_raw.cpu().numpy().copy()
        if plog is not None:
            out["packet_log"] = plog.cpu().numpy()
        return out
