"""Python binding of the MI355X EM-shower transport library (libems.so).

Argument marshalling only: every step of the transport runs in the HIP
kernels of ``csrc/``.  PyTorch supplies the device workspace (a uint8 tensor)
and the HIP stream.  If the compiled library is missing this module raises
on import -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libems.so")

ABI_VERSION = 8
OK, E_INVALID, E_CAPACITY, E_DEVICE, E_STATE, E_BUSY, E_TIMEOUT, E_VERSION = 0, -1, -2, -3, -4, -5, -6, -7
FP64, MIXED = 0, 1
# e- secondaries below this energy take their first step in the short-electron
# launch (ems_config.short_electron_MeV; 0 turns it off), by form.  Off by
# default: it pays off only for large e- populations in the mixed form
SHORT_ELECTRON_MEV = {0: 0.0, 1: 0.0}
F_STEPLOG, F_FULL_LEDGER, F_PROFILE, F_EVENT_LIVE, F_KERNEL_TIMING, F_NO_GRAPH, F_FULL_KERNELS = 1, 2, 4, 8, 16, 32, 64


class EmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ems error {code}: {msg}")
        self.code = code


class Material(C.Structure):
    _fields_ = [("Z", C.c_double), ("A_g_mol", C.c_double), ("density_g_cm3", C.c_double), ("I_eV", C.c_double),
                ("n_elements", C.c_uint32), ("el_Z", C.c_double * 4), ("el_A", C.c_double * 4),
                ("el_atoms", C.c_double * 4)]

    @classmethod
    def of(cls, m):
        """(Z, A, rho, I) for an element; (Z, A, rho, I, ((Z_i, A_i, atoms_i), ...))
        for a compound of 1..4 elements"""
        out = cls(*m[:4])
        if len(m) > 4:
            out.n_elements = len(m[4])  # above 4: rejected by the library
            for i, (z, a, n) in enumerate(m[4][:4]):
                out.el_Z[i], out.el_A[i], out.el_atoms[i] = z, a, n
        return out


class Geometry(C.Structure):
    _fields_ = [("n_slabs", C.c_uint32), ("z_mm", C.POINTER(C.c_double)), ("material", C.POINTER(C.c_uint32)),
                ("n_materials", C.c_uint32), ("materials", C.POINTER(Material)), ("half_xy_mm", C.c_double),
                ("n_boxes", C.c_uint32), ("box_lo", C.POINTER(C.c_double)), ("box_hi", C.POINTER(C.c_double)),
                ("box_material", C.POINTER(C.c_uint32)), ("world_lo", C.c_double * 3), ("world_hi", C.c_double * 3),
                ("world_material", C.c_uint32)]


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("precision", C.c_uint32), ("bz_tesla", C.c_double),
                ("gamma_cut_MeV", C.c_double), ("electron_cut_MeV", C.c_double), ("n_bins", C.c_uint32),
                ("emin_MeV", C.c_double), ("emax_MeV", C.c_double), ("dr_over_range", C.c_double),
                ("final_range_mm", C.c_double), ("lin_loss_limit", C.c_double), ("process_mask", C.c_uint32),
                ("flags", C.c_uint32), ("max_steps_per_track", C.c_uint32), ("seed", C.c_uint32),
                ("max_events", C.c_uint32), ("track_capacity", C.c_uint64), ("steps_per_launch", C.c_uint32),
                ("launch_blocks", C.c_uint32), ("steplog_capacity", C.c_uint64), ("profile_capacity", C.c_uint32),
                ("steps_per_visit", C.c_uint32), ("refill_below", C.c_uint32), ("interact_min", C.c_uint32),
                ("photon_steps_per_visit", C.c_uint32), ("photon_refill_below", C.c_uint32),
                ("exit_capacity", C.c_uint64), ("short_electron_MeV", C.c_double)]


class RunStats(C.Structure):
    _fields_ = [("iterations", C.c_uint64), ("steps", C.c_uint64 * 3), ("created", C.c_uint64 * 3),
                ("deferred", C.c_uint64), ("launches", C.c_uint64), ("peak_live", C.c_uint32 * 3),
                ("steplog_overflow", C.c_uint32), ("run_ms", C.c_double), ("step_kernel_ms", C.c_double),
                ("visits", C.c_uint64 * 3), ("made_by", C.c_uint64 * 2), ("kernel_ms", C.c_double * 3),
                ("graph_launches", C.c_uint64), ("short_steps", C.c_uint64)]


class LoadRequest(C.Structure):
    _fields_ = [("tracks", C.c_void_p), ("n_tracks", C.c_uint32), ("event_key", C.c_uint32),
                ("arrival_ns", C.c_uint64)]


class ServerInfo(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("in_flight", C.c_uint64),
                ("queued", C.c_uint64), ("admitted_bytes", C.c_uint64), ("admit_cap_bytes", C.c_uint64),
                ("peak_admitted_bytes", C.c_uint64), ("primaries_completed", C.c_uint64), ("chunks", C.c_uint64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("max_ms", C.c_double),
                ("wall_s", C.c_double), ("primaries_per_s", C.c_double), ("exits_dropped", C.c_uint64)]


LEDGER_DTYPE = np.dtype([("edep", "<f8"), ("escaped", "<f8", (3,)), ("killed", "<f8"), ("charged_len", "<f8"),
                         ("n_steps", "<u8"), ("n_created", "<u8", (3,)), ("n_null", "<u8"), ("n_pair", "<u4"),
                         ("n_annih", "<u4")], align=True)
STEP_DTYPE = np.dtype([("event", "<u4"), ("species", "<u4"), ("id", "<u8"), ("step", "<u4"), ("slab_after", "<i4"),
                       ("limiter", "<u4"), ("process", "<u4"), ("e_before", "<f8"), ("e_after", "<f8"),
                       ("pos_after", "<f8", (3,)), ("step_len", "<f8"), ("edep", "<f8")], align=True)
PRIMARY_DTYPE = np.dtype([("event", "<u4"), ("species", "<u4"), ("ekin", "<f8"), ("pos", "<f8", (3,)),
                          ("dir", "<f8", (3,))], align=True)

_lib = None


def lib():
    """Loads libems.so (after torch, so both use the same HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        try:
            import torch  # noqa: F401  (loads the HIP runtime torch uses)
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
        sig = {
            "ems_workspace_bytes": [C.POINTER(Config), C.POINTER(Geometry), C.POINTER(u64)],
            "ems_create": [C.POINTER(Config), C.POINTER(Geometry), vp, u64, vp, C.POINTER(vp)],
            "ems_create_static": [C.POINTER(Config), C.POINTER(Geometry), vp, C.POINTER(vp)],
            "ems_set_event_keys": [vp, u32, u32, vp],
            "ems_enqueue": [vp, vp, u64],
            "ems_enqueue_device": [vp, vp, u64],
            "ems_read_edep_device": [vp, u32, u32, vp],
            "ems_run": [vp],
            "ems_read_edep": [vp, u32, u32, vp],
            "ems_read_ledger": [vp, u32, u32, vp],
            "ems_reset_tallies": [vp],
            "ems_read_steplog": [vp, vp, u64, C.POINTER(u64)],
            "ems_read_profile": [vp, vp, u32, C.POINTER(u32)],
            "ems_read_exits": [vp, vp, u64, C.POINTER(u64)],
            "ems_stats": [vp, C.POINTER(RunStats)],
            "ems_destroy": [vp],
            "ems_host_tables": [C.POINTER(Config), C.POINTER(Geometry), vp, u64],
            "ems_export_tables": [vp, vp, u64],
            "ems_debug_host_transport": [C.POINTER(Config), C.POINTER(Geometry), vp, u64, u32, vp, vp, vp, vp, u64,
                                         C.POINTER(u64)],
            "ems_server_create": [C.POINTER(Config), C.POINTER(Geometry), vp, u64, vp, u64, C.POINTER(vp)],
            "ems_server_submit": [vp, vp, u32, u32, C.POINTER(u64)],
            "ems_server_submit_at": [vp, vp, u32, u32, u64, C.POINTER(u64)],
            "ems_server_wait": [vp, u64, C.c_int64, vp, vp],
            "ems_server_wait_exits": [vp, u64, C.c_int64, vp, vp, vp, u64, C.POINTER(u64)],
            "ems_server_poll": [vp, u64, C.POINTER(C.c_int)],
            "ems_server_flush": [vp],
            "ems_server_stats": [vp, C.POINTER(ServerInfo)],
            "ems_server_reset_stats": [vp],
            "ems_server_destroy": [vp],
            "ems_server_drive": [vp, vp, vp, u32, u32, C.POINTER(C.c_double), C.POINTER(u64)],
            "ems_probe_atomics": [vp, u64, u64, vp, C.POINTER(C.c_double)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.ems_last_error.argtypes = []
        L.ems_last_error.restype = C.c_char_p
        L.ems_abi_version.argtypes = []
        L.ems_abi_version.restype = C.c_uint32
        if L.ems_abi_version() != ABI_VERSION:
            raise ImportError("libems.so ABI version mismatch")
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise EmsError(rc, lib().ems_last_error().decode())
    return rc


class _GeoHolder:
    """Keeps the arrays a Geometry struct points to alive."""

    def __init__(self, geometry):
        self.mat = np.ascontiguousarray(geometry.material, dtype=np.uint32)
        self.mats = (Material * len(geometry.materials))(*[Material.of(m) for m in geometry.materials])
        g = Geometry()
        if hasattr(geometry, "world_lo"):  # boxes
            self.lo = np.ascontiguousarray(geometry.lo, dtype=np.float64)
            self.hi = np.ascontiguousarray(geometry.hi, dtype=np.float64)
            g.n_boxes = len(self.mat)
            g.box_lo = self.lo.ctypes.data_as(C.POINTER(C.c_double))
            g.box_hi = self.hi.ctypes.data_as(C.POINTER(C.c_double))
            g.box_material = self.mat.ctypes.data_as(C.POINTER(C.c_uint32))
            g.world_lo[:] = geometry.world_lo
            g.world_hi[:] = geometry.world_hi
            g.world_material = int(geometry.world_material)
            self.n_slabs = len(self.mat) + 1  # deposit columns: boxes, then the world
        else:
            self.z = np.ascontiguousarray(geometry.z_mm, dtype=np.float64)
            g.n_slabs = len(self.mat)
            g.z_mm = self.z.ctypes.data_as(C.POINTER(C.c_double))
            g.material = self.mat.ctypes.data_as(C.POINTER(C.c_uint32))
            g.half_xy_mm = float(geometry.half_xy_mm)
            self.n_slabs = len(self.mat)
        g.n_materials = len(geometry.materials)
        g.materials = self.mats
        self.g = g


def make_config(run, max_events, track_capacity=1 << 20, precision=FP64, flags=0, steps_per_launch=16,
                launch_blocks=0, steplog_capacity=0, profile_capacity=0, steps_per_visit=16, refill_below=32,
                interact_min=24, exit_capacity=0, photon_steps_per_visit=None, photon_refill_below=None,
                short_electron_MeV=None):
    """Config struct from a run description (any object with the physics
    fields: bz_tesla, cuts, grid, step function, mask, watchdog, seed).  The
    launch parameters (steps_per_visit, refill_below, interact_min, the
    photon kernel's photon_steps_per_visit and photon_refill_below, and the
    short-electron threshold short_electron_MeV) shape the kernels' work and
    change no result."""
    c = Config()
    c.abi_version = ABI_VERSION
    c.precision = precision
    for f in ("bz_tesla", "gamma_cut_MeV", "electron_cut_MeV", "n_bins", "emin_MeV", "emax_MeV", "dr_over_range",
              "final_range_mm", "lin_loss_limit", "process_mask", "max_steps_per_track", "seed"):
        setattr(c, f, getattr(run, f))
    c.flags = flags
    c.max_events = max_events
    c.track_capacity = track_capacity
    c.steps_per_launch = steps_per_launch
    c.launch_blocks = launch_blocks
    c.steplog_capacity = steplog_capacity
    c.profile_capacity = profile_capacity
    c.steps_per_visit = steps_per_visit
    c.refill_below = refill_below
    c.interact_min = interact_min
    # the photon kernel's visit length and refill threshold: the shared ones
    # unless given
    c.photon_steps_per_visit = steps_per_visit if photon_steps_per_visit is None else photon_steps_per_visit
    c.photon_refill_below = refill_below if photon_refill_below is None else photon_refill_below
    c.exit_capacity = exit_capacity
    c.short_electron_MeV = SHORT_ELECTRON_MEV[precision] if short_electron_MeV is None else short_electron_MeV
    return c


def workspace_bytes(config, geometry) -> int:
    gh = _GeoHolder(geometry)
    n = C.c_uint64()
    _check(lib().ems_workspace_bytes(C.byref(config), C.byref(gh.g), C.byref(n)))
    return n.value


def host_tables(config, geometry) -> np.ndarray:
    gh = _GeoHolder(geometry)
    nodes = config.n_bins + 1
    out = np.empty(len(geometry.materials) * 11 * nodes)
    _check(lib().ems_host_tables(C.byref(config), C.byref(gh.g), out.ctypes.data_as(C.c_void_p), out.size))
    return out.reshape(len(geometry.materials), 11, nodes)


def _prim(prim):
    p = np.ascontiguousarray(prim)
    if p.dtype.itemsize != 64:
        raise ValueError("primaries must be 64-byte records")
    return p


def debug_host_transport(config, geometry, prim, n_events, keys=None, log_cap=0):
    """Runs the library's step code on the host (test hook)."""
    gh = _GeoHolder(geometry)
    p = _prim(prim)
    edep = np.zeros((n_events, gh.n_slabs))
    led = np.zeros(n_events, dtype=LEDGER_DTYPE)
    log = np.zeros(log_cap, dtype=STEP_DTYPE) if log_cap else None
    n = C.c_uint64()
    k = None if keys is None else np.ascontiguousarray(keys, dtype=np.uint32)
    _check(lib().ems_debug_host_transport(
        C.byref(config), C.byref(gh.g), p.ctypes.data_as(C.c_void_p), len(p), n_events,
        None if k is None else k.ctypes.data_as(C.c_void_p), edep.ctypes.data_as(C.c_void_p),
        led.ctypes.data_as(C.c_void_p), None if log is None else log.ctypes.data_as(C.c_void_p), log_cap,
        C.byref(n)))
    out = dict(edep=edep, ledger=led, n_log=n.value)
    if log is not None:
        out["log"] = log[: min(log_cap, n.value)]
    return out


class Transport:
    """One transport context on the current HIP device.

    The workspace is a torch uint8 tensor on the device; the stream is the
    given torch stream, by default a stream of its own (default priority):
    chunks of iterations are replayed as captured graphs, which the null
    stream does not allow.  With static_workspace=True the context runs in
    the library's static device workspace instead (ems_create_static: no
    device allocation by the library or by this wrapper; one such context
    per device at a time)."""

    def __init__(self, config, geometry, stream=None, device="cuda", static_workspace=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the transport runs only on the GPU")
        self.config = config
        self._gh = _GeoHolder(geometry)
        self.n_slabs = self._gh.n_slabs
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        if static_workspace:
            self.workspace = None
            _check(lib().ems_create_static(C.byref(config), C.byref(self._gh.g),
                                           C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        else:
            nbytes = workspace_bytes(config, geometry)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            _check(lib().ems_create(C.byref(config), C.byref(self._gh.g), C.c_void_p(self._ws_ptr), nbytes,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ems_destroy(self._h)
            self._h = None
        self.workspace = None  # device memory back to the allocator

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_event_keys(self, keys, first_row=0):
        k = np.ascontiguousarray(keys, dtype=np.uint32)
        _check(lib().ems_set_event_keys(self._h, first_row, len(k), k.ctypes.data_as(C.c_void_p)))

    def enqueue(self, prim):
        p = _prim(prim)
        _check(lib().ems_enqueue(self._h, p.ctypes.data_as(C.c_void_p), len(p)))

    def enqueue_device(self, prim):
        """Primaries already in device memory: a contiguous CUDA tensor holding
        whole 64-byte primary records (e.g. a uint8 copy of a PRIMARY_DTYPE
        array)."""
        nbytes = prim.numel() * prim.element_size()
        if not prim.is_cuda or not prim.is_contiguous() or nbytes % PRIMARY_DTYPE.itemsize:
            raise ValueError("primaries must be a contiguous device tensor of whole 64-byte records")
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(prim.device))  # the records are written
        prim.record_stream(self.stream)  # and stay allocated until the library's stream has read them
        _check(lib().ems_enqueue_device(self._h, C.c_void_p(prim.data_ptr()), nbytes // PRIMARY_DTYPE.itemsize))

    def run(self):
        _check(lib().ems_run(self._h))

    def edep(self, first=0, n=None):
        n = self.config.max_events - first if n is None else n
        out = np.empty((n, self.n_slabs))
        _check(lib().ems_read_edep(self._h, first, n, out.ctypes.data_as(C.c_void_p)))
        return out

    def edep_device(self, out, first=0):
        """Deposits of rows [first, first + out.shape[0]) into `out`, a
        contiguous float64 CUDA tensor of shape (rows, n_slabs), copied on the
        context's stream; the caller's current stream waits for the copy."""
        import torch
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.dim() == 2
                and out.shape[1] == self.n_slabs):
            raise ValueError("out must be a contiguous float64 device tensor of shape (rows, n_slabs)")
        self.stream.wait_stream(torch.cuda.current_stream(out.device))  # earlier uses of out are done
        _check(lib().ems_read_edep_device(self._h, first, out.shape[0], C.c_void_p(out.data_ptr())))
        out.record_stream(self.stream)
        torch.cuda.current_stream(out.device).wait_stream(self.stream)  # later reads see the copy
        return out

    def ledger(self, first=0, n=None):
        n = self.config.max_events - first if n is None else n
        out = np.zeros(n, dtype=LEDGER_DTYPE)
        _check(lib().ems_read_ledger(self._h, first, n, out.ctypes.data_as(C.c_void_p)))
        return out

    def reset(self):
        _check(lib().ems_reset_tallies(self._h))

    def steplog(self):
        n = C.c_uint64()
        _check(lib().ems_read_steplog(self._h, None, 0, C.byref(n)))
        cap = min(n.value, self.config.steplog_capacity)
        out = np.zeros(cap, dtype=STEP_DTYPE)
        _check(lib().ems_read_steplog(self._h, out.ctypes.data_as(C.c_void_p), cap, C.byref(n)))
        return out, n.value

    def profile(self):
        n = C.c_uint32()
        _check(lib().ems_read_profile(self._h, None, 0, C.byref(n)))
        cap = min(n.value, self.config.profile_capacity)
        out = np.zeros((cap, 3), dtype=np.uint32)
        _check(lib().ems_read_profile(self._h, out.ctypes.data_as(C.c_void_p), cap, C.byref(n)))
        return out, n.value

    def exits(self):
        """Tracks that left the stack since the last reset (primary records:
        event row, species, kinetic energy, exit point, direction) and the
        number of exits including those beyond exit_capacity."""
        n = C.c_uint64()
        _check(lib().ems_read_exits(self._h, None, 0, C.byref(n)))
        out = np.zeros(min(n.value, self.config.exit_capacity), dtype=PRIMARY_DTYPE)
        if len(out):
            _check(lib().ems_read_exits(self._h, out.ctypes.data_as(C.c_void_p), len(out), C.byref(n)))
        return out, n.value

    def export_tables(self):
        """The tables this context uploaded, read back from the device:
        [n_materials, 11, n_bins + 1] in the order of host_tables (FP32
        values widened in the mixed form)."""
        nm = self._gh.g.n_materials
        out = np.empty(nm * 11 * (self.config.n_bins + 1))
        _check(lib().ems_export_tables(self._h, out.ctypes.data_as(C.c_void_p), out.size))
        return out.reshape(nm, 11, self.config.n_bins + 1)

    def stats(self):
        s = RunStats()
        _check(lib().ems_stats(self._h, C.byref(s)))
        return dict(iterations=s.iterations, steps=list(s.steps), created=list(s.created), deferred=s.deferred,
                    launches=s.launches, peak_live=list(s.peak_live), steplog_overflow=s.steplog_overflow,
                    run_ms=s.run_ms, step_kernel_ms=s.step_kernel_ms, visits=list(s.visits),
                    made_by=list(s.made_by), kernel_ms=list(s.kernel_ms), graph_launches=s.graph_launches,
                    short_steps=s.short_steps)


def probe_atomics(cells, n_ops, stream=None):
    """FP64 atomic-add throughput: n_ops adds spread uniformly over the
    cells of `cells` (a float64 CUDA tensor, zeroed and left holding the
    counts); returns the device time in ms."""
    import torch
    if not (cells.is_cuda and cells.dtype == torch.float64 and cells.is_contiguous()):
        raise ValueError("cells must be a contiguous float64 device tensor")
    s = stream if stream is not None else torch.cuda.current_stream()
    ms = C.c_double()
    _check(lib().ems_probe_atomics(C.c_void_p(cells.data_ptr()), cells.numel(), int(n_ops),
                                   C.c_void_p(s.cuda_stream), C.byref(ms)))
    return ms.value


class Server:
    """Continuous-batching offload server (one driver thread on the device).

    submit() and wait() may be called from any number of threads; ctypes
    releases the GIL during the calls."""

    def __init__(self, config, geometry, admit_cap_bytes, stream=None, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the server runs only on the GPU")
        self.config = config
        self._gh = _GeoHolder(geometry)
        self.n_slabs = self._gh.n_slabs
        sized = Config.from_buffer_copy(config)
        sized.flags |= F_EVENT_LIVE  # the server's context keeps per-event live counters
        nbytes = workspace_bytes(sized, geometry)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.Stream()
        torch.cuda.synchronize()
        h = C.c_void_p()
        _check(lib().ems_server_create(C.byref(config), C.byref(self._gh.g), C.c_void_p(ptr), nbytes,
                                       C.c_void_p(self.stream.cuda_stream), admit_cap_bytes, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ems_server_destroy(self._h)
            self._h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, tracks, key, arrival_ns=0):
        """Queues one request; its latency counts from arrival_ns (a
        time.monotonic_ns() value, e.g. a scheduled arrival) if given and
        not later than now, else from this call."""
        p = _prim(tracks)
        t = C.c_uint64()
        _check(lib().ems_server_submit_at(self._h, p.ctypes.data_as(C.c_void_p), len(p), int(key),
                                          int(arrival_ns), C.byref(t)))
        return t.value

    def wait(self, ticket, timeout_s=None, exits=False):
        """(edep, ledger) of a finished request, plus its outgoing tracks
        (primary records, event field 0) when exits=True."""
        edep = np.empty(self.n_slabs)
        led = np.zeros(1, dtype=LEDGER_DTYPE)
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        if not exits:
            _check(lib().ems_server_wait(self._h, ticket, us, edep.ctypes.data_as(C.c_void_p),
                                         led.ctypes.data_as(C.c_void_p)))
            return edep, led[0]
        cap = 1024
        while True:
            buf = np.zeros(cap, dtype=PRIMARY_DTYPE)
            n = C.c_uint64()
            rc = lib().ems_server_wait_exits(self._h, ticket, us, edep.ctypes.data_as(C.c_void_p),
                                             led.ctypes.data_as(C.c_void_p), buf.ctypes.data_as(C.c_void_p),
                                             cap, C.byref(n))
            if rc == E_CAPACITY and n.value > cap:
                cap = int(n.value)  # the result is kept for the retry
                continue
            _check(rc)
            return edep, led[0], buf[: n.value]

    def drive(self, producers, window=64):
        """Native producer threads (ems_server_drive): producers[p] is a list
        of (tracks, event_key, arrival_ns) submitted in order by thread p
        (arrival_ns 0: closed loop with `window` outstanding; else at that
        time.monotonic_ns() instant, latency counted from it).  Returns
        (largest submission lag in ms, monotonic time of the last
        submission in ns)."""
        keep, flat, first = [], [], [0]
        for reqs in producers:
            for tracks, key, arrival in reqs:
                p = _prim(tracks)
                keep.append(p)
                flat.append(LoadRequest(p.ctypes.data, len(p), int(key), int(arrival)))
            first.append(len(flat))
        arr = (LoadRequest * len(flat))(*flat)
        fst = (C.c_uint64 * len(first))(*first)
        lag, last = C.c_double(), C.c_uint64()
        _check(lib().ems_server_drive(self._h, arr, fst, len(producers), int(window), C.byref(lag), C.byref(last)))
        return lag.value, last.value

    def poll(self, ticket):
        d = C.c_int()
        _check(lib().ems_server_poll(self._h, ticket, C.byref(d)))
        return bool(d.value)

    def flush(self):
        _check(lib().ems_server_flush(self._h))

    def reset_stats(self):
        _check(lib().ems_server_reset_stats(self._h))

    def stats(self):
        s = ServerInfo()
        _check(lib().ems_server_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerInfo._fields_}
