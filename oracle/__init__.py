"""ctypes wrapper of the plain FP64 CPU oracle (``ems_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The GPU library never imports this package
and this package never imports the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ems_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

N_TABLES = 11
TABLE_NAMES = ["sigma_compton", "sigma_phot", "sigma_conv", "S_e-", "R_e-", "sigma_moller",
               "sigma_brem", "S_e+", "R_e+", "sigma_bhabha", "sigma_annih"]

# formula ids (see ems_oracle.h)
F = dict(SIGMA_KN=0, SIGMA_PE=1, SIGMA_PAIR=2, DSDE_PAIR=3, SIGMA_BREM=4, DSDK_BREM=5,
         SBREM=6, SIGMA_MOLLER=7, DSDE_MOLLER=8, SIGMA_BHABHA=9, DSDE_BHABHA=10,
         SION_E=11, SION_P=12, SIGMA_ANNIH=13, DSDE_COMPTON=14, PAIR_FMAX=15, PAIR_F=16,
         BREM_BOUND=17, BREM_F=18, X0=19, HIGHLAND=20, FLUCT_VAR_E=21, FLUCT_VAR_P=22)
SAMPLERS = dict(compton=0, pair=1, brem=2, moller=3, bhabha=4, annih=5)

LIMITERS = dict(ZPLANE=0, WALL=1, SAFETY=2, CONT=3, DISCRETE=4, STOPPED=5, SUBCUT=6,
                ESCAPE_SAFETY=7)
PROCESSES = dict(NONE=0, COMPTON=1, PHOT=2, CONV=3, MOLLER=4, BHABHA=5, BREM=6, ANNIH=7,
                 ANNIH_REST=8, NULL=9)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: plain IEEE double, no contraction."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Material(C.Structure):
    _fields_ = [("Z", C.c_double), ("A_g_mol", C.c_double), ("density_g_cm3", C.c_double),
                ("I_eV", C.c_double), ("n_elements", C.c_uint32), ("el_Z", C.c_double * 4),
                ("el_A", C.c_double * 4), ("el_atoms", C.c_double * 4)]


def material_struct(m) -> Material:
    """(Z, A, rho, I) for an element, (Z, A, rho, I, ((Z, A, atoms), ...))
    for a compound."""
    s = Material(*m[:4])
    if len(m) > 4:
        els = m[4]
        if not 1 <= len(els) <= 4:
            raise ValueError("a compound has 1..4 elements")
        s.n_elements = len(els)
        for i, (z, a, n) in enumerate(els):
            s.el_Z[i], s.el_A[i], s.el_atoms[i] = z, a, n
    return s


class Setup(C.Structure):
    _fields_ = [("n_slabs", C.c_uint32), ("z_mm", C.POINTER(C.c_double)),
                ("material", C.POINTER(C.c_uint32)), ("n_materials", C.c_uint32),
                ("materials", C.POINTER(Material)), ("half_xy_mm", C.c_double),
                ("bz_tesla", C.c_double), ("gamma_cut_MeV", C.c_double),
                ("electron_cut_MeV", C.c_double), ("n_bins", C.c_uint32),
                ("emin_MeV", C.c_double), ("emax_MeV", C.c_double),
                ("dr_over_range", C.c_double), ("final_range_mm", C.c_double),
                ("lin_loss_limit", C.c_double), ("process_mask", C.c_uint32),
                ("max_steps_per_track", C.c_uint32), ("seed", C.c_uint32)]


class Boxes(C.Structure):
    _fields_ = [("n_boxes", C.c_uint32), ("lo", C.POINTER(C.c_double)), ("hi", C.POINTER(C.c_double)),
                ("material", C.POINTER(C.c_uint32)), ("world_lo", C.c_double * 3), ("world_hi", C.c_double * 3),
                ("world_material", C.c_uint32)]


class Ledger(C.Structure):
    _fields_ = [("edep", C.c_double), ("escaped", C.c_double * 3), ("killed", C.c_double),
                ("charged_len", C.c_double), ("n_steps", C.c_uint64),
                ("n_created", C.c_uint64 * 3), ("n_null", C.c_uint64),
                ("n_pair", C.c_uint32), ("n_annih", C.c_uint32)]


LEDGER_DTYPE = np.dtype([("edep", "<f8"), ("escaped", "<f8", (3,)), ("killed", "<f8"),
                         ("charged_len", "<f8"), ("n_steps", "<u8"), ("n_created", "<u8", (3,)),
                         ("n_null", "<u8"), ("n_pair", "<u4"), ("n_annih", "<u4")], align=True)
assert LEDGER_DTYPE.itemsize == C.sizeof(Ledger)

STEP_DTYPE = np.dtype([("event", "<u4"), ("species", "<u4"), ("id", "<u8"), ("step", "<u4"),
                       ("slab_after", "<i4"), ("limiter", "<u4"), ("process", "<u4"),
                       ("e_before", "<f8"), ("e_after", "<f8"), ("pos_after", "<f8", (3,)),
                       ("step_len", "<f8"), ("edep", "<f8")], align=True)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        vp = C.c_void_p
        L.or_create.argtypes = [C.POINTER(Setup), C.POINTER(vp)]
        L.or_create.restype = C.c_int
        L.or_destroy.argtypes = [vp]
        L.or_destroy.restype = None
        L.or_run.argtypes = [vp, vp, C.c_uint64, C.c_uint32, vp, vp, vp, vp, C.c_uint64,
                             C.POINTER(C.c_uint64), vp, C.c_uint32, C.POINTER(C.c_uint32), C.c_int]
        L.or_run.restype = C.c_int
        L.or_run_exits.argtypes = list(L.or_run.argtypes) + [vp, C.c_uint64, C.POINTER(C.c_uint64)]
        L.or_run_exits.restype = C.c_int
        L.or_table_count.argtypes = [vp]
        L.or_table_count.restype = C.c_uint64
        L.or_export_tables.argtypes = [vp, vp, C.c_uint64]
        L.or_export_tables.restype = C.c_int
        L.or_table_lookup.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_double]
        L.or_table_lookup.restype = C.c_double
        L.or_inverse_range.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_double]
        L.or_inverse_range.restype = C.c_double
        L.or_sigma_bound.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_double, C.c_double]
        L.or_sigma_bound.restype = C.c_double
        L.or_sigma_total.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_double]
        L.or_sigma_total.restype = C.c_double
        L.or_formula.argtypes = [C.c_int, C.POINTER(Material), C.c_double, C.c_double, C.c_double]
        L.or_formula.restype = C.c_double
        L.or_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.or_philox.restype = None
        L.or_uniform.argtypes = [C.POINTER(C.c_uint32), C.c_uint64, C.c_uint32, C.c_uint32]
        L.or_uniform.restype = C.c_double
        L.or_child_id.argtypes = [C.POINTER(C.c_uint32), C.c_uint64, C.c_uint32, C.c_uint32]
        L.or_child_id.restype = C.c_uint64
        L.or_sample.argtypes = [vp, C.c_int, C.c_uint32, C.c_double, C.POINTER(C.c_double),
                                C.POINTER(C.c_uint32), C.c_uint64, C.c_uint32, C.POINTER(C.c_double)]
        L.or_sample.restype = C.c_int
        L.or_sample_along.argtypes = [vp, C.c_int, C.c_uint32, C.c_double, C.c_double, C.c_double,
                                      C.POINTER(C.c_double), C.POINTER(C.c_uint32), C.c_uint64, C.c_uint32,
                                      C.POINTER(C.c_double)]
        L.or_sample_along.restype = C.c_int
        L.or_create_boxes.argtypes = [C.POINTER(Setup), C.POINTER(Boxes), C.POINTER(vp)]
        L.or_create_boxes.restype = C.c_int
        L.or_geo_locate.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_geo_locate.restype = C.c_int
        L.or_geo_distance.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.or_geo_distance.restype = C.c_double
        L.or_geo_helix_distance.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                                            C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.or_geo_helix_distance.restype = C.c_double
        _lib = L
    return _lib


def _u32(a):
    return (C.c_uint32 * len(a))(*[int(x) & 0xFFFFFFFF for x in a])


def philox(ctr, key):
    out = (C.c_uint32 * 4)()
    lib().or_philox(_u32(ctr), _u32(key), out)
    return list(out)


def uniform(key, track_id, step, i):
    return lib().or_uniform(_u32(key), track_id, step, i)


def child_id(key, track_id, step, k):
    return lib().or_child_id(_u32(key), track_id, step, k)


def formula(which, material, cut, E, arg2=0.0):
    m = material_struct(material)
    w = F[which] if isinstance(which, str) else which
    return lib().or_formula(w, C.byref(m), cut, E, arg2)


class Oracle:
    """Oracle context: tables built once, then any number of runs."""

    def __init__(self, geometry, config):
        self.geo = geometry
        self.cfg = config
        boxes = hasattr(geometry, "world_lo")
        self._mat = np.ascontiguousarray(geometry.material, dtype=np.uint32)
        self._mats = (Material * len(geometry.materials))(*[material_struct(m) for m in geometry.materials])
        s = Setup()
        if boxes:
            self._lo = np.ascontiguousarray(geometry.lo, dtype=np.float64)
            self._hi = np.ascontiguousarray(geometry.hi, dtype=np.float64)
            b = Boxes()
            b.n_boxes = geometry.n_boxes
            b.lo = self._lo.ctypes.data_as(C.POINTER(C.c_double))
            b.hi = self._hi.ctypes.data_as(C.POINTER(C.c_double))
            b.material = self._mat.ctypes.data_as(C.POINTER(C.c_uint32))
            b.world_lo[:] = geometry.world_lo
            b.world_hi[:] = geometry.world_hi
            b.world_material = geometry.world_material
            self._boxes = b
        else:
            self._z = np.ascontiguousarray(geometry.z_mm, dtype=np.float64)
            s.n_slabs = geometry.n_slabs
            s.z_mm = self._z.ctypes.data_as(C.POINTER(C.c_double))
            s.material = self._mat.ctypes.data_as(C.POINTER(C.c_uint32))
            s.half_xy_mm = geometry.half_xy_mm
        s.n_materials = len(geometry.materials)
        s.materials = self._mats
        for f in ("bz_tesla", "gamma_cut_MeV", "electron_cut_MeV", "n_bins", "emin_MeV", "emax_MeV",
                  "dr_over_range", "final_range_mm", "lin_loss_limit", "process_mask",
                  "max_steps_per_track", "seed"):
            setattr(s, f, getattr(config, f))
        self._setup = s
        h = C.c_void_p()
        if boxes:
            rc = lib().or_create_boxes(C.byref(s), C.byref(self._boxes), C.byref(h))
        else:
            rc = lib().or_create(C.byref(s), C.byref(h))
        if rc != 0:
            raise ValueError(f"or_create failed ({rc})")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tables ---------------------------------------------------------
    def tables(self) -> np.ndarray:
        n = lib().or_table_count(self._h)
        out = np.empty(n, dtype=np.float64)
        rc = lib().or_export_tables(self._h, out.ctypes.data_as(C.c_void_p), n)
        assert rc == 0
        return out.reshape(len(self.geo.materials), N_TABLES, self.cfg.n_bins + 1)

    def lookup(self, material, table, E):
        t = TABLE_NAMES.index(table) if isinstance(table, str) else table
        return lib().or_table_lookup(self._h, material, t, E)

    def inverse_range(self, material, species, r):
        return lib().or_inverse_range(self._h, material, species, r)

    def sigma_bound(self, material, species, a, b):
        """null-collision bound of an e-/e+ step spanning [a, b] MeV"""
        return lib().or_sigma_bound(self._h, material, species, a, b)

    def sigma_total(self, material, species, E):
        """right-continuous interpolated discrete total of e-/e+ at E"""
        return lib().or_sigma_total(self._h, material, species, E)

    def sample(self, which, material, E, key, track_id, step, direction=(0.0, 0.0, 1.0)):
        out = (C.c_double * 16)()
        d = (C.c_double * 3)(*direction)
        w = SAMPLERS[which] if isinstance(which, str) else which
        rc = lib().or_sample(self._h, w, material, E, d, _u32(key), track_id, step, out)
        if rc != 0:
            raise ValueError("or_sample rejected its arguments")
        return np.array(out[:])

    def sample_along(self, which, material, T, s, key, track_id, step, mean=0.0, direction=(0.0, 0.0, 1.0)):
        """which: 'msc' -> [theta0, ux, uy, uz]; 'fluct_e-' / 'fluct_e+' ->
        [loss, variance]"""
        out = (C.c_double * 4)()
        d = (C.c_double * 3)(*direction)
        w = dict(msc=0, **{"fluct_e-": 1, "fluct_e+": 2})[which]
        rc = lib().or_sample_along(self._h, w, material, T, s, mean, d, _u32(key), track_id, step, out)
        if rc != 0:
            raise ValueError("or_sample_along rejected its arguments")
        return np.array(out[:])

    def geo_locate(self, p, u):
        return lib().or_geo_locate(self._h, (C.c_double * 3)(*p), (C.c_double * 3)(*u))

    def geo_distance(self, v, p, u):
        """(distance, axis, face coordinate) to the next boundary"""
        ax = C.c_int()
        f = C.c_double()
        d = lib().or_geo_distance(self._h, v, (C.c_double * 3)(*p), (C.c_double * 3)(*u), C.byref(ax), C.byref(f))
        return d, ax.value, f.value

    def geo_helix_distance(self, v, p, u, kappa, smax=float("inf")):
        """(path length, axis, face coordinate) to the next boundary along the
        helix of signed curvature kappa (1/mm) about z, searched up to smax"""
        ax = C.c_int()
        f = C.c_double()
        d = lib().or_geo_helix_distance(self._h, v, (C.c_double * 3)(*p), (C.c_double * 3)(*u), float(kappa),
                                        float(smax), C.byref(ax), C.byref(f))
        return d, ax.value, f.value

    # -- transport ------------------------------------------------------
    def run(self, prim: np.ndarray, n_events: int | None = None, event_keys=None,
            log_cap: int = 0, profile_cap: int = 0, stack_order: int = 0, exit_cap: int = 0):
        """Transport the primaries; returns a dict with edep [n_events, n_slabs],
        ledger (structured array), and optionally the step log / profile and
        the tracks leaving the stack (primary-record layout)."""
        prim = np.ascontiguousarray(prim)
        if n_events is None:
            n_events = int(prim["event"].max()) + 1 if len(prim) else 0
        edep = np.zeros((n_events, self.geo.n_cols), dtype=np.float64)
        ledger = np.zeros(n_events, dtype=LEDGER_DTYPE)
        keys = None
        if event_keys is not None:
            keys = np.ascontiguousarray(event_keys, dtype=np.uint32)
        log = np.zeros(log_cap, dtype=STEP_DTYPE) if log_cap else None
        log_n = C.c_uint64(0)
        prof = np.zeros((profile_cap, 3), dtype=np.uint64) if profile_cap else None
        prof_len = C.c_uint32(0)
        exits = np.zeros(exit_cap, dtype=prim.dtype) if exit_cap else None
        exits_n = C.c_uint64(0)
        rc = lib().or_run_exits(self._h, prim.ctypes.data_as(C.c_void_p), len(prim), n_events,
                                None if keys is None else keys.ctypes.data_as(C.c_void_p),
                                edep.ctypes.data_as(C.c_void_p), ledger.ctypes.data_as(C.c_void_p),
                                None if log is None else log.ctypes.data_as(C.c_void_p), log_cap,
                                C.byref(log_n),
                                None if prof is None else prof.ctypes.data_as(C.c_void_p), profile_cap,
                                C.byref(prof_len), stack_order,
                                None if exits is None else exits.ctypes.data_as(C.c_void_p), exit_cap,
                                C.byref(exits_n) if exit_cap else None)
        if rc != 0:
            raise ValueError(f"or_run failed ({rc})")
        out = dict(edep=edep, ledger=ledger, n_log=int(log_n.value), n_iter=int(prof_len.value))
        if exits is not None:
            out["n_exits"] = int(exits_n.value)
            out["exits"] = exits[: min(exit_cap, int(exits_n.value))]
        if log is not None:
            out["log"] = log[: min(log_cap, int(log_n.value))]
        if prof is not None:
            out["profile"] = prof[: min(profile_cap, int(prof_len.value))]
        return out
