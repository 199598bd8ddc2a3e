"""ctypes wrapper of the serial C oracle (test infrastructure only).

The wrapper only marshals arguments; every step of the method runs in kmco.c.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

METROPOLIS, BARKER = 0, 1
SCHED_RANDOM_PERM, SCHED_PALINDROME = 0, 1
INIT_RANDOM, INIT_ALL_UP, INIT_GIVEN = 0, 1, 2
F_SCORE, F_CHECK = 1, 2


class Desc(C.Structure):
    _fields_ = [("J", C.c_double), ("h", C.c_double), ("T", C.c_double),
                ("L", C.c_int32), ("tile", C.c_int32),
                ("steps_per_visit", C.c_int32), ("rate_model", C.c_int32),
                ("schedule", C.c_int32), ("init", C.c_int32),
                ("tile_rows", C.c_int32), ("dims", C.c_int32), ("time_slice", C.c_double)]


class Record(C.Structure):
    _fields_ = [("sweep", C.c_int64), ("M", C.c_int64), ("B", C.c_int64),
                ("events", C.c_int64), ("steps", C.c_int64), ("t", C.c_double)]


RECORD_DTYPE = np.dtype([("sweep", "<i8"), ("M", "<i8"), ("B", "<i8"),
                         ("events", "<i8"), ("steps", "<i8"), ("t", "<f8")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.kmco_philox.argtypes = [P, P, P]
        L.kmco_rates.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32,
                                 P, P, P, P]
        L.kmco_rates_z.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                   P, P, P, P]
        L.kmco_schedule_index.argtypes = [C.c_uint64, C.c_int32, C.c_int64]
        L.kmco_schedule_index.restype = C.c_int32
        L.kmco_perm_from_index.argtypes = [C.c_int32, P]
        L.kmco_schedule_index_n.argtypes = [C.c_uint64, C.c_int32, C.c_int64, C.c_int32]
        L.kmco_schedule_index_n.restype = C.c_int32
        L.kmco_perm_from_index_n.argtypes = [C.c_int32, C.c_int32, P]
        L.kmco_get_partition.argtypes = [P, P, P]
        L.kmco_tick_slot.argtypes = [C.c_uint64, C.c_int32, C.c_int64, C.c_int32,
                                     C.c_int32, C.c_uint32, C.c_uint32, P]
        L.kmco_tick_slot.restype = C.c_uint32
        L.kmco_create.argtypes = [C.POINTER(Desc), C.c_uint64, C.c_int32, P]
        L.kmco_create.restype = P
        L.kmco_run.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, P, C.c_int64, P, P]
        L.kmco_run.restype = C.c_int64
        L.kmco_get_spins.argtypes = [P, P]
        L.kmco_get_domain_clocks.argtypes = [P, P, P]
        L.kmco_get_domain_events.argtypes = [P, P]
        L.kmco_check_failures.argtypes = [P]
        L.kmco_check_failures.restype = C.c_int64
        L.kmco_get_retries.argtypes = [P, P, P]
        L.kmco_slice_log.argtypes = [C.c_double]
        L.kmco_slice_log.restype = C.c_double
        L.kmco_count_retry_ticks.argtypes = [C.c_uint64, C.c_int32, C.c_int64, C.c_int32,
                                             C.c_int32, C.c_uint32, C.c_uint32]
        L.kmco_count_retry_ticks.restype = C.c_int64
        L.kmco_destroy.argtypes = [P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().kmco_philox(_ptr(c), _ptr(k), _ptr(o))
    return o


def rates(J, h, T, model=METROPOLIS, z=4):
    """Class rate table for z neighbours (4: square lattice, 2: ring)."""
    r = np.zeros(10, np.uint64)
    w, gJ, gh = (np.zeros(10) for _ in range(3))
    if lib().kmco_rates_z(J, h, T, model, z, _ptr(r), _ptr(w), _ptr(gJ), _ptr(gh)):
        raise ValueError("invalid rate parameters")
    return r, w, gJ, gh


def schedule_index(seed, replica, sweep):
    return lib().kmco_schedule_index(seed, replica, sweep)


def perm_from_index(idx):
    p = np.zeros(4, np.int32)
    lib().kmco_perm_from_index(idx, _ptr(p))
    return p


def schedule_index_n(seed, replica, sweep, n_perm):
    return lib().kmco_schedule_index_n(seed, replica, sweep, n_perm)


def perm_from_index_n(idx, n):
    p = np.zeros(n, np.int32)
    lib().kmco_perm_from_index_n(idx, n, _ptr(p))
    return p


def slice_log(u):
    """The logarithm the time-slice variant decides with (kmco_slice_log)."""
    return lib().kmco_slice_log(float(u))


def count_retry_ticks(seed, replica, sweep, domain, visit, n_ticks, n):
    """Ticks t < n_ticks of one visit whose slot in [0, n) is redrawn."""
    return lib().kmco_count_retry_ticks(seed, replica, sweep, domain, visit, n_ticks, n)


def tick_slot(seed, replica, sweep, domain, visit, tick, n):
    r = C.c_int32(0)
    v = lib().kmco_tick_slot(seed, replica, sweep, domain, visit, tick, n,
                             C.byref(r))
    return v, r.value


class Replica:
    """One replica of the oracle: lattice, clocks and counters."""

    def __init__(self, L, tile, J=1.0, h=0.0, T=2.5, steps_per_visit=0,
                 rate_model=METROPOLIS, schedule=SCHED_RANDOM_PERM,
                 init=INIT_RANDOM, seed=1, replica=0, spins=None, tile_rows=0, dims=2,
                 time_slice=0.0):
        self.desc = Desc(J, h, T, L, tile, steps_per_visit, rate_model,
                         schedule, init, tile_rows, dims, time_slice)
        self.L, self.tile = L, tile
        self.ring = dims == 1
        self.tile_rows = 1 if self.ring else (tile_rows or tile)
        self.nd = tile * self.tile_rows
        self.ND = (L // tile) * ((1 if self.ring else L) // self.tile_rows)
        self.NI = steps_per_visit or self.nd
        given = None
        if spins is not None:
            self._given = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
            given = _ptr(self._given)
        self._h = lib().kmco_create(C.byref(self.desc), seed, replica, given)
        if not self._h:
            raise ValueError("oracle rejected the replica description")

    def run(self, n_sweeps, record_every=1, score=False, check=False, score_abs=False):
        """Records of n_sweeps sweeps; with score, also the score bins
        [n_bins, 2]; with score_abs as well, the bins' sums of absolute
        terms (the scale of rounding differences)."""
        cap = -(-n_sweeps // record_every) if n_sweeps else 0
        rec = np.zeros(max(cap, 1), RECORD_DTYPE)
        sc = np.zeros((max(cap, 1), 2))
        sa = np.zeros((max(cap, 1), 2))
        flags = (F_SCORE if (score or score_abs) else 0) | (F_CHECK if check else 0)
        n = lib().kmco_run(self._h, n_sweeps, record_every, flags, _ptr(rec), cap,
                           _ptr(sc), _ptr(sa) if score_abs else None)
        if n < 0:
            raise ValueError("oracle run failed")
        if score_abs:
            return rec[:n], sc[:cap], sa[:cap]
        if score:
            return rec[:n], sc[:cap]
        return rec[:n]

    def retries(self):
        """(ticks whose slot was redrawn, redraws) over all runs so far."""
        t, d = C.c_int64(0), C.c_int64(0)
        lib().kmco_get_retries(self._h, C.byref(t), C.byref(d))
        return t.value, d.value

    def spins(self):
        out = np.zeros((self.L,) if self.ring else (self.L, self.L), np.int8)
        lib().kmco_get_spins(self._h, _ptr(out))
        return out

    def domain_clocks(self):
        s = np.zeros(self.ND)
        c = np.zeros(self.ND)
        lib().kmco_get_domain_clocks(self._h, _ptr(s), _ptr(c))
        return s, c

    def domain_events(self):
        e = np.zeros(self.ND, np.int64)
        lib().kmco_get_domain_events(self._h, _ptr(e))
        return e

    def partition(self):
        """(colour of each domain, row-major over the domain grid; number of
        colours)."""
        col = np.zeros(self.ND, np.int32)
        n = C.c_int32(0)
        lib().kmco_get_partition(self._h, _ptr(col), C.byref(n))
        return col, n.value

    def check_failures(self):
        return lib().kmco_check_failures(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().kmco_destroy(h)
            self._h = None
