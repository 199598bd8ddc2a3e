"""Python binding of libkmc (argument marshalling only).

Every function here has the name of the C call it wraps (include/kmc.h) and
does nothing but convert arguments; every step of the method runs in the
HIP kernels of libkmc.so.  PyTorch provides the device memory (libkmc's
allocations go through torch's caching allocator) and the HIP stream.
There is no fallback: when libkmc.so is missing or no GPU is present the
calls raise.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkmc.so")

KMC_OK, KMC_EINVAL, KMC_ENOMEM, KMC_EDEVICE, KMC_ESTATE, KMC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RATE_METROPOLIS, RATE_BARKER = 0, 1
SCHED_RANDOM_PERM, SCHED_PALINDROME = 0, 1
INIT_RANDOM, INIT_ALL_UP, INIT_GIVEN = 0, 1, 2
F_CHECKPOINT, F_PERSISTENT, F_GRAPH, F_NO_MULTI, F_DEVICE_OUT, F_MULTI, F_SCORE, F_TIMING = (
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40, 0x80)
F_FLOW = 0x100
F_RESIDENT = 0x200
FLOW_MAX_SWEEPS = 64  # sweeps of one dataflow launch (KMC_F_FLOW)

STATUS_NAMES = {0: "KMC_OK", -1: "KMC_EINVAL", -2: "KMC_ENOMEM", -3: "KMC_EDEVICE",
                -4: "KMC_ESTATE", -5: "KMC_EUNSUPPORTED"}


class KmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ReplicaDesc(C.Structure):
    _fields_ = [("J", C.c_double), ("h", C.c_double), ("T", C.c_double),
                ("L", C.c_int32), ("tile", C.c_int32), ("steps_per_visit", C.c_int32),
                ("rate_model", C.c_int32), ("schedule", C.c_int32), ("init", C.c_int32),
                ("tile_rows", C.c_int32), ("dims", C.c_int32), ("time_slice", C.c_double)]


RECORD_DTYPE = np.dtype([("sweep", "<i8"), ("M", "<i8"), ("B", "<i8"),
                         ("events", "<i8"), ("steps", "<i8"), ("t", "<f8")])

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None
_torch_hooks = None


def lib():
    """Loads libkmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "or python -m paper_1403_4674_amd.build")
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        sigs = {
            "kmc_set_device_allocator": ([_ALLOC_FN, _FREE_FN, P], I32),
            "kmc_rate_table": ([C.c_double, C.c_double, C.c_double, I32, P, P, P, P], I32),
            "kmc_init_lattice": ([C.POINTER(P), C.POINTER(ReplicaDesc), I32, C.c_uint64, P,
                                  P], I32),
            "kmc_run_schedule": ([P, I64, I32, C.c_uint32], I32),
            "kmc_observables": ([P, P, I64, C.POINTER(I64), C.c_uint32], I32),
            "kmc_backward_score": ([P, P, I64, C.c_uint32], I32),
            "kmc_get_spins": ([P, I32, P], I32),
            "kmc_get_domain_state": ([P, I32, P, P, P], I32),
            "kmc_get_domain_clocks": ([P, I32, P, P], I32),
            "kmc_get_info": ([P, I32, C.POINTER(I32), C.POINTER(I32)], I32),
            "kmc_get_timing": ([P, C.POINTER(C.c_double), C.POINTER(I64)], I32),
            "kmc_exact_sweeps": ([C.POINTER(ReplicaDesc), P, P, I64, C.c_uint32, P], I32),
            "kmc_exact_sweeps_static": ([C.POINTER(ReplicaDesc), P, I64, C.c_uint32, P], I32),
            "kmc_set_wait_limit": ([P, I64], I32),
            "kmc_last_error": ([P], C.c_char_p),
            "kmc_destroy": ([P], None),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    """Names the C-ABI exports (checked against include/kmc.h by the tests)."""
    L = lib()
    names = ["kmc_set_device_allocator", "kmc_rate_table", "kmc_init_lattice",
             "kmc_run_schedule", "kmc_observables", "kmc_backward_score", "kmc_get_spins",
             "kmc_get_domain_state", "kmc_get_domain_clocks", "kmc_get_info",
             "kmc_get_timing", "kmc_last_error",
             "kmc_destroy", "kmc_exact_sweeps", "kmc_exact_sweeps_static",
             "kmc_set_wait_limit"]
    return [n for n in names if hasattr(L, n)]


def _check(status, ctx=None):
    if status != KMC_OK:
        msg = lib().kmc_last_error(ctx).decode() if ctx else ""
        raise KmcError(status, msg)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def use_torch_allocator():
    """Routes libkmc's device allocations through torch's caching allocator."""
    global _torch_hooks
    import torch
    if _torch_hooks is None:
        def alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(nbytes)
            except Exception:
                return None

        def free(ptr, user):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:  # interpreter shutdown: torch already torn down
                pass

        _torch_hooks = (_ALLOC_FN(alloc), _FREE_FN(free))
    _check(lib().kmc_set_device_allocator(_torch_hooks[0], _torch_hooks[1], None))


def kmc_rate_table(J, h, T, rate_model=RATE_METROPOLIS):
    r = np.zeros(10, np.uint64)
    w, gJ, gh = (np.zeros(10) for _ in range(3))
    _check(lib().kmc_rate_table(J, h, T, rate_model, _ptr(r), _ptr(w), _ptr(gJ), _ptr(gh)))
    return r, w, gJ, gh


def make_descs(descs):
    arr = (ReplicaDesc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = ReplicaDesc(float(d.get("J", 1.0)), float(d.get("h", 0.0)),
                             float(d["T"]), int(d["L"]), int(d["tile"]),
                             int(d.get("steps_per_visit", 0)),
                             int(d.get("rate_model", RATE_METROPOLIS)),
                             int(d.get("schedule", SCHED_RANDOM_PERM)),
                             int(d.get("init", INIT_RANDOM)),
                             int(d.get("tile_rows", 0)),
                             int(d.get("dims", 0)),
                             float(d.get("time_slice", 0.0)))
    return arr


EXACT_QUANTISED = 0x1


def kmc_exact_sweeps(desc, p, work, n_sweeps, quantised=True, stream=None):
    """Exact propagation of a distribution over the 2^(L*L) configurations of
    one replica (desc: a descriptor dict) through n_sweeps sweeps, in place
    in p (a float64 CUDA tensor of 2^(L*L) entries); work: a float64 CUDA
    tensor of 3 * 2^(L*L) entries.  Runs on torch's current stream."""
    import torch
    n = 1 << (int(desc["L"]) if desc.get("dims", 0) == 1 else int(desc["L"]) ** 2)
    for t, size in ((p, n), (work, 3 * n)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() >= size):
            raise ValueError("p and work must be contiguous float64 CUDA tensors of 2^N and 3 2^N")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    arr = make_descs([desc])
    _check(lib().kmc_exact_sweeps(arr, C.c_void_p(p.data_ptr()), C.c_void_p(work.data_ptr()),
                                  int(n_sweeps), EXACT_QUANTISED if quantised else 0,
                                  C.c_void_p(stream) if stream else None))


def kmc_exact_sweeps_static(desc, p, n_sweeps, quantised=True, stream=None):
    """kmc_exact_sweeps without a workspace (the library's own buffer; at
    most 16 sites): p is a float64 CUDA tensor of 2^(L*L) entries, updated in
    place on torch's current stream."""
    import torch
    n = 1 << (int(desc["L"]) if desc.get("dims", 0) == 1 else int(desc["L"]) ** 2)
    if not (p.is_cuda and p.dtype == torch.float64 and p.is_contiguous() and p.numel() >= n):
        raise ValueError("p must be a contiguous float64 CUDA tensor of 2^N entries")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    arr = make_descs([desc])
    _check(lib().kmc_exact_sweeps_static(arr, C.c_void_p(p.data_ptr()), int(n_sweeps),
                                         EXACT_QUANTISED if quantised else 0,
                                         C.c_void_p(stream) if stream else None))


def kmc_init_lattice(descs, seed, given_spins=None, stream=None):
    """descs: list of dicts with keys L, tile, T and optional J, h,
    steps_per_visit, rate_model, schedule, init, tile_rows (domain height;
    0 or absent: square domains), dims (1: a ring of L sites), time_slice
    (> 0: the rejection-free variant with fixed time slices).  stream: a hipStream_t
    handle (int) or None for torch's current stream.  Returns the context."""
    arr = make_descs(descs)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    g = None
    if given_spins is not None:
        g = np.ascontiguousarray(np.concatenate([np.asarray(x, np.int8).reshape(-1)
                                                 for x in given_spins]))
    ctx = C.c_void_p()
    st = lib().kmc_init_lattice(C.byref(ctx), arr, len(descs), C.c_uint64(seed),
                                _ptr(g) if g is not None else None,
                                C.c_void_p(stream) if stream else None)
    _check(st)
    return ctx


def kmc_run_schedule(ctx, n_sweeps, record_every=1, flags=0):
    _check(lib().kmc_run_schedule(ctx, n_sweeps, record_every, flags), ctx)


def kmc_observables(ctx, n_rep):
    """All records so far as a [n_rep, n_rec] structured array (synchronises)."""
    n = C.c_int64(0)
    _check(lib().kmc_observables(ctx, None, 0, C.byref(n), 0), ctx)
    out = np.zeros((n_rep, max(n.value, 1)), RECORD_DTYPE)
    if n.value:
        _check(lib().kmc_observables(ctx, _ptr(out), n.value, C.byref(n), 0), ctx)
    return out[:, :n.value]


def kmc_observables_device(ctx, out_tensor, capacity):
    """Enqueues a copy of the records into a device tensor of
    n_rep * capacity * 48 bytes (no synchronisation)."""
    n = C.c_int64(0)
    _check(lib().kmc_observables(ctx, C.c_void_p(out_tensor.data_ptr()), capacity,
                                 C.byref(n), F_DEVICE_OUT), ctx)
    return n.value


def kmc_backward_score(ctx, n_rep, n_bins, out_tensor=None):
    """Score bins [n_rep, n_bins, 2] of the last checkpointed run.  With a
    device tensor the result is written there asynchronously."""
    if out_tensor is not None:
        _check(lib().kmc_backward_score(ctx, C.c_void_p(out_tensor.data_ptr()), n_bins,
                                        F_DEVICE_OUT), ctx)
        return out_tensor
    out = np.zeros((n_rep, n_bins, 2))
    _check(lib().kmc_backward_score(ctx, _ptr(out), n_bins, 0), ctx)
    return out


def kmc_get_spins(ctx, replica, L, ring=False):
    out = np.zeros((L,) if ring else (L, L), np.int8)
    _check(lib().kmc_get_spins(ctx, replica, _ptr(out)), ctx)
    return out


def kmc_get_domain_state(ctx, replica):
    nd = C.c_int32(0)
    _check(lib().kmc_get_info(ctx, replica, None, C.byref(nd)), ctx)
    s, c = np.zeros(nd.value), np.zeros(nd.value)
    e = np.zeros(nd.value, np.int64)
    _check(lib().kmc_get_domain_state(ctx, replica, _ptr(s), _ptr(c), _ptr(e)), ctx)
    return s, c, e


def kmc_get_domain_clocks(ctx, replica):
    nd = C.c_int32(0)
    _check(lib().kmc_get_info(ctx, replica, None, C.byref(nd)), ctx)
    t, c = np.zeros(nd.value), np.zeros(nd.value)
    _check(lib().kmc_get_domain_clocks(ctx, replica, _ptr(t), _ptr(c)), ctx)
    return t, c


def kmc_get_timing(ctx):
    """(milliseconds, launches) of the hot-kernel launches timed since the
    last call (runs with F_TIMING)."""
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    _check(lib().kmc_get_timing(ctx, C.byref(ms), C.byref(n)), ctx)
    return ms.value, n.value


def kmc_destroy(ctx):
    if ctx:
        lib().kmc_destroy(ctx)


class Lattice:
    """Owns one libkmc context: a batch of replicas on the current GPU."""

    def __init__(self, descs, seed, given_spins=None, stream=None, torch_alloc=True):
        if torch_alloc:
            use_torch_allocator()
        self.descs = [dict(d) for d in descs]
        self.n_rep = len(descs)
        self.ctx = kmc_init_lattice(descs, seed, given_spins, stream)

    def run(self, n_sweeps, record_every=1, flags=0):
        kmc_run_schedule(self.ctx, n_sweeps, record_every, flags)

    def records(self):
        return kmc_observables(self.ctx, self.n_rep)

    def spins(self, replica=0):
        d = self.descs[replica]
        return kmc_get_spins(self.ctx, replica, d["L"], d.get("dims", 0) == 1)

    def domain_state(self, replica=0):
        return kmc_get_domain_state(self.ctx, replica)

    def domain_clocks(self, replica=0):
        return kmc_get_domain_clocks(self.ctx, replica)

    def set_wait_limit(self, max_polls):
        """Bound of each dataflow wait (a hook for testing the failure path)."""
        _check(lib().kmc_set_wait_limit(self.ctx, int(max_polls)), self.ctx)

    def timing(self):
        return kmc_get_timing(self.ctx)

    def score(self, n_bins, out_tensor=None):
        return kmc_backward_score(self.ctx, self.n_rep, n_bins, out_tensor)

    def close(self):
        if self.ctx:
            kmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
