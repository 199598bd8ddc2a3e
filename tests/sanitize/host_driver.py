"""Drives the host paths of a libkmc built with host-side AddressSanitizer
and UndefinedBehaviorSanitizer that need no GPU: rate tables, descriptor
validation of every entry point (rejected before any device call), error
strings.  Run by tests/test_sanitize.py in a process of its own with the
sanitizer runtime preloaded; argv[1] is the library."""
import ctypes as C
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from paper_1403_4674_amd import kmc  # noqa: E402

kmc.LIB_PATH = sys.argv[1]
L = kmc.lib()


def P(a):
    return a.ctypes.data_as(C.c_void_p)


r, w, gJ, gh = np.zeros(10, np.uint64), np.zeros(10), np.zeros(10), np.zeros(10)
for model in (0, 1):
    assert L.kmc_rate_table(1.0, 0.1, 2.0, model, P(r), P(w), P(gJ), P(gh)) == kmc.KMC_OK
assert L.kmc_rate_table(1.0, 0.1, -2.0, 0, P(r), P(w), P(gJ), P(gh)) == kmc.KMC_EINVAL
assert L.kmc_rate_table(float("nan"), 0.1, 2.0, 0, P(r), P(w), P(gJ), P(gh)) == kmc.KMC_EINVAL
ctx = C.c_void_p()
bad = [dict(L=10, tile=3, T=2.0), dict(L=16, tile=8, T=0.0), dict(L=16, tile=8, T=2.0, dims=3),
       dict(L=8, tile=3, T=2.0, dims=1), dict(L=16, tile=8, T=2.0, time_slice=-1.0),
       dict(L=2, tile=2, T=2.0), dict(L=256, tile=130, T=2.0), dict(L=16, tile=8, T=2.0,
                                                                    rate_model=7)]
for d in bad:
    assert L.kmc_init_lattice(C.byref(ctx), kmc.make_descs([d]), 1, 1, None, None) == \
        kmc.KMC_EINVAL, d
p = C.c_void_p(16)
assert L.kmc_exact_sweeps(kmc.make_descs([dict(L=6, tile=6, T=2.0)]), p, p, 1, 0, None) == \
    kmc.KMC_EINVAL
assert L.kmc_exact_sweeps_static(kmc.make_descs([dict(L=5, tile=5, T=2.0)]), p, 1, 0,
                                 None) == kmc.KMC_EINVAL
assert L.kmc_exact_sweeps(kmc.make_descs([dict(L=3, tile=1, T=2.0)]), p, p, 1, 0, None) == \
    kmc.KMC_EUNSUPPORTED
assert L.kmc_run_schedule(None, 1, 1, 0) == kmc.KMC_EINVAL
assert L.kmc_last_error(None) == b"null context"
L.kmc_destroy(None)
print("host driver: ok", flush=True)
