"""Failure handling forced from the host (needs an MI355X).

Device allocations are routed through a counting allocator hook
(kmc_set_device_allocator) that fails the k-th request.  For every k up to
the number a context needs, kmc_init_lattice must return KMC_ENOMEM and
release every allocation it made; a failure inside kmc_run_schedule (its
record, checkpoint and dataflow buffers) and inside kmc_backward_score
(replay buffers, bins) must be reported as KMC_ENOMEM, and destroying the
context must then release everything.  No kernel is made to fail: every
launch that runs, runs normally.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1403_4674_amd import kmc
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


class CountingAllocator:
    def __init__(self, torch):
        self.torch = torch
        self.fail_at = 0      # 1-based request to fail; 0: never
        self.requests = 0
        self.live = {}

    def hooks(self):
        def alloc(nbytes, user):
            self.requests += 1
            if self.requests == self.fail_at:
                return None
            p = self.torch.cuda.caching_allocator_alloc(nbytes)
            self.live[p] = nbytes
            return p

        def free(ptr, user):
            self.live.pop(ptr)
            self.torch.cuda.caching_allocator_delete(ptr)

        self._keep = (kmc._ALLOC_FN(alloc), kmc._FREE_FN(free))
        return self._keep


DESCS = [dict(L=32, tile=8, T=2.3, h=0.1), dict(L=24, tile=12, T=2.0),
         dict(L=64, tile=32, T=2.5, schedule=kmc.SCHED_PALINDROME)]


def init(descs):
    ctx = C.c_void_p()
    st = kmc.lib().kmc_init_lattice(C.byref(ctx), kmc.make_descs(descs), len(descs), 7, None,
                                    None)
    return st, ctx


def test_allocation_failures_are_reported_without_leaks():
    import torch
    assert torch.cuda.is_available()
    L = kmc.lib()
    A = CountingAllocator(torch)
    try:
        assert L.kmc_set_device_allocator(*A.hooks(), None) == kmc.KMC_OK
        st, ctx = init(DESCS)
        assert st == kmc.KMC_OK
        n_init = A.requests
        L.kmc_destroy(ctx)
        assert not A.live and n_init > 5
        say(f"allocation failures: {n_init} requests at init")
        for k in range(1, n_init + 1):
            A.requests, A.fail_at = 0, k
            st, ctx = init(DESCS)
            assert st == kmc.KMC_ENOMEM, (k, st)
            assert not A.live, (k, len(A.live))
        # failures inside a run (its records, checkpoint copies, dataflow
        # slots, score bins), at each of its requests: the run is refused
        # before anything is enqueued, and the same run then succeeds
        recovered = {}
        for flags in (kmc.F_CHECKPOINT, kmc.F_FLOW, kmc.F_SCORE,
                      kmc.F_FLOW | kmc.F_CHECKPOINT):
            for j in range(1, 5):
                A.requests, A.fail_at = 0, 0
                st, ctx = init(DESCS)
                assert st == kmc.KMC_OK
                A.fail_at = A.requests + j
                st = L.kmc_run_schedule(ctx, 4, 1, flags)
                if st == kmc.KMC_OK:  # the run needs fewer than j requests
                    L.kmc_destroy(ctx)
                    assert not A.live
                    break
                assert st == kmc.KMC_ENOMEM, (flags, j, st)
                assert b"allocation" in L.kmc_last_error(ctx)
                A.fail_at = 0
                assert L.kmc_run_schedule(ctx, 4, 1, flags) == kmc.KMC_OK  # recovers
                recovered[(flags, j)] = kmc.kmc_observables(ctx, len(DESCS))
                L.kmc_destroy(ctx)
                assert not A.live, (flags, j)
        # the replay's buffers in kmc_backward_score
        A.requests, A.fail_at = 0, 0
        st, ctx = init(DESCS)
        assert L.kmc_run_schedule(ctx, 4, 2, kmc.F_CHECKPOINT) == kmc.KMC_OK
        A.fail_at = A.requests + 1
        out = np.zeros((len(DESCS), 2, 2))
        assert L.kmc_backward_score(ctx, out.ctypes.data_as(C.c_void_p), 2, 0) == \
            kmc.KMC_ENOMEM
        L.kmc_destroy(ctx)
        assert not A.live
    finally:
        kmc.use_torch_allocator()
    # a recovered context holds what an untouched one holds after the run
    for (flags, j), rec in recovered.items():
        ref = kmc.Lattice(DESCS, 7)
        ref.run(4, 1, flags)
        assert np.array_equal(rec, ref.records()), (flags, j)
        ref.close()
