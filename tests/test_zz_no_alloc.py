"""kmc_exact_sweeps_static, the allocation-free form of kmc_exact_sweeps,
against kmc_exact_sweeps through the C-ABI (needs an MI355X).

Both run the same kernels in the same order on the same start vector, so the
propagated distributions must agree bit for bit.  Two calls in a row share
the library's buffer: a 4 x 4 lattice (the largest the buffer holds), then a
smaller 3 x 3 one, so the second call must not read anything the first left.
"""
import numpy as np
import pytest

from paper_1403_4674_amd import kmc
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

CASES = [dict(L=4, tile=2, T=2.3, h=0.15, steps_per_visit=3),
         dict(L=3, tile=3, tile_rows=1, T=2.0, h=-0.1, rate_model=kmc.RATE_BARKER,
              schedule=kmc.SCHED_PALINDROME, steps_per_visit=2)]


def start_vector(n_sites, seed):
    rng = np.random.default_rng(seed)
    p = rng.random(1 << n_sites)
    return p / p.sum()


def test_static_equals_workspace_form_twice():
    import torch
    assert torch.cuda.is_available()
    for k, d in enumerate(CASES):
        n = d["L"] ** 2
        say(f"exact sweeps without allocation: call {k + 1}, {d['L']}x{d['L']}")
        p0 = torch.tensor(start_vector(n, 7 + k), dtype=torch.float64, device="cuda")
        ref = p0.clone()
        work = torch.empty(3 << n, dtype=torch.float64, device="cuda")
        kmc.kmc_exact_sweeps(d, ref, work, 3, quantised=True)
        got = p0.clone()
        kmc.kmc_exact_sweeps_static(d, got, 3, quantised=True)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(g, r), np.abs(g - r).max()
        assert abs(g.sum() - 1.0) < 1e-12
        assert not np.array_equal(g, p0.cpu().numpy())  # the sweeps moved it
