"""The 2D parallelisation study on the GPU (needs an MI355X): the batched
trajectories of every setting (unpartitioned reference as one periodic
domain, a checkerboard of 6x6 domains, four 12x3 stripes) are the oracle's, bit for bit,
and the analysis runs on them."""
import numpy as np
import pytest

from paper_1403_4674_amd import analysis, experiments, kmc
from tests.gpu_helpers import assert_records_equal, oracle_for, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_small_study_trajectories_match_oracle(torch_cuda, oracle_lib):
    L, n_traj = 12, 24
    settings = [("reference", 12, 12, 144), ("cb4 NI=2", 6, 6, 2), ("stripes4 NI=5", 3, 12, 5)]
    say("12x12 study, 24 trajectories per setting")
    res = experiments.run_study(kmc, L, n_traj, total_steps=6000, settings=settings,
                                verbose=False)
    ic = analysis.circle_initial_condition(L)
    for r, (label, B, By, NI) in zip(res, settings):
        rec = r["rec"]
        assert rec.shape[0] == n_traj and rec["steps"][0, 0] == 0
        seed = 2024 + res.index(r)
        for rho in (0, n_traj - 1):
            d = dict(L=L, tile=B, tile_rows=By, T=2.4, steps_per_visit=NI,
                     rate_model=kmc.RATE_BARKER, init=kmc.INIT_GIVEN)
            o = oracle_for(oracle_lib, d, seed, rho, ic)
            every = int(round(rec["sweep"][rho, 2] - rec["sweep"][rho, 1]))
            n_sweeps = int(rec["sweep"][rho, -1])
            orec = o.run(n_sweeps, every)
            assert_records_equal(rec[rho, 1:], orec, f"{label} trajectory {rho}")
    rows = experiments.analyse(res, L, max_lag_samples=20)
    assert rows[0]["eta"] == 1.0 and rows[0]["chi2"] == pytest.approx(0.0, abs=1e-12)
    assert all(np.isfinite(r["tau_steps"]) and r["tau_steps"] > 0 for r in rows)
