"""The slot-retry rule on the GPU, in every execution form.

A tick selects its site with probability exactly 1/n_d (App. A,
Eq. (Glauber_TM)): the slot is a Lemire multiply of word 1 by n_d, and the
(2^32 mod n_d) smallest low halves are rejected and redrawn on the retry
streams.  For the domain sizes here that happens with probability 2.6e-8
(12 x 12), 7.1e-7 (61 x 61) and 1.7e-6 (100 x 100) per tick, so ordinary
runs compared with the oracle almost never reach it.  The seeds below were
found by tests/golden/retry_cases.py, which asks the oracle which counters
are rejected; the CPU test re-checks through full oracle runs that each case
redraws, and every GPU run is compared bit for bit with those oracle runs.
"""
import numpy as np
import pytest

from paper_1403_4674_amd import kmc
from tests.gpu_helpers import (assert_replica_equal, assert_score_close, oracle_for,
                               oracle_score, say)

# name -> (descriptor, replicas, seed, sweeps)
CASES = {
    "checker24_tile12": (dict(L=24, tile=12, T=2.2, h=0.1), 16, 5257, 3),
    "checker122_tile61": (dict(L=122, tile=61, T=2.4, h=-0.05), 2, 1, 2),
    "single100": (dict(L=100, tile=100, T=2.4, rate_model=kmc.RATE_BARKER), 1, 3, 3),
}

FORMS = {
    "phase": 0,
    "flow": kmc.F_FLOW,
    "persistent": kmc.F_PERSISTENT | kmc.F_NO_MULTI,
    "multi": kmc.F_PERSISTENT | kmc.F_MULTI,
    "resident": kmc.F_RESIDENT,
}

# forms that hold each case: the multi-slot kernel takes domains of at most
# 16 x 16, and domains over 64 sites a side run in the resident form only
CASE_FORMS = [("checker24_tile12", f) for f in FORMS] + \
             [("checker122_tile61", f) for f in ("phase", "flow", "persistent", "resident")] + \
             [("single100", "resident")]


def oracle_runs(kmco, name):
    desc, n_rep, seed, sweeps = CASES[name]
    oras, recs, redraws = [], [], 0
    for rho in range(n_rep):
        o = oracle_for(kmco, desc, seed, rho)
        recs.append(o.run(sweeps, 1))
        redraws += o.retries()[0]
        oras.append(o)
    return oras, recs, redraws


@pytest.mark.parametrize("name", list(CASES))
def test_cases_reach_the_retry_rule(oracle_lib, name):
    _, _, redraws = oracle_runs(oracle_lib, name)
    assert redraws >= 1, name


@pytest.mark.gpu
@pytest.mark.parametrize("name,form", CASE_FORMS)
def test_retry_rule_bit_exact(oracle_lib, name, form):
    import torch
    assert torch.cuda.is_available()
    desc, n_rep, seed, sweeps = CASES[name]
    say(f"retry rule: {name} ({n_rep} replicas, seed {seed}), form {form}")
    oras, recs, redraws = oracle_runs(oracle_lib, name)
    assert redraws >= 1
    lat = kmc.Lattice([desc] * n_rep, seed)
    lat.run(sweeps, 1, FORMS[form])
    g = lat.records()
    for rho in range(n_rep):
        assert_replica_equal(lat, rho, oras[rho], g[rho], recs[rho], f"{name} {form} {rho}")
    lat.close()


@pytest.mark.gpu
@pytest.mark.parametrize("form", ["flow", "multi"])
def test_retry_rule_score(oracle_lib, form):
    import torch
    assert torch.cuda.is_available()
    desc, n_rep, seed, sweeps = CASES["checker24_tile12"]
    say(f"retry rule with the fused score, form {form}")
    lat = kmc.Lattice([desc] * n_rep, seed)
    lat.run(sweeps, 1, FORMS[form] | kmc.F_SCORE)
    sc = lat.score(sweeps)
    redraws = 0
    for rho in range(n_rep):
        o, rec, osc, mag = oracle_score(oracle_lib, desc, seed, rho, sweeps, 1)
        redraws += o.retries()[0]
        assert np.array_equal(lat.spins(rho), o.spins()), rho
        assert_score_close(sc[rho], osc, mag, f"score {form} {rho}")
    assert redraws >= 1
