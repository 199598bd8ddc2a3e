"""Shared helpers of the GPU tests: oracle replicas for the same descriptors
and element-by-element comparisons."""
import numpy as np

RTOL_T = 1e-12
# score bins: |GPU - oracle| <= SCORE_REL * (sum over the bin of the absolute
# values of its terms, as the oracle reports them).  Scores are zero-mean
# sums of O(1) terms, so a relative bound on the value itself is ill-posed.
SCORE_REL = 1e-12


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def oracle_for(kmco, desc, seed, rho, spins=None):
    return kmco.Replica(desc["L"], desc["tile"], J=desc.get("J", 1.0), h=desc.get("h", 0.0),
                        T=desc["T"], steps_per_visit=desc.get("steps_per_visit", 0),
                        rate_model=desc.get("rate_model", 0),
                        schedule=desc.get("schedule", 0), init=desc.get("init", 0),
                        seed=seed, replica=rho, spins=spins,
                        tile_rows=desc.get("tile_rows", 0), dims=desc.get("dims", 2) or 2,
                        time_slice=desc.get("time_slice", 0.0))


def assert_records_equal(gpu, ora, what=""):
    """Integer fields bit-exact, simulated time within 1e-12 relative."""
    assert gpu.shape == ora.shape, (what, gpu.shape, ora.shape)
    for f in ("sweep", "M", "B", "events", "steps"):
        bad = np.nonzero(gpu[f] != ora[f])[0]
        assert bad.size == 0, (what, f, bad[:5], gpu[f][bad[:5]], ora[f][bad[:5]])
    np.testing.assert_allclose(gpu["t"], ora["t"], rtol=RTOL_T, atol=0, err_msg=what)


def assert_replica_equal(lat, rho, ora, gpu_rec=None, ora_rec=None, what=""):
    L = lat.descs[rho]["L"]
    g = lat.spins(rho)
    o = ora.spins()
    diff = np.argwhere(g != o)
    assert diff.size == 0, (what, "spins differ at", diff[:5])
    s, c, e = lat.domain_state(rho)
    t, tc = lat.domain_clocks(rho)  # the clocks-only call returns the same
    assert np.array_equal(t, s) and np.array_equal(tc, c), (what, "domain clocks")
    os_, oc = ora.domain_clocks()
    assert np.array_equal(e, ora.domain_events()), (what, "domain events")
    np.testing.assert_allclose(s + c, os_ + oc, rtol=RTOL_T, atol=0, err_msg=what)
    if gpu_rec is not None:
        assert_records_equal(gpu_rec, ora_rec, what)
    assert g.shape == ((L,) if lat.descs[rho].get("dims", 0) == 1 else (L, L))


def oracle_score(kmco, desc, seed, rho, sweeps, every, pre=0, spins=None):
    """The oracle's records, score bins and bin magnitudes (sums of absolute
    terms) of one replica after `pre` unscored sweeps."""
    o = oracle_for(kmco, desc, seed, rho, spins)
    if pre:
        o.run(pre, 1)
    rec, sc, sa = o.run(sweeps, every, score_abs=True)
    return o, rec, sc, sa


def assert_score_close(gpu, ref, mag, what=""):
    """Score bins within SCORE_REL of the bins' sums of absolute terms."""
    gpu, ref, mag = (np.asarray(x, np.float64) for x in (gpu, ref, mag))
    assert gpu.shape == ref.shape == mag.shape, (what, gpu.shape, ref.shape, mag.shape)
    err = np.abs(gpu - ref)
    bound = SCORE_REL * mag
    bad = np.argwhere(err > bound)
    assert bad.size == 0, (what, bad[:4], err[tuple(bad[0])], bound[tuple(bad[0])])
