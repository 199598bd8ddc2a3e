"""Backward score replay and autograd on the GPU (needs an MI355X).

* kmc_backward_score bins equal the oracle's score bins within 1e-12 of the
  bin's sum of absolute terms (the oracle adds the per-tick terms in event
  order, the kernel per class, per visit and per wavefront);
* the replay does not disturb the live state;
* KmcFunction's gradient equals the likelihood-ratio estimate formed from
  the oracle's records and score bins;
* on the differentiable workload the windowed LR derivative d<M>/dh agrees
  with the fluctuation identity beta Var(M) and with common-random-number
  central differences.
"""
import numpy as np
import pytest

from paper_1403_4674_amd import kmc, workloads
from tests.gpu_helpers import assert_score_close, oracle_for, oracle_score, say

pytestmark = pytest.mark.gpu

DESCS = [dict(L=16, tile=8, T=2.5, h=0.1, steps_per_visit=64),
         dict(L=32, tile=16, T=2.0, h=-0.2, rate_model=kmc.RATE_BARKER),
         dict(L=24, tile=12, T=3.0, h=0.3, J=0.8),
         dict(L=64, tile=32, T=2.3, h=0.0, steps_per_visit=300)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def oracle_bins(kmco, descs, seed, sweeps, rec_every):
    out = []
    for rho, d in enumerate(descs):
        o = oracle_for(kmco, d, seed, rho)
        _, sc = o.run(sweeps, rec_every, score=True)
        out.append(sc)
    return np.array(out)


@pytest.mark.parametrize("flags", [0, kmc.F_PERSISTENT])
def test_backward_score_matches_oracle(torch_cuda, oracle_lib, flags):
    sweeps, every = 22, 5
    say(f"score replay flags={flags}")
    lat = kmc.Lattice(DESCS, 9)
    lat.run(3, 1, flags)  # the replay starts from a non-trivial state
    o_pre = [oracle_for(oracle_lib, d, 9, r) for r, d in enumerate(DESCS)]
    for o in o_pre:
        o.run(3, 1)
    lat.run(sweeps, every, flags | kmc.F_CHECKPOINT)
    g = lat.score(-(-sweeps // every))
    ref, mag = [], []
    for o in o_pre:
        _, sc, sa = o.run(sweeps, every, score_abs=True)
        ref.append(sc)
        mag.append(sa)
    ref, mag = np.array(ref), np.array(mag)
    assert g.shape == ref.shape == (len(DESCS), 5, 2)
    for rho in range(len(DESCS)):
        assert_score_close(g[rho], ref[rho], mag[rho], f"replica {rho}")
    assert np.abs(ref).max() > 1.0


def test_backward_needs_checkpoint_and_keeps_state(torch_cuda, oracle_lib):
    lat = kmc.Lattice(DESCS[:2], 3)
    lat.run(4, 2)
    with pytest.raises(kmc.KmcError) as e:
        lat.score(2)
    assert e.value.status == kmc.KMC_ESTATE
    lat.run(6, 3, kmc.F_CHECKPOINT)
    before = [lat.spins(r) for r in range(2)], lat.records()
    lat.score(2)
    after = [lat.spins(r) for r in range(2)], lat.records()
    assert all(np.array_equal(a, b) for a, b in zip(before[0], after[0]))
    assert np.array_equal(before[1], after[1])
    with pytest.raises(kmc.KmcError):
        lat.score(1)  # capacity below the number of intervals
    lat.run(5, 5)  # the live run continues as if nothing happened
    for rho, d in enumerate(DESCS[:2]):
        o = oracle_for(oracle_lib, d, 3, rho)
        o.run(4, 2)
        o.run(6, 3)
        o.run(5, 5)
        assert np.array_equal(lat.spins(rho), o.spins())


def test_autograd_equals_oracle_lr_estimate(torch_cuda, oracle_lib):
    import torch

    from paper_1403_4674_amd.autograd import KmcFunction
    base = [dict(L=16, tile=8, T=2.4, steps_per_visit=64) for _ in range(6)]
    Jv = np.array([1.0, 0.9, 1.1, 1.0, 0.95, 1.05])
    hv = np.array([0.1, -0.1, 0.0, 0.2, 0.05, -0.15])
    J = torch.tensor(Jv, dtype=torch.float64, device="cuda", requires_grad=True)
    h = torch.tensor(hv, dtype=torch.float64, device="cuda", requires_grad=True)
    say("autograd vs oracle LR")
    obs = KmcFunction.apply(J, h, base, 21, 12, 3, True)
    w = torch.linspace(0.5, 1.5, obs.shape[1], dtype=torch.float64, device="cuda")
    loss = (obs[..., 0] * w).sum() + (obs[..., 1] * w * 2).sum()
    loss.backward()
    # the same estimator from the oracle's records and score bins
    descs = [dict(b, J=float(a), h=float(c)) for b, a, c in zip(base, Jv, hv)]
    O, S, Ms, Bs = [], [], [], []
    for rho, d in enumerate(descs):
        o = oracle_for(oracle_lib, d, 21, rho)
        rec, sc = o.run(12, 3, score=True)
        N = 256.0
        m = rec["M"] / N
        e = (-d["J"] * rec["B"] - d["h"] * rec["M"]) / N
        O.append(m * w.cpu().numpy() + 2 * e * w.cpu().numpy())
        S.append(np.cumsum(sc, axis=0))
        Ms.append(rec["M"] / N)
        Bs.append(rec["B"] / N)
    O, S = np.array(O), np.array(S)
    base_loo = (O.sum(0, keepdims=True) - O) / (len(descs) - 1)
    lr = ((O - base_loo)[..., None] * S).sum(1)
    wn = 2 * w.cpu().numpy()
    gJ = lr[:, 0] - (wn * np.array(Bs)).sum(1)
    gh = lr[:, 1] - (wn * np.array(Ms)).sum(1)
    np.testing.assert_allclose(J.grad.cpu().numpy(), gJ, rtol=1e-9, atol=1e-8)
    np.testing.assert_allclose(h.grad.cpu().numpy(), gh, rtol=1e-9, atol=1e-8)


def test_fluctuation_identity_and_crn_differences(torch_cuda):
    """Differentiable workload at reduced length: 1024 replicas of 64x64,
    T = 2.5, h ~ U[-0.2, 0.2] (the workload's draw), 32x32 domains.  The
    autocorrelation of M decays as exp(-s/60 sweeps) here, so the LR window
    of 400 sweeps leaves a truncation bias below 0.2%."""
    from paper_1403_4674_amd.autograd import windowed_lr_derivative
    seed, descs, _ = workloads.differentiable_1024()
    sweeps, every, window, burn = 4000, 4, 100, 50
    say("fluctuation identity, 1024 x 64^2 x 4000 sweeps")
    lat = kmc.Lattice(descs, seed)
    lat.run(400, 400, kmc.F_PERSISTENT)  # equilibrate
    lat.run(sweeps, every, kmc.F_PERSISTENT | kmc.F_CHECKPOINT)
    rec = lat.records()[:, 1:]
    bins = lat.score(sweeps // every)
    M = rec["M"].astype(np.float64)
    Bd = rec["B"].astype(np.float64)
    J = np.array([x["J"] for x in descs])[:, None]
    h = np.array([x["h"] for x in descs])[:, None]
    E = -J * Bd - h * M
    beta = 1.0 / 2.5

    def zscore(diff):
        return diff.mean() / (diff.std(ddof=1) / np.sqrt(diff.size))

    # d<M>/dh = beta Var(M)
    lr_h = windowed_lr_derivative(M, bins[..., 1], window, burn)
    fi_h = beta * M[:, burn:].var(axis=1)
    z = zscore(lr_h - fi_h)
    assert abs(z) < 4.5, (lr_h.mean(), fi_h.mean(), z)
    assert fi_h.mean() > 50.0
    # d<E>/dJ = -<B> + beta Cov(E, B); the LR part is the covariance term
    lr_J = windowed_lr_derivative(E, bins[..., 0], window, burn)
    Ec = E[:, burn:] - E[:, burn:].mean(1, keepdims=True)
    Bc = Bd[:, burn:] - Bd[:, burn:].mean(1, keepdims=True)
    fi_J = beta * (Ec * Bc).mean(1)
    z = zscore(lr_J - fi_J)
    assert abs(z) < 4.5, (lr_J.mean(), fi_J.mean(), z)
    # common-random-number central differences in h (dh = 1e-3)
    dh = 1e-3
    plus = kmc.Lattice([dict(x, h=x["h"] + dh) for x in descs], seed)
    minus = kmc.Lattice([dict(x, h=x["h"] - dh) for x in descs], seed)
    for l in (plus, minus):
        l.run(400, 400, kmc.F_PERSISTENT)
        l.run(sweeps, every, kmc.F_PERSISTENT)
    Mp = plus.records()[:, 1:]["M"][:, burn:].astype(np.float64).mean(1)
    Mm = minus.records()[:, 1:]["M"][:, burn:].astype(np.float64).mean(1)
    fd = (Mp - Mm) / (2 * dh)
    z2 = zscore(fd - fi_h)
    assert abs(z2) < 4.5, (fd.mean(), fi_h.mean(), z2)


def test_backward_score_multi_slot(torch_cuda, oracle_lib):
    from tests.test_gpu_parity import MULTI_MIX
    descs = MULTI_MIX
    say("score replay, multi-slot form")
    lat = kmc.Lattice(descs, 5)
    lat.run(7, 2, kmc.F_PERSISTENT | kmc.F_MULTI | kmc.F_CHECKPOINT)
    g = lat.score(4)
    ref = kmc.Lattice(descs, 5)
    ref.run(7, 2, kmc.F_PERSISTENT | kmc.F_NO_MULTI | kmc.F_CHECKPOINT)
    r = ref.score(4)
    for rho in range(len(descs)):
        _, _, sc, sa = oracle_score(oracle_lib, descs[rho], 5, rho, 7, 2)
        assert_score_close(g[rho], sc, sa, f"multi replica {rho}")
        assert_score_close(r[rho], sc, sa, f"one-domain replica {rho}")


@pytest.mark.parametrize("flags", [kmc.F_PERSISTENT, kmc.F_PERSISTENT | kmc.F_MULTI, 0])
def test_fused_score_equals_replay(torch_cuda, oracle_lib, flags):
    from tests.test_gpu_parity import MULTI_MIX
    descs = MULTI_MIX[:8] + DESCS
    say(f"fused score vs replay, flags {flags}")
    a = kmc.Lattice(descs, 17)
    b = kmc.Lattice(descs, 17)
    a.run(6, 3, flags | kmc.F_CHECKPOINT)
    b.run(6, 3, flags | kmc.F_SCORE)
    ga, gb = a.score(2), b.score(2)
    if flags & kmc.F_PERSISTENT:
        assert np.array_equal(ga, gb)  # same kernel, same state, no atomics
    else:  # visits add to the bins with atomics, in no fixed order
        for rho in range(len(descs)):
            _, _, sc, sa = oracle_score(oracle_lib, descs[rho], 17, rho, 6, 3)
            assert_score_close(ga[rho], sc, sa, f"replay {rho}")
            assert_score_close(gb[rho], sc, sa, f"fused {rho}")
    for rho in range(len(descs)):
        assert np.array_equal(a.spins(rho), b.spins(rho))
    assert np.array_equal(a.records(), b.records())
    with pytest.raises(kmc.KmcError):
        b.run(3, 1, kmc.F_GRAPH | kmc.F_SCORE)
