"""torch.autograd wrapper: gradients of kMC observables with respect to (J, h).

Forward runs the domain-decomposed kMC on the GPU through libkmc and returns
per-record observables; backward calls kmc_backward_score, whose kernel
replays the forward trajectory bit-exactly from its saved start state and
accumulates the likelihood-ratio score d ln P(path)/d(J, h) of every tick.
Then, for an observable O_k recorded at sweep endpoint k (Sec. 2.3),

    d E[O_k]/d theta = E[dO_k/d theta] + E[(O_k - b_k) S_k],

with S_k the score of all ticks up to record k and b_k a baseline that does
not depend on the replica's own path (the leave-one-out mean over replicas
of the batch), which keeps the estimator unbiased.
"""
import numpy as np
import torch

from . import kmc


class KmcFunction(torch.autograd.Function):
    """obs = KmcFunction.apply(J, h, base_descs, seed, n_sweeps, record_every,
    persistent, fused).  J, h: float64 tensors [n_rep].  obs: float64
    [n_rep, n_rec, 2] with (m, e) = (M/N, E/N) per site, E = -J B - h M.
    fused=False (default): the forward saves its start state and backward
    replays the run with the score kernel; fused=True: the forward also
    accumulates the score and backward only reads it."""

    @staticmethod
    def forward(ctx, J, h, base_descs, seed, n_sweeps, record_every, persistent=True,
                fused=False):
        Jh = J.detach().double().cpu().numpy()
        hh = h.detach().double().cpu().numpy()
        descs = [dict(d, J=float(a), h=float(b)) for d, a, b in zip(base_descs, Jh, hh)]
        lat = kmc.Lattice(descs, seed)
        flags = (kmc.F_SCORE if fused else kmc.F_CHECKPOINT) | \
            (kmc.F_PERSISTENT if persistent else 0)
        lat.run(n_sweeps, record_every, flags)
        rec = lat.records()
        N = np.array([d["L"] ** 2 for d in descs], dtype=np.float64)[:, None]
        M = rec["M"].astype(np.float64)
        B = rec["B"].astype(np.float64)
        m = M / N
        e = (-Jh[:, None] * B - hh[:, None] * M) / N
        obs = torch.from_numpy(np.stack([m, e], axis=-1)).to(J.device)
        ctx.lat = lat
        ctx.n_bins = -(-n_sweeps // record_every)
        ctx.n_rec = rec.shape[1]
        ctx.save_for_backward(obs, torch.from_numpy(M / N).to(J.device),
                              torch.from_numpy(B / N).to(J.device))
        return obs

    @staticmethod
    def backward(ctx, grad_obs):
        obs, m_site, b_site = ctx.saved_tensors
        dev = grad_obs.device
        n_rep = obs.shape[0]
        if dev.type == "cuda":
            bins = torch.empty((n_rep, ctx.n_bins, 2), dtype=torch.float64, device=dev)
            ctx.lat.score(ctx.n_bins, bins)
        else:
            bins = torch.from_numpy(ctx.lat.score(ctx.n_bins))
        S = torch.cumsum(bins, dim=1)[:, :ctx.n_rec, :]          # [n_rep, n_rec, 2]
        # O weighted by the incoming gradient, per replica and record
        G = (grad_obs * obs).sum(-1)                                # [n_rep, n_rec]
        if n_rep > 1:
            base = (G.sum(0, keepdim=True) - G) / (n_rep - 1)
        else:
            base = torch.zeros_like(G)
        lr = ((G - base)[..., None] * S).sum(1)                    # [n_rep, 2]
        # explicit dependence of e = (-J B - h M)/N on J and h
        gJ = lr[:, 0] - (grad_obs[..., 1] * b_site).sum(1)
        gh = lr[:, 1] - (grad_obs[..., 1] * m_site).sum(1)
        ctx.lat.close()
        return gJ, gh, None, None, None, None, None, None


def windowed_lr_derivative(O, bins, window, n_center):
    """Stationary derivative d<O>/d theta per replica from one long run.

    Estimates Cov(O(s), sum of the score over the `window` record intervals
    ending at s), averaged over records s.  O is centred by its mean over
    the first n_center records and only windows that start after them are
    used: score increments have zero mean given the past, so a centre taken
    from the past keeps the estimate unbiased (centring by the mean of the
    same records would correlate with the score and bias it by about
    -window/run_length).  O: [n_rep, n_rec]; bins: [n_rep, n_rec] score of
    one parameter per record interval.  numpy in, numpy out."""
    O = np.asarray(O, np.float64)
    bins = np.asarray(bins, np.float64)
    c = O[:, :n_center].mean(axis=1, keepdims=True)
    cs = np.concatenate([np.zeros((O.shape[0], 1)), np.cumsum(bins, axis=1)], axis=1)
    k = np.arange(n_center + window - 1, O.shape[1])
    if k.size == 0:
        raise ValueError("run too short for the window and the centring records")
    Sw = cs[:, k + 1] - cs[:, k + 1 - window]
    return ((O[:, k] - c) * Sw).mean(axis=1)
