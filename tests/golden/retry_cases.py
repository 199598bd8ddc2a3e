"""Finds seeds whose first sweeps contain ticks with a rejected slot draw.

The exact 1/n_d site selection (App. A, Eq. (Glauber_TM)) draws the slot by
a Lemire multiply with rejection of the (2^32 mod n_d) smallest low halves;
a rejected tick is redrawn on the retry streams.  For n_d that is not a
power of two this happens with probability (2^32 mod n_d)/2^32 per tick, so
a run compared with the GPU only reaches the rule if its counters are
chosen for it.  Whether a tick is rejected depends only on its counter
(seed, replica, sweep, domain | visit, tick) and n_d, never on the lattice,
so the search asks the oracle's kmco_count_retry_ticks and runs nothing
else.  The printed seeds are the ones tests/test_gpu_retry.py uses (its CPU
test re-checks, through full oracle runs, that each case does redraw).

Random colour order: every domain is visited once per sweep (visit 0).
"""
import sys

from oracle import kmco

# (name, L, domain side, n_replicas, sweeps to search)
CASES = [("checker24_tile12", 24, 12, 16, 2),
         ("checker122_tile61", 122, 61, 2, 2),
         ("single100", 100, 100, 1, 3)]


def first_seed(L, B, n_rep, sweeps, start=1, limit=200000):
    nd = B * B
    ND = (L // B) ** 2
    for seed in range(start, start + limit):
        hits = []
        for rho in range(n_rep):
            for w in range(sweeps):
                for d in range(ND):
                    k = kmco.count_retry_ticks(seed, rho, w, d, 0, nd, nd)
                    if k:
                        hits.append((rho, w, d, k))
        if hits:
            return seed, hits
    return None, []


def main():
    for name, L, B, n_rep, sweeps in CASES:
        seed, hits = first_seed(L, B, n_rep, sweeps)
        print(f"{name}: seed {seed}  (replica, sweep, domain, ticks) {hits}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
