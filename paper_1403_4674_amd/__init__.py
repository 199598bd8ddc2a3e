"""MI355X (gfx950) domain-decomposed sequential-update kinetic Monte Carlo.

Hot path: libkmc.so (HIP kernels + C-ABI, include/kmc.h); this package is
its thin Python binding plus the torch autograd wrapper and the tile
autotuner.
"""
from .kmc import (F_CHECKPOINT, F_DEVICE_OUT, F_GRAPH, F_PERSISTENT, INIT_ALL_UP,
                  INIT_GIVEN, INIT_RANDOM, RATE_BARKER, RATE_METROPOLIS, RECORD_DTYPE,
                  SCHED_PALINDROME, SCHED_RANDOM_PERM, KmcError, Lattice, kmc_backward_score,
                  kmc_destroy, kmc_get_domain_state, kmc_get_spins, kmc_init_lattice,
                  kmc_observables, kmc_rate_table, kmc_run_schedule)

__all__ = [
    "F_CHECKPOINT", "F_DEVICE_OUT", "F_GRAPH", "F_PERSISTENT", "INIT_ALL_UP", "INIT_GIVEN",
    "INIT_RANDOM", "RATE_BARKER", "RATE_METROPOLIS", "RECORD_DTYPE", "SCHED_PALINDROME",
    "SCHED_RANDOM_PERM", "KmcError", "Lattice", "kmc_backward_score", "kmc_destroy",
    "kmc_get_domain_state", "kmc_get_spins", "kmc_init_lattice", "kmc_observables",
    "kmc_rate_table", "kmc_run_schedule",
]
