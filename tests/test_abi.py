"""Host-side checks of the C-ABI library (no GPU needed).

* libkmc.so loads and exports every call declared in include/kmc.h;
* its host-built rate table is bit-equal to the oracle's (both are computed
  with the host libm exp; they share no code);
* invalid descriptors are rejected with KMC_EINVAL before any device call.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kmc():
    from paper_1403_4674_amd import kmc as k
    if not os.path.exists(k.LIB_PATH):
        from paper_1403_4674_amd import build
        build.build()
    return k


def declared_calls():
    with open(os.path.join(ROOT, "include", "kmc.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(kmc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_call(kmc):
    names = declared_calls()
    assert "kmc_init_lattice" in names and "kmc_backward_score" in names
    L = kmc.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(kmc.exported_symbols()) == names


@pytest.mark.parametrize("model", [0, 1])
def test_rate_table_bit_equal_to_oracle(kmc, oracle_lib, model):
    rng = np.random.default_rng(3)
    cases = [(1.0, 0.0, 2.5), (1.0, 0.0, 2.269), (1.0, 0.0, 1.5)]
    cases += [(float(a), float(b), float(c)) for a, b, c in
              zip(rng.uniform(-2, 2, 40), rng.uniform(-1, 1, 40), rng.uniform(0.3, 5, 40))]
    for J, h, T in cases:
        a = kmc.kmc_rate_table(J, h, T, model)
        b = oracle_lib.rates(J, h, T, model)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), (J, h, T)


def test_rate_table_rejects_bad_input(kmc):
    with pytest.raises(kmc.KmcError):
        kmc.kmc_rate_table(1.0, 0.0, 0.0)
    with pytest.raises(kmc.KmcError):
        kmc.kmc_rate_table(1.0, 0.0, 1.0, rate_model=7)


BAD = [
    dict(L=16, tile=6, T=2.0),    # L not a multiple of tile
    dict(L=2, tile=2, T=2.0),     # one domain with fewer than three rows
    dict(L=12, tile=4, tile_rows=5, T=2.0),    # L not a multiple of tile_rows
    dict(L=16, tile=8, tile_rows=-1, T=2.0),   # tile_rows below 0
    dict(L=256, tile=16, tile_rows=256, T=2.0),  # tile_rows above 128
    dict(L=192, tile=96, T=2.0),  # domains over 64 sites a side with L > 128
    dict(L=2, tile=1, tile_rows=2, T=2.0),     # wrapped column with two sites
    dict(L=2, tile=2, tile_rows=1, T=2.0),     # wrapped row with two sites
    dict(L=8, tile=0, T=2.0),     # tile below 1
    dict(L=20, tile=8, T=2.0),    # L not a multiple of tile
    dict(L=256, tile=128, T=2.0), # tile above 64
    dict(L=16, tile=8, T=0.0),    # T must be positive
    dict(L=16, tile=8, T=float("nan")),
    dict(L=16, tile=8, T=2.0, steps_per_visit=-1),
    dict(L=16, tile=8, T=2.0, rate_model=3),
    dict(L=16, tile=8, T=2.0, schedule=5),
    dict(L=16, tile=8, T=2.0, init=9),
]


@pytest.mark.parametrize("bad", BAD)
def test_init_rejects_invalid_descriptor(kmc, bad):
    arr = kmc.make_descs([dict(L=16, tile=8, T=2.0), bad])
    ctx = C.c_void_p()
    st = kmc.lib().kmc_init_lattice(C.byref(ctx), arr, 2, C.c_uint64(1), None, None)
    assert st == kmc.KMC_EINVAL and not ctx.value


def test_calls_reject_null_context(kmc):
    L = kmc.lib()
    assert L.kmc_run_schedule(None, 1, 1, 0) == kmc.KMC_EINVAL
    assert L.kmc_backward_score(None, None, 0, 0) == kmc.KMC_EINVAL
    assert L.kmc_get_spins(None, 0, None) == kmc.KMC_EINVAL
    assert L.kmc_set_wait_limit(None, 5) == kmc.KMC_EINVAL
    assert L.kmc_get_domain_clocks(None, 0, None, None) == kmc.KMC_EINVAL
    assert L.kmc_get_domain_state(None, 0, None, None, None) == kmc.KMC_EINVAL
    assert L.kmc_last_error(None) == b"null context"


def test_exact_sweeps_rejects_bad_arguments(kmc):
    """Validation happens before any device call (no GPU needed)."""
    L = kmc.lib()
    p = C.c_void_p(16)  # never dereferenced: every call below fails validation
    big = kmc.make_descs([dict(L=6, tile=6, T=2.0)])          # 36 sites > 26
    assert L.kmc_exact_sweeps(big, p, p, 1, 0, None) == kmc.KMC_EINVAL
    bad = kmc.make_descs([dict(L=4, tile=3, T=2.0)])          # L not a multiple of tile
    assert L.kmc_exact_sweeps(bad, p, p, 1, 0, None) == kmc.KMC_EINVAL
    nine = kmc.make_descs([dict(L=3, tile=1, T=2.0)])         # 9 colours, random orders
    assert L.kmc_exact_sweeps(nine, p, p, 1, 0, None) == kmc.KMC_EUNSUPPORTED
    ok = kmc.make_descs([dict(L=4, tile=2, T=2.0)])
    assert L.kmc_exact_sweeps(ok, None, p, 1, 0, None) == kmc.KMC_EINVAL
    assert L.kmc_exact_sweeps(ok, p, p, -1, 0, None) == kmc.KMC_EINVAL
    # the allocation-free form holds at most 16 sites in its own buffer
    five = kmc.make_descs([dict(L=5, tile=5, T=2.0)])         # 25 sites > 16
    assert L.kmc_exact_sweeps_static(five, p, 1, 0, None) == kmc.KMC_EINVAL
    assert L.kmc_exact_sweeps_static(big, p, 1, 0, None) == kmc.KMC_EINVAL
    assert L.kmc_exact_sweeps_static(bad, p, 1, 0, None) == kmc.KMC_EINVAL
    assert L.kmc_exact_sweeps_static(nine, p, 1, 0, None) == kmc.KMC_EUNSUPPORTED
    assert L.kmc_exact_sweeps_static(ok, None, 1, 0, None) == kmc.KMC_EINVAL
    assert L.kmc_exact_sweeps_static(ok, p, -1, 0, None) == kmc.KMC_EINVAL
    L.kmc_destroy(None)


def test_allocator_hooks_must_come_in_pairs(kmc):
    L = kmc.lib()
    alloc = kmc._ALLOC_FN(lambda n, u: None)
    assert L.kmc_set_device_allocator(alloc, C.cast(None, kmc._FREE_FN), None) == kmc.KMC_EINVAL
    assert L.kmc_set_device_allocator(C.cast(None, kmc._ALLOC_FN),
                                      C.cast(None, kmc._FREE_FN), None) == kmc.KMC_OK


def test_header_compiles_as_plain_c(tmp_path):
    """include/kmc.h is a C header: plain C11 with no HIP or torch types."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text(
        '#include "kmc.h"\n'
        "#include <stddef.h>\n"
        "int main(void) {\n"
        "    kmc_rate_model m = KMC_RATE_BARKER;\n"
        "    kmc_schedule s = KMC_SCHED_PALINDROME;\n"
        "    kmc_init i = KMC_INIT_ALL_UP;\n"
        "    kmc_replica_desc d = {0};\n"
        "    kmc_record r = {0};\n"
        "    _Static_assert(sizeof(kmc_replica_desc) == 64, \"descriptor size\");\n"
        "    _Static_assert(offsetof(kmc_replica_desc, time_slice) == 56, \"slice\");\n"
        "    kmc_status (*f)(kmc_ctx *, int32_t, double *, double *) = kmc_get_domain_clocks;\n"
        "    (void)d; (void)r; (void)f;\n"
        "    return (int)m + (int)s + (int)i - 3;\n"
        "}\n")
    exe = tmp_path / "use"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-c", "-I",
                    os.path.join(ROOT, "include"), str(src), "-o", str(exe) + ".o"],
                   check=True)



def test_descriptor_layout(kmc):
    """The descriptor as the C header lays it out (64 bytes: three doubles,
    eight int32 fields, the time slice), and refusals that need no GPU."""
    import ctypes
    assert ctypes.sizeof(kmc.ReplicaDesc) == 64
    assert kmc.ReplicaDesc.time_slice.offset == 56 and kmc.ReplicaDesc.dims.offset == 52
    L = kmc.lib()
    p = C.c_void_p(16)
    sl = kmc.make_descs([dict(L=4, tile=2, T=2.0, time_slice=0.5)])
    assert L.kmc_exact_sweeps(sl, p, p, 1, 0, None) == kmc.KMC_EUNSUPPORTED
    neg = kmc.make_descs([dict(L=4, tile=2, T=2.0, time_slice=-1.0)])
    assert L.kmc_exact_sweeps(neg, p, p, 1, 0, None) == kmc.KMC_EINVAL
    ring = kmc.make_descs([dict(L=8, tile=3, T=2.0, dims=1)])   # 8 % 3 != 0
    assert L.kmc_exact_sweeps(ring, p, p, 1, 0, None) == kmc.KMC_EINVAL
