"""Host logic of the factor storage: the library's pool (its bookkeeping is
host code, compiled here with the host compiler over host memory chunks).
After every step of seeded sequences of allocations, deferred releases,
program launches and completions: live buffers lie inside one chunk, keep
their contents and never overlap each other, the free ranges or the
releases still pending; every element of every chunk is live, free or
pending; no two free ranges of a chunk touch.  With everything released the
free ranges merge back into one per chunk.  And the property the pool is
for: as low-rank factors grow, the memory freed by smaller ranks serves the
larger ones, so the chunks stay close to the peak of live storage."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_17116_amd", "csrc")
SHIM = os.path.join(ROOT, "tests", "host", "pool_shim.cpp")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("pool") / "libpoolshim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, SHIM, "-o", out], check=True)
    L = C.CDLL(out)
    dp = C.POINTER(C.c_double)
    L.pool_random.argtypes = [C.c_uint, C.c_int, C.c_size_t, C.c_size_t, dp]
    L.pool_growing_ranks.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_size_t, dp]
    return L


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_sequences_keep_the_invariants(lib, seed):
    out = np.zeros(2)
    rc = lib.pool_random(seed, 4000, 1 << 14, 6000, out.ctypes.data_as(C.POINTER(C.c_double)))
    assert rc == 0, f"check {rc // 100} failed"
    print(f"seed {seed}: capacity {out[0]:.0f}, peak live {out[1]:.0f}")


def test_growing_ranks_reuse_freed_memory(lib):
    """Each round holds the old factors (released, pending) and the new ones
    together, so no pool can hold less than that sum; the chunks must stay
    within 25% of it (a pool that reused only exact sizes would add a whole
    round's storage for every round)."""
    out = np.zeros(3)
    # 200 blocks of 256 rows, rank 8 -> 8 + 40 * 2 = 88
    rc = lib.pool_growing_ranks(200, 256, 8, 2, 40, 1 << 20, out.ctypes.data_as(C.POINTER(C.c_double)))
    assert rc == 0, f"check {rc // 100} failed"
    cap, peak, need = out
    print(f"capacity {cap:.0f} elements; peak live {peak:.0f}, live + pending {need:.0f}")
    assert cap <= 1.25 * need
