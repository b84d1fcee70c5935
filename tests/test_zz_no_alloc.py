"""The allocation-free matvec (cbie_matvec_noalloc) against cbie_matvec,
through the C-ABI: two calls in a row on one GPU, the second with a smaller
input (a smaller context and fewer right-hand sides), each checked against
the allocating entry point of its own context; a call larger than the
scratch array is refused with EINVAL before any device work."""
import numpy as np
import pytest

from synth import workloads as W

pytestmark = pytest.mark.gpu


def _ctx(spec, leaf):
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=leaf, eta=1.0, near_delta=1.0)
    s.fill()
    s.compress(1e-6)
    return s


def _check(s, nrhs, seed):
    import torch
    x = torch.from_numpy(W.random_complex((s.n, nrhs), seed=seed)).cuda()
    y_ref = s.matvec(x).cpu().numpy()
    y = s.matvec_noalloc(x).cpu().numpy()
    err = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    print(f"n {s.n}, nrhs {nrhs}: max |y - y_ref| / max |y_ref| = {err:.2e}")
    # the same FP64 sums, in another order (atomic accumulation)
    assert err <= 1e-13


def test_noalloc_matvec_matches_matvec_on_two_calls():
    from paper_2408_17116_amd import cbie
    big = _ctx(W.tiny_sphere(s=4, q=4, k0=6.0), leaf=64)      # 3072 unknowns
    small = _ctx(W.tiny_sphere(s=2, q=4, k0=3.0), leaf=32)    # 768 unknowns
    assert big.stats()["n_lr_blocks"] > 0 and small.stats()["n_lr_blocks"] > 0
    _check(big, 4, seed=1)
    _check(small, 1, seed=2)
    # too many right-hand sides for the scratch array: refused
    per_rhs = 2 * small.n + small.stats()["sum_rank"]
    nrhs = (1 << 23) // per_rhs + 1
    import torch
    x = torch.zeros((small.n, nrhs), dtype=torch.complex128, device="cuda")
    with pytest.raises(cbie.CbieError) as e:
        small.matvec_noalloc(x)
    assert e.value.code == cbie.EINVAL
    # and the scratch still serves a valid call afterwards
    _check(small, 2, seed=3)
    big.close()
    small.close()
