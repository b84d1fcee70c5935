"""Batched objects: one context holding several uneven scatterers (different
shapes, patch counts, Chebyshev orders and wavenumbers) is block diagonal.
Every step runs for all objects in shared batched launches; each object's
solution must equal the one from a context of its own, and the dense oracle
solution of that object."""
import numpy as np
import pytest

from oracle import dense, geometry as G, mfie
from synth import workloads as W

pytestmark = pytest.mark.gpu

OBJECTS = [
    W.ObjectSpec(axes=(1.0, 0.7, 0.5), center=(0.0, 0.0, 0.0), s=2, q=4, k0=3.0),
    W.ObjectSpec(axes=(0.6, 0.9, 1.2), center=(4.0, 0.0, 0.0), s=2, q=5, k0=4.5),
    W.ObjectSpec(axes=(0.8, 0.8, 0.8), center=(0.0, 5.0, 1.0), s=1, q=6, k0=2.0),
]


def _solve(objs, prec, tol):
    import torch
    from paper_2408_17116_amd import cbie
    s = cbie.Solver(objs)
    s.build_tree(leaf_size=128, eta=1.0, near_delta=1.0)
    s.fill()
    s.compress(tol)
    s.factor(prec)
    kh, pol = W.plane_waves(2, seed=17)
    b = s.rhs_planewave(kh, pol)
    x, it = s.solve(b, tol=1e-12, maxit=0 if prec == cbie.PREC_C128 else 30)
    st = s.stats()
    out = x.cpu().numpy(), b.cpu().numpy(), st
    s.close()
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", [0, 1], ids=["c128", "c64_ir"])
def test_batch_equals_single_objects_and_oracle(prec):
    tol = 1e-10
    xb, bb, st = _solve(OBJECTS, prec, tol)
    assert st["n_objects"] == len(OBJECTS)
    off = 0
    for o, spec in enumerate(OBJECTS):
        n = spec.n_unknowns
        xs, bs, _ = _solve([spec], prec, tol)
        # the right-hand sides of the batch are the objects' own, stacked
        assert np.abs(bb[off:off + n] - bs).max() <= 1e-14 * np.abs(bs).max()
        d = np.linalg.norm(xb[off:off + n] - xs) / np.linalg.norm(xs)
        nd = G.build_nodes(spec)
        A = mfie.dense_matrix(nd, spec.k0)
        kh, pol = W.plane_waves(2, seed=17)
        xo = dense.solve(A, mfie.rhs_planewave(nd, spec.k0, kh, pol))
        e = np.linalg.norm(xb[off:off + n] - xo) / np.linalg.norm(xo)
        print(f"prec {prec} object {o} (N {n}, q {spec.q}): batch vs single {d:.2e}, vs dense oracle {e:.2e}")
        assert d < 1e-8
        assert e < 1e-7
        off += n
    assert off == xb.shape[0]
