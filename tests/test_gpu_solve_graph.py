"""Substitutions replayed through the captured HIP graph.  The first solve
with a factorization records the substitution program and runs it eagerly;
every later substitution (refinement sweeps, later solves) launches the
graph.  Each replayed substitution, with eager work and synchronizations in
between, must reproduce bit for bit what the recorded program computes when
it is run eagerly (the replay off); a change of the number of right-hand
sides must record a new program.  Refined solves (their FP64 residual sums
blocks atomically, so they agree to rounding only) are compared with a
tolerance."""
import os

import numpy as np
import pytest

from oracle import geometry as G, mfie, dense
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _solve(s, b, replay, maxit=0):
    os.environ["CBIE_SOLVE_REPLAY"] = "1" if replay else "0"
    try:
        x, it = s.solve(b, tol=1e-12, maxit=maxit)
    finally:
        os.environ.pop("CBIE_SOLVE_REPLAY", None)
    return x.clone(), it


@pytest.mark.parametrize("prec", [0, 1], ids=["c128", "c64_ir"])
def test_graph_replays_equal_eager_runs(prec):
    import torch
    from paper_2408_17116_amd import cbie
    spec = W.tiny_sphere(s=3, q=5, k0=3.0)        # 2700 unknowns
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=100, eta=1.0, near_delta=1.0)
    s.fill()
    s.compress(1e-9)
    s.factor(prec)
    n = s.n
    bs = [torch.from_numpy(W.random_complex((n, 3), seed=10 + i)).cuda() for i in range(3)]
    y = torch.from_numpy(W.random_complex((n, 2), seed=99)).cuda()
    ref = [_solve(s, b, replay=False)[0] for b in bs]
    assert s.stats()["solve_replays"] == 0
    first, _ = _solve(s, bs[0], replay=True)           # records the program
    torch.cuda.synchronize()
    assert torch.equal(first, ref[0])
    for rep in range(3):
        for i, b in enumerate(bs):
            x, _ = _solve(s, b, replay=True)
            s.matvec(y)                                 # eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(x, ref[i]), (rep, i)
    nrep = s.stats()["solve_replays"]
    assert nrep >= 9
    # a different number of right-hand sides records a new program
    b2 = bs[1][:, :2].contiguous()
    x2, _ = _solve(s, b2, replay=True)
    x2r, _ = _solve(s, b2, replay=False)
    assert torch.equal(x2, x2r)
    x3, _ = _solve(s, bs[2], replay=True)
    assert torch.equal(x3, ref[2])
    # refined solves: every sweep's correction is a replay
    nd = G.build_nodes(spec)
    xo = dense.solve(mfie.dense_matrix(nd, spec.k0), bs[0].cpu().numpy())
    if prec == cbie.PREC_C64_IR:
        before = s.stats()["solve_replays"]
        xr, it = _solve(s, bs[0], replay=True, maxit=30)
        xe, ite = _solve(s, bs[0], replay=False, maxit=30)
        assert s.stats()["solve_replays"] == before + it + 1
        d = (torch.linalg.norm(xr - xe) / torch.linalg.norm(xe)).item()
        assert d < 1e-13
        first = xr
    e = np.linalg.norm(first.cpu().numpy() - xo) / np.linalg.norm(xo)
    print(f"prec {prec}: replays {s.stats()['solve_replays']}, vs dense oracle {e:.2e}")
    assert e < 1e-7
    s.close()

