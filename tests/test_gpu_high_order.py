"""Chebyshev orders above 8 (two nodes per lane in the near quadrature):
q = 10, the paper's 10 x 10 points per patch (Sec. IV-A, Table 1), and
q = 11, the largest order whose patch fits a 256-unknown leaf.  Checked
against the oracle row by row (far entries by the same Fejer rule, near
entries by its independent Duffy quadrature), then the complex64 H-LU with
FP64 refinement against exact oracle rows, and the surface current against
the Mie series, which q = 10 must approach more closely than q = 8 on the
same patches."""
import numpy as np
import pytest

from oracle import geometry as G, mfie, mie, post
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _solver(spec, leaf=256, tol=None):
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=leaf, eta=1.0, near_delta=1.0)
    s.fill()
    if tol is not None:
        s.compress(tol)
    return s


@pytest.mark.parametrize("q", [9, 10, 11])
def test_fill_rows_match_oracle(q):
    spec = W.tiny_sphere(s=2, q=q, k0=3.0)
    s = _solver(spec, leaf=2 * q * q)
    A = s.export_dense()
    nd = G.build_nodes(spec)
    rows = W.sample_indices(2 * nd.size, 6, seed=q)
    ref = mfie.matrix_rows(nd, spec.k0, rows)
    got = A[rows].cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    # the same rows with a finer rule (90 x 72 points): what is left of the
    # difference is the oracle's side
    s.fill(n_ang=90, n_rad=72)
    fine = s.export_dense()[rows].cpu().numpy()
    err_f = np.abs(fine - ref).max() / np.abs(ref).max()
    print(f"q {q}: rows err {err:.2e} (finer rule {err_f:.2e})")
    assert err < 1e-9
    s.close()


def test_q10_solve_residual_and_mie():
    import torch
    from paper_2408_17116_amd import cbie
    k0 = 2.0 * np.pi
    errs = {}
    for q in (8, 10):
        spec = W.ObjectSpec(axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), s=2, q=q, k0=k0)
        s = _solver(spec, tol=1e-8)
        s.factor(cbie.PREC_C64_IR)
        kh, pol = W.axial_wave()
        b = s.rhs_planewave(kh, pol)
        x, it = s.solve(b, tol=1e-11, maxit=30)
        x = x.cpu().numpy()[:, 0]
        nd = G.build_nodes(spec)
        rows = W.sample_indices(2 * nd.size, 6, seed=3)
        Ar = mfie.matrix_rows(nd, k0, rows)
        bo = mfie.rhs_planewave(nd, k0, kh, pol)[:, 0]
        res = np.abs(Ar @ x - bo[rows]).max() / np.abs(bo).max()
        J = post.surface_current(nd, x)
        Jm = mie.pec_surface_current(k0, 1.0, nd.r)
        errs[q] = post.weighted_rel_l2(nd, J, Jm)
        print(f"q {q}: {2 * nd.size} unknowns, {it} sweeps, sampled residual {res:.2e}, J vs Mie {errs[q]:.2e}")
        assert res < 1e-7
        s.close()
    # spectral convergence in the order on the same 24 patches
    assert errs[10] < 0.5 * errs[8]
    torch.cuda.synchronize()
