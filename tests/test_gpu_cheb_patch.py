"""Chebyshev-interpolated patches (generic surface input, the form a CAD
surface is handed over in) through the C-ABI, against the oracle: near
pairs identical and dense fills equal entry by entry (far entries to
rounding, near entries to the agreement of the two quadratures) on an
interpolated sphere and a torus, for both formulations; then full
pipelines on an interpolated sphere (against the Mie series) and a torus
(residual on exact oracle rows)."""
import numpy as np
import pytest

from oracle import geometry as G, mfie, mie, muller as Mu, post
from synth import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "sphere_s1q4": lambda: W.gnomonic_sphere_cheb(1, 4, 1.0, 10),
    "torus_6x3_q4": lambda: W.torus_cheb(6, 3, 4, 2.0, 10, R=1.0, rho=0.4),
}


def _solver(spec, leaf):
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=leaf, eta=1.0, near_delta=1.0)
    return s


def _near_mask(nd, pairs, upn):
    q2 = nd.q ** 2
    m = np.zeros((nd.size, nd.n_patches), dtype=bool)
    for (t, p, _u, _v, _s) in pairs:
        m[t, p] = True
    return np.repeat(np.repeat(m, upn, axis=0), upn * q2, axis=1)


@pytest.mark.parametrize("name", list(CASES))
def test_mfie_near_pairs_and_fill_match_oracle(name):
    spec = CASES[name]()
    s = _solver(spec, 2 * spec.q ** 2)
    t, p = s.near_pairs()
    s.fill()
    A = s.export_dense().cpu().numpy()
    s.close()
    nd = G.build_nodes(spec)
    pairs = mfie.near_pairs(nd)
    assert np.array_equal(t, np.array([e[0] for e in pairs])) and np.array_equal(p, np.array([e[1] for e in pairs]))
    Ao = mfie.dense_matrix(nd, spec.k0, pairs=pairs, workers=4)
    mask = _near_mask(nd, pairs, 2)
    scale = np.abs(Ao).max()
    far = np.abs(A - Ao)[~mask].max() / scale if (~mask).any() else 0.0   # s = 1: every pair is near
    near = np.abs(A - Ao)[mask].max() / scale
    print(f"{name}: {A.shape[0]} unknowns, {len(pairs)} near pairs; far {far:.2e}, near {near:.2e}")
    assert far < 1e-13 and near < 1e-9


def test_nmuller_fill_matches_oracle():
    spec = W.gnomonic_sphere_cheb(1, 3, 1.5, 8, form=W.FORM_NMULLER, eps_r=3.0)
    s = _solver(spec, 4 * spec.q ** 2)
    s.fill()
    A = s.export_dense().cpu().numpy()
    s.close()
    nd = G.build_nodes(spec)
    pairs = mfie.near_pairs(nd)
    Ao = Mu.dense_matrix(nd, spec.k0, spec.eps_r, pairs=pairs, workers=4)
    mask = _near_mask(nd, pairs, 4)
    scale = np.abs(Ao).max()
    far = np.abs(A - Ao)[~mask].max() / scale if (~mask).any() else 0.0
    near = np.abs(A - Ao)[mask].max() / scale
    print(f"N-Mueller: {A.shape[0]} unknowns; far {far:.2e}, near {near:.2e}")
    assert far < 1e-13 and near < 1e-9


def test_interpolated_sphere_against_mie():
    """Gnomonic cube sphere as 96 patches of degree 14, q = 8, k = 2 pi
    (12,288 unknowns), mixed pipeline: the current against the Mie series,
    next to the same solver on the library's own equiangular sphere."""
    from paper_2408_17116_amd import cbie
    errs = {}
    for name, spec in (("chebyshev", W.gnomonic_sphere_cheb(4, 8, 2 * np.pi, 14)),
                       ("equiangular", W.tiny_sphere(s=4, q=8, k0=2 * np.pi))):
        s = _solver(spec, 256)
        s.fill()
        s.compress(1e-6)
        s.factor(cbie.PREC_C64_IR)
        b = s.rhs_planewave(*W.axial_wave())
        x, it = s.solve(b, tol=1e-10, maxit=30)
        s.close()
        nd = G.build_nodes(spec)
        J = post.surface_current(nd, x.cpu().numpy()[:, 0])
        errs[name] = post.weighted_rel_l2(nd, J, mie.pec_surface_current(spec.k0, 1.0, nd.r))
        print(f"{name}: {spec.n_unknowns} unknowns, {it} sweeps, J vs Mie {errs[name]:.2e}")
    assert errs["chebyshev"] < 1e-2
    assert errs["chebyshev"] < 10 * errs["equiangular"]


def test_torus_pipeline_exact_rows():
    """A torus (R = 1, rho = 0.4) as 24 x 8 patches of degree 12, q = 6,
    k = 4 (13,824 unknowns), mixed pipeline: the residual of the solution on
    exact oracle rows."""
    from paper_2408_17116_amd import cbie
    spec = W.torus_cheb(24, 8, 6, 4.0, 12, R=1.0, rho=0.4)
    s = _solver(spec, 256)
    s.fill()
    s.compress(1e-8)
    s.factor(cbie.PREC_C64_IR)
    kh, pol = W.plane_waves(2, seed=5)
    b = s.rhs_planewave(kh, pol)
    x, it = s.solve(b, tol=1e-11, maxit=30)
    st = s.stats()
    s.close()
    nd = G.build_nodes(spec)
    rows = W.sample_indices(2 * nd.size, 8, seed=17)
    A = mfie.matrix_rows(nd, spec.k0, rows)
    bo = mfie.rhs_planewave(nd, spec.k0, kh, pol)
    res = np.abs(A @ x.cpu().numpy() - bo[rows]).max() / np.abs(bo).max()
    print(f"torus: {spec.n_unknowns} unknowns, CR {st['compression_rate']:.3f}, max rank {st['max_rank']}, "
          f"{it} sweeps; residual on 8 exact oracle rows {res:.2e}")
    assert res < 1e-6
