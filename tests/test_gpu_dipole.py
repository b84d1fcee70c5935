"""Point-dipole excitation (Sec. IV-A: the spiral antenna is fed by an
x-polarized dipole) through the C-ABI, against the oracle.

The right-hand sides of cbie_rhs_dipole must equal the oracle's entry by
entry (MFIE and N-Mueller, several dipoles, a context of objects with
different wavenumbers).  A PEC sphere excited by a dipole outside it is
then solved: the solution must leave a small residual on exact oracle rows
with the oracle's right-hand side, and a dipole moved far away must give
the plane-wave solution, scaled by the dipole's far-field factor."""
import numpy as np
import pytest

from oracle import dipole, geometry as G, mfie
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _dipoles(n, radius, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    pos = d / np.linalg.norm(d, axis=1)[:, None] * radius * rng.uniform(1.2, 2.0, n)[:, None]
    return pos, rng.standard_normal((n, 3))


@pytest.mark.parametrize("form", ["mfie", "nmuller"])
def test_rhs_matches_oracle(form):
    from paper_2408_17116_amd import cbie
    if form == "mfie":
        spec = W.tiny_sphere(s=2, q=4, k0=3.0)
    else:
        spec = W.ObjectSpec(axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), s=2, q=4, k0=2.0,
                            form=W.FORM_NMULLER, eps_r=4.0, mu_r=1.0)
    pos, mom = _dipoles(3, 1.0, seed=7)
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=64, eta=1.0, near_delta=1.0)
    b = s.rhs_dipole(pos, mom).cpu().numpy()
    s.close()
    nd = G.build_nodes(spec)
    ref = dipole.rhs_mfie(nd, spec.k0, pos, mom) if form == "mfie" else dipole.rhs_nmuller(nd, spec.k0, pos, mom)
    err = np.abs(b - ref).max() / np.abs(ref).max()
    print(f"{form}: {b.shape[0]} rows x {b.shape[1]} dipoles, max error {err:.2e}")
    assert err < 1e-13


def test_rhs_multi_object_context():
    from paper_2408_17116_amd import cbie
    objs = W.ellipsoid_batch(3, seed=1)
    pos, mom = _dipoles(2, 6.0, seed=3)
    s = cbie.Solver(objs)
    s.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
    b = s.rhs_dipole(pos, mom).cpu().numpy()
    s.close()
    off = 0
    for o in objs:
        nd = G.build_nodes(o)
        ref = dipole.rhs_mfie(nd, o.k0, pos, mom)
        err = np.abs(b[off:off + o.n_unknowns] - ref).max() / np.abs(ref).max()
        print(f"object k0 {o.k0:.3f}, {o.n_unknowns} unknowns: max error {err:.2e}")
        assert err < 1e-13
        off += o.n_unknowns


def test_dipole_excited_sphere_against_oracle_rows_and_plane_wave_limit():
    import torch
    from paper_2408_17116_amd import cbie
    spec = W.sphere_pec_small()                       # r = 1, k = 2 pi, 3,072 unknowns
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
    s.fill()
    s.compress(1e-8)
    s.factor(cbie.PREC_C64_IR)
    k = spec.k0
    D = 1e4
    pos = np.array([[0.0, 0.0, -2.0], [0.0, 0.0, -D]])
    mom = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    b = s.rhs_dipole(pos, mom)
    x, it = s.solve(b, tol=1e-12, maxit=30)
    kh, pol = W.axial_wave()
    xp, _ = s.solve(s.rhs_planewave(kh, pol), tol=1e-12, maxit=30)
    s.close()
    x, xp = x.cpu().numpy(), xp.cpu().numpy()[:, 0]
    nd = G.build_nodes(spec)
    rows = W.sample_indices(2 * nd.size, 8, seed=13)
    A = mfie.matrix_rows(nd, k, rows)
    bo = dipole.rhs_mfie(nd, k, pos[:1], mom[:1])[:, 0]
    res = np.abs(A @ x[:, 0] - bo[rows]).max() / np.abs(bo).max()
    c = -1j * k * np.exp(-1j * k * D) / (4 * np.pi * D)
    lim = np.linalg.norm(x[:, 1] / c - xp) / np.linalg.norm(xp)
    print(f"{it} sweeps; residual on 8 exact oracle rows {res:.2e}; distant dipole vs plane wave {lim:.2e}")
    assert res < 1e-7
    assert lim < 1e-3


def test_dipole_rhs_errors():
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([W.tiny_sphere(s=1, q=4, k0=1.0)])
    try:
        s.rhs_dipole([[0.0, 0.0, 3.0]], [[1.0, 0.0, 0.0]])
    except cbie.CbieError as e:
        assert e.code == cbie.ESTATE
    else:
        raise AssertionError("rhs_dipole before build_tree must fail")
    s.build_tree(leaf_size=64, eta=1.0, near_delta=1.0)
    with pytest.raises(ValueError):
        s.rhs_dipole([[0.0, 0.0, 3.0]], [[1.0, 0.0]])
    s.close()
