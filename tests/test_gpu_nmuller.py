"""N-Mueller formulation of a homogeneous dielectric body on the GPU (four
unknowns per node): the fill against the oracle entry by entry (far entries
with the Chebyshev-differentiated divergence, near entries from two
different quadratures), ACA of the explicit admissible blocks, the H-LU
solution against the dense oracle solution in both precisions, the dielectric
Mie series, and sampled rows at the dielectric-sphere workload."""
import numpy as np
import pytest

from oracle import geometry as G, mfie, mie, muller as Mu
from synth import workloads as W

pytestmark = pytest.mark.gpu

KH, POL = np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]])


def _spec(s, q, k0, er, axes=(1.0, 1.0, 1.0)):
    return W.ObjectSpec(axes=axes, center=(0.0, 0.0, 0.0), s=s, q=q, k0=k0, form=W.FORM_NMULLER,
                        eps_r=er, mu_r=1.0)


def _solver(spec, leaf=None):
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=leaf or 4 * spec.q ** 2, eta=1.0, near_delta=1.0)
    return s


CASES = [_spec(1, 4, 1.0, 4.0), _spec(2, 4, 2.0, 9.0, axes=(1.2, 0.8, 0.6))]


@pytest.mark.parametrize("spec", CASES, ids=["sphere_s1q4", "ell_s2q4"])
def test_fill_matches_oracle(spec):
    s = _solver(spec)
    s.fill()
    A = s.export_dense().cpu().numpy()
    nd = G.build_nodes(spec)
    Ao = Mu.dense_matrix(nd, spec.k0, spec.eps_r, 1.0, workers=8)
    pairs = mfie.near_pairs(nd)
    q2 = spec.q ** 2
    near = np.zeros((nd.size, nd.n_patches), dtype=bool)
    for (t, p, _u, _v, _s) in pairs:
        near[t, p] = True
    mask = np.repeat(np.repeat(near, 4, axis=0), 4 * q2, axis=1)
    scale = np.abs(Ao).max()
    far_err = np.abs(A - Ao)[~mask].max() / scale if (~mask).any() else 0.0
    near_err = np.abs(A - Ao)[mask].max() / scale
    print(f"N {A.shape[0]}: far {far_err:.2e} near {near_err:.2e}")
    assert far_err < 1e-13
    assert near_err < 1e-9
    s.close()


def test_aca_of_explicit_blocks_within_tolerance():
    import torch
    spec = _spec(3, 4, 3.0, 4.0)
    s = _solver(spec)
    s.fill()
    A = s.export_dense()
    for tol in (1e-4, 1e-7):
        s.compress(tol)
        st = s.stats()
        Ac = s.export_dense()
        err = (torch.linalg.norm(Ac - A) / torch.linalg.norm(A)).item()
        x = torch.from_numpy(W.random_complex((s.n, 2), seed=3)).cuda()
        y = s.matvec(x)
        mv = (torch.linalg.norm(y - Ac @ x) / torch.linalg.norm(Ac @ x)).item()
        print(f"tol {tol:g}: {st['n_lr_blocks']} blocks, max rank {st['max_rank']}, rel F err {err:.2e}, matvec {mv:.1e}")
        assert st["n_lr_blocks"] > 0
        assert err < 10 * tol
        assert mv < 1e-13
    s.close()


def test_aca_entries_on_the_fly_equal_explicit_copies():
    """The same admissible blocks compressed from explicit copies and from
    entries generated on the fly (divergence through the source patch's
    lines): both within the tolerance of the uncompressed fill, with the same
    ranks, and the two compressed operators equal to well below it."""
    import os
    import torch
    spec = _spec(3, 4, 3.0, 4.0)
    s = _solver(spec)
    s.fill()
    A = s.export_dense()
    old = os.environ.get("CBIE_NM_OTF_MIN")
    out = {}
    try:
        for name, lim in (("explicit", "1000000000"), ("on_the_fly", "0")):
            os.environ["CBIE_NM_OTF_MIN"] = lim
            s.compress(1e-7)
            out[name] = (s.export_dense(), s.block_features(1e-7)[1], s.stats())
    finally:
        if old is None:
            del os.environ["CBIE_NM_OTF_MIN"]
        else:
            os.environ["CBIE_NM_OTF_MIN"] = old
    (Ae, re, ste), (Ao, ro, sto) = out["explicit"], out["on_the_fly"]
    ee = (torch.linalg.norm(Ae - A) / torch.linalg.norm(A)).item()
    eo = (torch.linalg.norm(Ao - A) / torch.linalg.norm(A)).item()
    d = (torch.linalg.norm(Ao - Ae) / torch.linalg.norm(A)).item()
    print(f"{ste['n_lr_blocks']} blocks: explicit {ee:.2e}, on the fly {eo:.2e}, between them {d:.2e}; "
          f"ranks equal {np.array_equal(re, ro)} (max {re.max()} / {ro.max()}); "
          f"compress {ste['t_compress']:.3f} s / {sto['t_compress']:.3f} s")
    assert ee < 1e-6 and eo < 1e-6
    assert np.array_equal(re, ro) or d < 1e-8
    s.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["c128", "c64_ir"])
def test_hlu_solution_matches_dense_oracle(prec):
    from paper_2408_17116_amd import cbie
    spec = _spec(2, 4, 1.0, 4.0)
    s = _solver(spec)
    s.fill()
    s.compress(1e-10)
    s.factor(prec)
    b = s.rhs_planewave(KH, POL)
    x, it = s.solve(b, tol=1e-12, maxit=0 if prec == cbie.PREC_C128 else 30)
    nd = G.build_nodes(spec)
    bo = Mu.rhs_planewave(nd, spec.k0, KH, POL)
    assert np.abs(b.cpu().numpy()[:, 0] - bo[:, 0]).max() < 1e-14 * np.abs(bo).max()
    xo = np.linalg.solve(Mu.dense_matrix(nd, spec.k0, spec.eps_r, 1.0, workers=8), bo[:, 0])
    e = np.linalg.norm(x.cpu().numpy()[:, 0] - xo) / np.linalg.norm(xo)
    print(f"prec {prec}: vs dense oracle {e:.2e}, refinement sweeps {it}")
    assert e < 1e-8
    s.close()


def test_solution_converges_to_dielectric_mie_and_far_field():
    """eps_r = 4, ka = 1, 24 patches q = 6 (3456 unknowns): the oracle's own
    gap to Mie at this size is 2e-6 (J), 3e-6 (M)."""
    from paper_2408_17116_amd import cbie
    spec = _spec(2, 6, 1.0, 4.0)
    s = _solver(spec)
    s.fill()
    s.compress(1e-9)
    s.factor(cbie.PREC_C64_IR)
    x, it = s.solve(s.rhs_planewave(KH, POL), tol=1e-12, maxit=30)
    xn = x.cpu().numpy()[:, 0]
    nd = G.build_nodes(spec)
    J, M = Mu.currents(nd, xn)
    Jm, Mm = mie.dielectric_surface_currents(spec.k0, 1.0, 4.0, 1.0, nd.r)
    eJ = np.linalg.norm(J - Jm) / np.linalg.norm(Jm)
    eM = np.linalg.norm(M - Mm) / np.linalg.norm(Mm)
    th = np.arange(0, 181, 5)
    from oracle import post
    rh = post.plane_cut(th, 0.0)
    E = s.farfield(x, rh)[0]
    Eo = Mu.far_field(nd, spec.k0, xn, rh)
    ff = np.abs(E - Eo).max() / np.abs(Eo).max()
    sE, _ = mie.dielectric_rcs(spec.k0, 1.0, 4.0, 1.0, np.deg2rad(th))
    rcs = 4 * np.pi * np.sum(np.abs(E) ** 2, axis=1)
    er = np.abs(rcs - sE).max() / sE.max()
    print(f"J {eJ:.2e} M {eM:.2e}; far field vs oracle {ff:.1e}; RCS vs Mie {er:.2e}; sweeps {it}")
    assert eJ < 1e-5 and eM < 1e-5
    assert ff < 1e-12
    assert er < 1e-5
    s.close()


def test_sampled_rows_at_dielectric_sphere():
    """eps_r = 16, ka = 5, 96 patches q = 8, 24576 unknowns: rows of the
    filled operator (dense near blocks and plain-rule far entries) against
    rows the oracle computes one by one."""
    spec = W.sphere_dielectric()
    s = _solver(spec, leaf=256)
    s.fill()
    A = s.export_dense()
    rows = W.sample_indices(spec.n_unknowns, 4, seed=11)
    got = A[rows].cpu().numpy()
    del A
    nd = G.build_nodes(spec)
    ref = Mu.matrix_rows(nd, spec.k0, spec.eps_r, 1.0, rows)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"rows {rows}: err {err:.2e}")
    assert err < 1e-8
    s.close()


def test_dielectric_sphere_workload_end_to_end():
    """eps_r = 16, ka = 5, 24576 unknowns, ACA 1e-6, complex64 H-LU with FP64
    refinement: the residual against the stored operator, and the Mie series
    (its gap here is the discretization's: q = 8 points per patch side with
    the interior wavenumber 4 k0)."""
    import torch
    from oracle import post
    from paper_2408_17116_amd import cbie
    spec = W.sphere_dielectric()
    s = _solver(spec, leaf=256)
    s.fill()
    s.compress(1e-6)
    s.factor(cbie.PREC_C64_IR)
    b = s.rhs_planewave(KH, POL)
    x, it = s.solve(b, tol=1e-10, maxit=30)
    res = (torch.linalg.norm(s.matvec(x) - b) / torch.linalg.norm(b)).item()
    nd = G.build_nodes(spec)
    J, M = Mu.currents(nd, x.cpu().numpy()[:, 0])
    Jm, Mm = mie.dielectric_surface_currents(spec.k0, 1.0, spec.eps_r, 1.0, nd.r)
    eJ = np.linalg.norm(J - Jm) / np.linalg.norm(Jm)
    th = np.arange(0, 181)
    sE, sH = mie.dielectric_rcs(spec.k0, 1.0, spec.eps_r, 1.0, np.deg2rad(th))
    E0 = s.farfield(x, post.plane_cut(th, 0.0))[0]
    E90 = s.farfield(x, post.plane_cut(th, 90.0))[0]
    r0, r90 = 4 * np.pi * np.sum(np.abs(E0) ** 2, 1), 4 * np.pi * np.sum(np.abs(E90) ** 2, 1)
    erc = max(np.linalg.norm(r0 - sE) / np.linalg.norm(sE), np.linalg.norm(r90 - sH) / np.linalg.norm(sH))
    print(f"sweeps {it}, residual {res:.1e}, J vs Mie {eJ:.2e}, RCS vs Mie {erc:.2e}")
    assert res < 1e-9
    assert erc < 1e-4
    assert eJ < 2e-3
    s.close()
