"""GPU parity of ACA compression, FP64 H-matvec, plane-wave RHS and far
field against the oracle and against the exactly filled matrix."""
import numpy as np
import pytest

from oracle import geometry as G, mfie, post
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _filled(spec, leaf, tol=None):
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=leaf, eta=1.0, near_delta=1.0)
    s.fill()
    A_exact = s.export_dense()
    if tol is not None:
        s.compress(tol)
    return s, A_exact


def test_rhs_and_farfield_match_oracle():
    import torch
    spec = W.ObjectSpec(axes=(1.2, 0.8, 0.6), center=(0.1, 0.0, -0.1), s=2, q=5, k0=1.5)
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=50, eta=1.0)
    kh, pol = W.plane_waves(3, seed=5)
    b = s.rhs_planewave(kh, pol).cpu().numpy()
    nd = G.build_nodes(spec)
    bo = mfie.rhs_planewave(nd, spec.k0, kh, pol)
    assert np.abs(b - bo).max() < 1e-14 * np.abs(bo).max()
    x = W.random_complex((2 * nd.size, 2), seed=3)
    rh = post.plane_cut(np.linspace(0, 180, 19), 30.0)
    E = s.farfield(torch.from_numpy(x).cuda(), rh)
    for r in range(2):
        Eo = post.far_field(nd, spec.k0, x[:, r], rh)
        assert np.abs(E[r] - Eo).max() < 1e-12 * np.abs(Eo).max()


def test_matvec_dense_part_matches_oracle():
    import torch
    spec = W.tiny_sphere(s=1, q=4, k0=1.0)
    s, _ = _filled(spec, leaf=2 * 16, tol=1e-8)
    nd = G.build_nodes(spec)
    Ao = mfie.dense_matrix(nd, spec.k0)
    x = W.random_complex((2 * nd.size, 3), seed=1)
    y = s.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    yo = Ao @ x
    assert np.abs(y - yo).max() < 1e-9 * np.abs(yo).max()


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-8])
def test_aca_compression_error_bound(tol):
    import torch
    spec = W.tiny_sphere(s=4, q=4, k0=6.0)   # 96 patches, 3072 unknowns
    s, A = _filled(spec, leaf=64, tol=tol)
    st = s.stats()
    assert st["n_lr_blocks"] > 0 and st["max_rank"] > 0
    Ac = s.export_dense()
    err = (torch.linalg.norm(Ac - A) / torch.linalg.norm(A)).item()
    print(f"tol {tol:g}: rel F err {err:.2e}, CR {st['compression_rate']:.3f}, max rank {st['max_rank']}")
    assert err < 10 * tol
    # the H-matvec equals the compressed matrix applied densely
    x = torch.from_numpy(W.random_complex((A.shape[0], 2), seed=2)).cuda()
    y = s.matvec(x)
    yd = Ac @ x
    assert (torch.linalg.norm(y - yd) / torch.linalg.norm(yd)).item() < 1e-13


def test_no_near_pair_in_low_rank_blocks_and_full_cover():
    import torch
    spec = W.tiny_sphere(s=4, q=4, k0=6.0)
    s, A = _filled(spec, leaf=64, tol=1e-6)
    st = s.stats()
    # dense + low-rank blocks cover the matrix exactly once: the dense
    # entries plus the low-rank block areas add up to N^2
    N = A.shape[0]
    assert st["dense_entries"] <= N * N
    assert st["n_near_pairs"] > 0


def test_matvec_after_recompression_at_other_tolerances():
    """The matvec's per-block scratch layout depends on the ranks: after a
    new compress (ranks larger, then smaller) the product must still equal
    the compressed matrix applied densely."""
    import torch
    spec = W.tiny_sphere(s=4, q=4, k0=6.0)
    s, _ = _filled(spec, leaf=64, tol=1e-4)
    x = torch.from_numpy(W.random_complex((s.n, 2), seed=4)).cuda()
    s.matvec(x)
    for tol in (1e-9, 1e-3, 1e-7):
        s.compress(tol)
        y = s.matvec(x)
        yd = s.export_dense() @ x
        err = (torch.linalg.norm(y - yd) / torch.linalg.norm(yd)).item()
        print(f"tol {tol:g}: max rank {s.stats()['max_rank']}, matvec vs dense {err:.1e}")
        assert err < 1e-13


@pytest.mark.parametrize("form", ["mfie", "nmuller"])
def test_aca_in_rounds_of_a_small_workspace_budget(form, monkeypatch):
    """The ACA workspace is used in rounds that fit a budget (elements, here
    small enough for a few blocks per round): ranks, factors and the
    recorded workspace must equal those of a single round, also for the
    full-width redo of blocks whose predicted width was too small (a
    network with zero weights predicts log-rank 0, width 8)."""
    import torch
    from paper_2408_17116_amd import cbie
    if form == "mfie":
        spec, leaf = W.tiny_sphere(s=4, q=4, k0=6.0), 64
    else:
        spec = W.ObjectSpec(axes=(1.2, 0.8, 0.6), center=(0.0, 0.0, 0.0), s=3, q=4, k0=3.0,
                            form=W.FORM_NMULLER, eps_r=4.0, mu_r=1.0)
        leaf = 64
    s, _ = _filled(spec, leaf=leaf)
    s.set_rank_model(np.zeros(cbie.MLP_NPARAMS, np.float32), np.zeros(cbie.MLP_NFEAT, np.float32),
                     np.ones(cbie.MLP_NFEAT, np.float32), margin=0.0)
    out = {}
    for budget in (None, 20000):
        if budget is not None:
            monkeypatch.setenv("CBIE_ACA_BUDGET", str(budget))
        for mode in (cbie.RANK_ADAPTIVE, cbie.RANK_PREDICTED):
            s.compress(1e-6, mode=mode)
            _, r = s.block_features(1e-6)
            st = s.stats()
            out[budget, mode] = (s.export_dense(), r, st["aca_workspace_bytes"], st["aca_fallbacks"])
    ref = out[None, cbie.RANK_ADAPTIVE]
    assert ref[3] == 0 and ref[1].max() > 8
    print(f"{form}: {ref[1].size} blocks, max rank {ref[1].max()}, "
          f"fallbacks at width 8 {out[None, cbie.RANK_PREDICTED][3]}")
    for key, (A, r, ws, fb) in out.items():
        assert torch.equal(A, ref[0]), key
        assert np.array_equal(r, ref[1]), key
    for mode in (cbie.RANK_ADAPTIVE, cbie.RANK_PREDICTED):
        assert out[20000, mode][2:] == out[None, mode][2:]
    assert out[None, cbie.RANK_PREDICTED][3] > 0
    s.close()
