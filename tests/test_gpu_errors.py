"""Error paths of the C-ABI, forced from the host (every kernel exits
normally): calls out of order return ESTATE; a stage that fails after its
argument checks leaves the context in the preceding state, so a later call
that needs the stage is refused instead of reading stale tables; refinement
that cannot reach its tolerance returns ENOCONV with the sweep count; a
rank model that under-predicts every width falls back to the full width and
still meets the tolerance against the uncompressed fill."""
import numpy as np
import pytest

from synth import workloads as W

pytestmark = pytest.mark.gpu


def _spec():
    return W.tiny_sphere(s=3, q=4, k0=5.0)     # 54 patches, 1728 unknowns


def _status(fn, *args):
    from paper_2408_17116_amd import cbie
    try:
        fn(*args)
    except cbie.CbieError as e:
        return e.code
    return cbie.OK


def test_calls_out_of_order_return_estate():
    import torch
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([_spec()])
    x = torch.zeros((s.n, 1), dtype=torch.complex128, device="cuda")
    assert _status(s.fill) == cbie.ESTATE
    assert _status(s.compress, 1e-6) == cbie.ESTATE
    assert _status(s.factor, cbie.PREC_C64_IR) == cbie.ESTATE
    assert _status(s.matvec, x) == cbie.ESTATE
    assert _status(s.solve, x) == cbie.ESTATE
    s.build_tree(leaf_size=64, eta=1.0, near_delta=1.0)
    assert _status(s.compress, 1e-6) == cbie.ESTATE
    s.fill()
    assert _status(s.factor, cbie.PREC_C128) == cbie.ESTATE
    assert _status(s.matvec, x) == cbie.ESTATE
    s.compress(1e-6)
    assert _status(s.solve, x) == cbie.ESTATE
    s.close()


def test_failed_compress_downgrades_state():
    import torch
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([_spec()])
    s.build_tree(leaf_size=64, eta=1.0, near_delta=1.0)
    s.fill()
    s.compress(1e-6)
    s.factor(cbie.PREC_C64_IR)
    x = torch.from_numpy(W.random_complex((s.n, 2), seed=3)).cuda()
    y0 = s.matvec(x).cpu().numpy()
    # the rank-model check runs inside the stage, after the state was lowered
    assert _status(s.compress, 1e-6, cbie.RANK_PREDICTED) == cbie.EINVAL
    assert "rank model" in s.lib.cbie_last_error(s.h).decode()
    assert _status(s.matvec, x) == cbie.ESTATE
    assert _status(s.solve, x) == cbie.ESTATE
    assert _status(s.factor, cbie.PREC_C64_IR) == cbie.ESTATE
    s.compress(1e-6)
    y1 = s.matvec(x).cpu().numpy()
    assert np.abs(y1 - y0).max() <= 1e-12 * np.abs(y0).max()
    s.close()


def test_refinement_enoconv_and_sweep_count():
    import torch
    from paper_2408_17116_amd import cbie
    s = cbie.Solver([_spec()])
    s.build_tree(leaf_size=64, eta=1.0, near_delta=1.0)
    s.fill()
    s.compress(1e-6)
    s.factor(cbie.PREC_C64_IR)
    kh, pol = W.plane_waves(2, seed=1)
    b = s.rhs_planewave(kh, pol)
    # an unreachable tolerance: one sweep, then ENOCONV with the last iterate
    assert _status(s.solve, b, 1e-300, 1) == cbie.ENOCONV
    x, it = s.solve(b, tol=1e-300, maxit=1, raise_on_noconv=False)
    assert it == 1 and s.stats()["ir_iterations"] == 1
    assert torch.isfinite(torch.view_as_real(x)).all()
    # the same call with a reachable tolerance converges within the limit
    x2, it2 = s.solve(b, tol=1e-10, maxit=30)
    res = (torch.linalg.norm(s.matvec(x2) - b) / torch.linalg.norm(b)).item()
    assert res <= 1e-10 * np.sqrt(2) and it2 <= 30
    s.close()


def test_predicted_width_fallback_meets_tolerance():
    import torch
    from paper_2408_17116_amd import cbie
    tol = 1e-6
    s = cbie.Solver([_spec()])
    s.build_tree(leaf_size=64, eta=1.0, near_delta=1.0)
    s.fill()
    A_exact = s.export_dense().cpu().numpy()       # admissible blocks by the plain rule
    s.compress(tol)
    st_a = s.stats()
    assert st_a["aca_unconverged"] == 0 and st_a["n_lr_blocks"] > 0
    _, ranks_a = s.block_features(tol)
    # a network that predicts log-rank 0 everywhere: widths of 8 columns
    s.set_rank_model(np.zeros(cbie.MLP_NPARAMS, np.float32), np.zeros(8, np.float32), np.ones(8, np.float32), 0.25)
    s.compress(tol, mode=cbie.RANK_PREDICTED)
    st_p = s.stats()
    _, ranks_p = s.block_features(tol)
    assert st_p["aca_fallbacks"] > 0 and st_p["aca_fallbacks"] == int((ranks_a > 8).sum())
    assert np.array_equal(ranks_a, ranks_p)
    A_p = s.export_dense().cpu().numpy()
    err = np.linalg.norm(A_p - A_exact) / np.linalg.norm(A_exact)
    print(f"fallbacks {st_p['aca_fallbacks']} of {st_p['n_lr_blocks']}, |A_H - A| / |A| = {err:.2e}")
    assert err <= 10 * tol
    torch.cuda.synchronize()
    s.close()


def test_complex64_recompression_keeps_the_tolerance():
    """Recompression of formatted sums in a complex64 factorization builds
    its range basis in FP64 (an FP32 Gram matrix would drop every direction
    below ~3e-4 of the largest).  Forced to recompress after every 64
    appended columns (CBIE_KMAX), the complex64 factorization's plain
    substitution must leave a residual against the stored FP64 operator
    within a small factor of the complex128 one's: both are truncated at the
    same tolerance, and complex64 rounding adds ~1e-7 relative per entry."""
    import os
    import torch
    from paper_2408_17116_amd import cbie
    spec = W.tiny_sphere(s=4, q=4, k0=6.0)      # 3072 unknowns
    old = os.environ.get("CBIE_KMAX")
    os.environ["CBIE_KMAX"] = "64"
    try:
        s = cbie.Solver([spec])
        s.build_tree(leaf_size=64, eta=1.0, near_delta=1.0)
        s.fill()
        s.compress(1e-8)
        kh, pol = W.plane_waves(2, seed=8)
        b = s.rhs_planewave(kh, pol)
        res = {}
        for prec in (cbie.PREC_C128, cbie.PREC_C64_IR):
            s.factor(prec)
            x0, _ = s.solve(b, tol=1e-10, maxit=0)
            res[prec] = (torch.linalg.norm(s.matvec(x0) - b) / torch.linalg.norm(b)).item()
            x, it = s.solve(b, tol=1e-10, maxit=30)
            print(f"prec {prec}: substitution residual {res[prec]:.2e}, {it} sweeps to 1e-10")
        s.close()
    finally:
        if old is None:
            del os.environ["CBIE_KMAX"]
        else:
            os.environ["CBIE_KMAX"] = old
    assert res[cbie.PREC_C128] < 1e-6
    assert res[cbie.PREC_C64_IR] < 1e-4
