"""ACA oracle against dense SVD on admissible blocks of the MFIE matrix."""
import numpy as np
import pytest

from oracle import aca, geometry as G, mfie
from synth import workloads as W


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
def test_aca_on_far_block(eps):
    nd = G.build_nodes(W.sphere_pec_ka20())
    k = 20.0
    # source: patches 0..3 of face +x; target: patches of face -x (far away)
    q2 = 64
    src = np.arange(0, 4 * q2)
    tgt = np.arange(64 * q2, 68 * q2)
    blk = mfie.far_block(nd, k, tgt, src).reshape(2 * tgt.size, 2 * src.size)
    m, n = blk.shape
    U, V = aca.aca(lambda i: blk[i], lambda j: blk[:, j], m, n, eps)
    err = np.linalg.norm(blk - U @ V.T) / np.linalg.norm(blk)
    assert err < 10 * eps
    r_svd = aca.svd_rank(blk, eps)
    assert r_svd <= U.shape[1] <= 2 * r_svd + 4


def test_aca_exact_low_rank_and_zero_rows():
    rng = np.random.default_rng(1)
    A = (rng.standard_normal((40, 3)) + 1j * rng.standard_normal((40, 3))) @ \
        (rng.standard_normal((3, 30)) + 0j)
    A[0] = 0.0                                    # a zero first row must be skipped
    U, V = aca.aca(lambda i: A[i], lambda j: A[:, j], 40, 30, 1e-12)
    assert U.shape[1] == 3 or np.linalg.norm(A - U @ V.T) < 1e-10 * np.linalg.norm(A)
    assert np.linalg.norm(A - U @ V.T) < 1e-12 * np.linalg.norm(A)
