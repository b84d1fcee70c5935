"""Host control flow of the FP64 iterative refinement around the complex64
factorization (x = M b, then r = b - A x, x += M r), compiled here with the
host compiler over dense host vectors.  Pinned by cases whose iterates are
known in closed form: with A = I and M = (1 - e) I the k-th iterate is
(1 - e^(k+1)) b, so the residual ratio after k corrections is |e|^(k+1)
exactly; the tolerance is met by the last permitted correction, which must
be seen; a divergent factor (|e| > 1) never converges; a NaN in the
factorization is a failure, not convergence; maxit = 0 is the plain
substitution with no residual formed."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_17116_amd", "csrc")
SHIM = os.path.join(ROOT, "tests", "host", "refine_shim.cpp")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("refine") / "librefineshim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, SHIM, "-o", out], check=True)
    L = C.CDLL(out)
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
    L.refine_dense.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, C.c_double, C.c_int, ip, dp]
    return L


def _run(lib, A, M, B, tol, maxit):
    n, nrhs = B.shape
    a = np.asfortranarray(A, dtype=np.complex128)
    m = np.asfortranarray(M, dtype=np.complex128)
    b = np.asfortranarray(B, dtype=np.complex128)
    x = np.zeros((n, nrhs), np.complex128, order="F")
    info = np.zeros(4, np.int32)
    worst = C.c_double()
    dp = C.POINTER(C.c_double)
    lib.refine_dense(n, nrhs, a.ctypes.data_as(dp), m.ctypes.data_as(dp), b.ctypes.data_as(dp),
                     x.ctypes.data_as(dp), tol, maxit, info.ctypes.data_as(C.POINTER(C.c_int)), C.byref(worst))
    return x, dict(corrections=int(info[0]), residuals=int(info[1]), converged=bool(info[2]),
                   nonfinite=bool(info[3]), worst=worst.value)


def _rhs(n, nrhs, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs))


def test_contraction_closed_form(lib):
    n, e = 6, 0.1
    B = _rhs(n, 3)
    # ratios 0.1, 0.01, 0.001, 1e-4: tolerance 2e-4 is met after 3 corrections
    x, r = _run(lib, np.eye(n), (1 - e) * np.eye(n), B, 2e-4, 10)
    assert r["converged"] and r["corrections"] == 3 and r["residuals"] == 4
    assert abs(r["worst"] - e ** 4) < 1e-12
    np.testing.assert_allclose(x, (1 - e ** 4) * B, rtol=1e-13)


def test_last_permitted_correction_is_checked(lib):
    n, e = 5, 0.1
    B = _rhs(n, 2, seed=1)
    # the third correction reaches 1e-4 <= 2e-4: with maxit = 3 this converges
    _, r = _run(lib, np.eye(n), (1 - e) * np.eye(n), B, 2e-4, 3)
    assert r["converged"] and r["corrections"] == 3 and r["residuals"] == 4
    # with maxit = 2 it does not (ratio 1e-3 after two corrections)
    _, r = _run(lib, np.eye(n), (1 - e) * np.eye(n), B, 2e-4, 2)
    assert not r["converged"] and not r["nonfinite"] and r["corrections"] == 2
    assert abs(r["worst"] - e ** 3) < 1e-12


def test_divergent_factor_never_converges(lib):
    n = 4
    B = _rhs(n, 1, seed=2)
    _, r = _run(lib, np.eye(n), 2.5 * np.eye(n), B, 1e-8, 6)    # e = -1.5
    assert not r["converged"] and r["corrections"] == 6
    assert abs(r["worst"] - 1.5 ** 7) / 1.5 ** 7 < 1e-12


def test_nan_factor_is_failure(lib):
    n = 4
    B = _rhs(n, 2, seed=3)
    M = np.eye(n, dtype=complex)
    M[1, 2] = np.nan
    _, r = _run(lib, np.eye(n), M, B, 1e-8, 5)
    assert r["nonfinite"] and not r["converged"] and r["corrections"] == 0
    assert r["worst"] == np.inf


def test_maxit_zero_is_plain_substitution(lib):
    n = 4
    B = _rhs(n, 2, seed=4)
    x, r = _run(lib, np.eye(n), 0.5 * np.eye(n), B, 1e-12, 0)
    assert r["converged"] and r["residuals"] == 0 and r["corrections"] == 0
    np.testing.assert_allclose(x, 0.5 * B, rtol=1e-15)


def test_general_matrix_against_lapack(lib):
    rng = np.random.default_rng(5)
    n = 12
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 6 * np.eye(n)
    Minv = np.linalg.inv(A)
    M = Minv + 1e-3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / n
    B = _rhs(n, 4, seed=6)
    x, r = _run(lib, A, M, B, 1e-13, 40)
    assert r["converged"]
    np.testing.assert_allclose(x, np.linalg.solve(A, B), rtol=1e-11, atol=1e-12)
