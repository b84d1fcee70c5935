"""Host logic of the GMRES refinement (the factorization as the right
preconditioner of an FP64 Krylov iteration), compiled here with the host
compiler over dense host vectors.  Checked against what fixes it: with the
exact inverse as preconditioner one Krylov step solves the system; without a
preconditioner, on a well-conditioned nonsymmetric complex matrix, the
iterates converge to LAPACK's solution; and on a nearly singular operator
whose approximate inverse is perturbed at 1e-4 (stationary refinement
x += M (b - A x) diverges there: the spectral radius of I - M A exceeds 1)
GMRES reaches 1e-10 in a few steps, also across restarts (its FP64 floor
there, about the unit roundoff times ||A|| ||x|| / ||b|| ~ 1e-16 / 1e-6,
lies below)."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_17116_amd", "csrc")
SHIM = os.path.join(ROOT, "tests", "host", "gmres_shim.cpp")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("gmres") / "libgmresshim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, SHIM, "-o", out], check=True)
    L = C.CDLL(out)
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
    L.gmres_dense.argtypes = [C.c_int, dp, dp, dp, dp, C.c_double, C.c_int, C.c_int, ip, dp]
    return L


def _run(lib, A, M, b, tol, restart, max_iter, x0=None):
    n = A.shape[0]
    a = np.asfortranarray(A, dtype=np.complex128)
    m = np.asfortranarray(M, dtype=np.complex128)
    bb = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.zeros(n, np.complex128) if x0 is None else np.ascontiguousarray(x0, dtype=np.complex128)
    info = np.zeros(4, np.int32)
    rr = C.c_double()
    dp = lambda v: v.ctypes.data_as(C.POINTER(C.c_double))
    ok = lib.gmres_dense(n, dp(a), dp(m), dp(bb), dp(x), tol, restart, max_iter,
                         info.ctypes.data_as(C.POINTER(C.c_int)), C.byref(rr))
    return bool(ok), x, info, rr.value


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))


def test_exact_inverse_solves_in_one_step(lib):
    n = 40
    A = _rand(n, 1) + 10 * np.eye(n)
    b = _rand(n, 2)[:, 0]
    ok, x, info, rr = _run(lib, A, np.linalg.inv(A), b, 1e-12, 20, 50)
    assert ok and info[0] == 1 and rr < 1e-12
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-11 * np.linalg.norm(x)


def test_unpreconditioned_converges_to_lapack(lib):
    n = 60
    A = _rand(n, 3) / np.sqrt(n) + 3 * np.eye(n)    # eigenvalues in a disc around 3, radius ~1
    b = _rand(n, 4)[:, 0]
    ok, x, info, rr = _run(lib, A, np.eye(n), b, 1e-13, 60, 200)
    assert ok and rr < 1e-13
    # the least-squares residual the rotations track is the true one: the
    # first cycle stops at the tolerance, no restart (33 steps measured)
    assert info[1] == 1 and info[0] <= 40
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) < 1e-11 * np.linalg.norm(xs)
    # the residual GMRES tracked equals the one recomputed from x
    assert abs(rr - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) < 1e-14


@pytest.mark.parametrize("restart", [30, 4])
def test_nearly_singular_operator_where_stationary_refinement_diverges(lib, restart):
    n = 80
    rng = np.random.default_rng(5)
    U, _ = np.linalg.qr(_rand(n, 6))
    V, _ = np.linalg.qr(_rand(n, 7))
    sig = np.ones(n)
    sig[-3:] = [1e-5, 3e-6, 1e-6]                  # three near-resonant directions
    A = (U * sig) @ V.conj().T
    E = 1e-4 * _rand(n, 8) / np.sqrt(n)            # the factorization's truncation
    M = np.linalg.inv(A + E)
    b = _rand(n, 9)[:, 0]
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(n) - M @ A)))
    assert rho > 1                                  # plain refinement cannot converge
    x = M @ b
    for _ in range(30):
        x = x + M @ (b - A @ x)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) > 1e-6
    ok, xg, info, rr = _run(lib, A, M, b, 1e-10, restart, 200)
    print(f"restart {restart}: spectral radius of I - M A {rho:.1f}; GMRES {info[0]} steps, {info[1]} cycles, "
          f"residual {rr:.1e}")
    assert ok and rr < 1e-10
    assert np.linalg.norm(b - A @ xg) / np.linalg.norm(b) < 1e-10
    assert info[0] <= (12 if restart == 30 else 60)
