"""Host tables the kernels read (Sec. II-B), compiled here with the host
compiler from the library's source: every Fejer-1 rule the quadrature uses
(n = 1..96) integrates polynomials of degree below n exactly, has positive
weights summing to 2 and ascending first-kind Chebyshev nodes; every
differentiation matrix (q = 1..8) differentiates polynomials of degree below
q exactly at the nodes; and both agree with the oracle's independent
construction."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from oracle import cheb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_17116_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("rules") / "librulesshim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "rules_shim.cpp"), os.path.join(CSRC, "rules.cpp"), "-o", out],
                   check=True)
    L = C.CDLL(out)
    dp = C.POINTER(C.c_double)
    L.fejer_rule_c.argtypes = [C.c_int, dp, dp]
    L.cheb_diff_matrices_c.argtypes = [C.c_int, dp, C.c_int]
    L.cheb_diff_matrices_c.restype = C.c_int
    return L


def _fejer(lib, n):
    x, w = np.zeros(n), np.zeros(n)
    lib.fejer_rule_c(n, x.ctypes.data_as(C.POINTER(C.c_double)), w.ctypes.data_as(C.POINTER(C.c_double)))
    return x, w


def test_fejer_rules_are_exact_to_degree_n_minus_one(lib):
    for n in list(range(1, 25)) + [32, 40, 64, 96]:
        x, w = _fejer(lib, n)
        assert np.all(np.diff(x) > 0) and np.all(w > 0)
        assert np.allclose(x, -np.cos((2 * np.arange(n) + 1) * np.pi / (2 * n)), rtol=0, atol=1e-15)
        # Legendre moments: exact for degree < n (Legendre, not monomials, to stay well conditioned)
        for k in range(n):
            Pk = np.polynomial.legendre.Legendre.basis(k)(x)
            assert abs(np.dot(w, Pk) - (2.0 if k == 0 else 0.0)) < 4e-14 * max(1, n / 8), (n, k)
        xo, wo = cheb.fejer1(n)
        assert np.abs(xo - x).max() < 1e-15 and np.abs(wo - w).max() < 1e-14


def test_differentiation_matrices_are_exact_on_polynomials(lib):
    cap = sum(q * q for q in range(1, 9))
    out = np.zeros(cap)
    n = lib.cheb_diff_matrices_c(8, out.ctypes.data_as(C.POINTER(C.c_double)), cap)
    assert n == cap
    off = 0
    for q in range(1, 9):
        assert off == (q - 1) * q * (2 * q - 1) // 6
        D = out[off:off + q * q].reshape(q, q)
        off += q * q
        x, _ = _fejer(lib, q)
        for k in range(q):
            p = np.polynomial.chebyshev.Chebyshev.basis(k)
            assert np.abs(D @ p(x) - p.deriv()(x)).max() < 1e-12 * max(1, k * k), (q, k)
        Do = cheb.diff_matrix(q)
        assert np.abs(D - Do).max() < 1e-12 * max(1.0, np.abs(Do).max())
