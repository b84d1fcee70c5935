"""Thin ctypes binding of libcbie.so (argument marshalling only).

Every step of the solver runs in the library's HIP kernels; PyTorch only
provides device memory and the stream.  Device vectors are complex128
tensors; a block of nrhs vectors of length n is held as a contiguous
(nrhs, n) tensor, i.e. column-major (n, nrhs) with leading dimension n, in
the original unknown order (object, patch, node (k, l), component u/v).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbie.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, ENOCONV, ESINGULAR, EINTERNAL = 0, -1, -2, -3, -4, -5, -6, -7
MFIE_PEC, NMULLER = 0, 1
PREC_C128, PREC_C64_IR = 0, 1
RANK_ADAPTIVE, RANK_PREDICTED = 0, 1
ORDER_ENTIRE, ORDER_COMPONENT = 0, 1

EXPORTED = ["cbie_create", "cbie_build_tree", "cbie_fill", "cbie_compress", "cbie_factor",
            "cbie_solve", "cbie_matvec", "cbie_rhs_planewave", "cbie_farfield", "cbie_get_stats",
            "cbie_set_profiling", "cbie_get_near_pairs", "cbie_export_dense", "cbie_last_error",
            "cbie_destroy", "cbie_get_block_features", "cbie_set_rank_model", "cbie_mlp_forward",
            "cbie_mlp_grad", "cbie_mlp_train", "cbie_matvec_noalloc", "cbie_solve_gmres",
            "cbie_set_factor_tolerance", "cbie_set_factor_ordering", "cbie_rhs_dipole"]

MLP_NFEAT, MLP_NPARAMS = 8, 4801


class CbieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cbie error {code}: {msg}")
        self.code = code


class _Patch(C.Structure):
    _fields_ = [("face", C.c_int), ("i", C.c_int), ("j", C.c_int), ("split", C.c_int)]


class _Object(C.Structure):
    _fields_ = [("form", C.c_int), ("k0", C.c_double), ("axes", C.c_double * 3),
                ("center", C.c_double * 3), ("q", C.c_int), ("n_patches", C.c_int),
                ("patches", C.POINTER(_Patch)), ("eps_r", C.c_double), ("mu_r", C.c_double),
                ("patch_degree", C.c_int), ("patch_coeffs", C.POINTER(C.c_double))]


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_unknowns", "n_nodes", "n_patches", "n_objects", "n_clusters", "n_leaves",
        "n_dense_blocks", "n_lr_blocks", "n_near_pairs", "dense_entries", "lr_entries",
        "max_rank", "sum_rank")] + [
        ("compression_rate", C.c_double), ("t_tree", C.c_double), ("t_fill", C.c_double),
        ("t_compress", C.c_double), ("t_factor", C.c_double), ("t_solve", C.c_double),
        ("factor_flops", C.c_int64), ("n_kernel_launches", C.c_int64),
        ("ir_iterations", C.c_int64), ("quad_seconds", C.c_double),
        ("gemm_launches", C.c_int64), ("gemm_flops", C.c_double), ("gemm_seconds", C.c_double),
        ("aca_fallbacks", C.c_int64), ("aca_workspace_bytes", C.c_double), ("solve_replays", C.c_int64),
        ("aca_unconverged", C.c_int64), ("gemm_flops_alg", C.c_double), ("factor_flops_executed", C.c_int64),
        ("leaf_lu_launches", C.c_int64), ("leaf_lu_flops", C.c_double), ("leaf_lu_seconds", C.c_double),
        ("quad_points", C.c_double), ("quad_flops", C.c_double),
        ("solve_factor_bytes", C.c_double), ("far_fill_seconds", C.c_double), ("gemm_bytes_alg", C.c_double),
        ("gemm_flops_mfma", C.c_double), ("factor_mem_flushes", C.c_int64),
        ("t_factor_reorder", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libcbie.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "cbie_create": ([C.POINTER(_Object), i32, vp, C.POINTER(vp)], i32),
        "cbie_build_tree": ([vp, i32, dbl, dbl], i32),
        "cbie_fill": ([vp, i32, i32], i32),
        "cbie_compress": ([vp, dbl, i32], i32),
        "cbie_factor": ([vp, i32], i32),
        "cbie_solve": ([vp, i32, vp, vp, C.c_long, dbl, i32, C.POINTER(i32)], i32),
        "cbie_matvec": ([vp, i32, vp, vp, C.c_long], i32),
        "cbie_matvec_noalloc": ([vp, i32, vp, vp, C.c_long], i32),
        "cbie_solve_gmres": ([vp, i32, vp, vp, C.c_long, dbl, i32, i32, C.POINTER(i32)], i32),
        "cbie_set_factor_tolerance": ([vp, dbl], i32),
        "cbie_set_factor_ordering": ([vp, i32], i32),
        "cbie_rhs_planewave": ([vp, i32, vp, vp, vp, C.c_long], i32),
        "cbie_rhs_dipole": ([vp, i32, vp, vp, vp, C.c_long], i32),
        "cbie_farfield": ([vp, i32, vp, C.c_long, i32, vp, vp], i32),
        "cbie_get_stats": ([vp, vp, C.c_size_t], i32),
        "cbie_set_profiling": ([vp, i32], i32),
        "cbie_get_near_pairs": ([vp, i64, vp, vp, C.POINTER(i64)], i32),
        "cbie_export_dense": ([vp, vp, C.c_long], i32),
        "cbie_last_error": ([vp], C.c_char_p),
        "cbie_destroy": ([vp], None),
        "cbie_get_block_features": ([vp, dbl, i64, vp, vp, C.POINTER(i64)], i32),
        "cbie_set_rank_model": ([vp, vp, vp, vp, C.c_float], i32),
        "cbie_mlp_forward": ([vp, vp, vp, vp, vp, i64, vp], i32),
        "cbie_mlp_grad": ([vp, vp, vp, vp, vp, vp, i64, vp, vp], i32),
        "cbie_mlp_train": ([vp, vp, vp, vp, vp, vp, vp, i64, i32, C.c_float, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Solver:
    """One context: a set of independent objects (block-diagonal system)."""

    def __init__(self, objects, stream=None):
        import torch
        self.torch = torch
        self.lib = load()
        if not isinstance(objects, (list, tuple)):
            objects = [objects]
        self.objects = list(objects)
        objs = (_Object * len(objects))()
        self._keep = []
        for o, spec in enumerate(objects):
            objs[o].form = spec.form
            objs[o].k0 = spec.k0
            objs[o].axes = (C.c_double * 3)(*spec.axes)
            objs[o].center = (C.c_double * 3)(*spec.center)
            objs[o].q = spec.q
            coeffs = getattr(spec, "coeffs", None)
            if coeffs is not None:
                # Chebyshev-interpolated patches: (n_patches, 3, d + 1, d + 1)
                cf = np.ascontiguousarray(coeffs, dtype=np.float64)
                if cf.ndim != 4 or cf.shape[1] != 3 or cf.shape[2] != cf.shape[3]:
                    raise ValueError("coeffs must be (n_patches, 3, d + 1, d + 1)")
                self._keep.append(cf)
                objs[o].n_patches = cf.shape[0]
                objs[o].patch_degree = cf.shape[2] - 1
                objs[o].patch_coeffs = cf.ctypes.data_as(C.POINTER(C.c_double))
            else:
                pts = spec.patches()
                arr = (_Patch * len(pts))(*[_Patch(f, i, j, s) for (f, i, j, s) in pts])
                self._keep.append(arr)
                objs[o].n_patches = len(pts)
                objs[o].patches = arr
            eps, mu = complex(getattr(spec, "eps_r", 1.0)), complex(getattr(spec, "mu_r", 1.0))
            if eps.imag != 0 or mu.imag != 0:
                raise ValueError("lossless interior materials only (real eps_r, mu_r)")
            objs[o].eps_r = eps.real
            objs[o].mu_r = mu.real
        self.n = sum(s.n_unknowns for s in objects)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.cbie_create(objs, len(objects), C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != OK:
            raise CbieError(st, "cbie_create failed")
        self.h = h

    def _check(self, st):
        if st != OK:
            raise CbieError(st, self.lib.cbie_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.cbie_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ stages
    def build_tree(self, leaf_size=256, eta=1.0, near_delta=1.0):
        self._check(self.lib.cbie_build_tree(self.h, leaf_size, eta, near_delta))

    def fill(self, n_ang=0, n_rad=0):
        self._check(self.lib.cbie_fill(self.h, n_ang, n_rad))

    def compress(self, tol=1e-6, mode=RANK_ADAPTIVE):
        self._check(self.lib.cbie_compress(self.h, tol, mode))

    def factor(self, prec=PREC_C128):
        self._check(self.lib.cbie_factor(self.h, prec))

    def set_factor_tolerance(self, tol):
        """Truncation tolerance of later factorizations (0: the compress tolerance)."""
        self._check(self.lib.cbie_set_factor_tolerance(self.h, tol))

    def set_factor_ordering(self, ordering):
        """ORDER_ENTIRE (default) or ORDER_COMPONENT for later factorizations."""
        self._check(self.lib.cbie_set_factor_ordering(self.h, ordering))

    def _cols(self, v):
        """(n,) or (n, m) complex128 cuda tensor -> contiguous (m, n) tensor."""
        t = self.torch
        v = t.as_tensor(v)
        if v.dim() == 1:
            v = v[:, None]
        return v.to(device="cuda", dtype=t.complex128).t().contiguous()

    def solve(self, b, tol=1e-10, maxit=0, raise_on_noconv=True):
        bc = self._cols(b)
        x = self.torch.empty_like(bc)
        it = C.c_int(0)
        st = self.lib.cbie_solve(self.h, bc.shape[0], _ptr(bc), _ptr(x), self.n, tol, maxit, C.byref(it))
        if st == ENOCONV and not raise_on_noconv:
            return x.t(), it.value
        self._check(st)
        return x.t(), it.value

    def solve_gmres(self, b, tol=1e-10, restart=30, maxit=200, raise_on_noconv=True):
        """GMRES-based refinement (the factorization as right preconditioner
        of FP64 GMRES); returns (x, Krylov steps over all columns)."""
        bc = self._cols(b)
        x = self.torch.empty_like(bc)
        it = C.c_int(0)
        st = self.lib.cbie_solve_gmres(self.h, bc.shape[0], _ptr(bc), _ptr(x), self.n, tol, restart, maxit,
                                       C.byref(it))
        if st == ENOCONV and not raise_on_noconv:
            return x.t(), it.value
        self._check(st)
        return x.t(), it.value

    def matvec(self, x):
        xc = self._cols(x)
        y = self.torch.empty_like(xc)
        self._check(self.lib.cbie_matvec(self.h, xc.shape[0], _ptr(xc), _ptr(y), self.n))
        return y.t()

    def matvec_noalloc(self, x, y=None):
        """y = A_H x through the allocation-free entry point; y (same shape
        as the (m, n) column block of x) may be passed in."""
        xc = self._cols(x)
        if y is None:
            y = self.torch.empty_like(xc)
        self._check(self.lib.cbie_matvec_noalloc(self.h, xc.shape[0], _ptr(xc), _ptr(y), self.n))
        return y.t()

    def rhs_planewave(self, khat, pol):
        khat = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
        pol = np.ascontiguousarray(np.atleast_2d(pol), dtype=np.float64)
        nw = khat.shape[0]
        b = self.torch.empty((nw, self.n), dtype=self.torch.complex128, device="cuda")
        self._check(self.lib.cbie_rhs_planewave(self.h, nw, khat.ctypes.data_as(C.c_void_p),
                                                pol.ctypes.data_as(C.c_void_p), _ptr(b), self.n))
        return b.t()

    def rhs_dipole(self, pos, moment):
        """Right-hand sides of point electric dipoles (positions, current
        moments: (n, 3) each), one column per dipole."""
        pos = np.ascontiguousarray(np.atleast_2d(pos), dtype=np.float64)
        moment = np.ascontiguousarray(np.atleast_2d(moment), dtype=np.float64)
        if pos.shape != moment.shape or pos.shape[1] != 3:
            raise ValueError("pos and moment must both be (n, 3)")
        nd = pos.shape[0]
        b = self.torch.empty((nd, self.n), dtype=self.torch.complex128, device="cuda")
        self._check(self.lib.cbie_rhs_dipole(self.h, nd, pos.ctypes.data_as(C.c_void_p),
                                             moment.ctypes.data_as(C.c_void_p), _ptr(b), self.n))
        return b.t()

    def farfield(self, x, rhat):
        xc = self._cols(x)
        rhat = np.ascontiguousarray(np.atleast_2d(rhat), dtype=np.float64)
        out = np.empty((xc.shape[0], rhat.shape[0], 3), dtype=np.complex128)
        self._check(self.lib.cbie_farfield(self.h, xc.shape[0], _ptr(xc), self.n, rhat.shape[0],
                                           rhat.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p)))
        return out

    def set_profiling(self, on=True):
        """Time every batched GEMM launch with HIP events (gemm_seconds)."""
        self._check(self.lib.cbie_set_profiling(self.h, 1 if on else 0))

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.cbie_get_stats(self.h, C.byref(s), C.sizeof(s)))
        return {name: getattr(s, name) for name, _ in Stats._fields_}

    def near_pairs(self):
        cnt = C.c_int64(0)
        self._check(self.lib.cbie_get_near_pairs(self.h, 0, None, None, C.byref(cnt)))
        t = np.empty(cnt.value, dtype=np.int32)
        p = np.empty(cnt.value, dtype=np.int32)
        self._check(self.lib.cbie_get_near_pairs(self.h, cnt.value, t.ctypes.data_as(C.c_void_p),
                                                 p.ctypes.data_as(C.c_void_p), C.byref(cnt)))
        return t, p

    def block_features(self, aca_tol):
        """(features (count, 8) float32, ranks (count,) int32; -1 before
        compress) of the admissible blocks, in low-rank block order."""
        cnt = C.c_int64(0)
        self._check(self.lib.cbie_get_block_features(self.h, aca_tol, 0, None, None, C.byref(cnt)))
        f = np.empty((cnt.value, MLP_NFEAT), dtype=np.float32)
        r = np.empty(cnt.value, dtype=np.int32)
        self._check(self.lib.cbie_get_block_features(self.h, aca_tol, cnt.value, f.ctypes.data_as(C.c_void_p),
                                                     r.ctypes.data_as(C.c_void_p), C.byref(cnt)))
        return f, r

    def set_rank_model(self, params, mean, sdev, margin=0.25):
        """Model for compress(mode=RANK_PREDICTED) (host arrays, copied)."""
        p = np.ascontiguousarray(params, dtype=np.float32)
        m = np.ascontiguousarray(mean, dtype=np.float32)
        d = np.ascontiguousarray(sdev, dtype=np.float32)
        if p.size != MLP_NPARAMS or m.size != MLP_NFEAT or d.size != MLP_NFEAT:
            raise ValueError("rank model sizes")
        self._check(self.lib.cbie_set_rank_model(self.h, p.ctypes.data_as(C.c_void_p), m.ctypes.data_as(C.c_void_p),
                                                 d.ctypes.data_as(C.c_void_p), float(margin)))

    def export_dense(self):
        A = self.torch.empty((self.n, self.n), dtype=self.torch.complex128, device="cuda")
        self._check(self.lib.cbie_export_dense(self.h, _ptr(A), self.n))
        return A.t()   # the library writes column-major


# ------------------------------------------------------------------ network
def _f32(t, n=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError("expected a contiguous float32 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return _ptr(t)


def _mlp_check(st, what):
    if st != OK:
        raise CbieError(st, what)


def mlp_forward(params, mean, sdev, X):
    """y[i] = network((X[i] - mean) / sdev); X (n, 8) raw features."""
    import torch
    n = X.shape[0]
    y = torch.empty(n, dtype=torch.float32, device=X.device)
    _mlp_check(load().cbie_mlp_forward(C.c_void_p(torch.cuda.current_stream().cuda_stream), _f32(params, MLP_NPARAMS),
                                       _f32(mean, MLP_NFEAT), _f32(sdev, MLP_NFEAT), _f32(X, n * MLP_NFEAT), n,
                                       _f32(y)), "cbie_mlp_forward")
    return y


def mlp_grad(params, mean, sdev, X, t):
    """(loss, gradient) of mean (y - t)^2 over all samples."""
    import torch
    n = X.shape[0]
    g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=X.device)
    L = torch.empty(1, dtype=torch.float32, device=X.device)
    _mlp_check(load().cbie_mlp_grad(C.c_void_p(torch.cuda.current_stream().cuda_stream), _f32(params, MLP_NPARAMS),
                                    _f32(mean, MLP_NFEAT), _f32(sdev, MLP_NFEAT), _f32(X, n * MLP_NFEAT),
                                    _f32(t, n), n, _f32(g), _f32(L)), "cbie_mlp_grad")
    return L, g


def mlp_train(params, mean, sdev, X, t, order, batch, lr):
    """Adam on consecutive runs of `batch` sample indices of `order` (int32
    CUDA tensor); params (float32 CUDA) updated in place; per-step losses."""
    import torch
    n = X.shape[0]
    if not (order.is_cuda and order.dtype == torch.int32 and order.is_contiguous()):
        raise TypeError("order: contiguous int32 CUDA tensor")
    if order.numel() and (int(order.min()) < 0 or int(order.max()) >= n):
        raise ValueError("order holds an index outside the samples")
    nsteps = order.numel() // batch
    losses = torch.empty(max(nsteps, 1), dtype=torch.float32, device=X.device)
    _mlp_check(load().cbie_mlp_train(C.c_void_p(torch.cuda.current_stream().cuda_stream), _f32(params, MLP_NPARAMS),
                                     _f32(mean, MLP_NFEAT), _f32(sdev, MLP_NFEAT), _f32(X, n * MLP_NFEAT),
                                     _f32(t, n), _ptr(order), nsteps, batch, float(lr), _f32(losses)),
               "cbie_mlp_train")
    return losses[:nsteps]
