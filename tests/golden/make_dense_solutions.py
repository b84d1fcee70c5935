"""Dense oracle solutions of the full-size workloads, for the GPU tests and
the benchmark's accuracy check.

For each workload the script assembles the dense complex128 CBIE matrix with
the oracle's own routines (Fejer rule for far pairs, the oracle's Duffy
quadrature for self and near pairs, eq. 20), factors it with LAPACK's
partial-pivot LU (the plain definition x = A^-1 b of what the H-matrix
method approximates, Sec. III) and solves for seeded plane waves (eqs. 19,
22).  It calls only oracle/ and the seeded inputs of synth/.

After the solve, a seeded sample of rows is recomputed one by one with the
oracle's row routine (matrix_rows) and the residual of the stored solution
on those rows is recorded: it checks the row routine against the dense
assembly at full size and the solution against the matrix it solves.

    python tests/golden/make_dense_solutions.py sphere_ka20     # 49152 unknowns, ~32 min on 8 cores, 40 GB
    python tests/golden/make_dense_solutions.py dielectric      # 24576 unknowns
    python tests/golden/make_dense_solutions.py batch_subset    # 4 seeded objects of the 64-ellipsoid batch
    python tests/golden/make_dense_solutions.py resonance       # 38400 unknowns, eps_d 10.5074 (Sec. IV-B)
    python tests/golden/make_dense_solutions.py stretched       # 12288 unknowns: the 196,608-unknown ellipsoid's
                                                                # shape and patch size, scaled down 4x
    python tests/golden/make_dense_solutions.py component_small # 768-unknown MFIE and 1536-unknown N-Mueller
                                                                # spheres: dense solve and the component-wise
                                                                # block solve (Sec. III-A, eqs. 22-28)
"""
from __future__ import annotations

import os
import sys
import time
from multiprocessing import Pool

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dense, geometry as G, mfie, muller  # noqa: E402
from synth import workloads as W  # noqa: E402

_ND = None
_ARGS = None


def _init(nd, args):
    global _ND, _ARGS
    _ND, _ARGS = nd, args


def _near_chunk(chunk):
    form, k0, eps_r = _ARGS
    if form == W.FORM_MFIE_PEC:
        return [mfie.singular_block(_ND, k0, t, p, u, v) for (t, p, u, v, _s) in chunk]
    md = muller.Media(k0, eps_r)
    return [muller.singular_block(_ND, md, t, p, u, v) for (t, p, u, v, _s) in chunk]


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def dense_solve(spec, kh, pol, workers=8, n_check=8, seed=11):
    """Assemble, factor and solve; returns (x, record)."""
    nd = G.build_nodes(spec)
    n, q2 = nd.size, nd.q * nd.q
    upn = spec.unknowns_per_node
    N = upn * n
    t0 = time.time()
    pairs = mfie.near_pairs(nd)
    log(f"N = {N}: {len(pairs)} near pairs ({time.time() - t0:.0f} s)")
    size = max(1, len(pairs) // (40 * workers))
    chunks = [pairs[i:i + size] for i in range(0, len(pairs), size)]
    args = (spec.form, spec.k0, spec.eps_r)
    blocks = []
    with Pool(workers, initializer=_init, initargs=(nd, args)) as pool:
        for ci, res in enumerate(pool.imap(_near_chunk, chunks)):
            blocks.extend(res)
            if ci % 40 == 0:
                log(f"near chunks {ci + 1}/{len(chunks)}")
    log(f"near blocks done ({time.time() - t0:.0f} s)")
    # A in Fortran order: AT is C-ordered A^T, so LAPACK factors A in place
    AT = np.empty((N, N), dtype=complex)
    A = AT.T
    idx = np.arange(n)
    if spec.form == W.FORM_MFIE_PEC:
        for a0 in range(0, n, 256):
            ti = idx[a0:a0 + 256]
            with np.errstate(divide="ignore", invalid="ignore"):
                A[2 * a0:2 * (a0 + ti.size)] = mfie.far_block(nd, spec.k0, ti, idx).reshape(2 * ti.size, N)
    else:
        md = muller.Media(spec.k0, spec.eps_r)
        for p in range(nd.n_patches):
            for a0 in range(0, n, 1024):
                ti = idx[a0:a0 + 1024]
                blk = muller.far_patch(nd, md, ti, p)                       # [i, c, j, a]
                A[4 * a0:4 * (a0 + ti.size), 4 * p * q2:4 * (p + 1) * q2] = blk.reshape(4 * ti.size, 4 * q2)
    log(f"far entries done ({time.time() - t0:.0f} s)")
    for (t, p, _u, _v, _s), blk in zip(pairs, blocks):
        A[upn * t:upn * (t + 1), upn * p * q2:upn * (p + 1) * q2] = blk.reshape(upn, upn * q2)
    del blocks
    diag = np.full(upn, 0.5) if upn == 2 else muller.Media(spec.k0, spec.eps_r).diag
    A[np.arange(N), np.arange(N)] += np.tile(diag, n)
    B = mfie.rhs_planewave(nd, spec.k0, kh, pol) if upn == 2 else muller.rhs_planewave(nd, spec.k0, kh, pol)
    log(f"assembled ({time.time() - t0:.0f} s); LU of {N} x {N}")
    lu, piv = sla.lu_factor(A, overwrite_a=True, check_finite=False)
    log(f"LU done ({time.time() - t0:.0f} s)")
    x = sla.lu_solve((lu, piv), B, check_finite=False)
    del lu, AT, A
    rows = W.sample_indices(N, n_check, seed=seed)
    if upn == 2:
        R = mfie.matrix_rows(nd, spec.k0, rows)
    else:
        R = muller.matrix_rows(nd, spec.k0, spec.eps_r, spec.mu_r, rows=rows)
    res = np.abs(R @ x - B[rows]).max() / np.abs(B).max()
    log(f"row check: max |A x - b| / max |b| over {rows.size} recomputed rows = {res:.2e}")
    rec = {"n_unknowns": N, "near_pairs": len(pairs), "check_rows": rows, "check_residual": res,
           "seconds": time.time() - t0}
    return x, rec


def main():
    which = sys.argv[1]
    if which == "sphere_ka20":
        spec = W.sphere_pec_ka20()
        kh, pol = W.plane_waves(16, seed=0)
        x, rec = dense_solve(spec, kh, pol)
        np.savez(os.path.join(HERE, "sphere_ka20_49152_dense.npz"), x=x, khat=kh, pol=pol, **rec)
    elif which == "dielectric":
        spec = W.sphere_dielectric()
        kh, pol = W.axial_wave()
        x, rec = dense_solve(spec, kh, pol)
        np.savez(os.path.join(HERE, "dielectric_24576_dense.npz"), x=x, khat=kh, pol=pol, **rec)
    elif which == "batch_subset":
        objs = W.ellipsoid_batch(64, seed=0)
        kh, pol = W.plane_waves(32, seed=4)
        pick = W.sample_indices(64, 4, seed=7)
        out = {"objects": pick, "khat": kh[:4], "pol": pol[:4]}
        for o in pick:
            x, rec = dense_solve(objs[o], kh[:4], pol[:4])
            out[f"x{o}"] = x
            out[f"check_residual{o}"] = rec["check_residual"]
        np.savez(os.path.join(HERE, "ellipsoid_batch_subset_dense.npz"), **out)
    elif which == "resonance":
        spec = W.ObjectSpec(axes=(2.0, 2.0, 2.0), center=(0.0, 0.0, 0.0), s=5, q=8, k0=2.0 * np.pi,
                            form=W.FORM_NMULLER, eps_r=10.5074, mu_r=1.0)
        kh, pol = W.axial_wave()
        x, rec = dense_solve(spec, kh, pol)
        np.savez(os.path.join(HERE, "resonance_38400_dense.npz"), x=x, khat=kh, pol=pol, **rec)
    elif which == "stretched":
        spec = W.ObjectSpec(axes=(2.0, 1.0, 0.5), center=(0.0, 0.0, 0.0), s=4, q=8, k0=5.0)
        kh, pol = W.plane_waves(1, seed=0)
        x, rec = dense_solve(spec, kh, pol)
        np.savez(os.path.join(HERE, "stretched_ellipsoid_12288_dense.npz"), x=x, khat=kh, pol=pol, **rec)
    elif which == "component_small":
        out = {}
        spec = W.tiny_sphere(s=2, q=4, k0=3.0)
        nd = G.build_nodes(spec)
        A = mfie.dense_matrix(nd, spec.k0, workers=8)
        kh, pol = W.plane_waves(3, seed=11)
        b = mfie.rhs_planewave(nd, spec.k0, kh, pol)
        out.update(mfie_khat=kh, mfie_pol=pol, mfie_x=dense.solve(A, b), mfie_xc=dense.component_block_solve(A, b, 2))
        spec = W.ObjectSpec(axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), s=2, q=4, k0=2.0,
                            form=W.FORM_NMULLER, eps_r=4.0, mu_r=1.0)
        nd = G.build_nodes(spec)
        A = muller.dense_matrix(nd, spec.k0, spec.eps_r, workers=8)
        kh, pol = W.axial_wave()
        b = muller.rhs_planewave(nd, spec.k0, kh, pol)
        out.update(nm_khat=kh, nm_pol=pol, nm_x=dense.solve(A, b), nm_xc=dense.component_block_solve(A, b, 4))
        for k in ("mfie", "nm"):
            d = np.linalg.norm(out[k + "_x"] - out[k + "_xc"]) / np.linalg.norm(out[k + "_x"])
            log(f"{k}: component block solve vs dense solve {d:.2e}")
        np.savez(os.path.join(HERE, "component_small_dense.npz"), **out)
    else:
        raise SystemExit(f"unknown workload {which}")


if __name__ == "__main__":
    main()
