"""Benchmark: H build + factor + solve of the CBIE MFIE system on one MI355X.

Workload: PEC sphere r = 1 m, ka = 20, 384 patches, q = 8 (49152 unknowns),
leaf 256, eta = 1, ACA tolerance 1e-6, 16 seeded plane waves.  One step is
the whole hot path: geometry + near classification + cluster/block trees,
fill (far rule + change-of-variables near quadrature), ACA compression,
H-LU, and the 16-right-hand-side solve.  Two pipelines are timed:
  mixed  compression with the widths of the rank network, complex64 H-LU,
         FP64 iterative refinement to 1e-9 (the reported value)
  fp64   adaptive compression, complex128 H-LU, FP64 iterative refinement
         to the same 1e-9
Inputs (patch tables, wave directions) are generated, and the rank network
is trained on the GPU from the adaptive ranks of other workloads (the
3072-unknown sphere and 24 seeded ellipsoids), before the timed region;
every step rebuilds everything from the inputs on the GPU.  After the timed
steps each pipeline's solution is compared with the dense oracle solution
stored under tests/golden (complex128 LAPACK solve of the same matrix,
written by tests/golden/make_dense_solutions.py), when that file exists.

A second workload is reported beside it (not the value): the dielectric
sphere eps_r = 16, ka = 5, 96 patches q = 8, 24576 unknowns, N-Mueller
formulation, one plane wave, one step per pipeline after one warmup.
And a third: the batch of 64 seeded PEC ellipsoids (semi-axes U[0.5, 2] m,
ka U[2, 12], 24-150 patches, q 6-8; 548208 unknowns in all) with 32 plane
waves per object, in one context (every stage in shared launches), mixed
pipeline, one step.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-dielectric] [--no-batch]
python bench.py --large-ellipsoid   (the PEC ellipsoid of semi-axes (8, 4, 2) m,
                                ka = 40, 196608 unknowns, ACA 1e-8: the rank
                                network trained on the GPU from the adaptive
                                ranks of the small sphere and 24 seeded
                                ellipsoids; adaptive vs predicted-width
                                compression; complex64 H-LU + refinement and
                                a one-wave solve; one JSON line, about 2 min)
python bench.py --high-contrast 50,100,200,300   (the 1-wavelength dielectric
                                sphere of the high-contrast study on 98,304
                                unknowns, ACA 1e-8: one JSON line per eps)
python bench.py --sphere-scaling 2,4,8,16,26   (the 3-wavelength-radius PEC sphere
                                at q = 10 from 4,800 to 811,200 unknowns: phase
                                times and storage per size, one JSON line each)
python bench.py --copy-probe   (a plain 1 GiB read + 1 GiB write elementwise
                                kernel, three launches: the reference for
                                scaling HBM traffic counters)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def run_pipeline(cbie, spec, kh, pol, prec, ir_tol, profile=True, model=None, factor_tol=0.0, aca_tol=1e-6):
    """One step: tree, fill, compress (predicted widths when a rank model is
    given), factor (truncation at factor_tol, 0: the ACA tolerance), right-hand
    sides and the refined solve."""
    s = cbie.Solver([spec])
    s.set_profiling(profile)
    s.set_factor_tolerance(factor_tol)
    s.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
    s.fill()
    if model is not None:
        s.set_rank_model(*model)
        s.compress(aca_tol, mode=cbie.RANK_PREDICTED)
    else:
        s.compress(aca_tol)
    s.factor(prec)
    b = s.rhs_planewave(kh, pol)
    x, it = s.solve(b, tol=ir_tol, maxit=20)
    st = s.stats()
    st["ir_iterations"] = it
    return s, x, st


def golden(name):
    """Stored dense oracle solution (tests/golden), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    return np.load(path)


def accuracy(x, x_ref):
    """Relative L2 error of the unknowns against the dense oracle solution:
    over all columns, and the worst column."""
    import numpy as np
    x = np.asarray(x)
    d = np.linalg.norm(x - x_ref, axis=0) / np.linalg.norm(x_ref, axis=0)
    return {"rel_l2": float(np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)), "worst_column": float(d.max())}


def train_rank_model(cbie, W):
    """Rank network trained on the GPU (project kernels) from the adaptive
    ranks of the 3072-unknown sphere and 24 seeded ellipsoids at every decade
    of tolerance 1e-3..1e-9.  Returns ((params, mean, sdev, margin), info)."""
    import numpy as np
    import torch
    tols = [10.0 ** -e for e in range(3, 10)]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    t0 = time.perf_counter()
    F, R = [], []
    for objs in ([W.sphere_pec_small()], W.ellipsoid_batch(24, seed=3)):
        s = cbie.Solver(objs)
        s.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
        s.fill()
        for tol in tols:
            s.compress(tol)
            f, r = s.block_features(tol)
            F.append(f)
            R.append(r)
        s.close()
    F, R = np.concatenate(F), np.concatenate(R)
    mean = F.mean(0).astype(np.float32)
    sdev = np.maximum(F.std(0), 1e-3).astype(np.float32)
    steps, batch = 4000, 256
    rng = np.random.default_rng(0)
    order = np.concatenate([rng.permutation(F.shape[0]) for _ in range(steps * batch // F.shape[0] + 1)])
    p = dev(W.mlp_initial_weights(0))
    losses = cbie.mlp_train(p, dev(mean), dev(sdev), dev(F), dev(np.log(np.maximum(R, 1)).astype(np.float32)),
                            dev(order[:steps * batch].astype(np.int32)), batch, 2e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"[bench] rank network: {F.shape[0]} samples, {t_train:.1f} s", file=sys.stderr, flush=True)
    info = {"samples": int(F.shape[0]), "steps": steps, "seconds": t_train,
            "loss_first": float(losses[:20].mean()), "loss_last": float(losses[-100:].mean())}
    return (p.cpu().numpy(), mean, sdev, 0.25), info


def compress_modes(cbie, spec, model):
    """Adaptive against predicted-width compression of one filled context:
    seconds, ACA workspace, fallbacks, and whether the ranks agree."""
    import numpy as np
    import torch
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
    s.fill()
    s.set_rank_model(*model)
    out, ranks = {}, {}
    for name, mode in (("adaptive", cbie.RANK_ADAPTIVE), ("predicted", cbie.RANK_PREDICTED)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.compress(1e-6, mode=mode)
        torch.cuda.synchronize()
        st = s.stats()
        ranks[name] = s.block_features(1e-6)[1]
        out[name] = {"seconds": time.perf_counter() - t1, "aca_workspace_GiB": st["aca_workspace_bytes"] / 2 ** 30,
                     "fallbacks": st["aca_fallbacks"], "unconverged": st["aca_unconverged"]}
    out["ranks_equal"] = bool(np.array_equal(ranks["adaptive"], ranks["predicted"]))
    s.close()
    return out


def dielectric(cbie, W, precs, names):
    """N-Mueller workload: seconds and unknowns/s per pipeline (one warmup,
    one timed step, both refined to 1e-10), refinement sweeps, the residual
    against the stored operator and the error against the stored dense
    oracle solution."""
    import numpy as np
    import torch
    spec = W.sphere_dielectric()
    kh, pol = np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]])
    gold = golden("dielectric_24576_dense.npz")
    # ACA 1e-7: at 1e-6 the compression error, amplified by the conditioning
    # of the eps_r = 16 system, leaves 1.7e-5 against the dense solution
    out = {"workload": "dielectric sphere eps_r=16, ka=5, 96 patches q=8, 24576 unknowns, N-Mueller, "
                       "leaf 256, eta 1, ACA 1e-7, 1 plane wave"}
    for name in names:
        prec = precs[name]
        s, x, st = run_pipeline(cbie, spec, kh, pol, prec, 1e-10, profile=False, aca_tol=1e-7)
        s.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, x, st = run_pipeline(cbie, spec, kh, pol, prec, 1e-10, profile=False, aca_tol=1e-7)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b = s.rhs_planewave(kh, pol)
        res = (torch.linalg.norm(s.matvec(x) - b) / torch.linalg.norm(b)).item()
        s.close()
        out[name] = {"seconds": dt, "unknowns_per_s": spec.n_unknowns / dt, "ir_iterations": st["ir_iterations"],
                     "residual": res, "phases_s": {p: st["t_" + p] for p in ("tree", "fill", "compress", "factor",
                                                                               "solve")}}
        if gold is not None:
            out[name]["accuracy_vs_dense_oracle"] = accuracy(x.cpu().numpy(), gold["x"])
        print(f"[bench] dielectric {name}: {dt:.2f} s", file=sys.stderr, flush=True)
    return out


def nm_compress_modes(cbie, W):
    """Compression of the dielectric sphere (ACA 1e-7) with N-Mueller blocks
    filled explicitly and compressed from their copies, with entries
    generated on the fly, and with the default split between the two (by
    block size): seconds, ranks, and whether the ranks agree."""
    import numpy as np
    import torch
    s = cbie.Solver([W.sphere_dielectric()])
    s.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
    s.fill()
    out, ranks = {}, {}
    old = os.environ.get("CBIE_NM_OTF_MIN")
    try:
        for name, lim in (("explicit", "1000000000"), ("on_the_fly", "0"), ("default", old)):
            if lim is None:
                os.environ.pop("CBIE_NM_OTF_MIN", None)
            else:
                os.environ["CBIE_NM_OTF_MIN"] = lim
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.compress(1e-7)
            torch.cuda.synchronize()
            out[name] = {"seconds": time.perf_counter() - t0, "max_rank": s.stats()["max_rank"]}
            ranks[name] = s.block_features(1e-7)[1]
    finally:
        if old is None:
            os.environ.pop("CBIE_NM_OTF_MIN", None)
        else:
            os.environ["CBIE_NM_OTF_MIN"] = old
    out["ranks_equal"] = bool(np.array_equal(ranks["explicit"], ranks["on_the_fly"]))
    s.close()
    return out


def ellipsoid_batch(cbie, W):
    """The 64-object batch in one context, mixed pipeline, one step."""
    import numpy as np
    import torch
    objs = W.ellipsoid_batch(64, seed=0)
    kh, pol = W.plane_waves(32, seed=4)
    N = sum(o.n_unknowns for o in objs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = cbie.Solver(objs)
    s.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
    s.fill()
    s.compress(1e-6)
    s.factor(cbie.PREC_C64_IR)
    b = s.rhs_planewave(kh, pol)
    x, it = s.solve(b, tol=1e-10, maxit=20)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = s.stats()
    res = (torch.linalg.norm(s.matvec(x) - b) / torch.linalg.norm(b)).item()
    out = {"workload": "64 PEC ellipsoids (seed 0), 548208 unknowns, 32 plane waves each, one context, "
                       "leaf 256, eta 1, ACA 1e-6, mixed pipeline",
           "seconds": dt, "unknowns_per_s": N / dt, "ir_iterations": it, "residual": res,
           "phases_s": {p: st["t_" + p] for p in ("tree", "fill", "compress", "factor", "solve")}}
    gold = golden("ellipsoid_batch_subset_dense.npz")
    if gold is not None:
        off = np.concatenate([[0], np.cumsum([o.n_unknowns for o in objs])])
        xs = x.cpu().numpy()
        errs = {}
        for o in gold["objects"]:
            o = int(o)
            xr = gold[f"x{o}"]
            errs[str(o)] = accuracy(xs[off[o]:off[o + 1], :xr.shape[1]], xr)["rel_l2"]
        out["accuracy_vs_dense_oracle"] = {"objects": errs, "worst": max(errs.values())}
    s.close()
    print(f"[bench] ellipsoid batch: {dt:.2f} s", file=sys.stderr, flush=True)
    return out


def large_ellipsoid(cbie, W):
    """Rank network trained on the GPU, then the 196608-unknown ellipsoid
    compressed adaptively and with predicted widths (same ranks), factored
    in complex64 and solved with FP64 refinement.  ACA 1e-8: the operator's
    smallest singular value is near 1.5e-3 (an interior resonance of the
    MFIE at this size), which amplifies the compression error about
    800-fold; at 1e-6 the solution would miss 1e-5."""
    import numpy as np
    import torch
    model, info = train_rank_model(cbie, W)
    spec = W.ellipsoid_pec_large()
    s = cbie.Solver([spec])
    s.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
    s.fill()
    out = {"workload": "PEC ellipsoid semi-axes (8, 4, 2) m, ka = 40, 1536 patches q = 8, 196608 unknowns, "
                       "leaf 256, eta 1, ACA 1e-8, 1 plane wave, mixed pipeline",
           "training": info, "fill_s": s.stats()["t_fill"]}
    ranks = {}
    s.set_rank_model(*model)
    for name, mode in (("adaptive", cbie.RANK_ADAPTIVE), ("predicted", cbie.RANK_PREDICTED)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.compress(1e-8, mode=mode)
        torch.cuda.synchronize()
        st = s.stats()
        ranks[name] = s.block_features(1e-8)[1]
        out[name] = {"seconds": time.perf_counter() - t1, "aca_workspace_GiB": st["aca_workspace_bytes"] / 2 ** 30,
                     "fallbacks": st["aca_fallbacks"], "unconverged": st["aca_unconverged"],
                     "lr_blocks": st["n_lr_blocks"], "max_rank": st["max_rank"]}
        print(f"[bench] large ellipsoid, {name} compress: {out[name]['seconds']:.2f} s", file=sys.stderr, flush=True)
    out["ranks_equal"] = bool(np.array_equal(ranks["adaptive"], ranks["predicted"]))
    kh, pol = W.plane_waves(1, seed=0)
    t1 = time.perf_counter()
    s.factor(cbie.PREC_C64_IR)
    b = s.rhs_planewave(kh, pol)
    x, it = s.solve(b, tol=1e-10, maxit=30)
    torch.cuda.synchronize()
    st = s.stats()
    out["factor_solve"] = {"seconds": time.perf_counter() - t1, "factor_s": st["t_factor"], "solve_s": st["t_solve"],
                           "factor_flops": st["factor_flops"], "ir_iterations": it,
                           "residual": (torch.linalg.norm(s.matvec(x) - b) / torch.linalg.norm(b)).item()}
    s.close()
    return out


def sphere_scaling(cbie, W, splits):
    """The paper's scaling study (Sec. IV-A, Fig. 4): PEC sphere of radius
    3 wavelengths (ka = 6 pi), 10 x 10 points per patch, cube-sphere faces
    split s x s (6 s^2 patches, 1200 s^2 unknowns: 4,800 at s = 2 up to
    811,200 at s = 26), ACA 1e-4, axial wave, mixed pipeline.  Times of each
    phase, compression rate, storage and the residual against the stored
    operator, one size at a time (one JSON line each)."""
    import numpy as np
    import torch
    kh, pol = W.axial_wave()
    for s_ in splits:
        spec = W.ObjectSpec(axes=(3.0, 3.0, 3.0), center=(0.0, 0.0, 0.0), s=s_, q=10, k0=2.0 * np.pi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv = cbie.Solver([spec])
        sv.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
        sv.fill()
        sv.compress(1e-4)
        sv.factor(cbie.PREC_C64_IR)
        b = sv.rhs_planewave(kh, pol)
        x, it = sv.solve(b, tol=1e-10, maxit=30)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = sv.stats()
        res = (torch.linalg.norm(sv.matvec(x) - b) / torch.linalg.norm(b)).item()
        sv.close()
        rec = {"sphere_scaling": {"radius_wavelengths": 3, "q": 10, "patches": 6 * s_ * s_,
                                  "unknowns": spec.n_unknowns, "seconds": dt,
                                  "phases_s": {p: st["t_" + p] for p in ("tree", "fill", "compress", "factor", "solve")},
                                  "compression_rate": st["compression_rate"], "max_rank": st["max_rank"],
                                  "lr_entries": st["lr_entries"], "dense_entries": st["dense_entries"],
                                  "factor_flops": st["factor_flops"], "ir_iterations": it, "residual": res}}
        print(json.dumps(rec), flush=True)


def high_contrast(cbie, W, eps_list):
    """The paper's high-contrast study (Sec. IV-B, Fig. 8): dielectric sphere
    one exterior wavelength across (radius 0.5 m, k0 = 2 pi, mu_d = 1) on one
    fixed mesh (faces split 8 x 8, q = 8: 98,304 unknowns, which resolves the
    interior wavelength up to eps_d = 300), ACA 1e-8, complex64 H-LU refined
    to 1e-10, axial wave.  Time of each phase, ranks, sweeps and the residual
    against the stored operator per permittivity (one JSON line each); the
    currents' error against the Mie series is checked by
    tests/test_gpu_high_contrast.py."""
    import numpy as np
    import torch
    kh, pol = W.axial_wave()
    for eps in eps_list:
        spec = W.ObjectSpec(axes=(0.5, 0.5, 0.5), center=(0.0, 0.0, 0.0), s=8, q=8, k0=2.0 * np.pi,
                            form=W.FORM_NMULLER, eps_r=eps, mu_r=1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv = cbie.Solver([spec])
        sv.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
        sv.fill()
        sv.compress(1e-8)
        sv.factor(cbie.PREC_C64_IR)
        b = sv.rhs_planewave(kh, pol)
        x, it = sv.solve(b, tol=1e-10, maxit=30)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = sv.stats()
        res = (torch.linalg.norm(sv.matvec(x) - b) / torch.linalg.norm(b)).item()
        sv.close()
        rec = {"high_contrast": {"eps_r": eps, "unknowns": spec.n_unknowns, "seconds": dt,
                                 "phases_s": {p: st["t_" + p] for p in ("tree", "fill", "compress", "factor", "solve")},
                                 "compression_rate": st["compression_rate"], "max_rank": st["max_rank"],
                                 "ir_iterations": it, "residual": res}}
        print(json.dumps(rec), flush=True)


def gemm_traffic(pipeline):
    """HBM bytes per k_zgemm launch from the committed counter runs
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size), or
    None when the GEMM kernel or the scheduler that forms its launches has
    changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_zgemm_traffic_sphere_ka20_49152_mixed.json")
    if pipeline != "mixed" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for src, sha in rec["source_sha256"].items():
        if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != sha:
            return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(spec, kh, pol, budget_s=20.0):
    """Time the oracle (dense fill by rows + LAPACK LU + solve) on a bounded
    sample and scale it to the full workload's unknowns/s."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import geometry as G, mfie
    from synth import workloads as W

    nd = G.build_nodes(spec)
    N = 2 * nd.size
    rows = W.sample_indices(N, 4, seed=1)
    t0 = time.perf_counter()
    mfie.matrix_rows(nd, spec.k0, rows)
    t_row = (time.perf_counter() - t0) / rows.size
    n_lu = 3000
    A = W.random_complex((n_lu, n_lu), seed=2)
    t0 = time.perf_counter()
    lu = sla.lu_factor(A, check_finite=False)
    t_lu_s = time.perf_counter() - t0
    B = W.random_complex((n_lu, 16), seed=3)
    t0 = time.perf_counter()
    sla.lu_solve(lu, B, check_finite=False)
    t_sv_s = time.perf_counter() - t0
    t_fill = t_row * N
    t_lu = t_lu_s * (N / n_lu) ** 3
    t_sv = t_sv_s * (N / n_lu) ** 2
    total = t_fill + t_lu + t_sv
    threads = os.cpu_count()
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        pass
    return {"value": N / total, "unit": "unknowns/s", "cores": threads, "kind": "oracle",
            "sample": (f"oracle fill of {rows.size} exact rows ({t_row:.2f} s/row) scaled to {N} rows; "
                       f"LAPACK zgetrf/zgetrs on a {n_lu}x{n_lu} complex128 matrix (16 rhs) scaled by "
                       f"(N/{n_lu})^3 and ^2; projected dense solve {total:.0f} s"),
            "seconds_projected": total}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--pipelines", default="mixed,fp64")
    ap.add_argument("--no-dielectric", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--large-ellipsoid", action="store_true")
    ap.add_argument("--sphere-scaling", default="",
                    help="comma-separated face splits s of the 3-wavelength sphere at q = 10 (e.g. 2,4,8,16,26)")
    ap.add_argument("--high-contrast", default="",
                    help="comma-separated permittivities of the 1-wavelength dielectric sphere (e.g. 50,100,200,300)")
    ap.add_argument("--factor-tol", type=float, default=0.0,
                    help="truncation tolerance of the mixed leg's factorization (0: the ACA tolerance)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = 1 << 28                                   # float32: 1 GiB
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe": {"launches": 3, "bytes_read_per_launch": 4 * n,
                                         "bytes_written_per_launch": 4 * n}}))
        return
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the H-matrix solve of one object is not "
              "sharded); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2408_17116_amd import cbie
    from synth import workloads as W

    if args.large_ellipsoid:
        print(json.dumps({"large_ellipsoid": large_ellipsoid(cbie, W)}))
        return
    if args.sphere_scaling:
        sphere_scaling(cbie, W, [int(v) for v in args.sphere_scaling.split(",")])
        return
    if args.high_contrast:
        high_contrast(cbie, W, [float(v) for v in args.high_contrast.split(",")])
        return
    spec = W.sphere_pec_ka20()
    kh, pol = W.plane_waves(16, seed=0)
    N = spec.n_unknowns
    precs = {"mixed": cbie.PREC_C64_IR, "fp64": cbie.PREC_C128}
    names = args.pipelines.split(",")
    model, train_info = train_rank_model(cbie, W) if "mixed" in names else (None, None)
    results = {}
    for name in names:
        prec = precs[name]
        mdl = model if name == "mixed" else None
        ftol = args.factor_tol if name == "mixed" else 0.0
        for _ in range(args.warmup):
            s, x, st = run_pipeline(cbie, spec, kh, pol, prec, 1e-9, model=mdl, factor_tol=ftol)
            s.close()
            print(f"[bench] warmup {name} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for k in range(args.steps):
            s, x, st = run_pipeline(cbie, spec, kh, pol, prec, 1e-9, model=mdl, factor_tol=ftol)
            stats.append(st)
            s.close()
            print(f"[bench] step {k} {name}: " + ", ".join(f"{p} {st['t_' + p]:.3f}s" for p in
                  ("tree", "fill", "compress", "factor", "solve")), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        results[name] = (dt, stats[-1], x)

    gold = golden("sphere_ka20_49152_dense.npz")
    name0 = "mixed" if "mixed" in results else list(results)[0]
    dt, st, _ = results[name0]
    line = {
        "metric": "H build+factor+solve s & unknowns/s, mixed vs FP64 H-LU, at 1e-5 rel err",
        "value": N / dt, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+f64" if name0 == "mixed" else "c128", "data": "synthetic",
        "config": {"workload": "PEC sphere ka=20, 384 patches q=8, 49152 unknowns, leaf 256, eta 1, "
                               "ACA 1e-6, 16 plane waves", "pipeline": name0},
        "roofline": gemm_roofline(st, name0),
        "rooflines": phase_rooflines(st, name0, N),
        "phases_s": {p: st["t_" + p] for p in ("tree", "fill", "compress", "factor", "solve")},
        "stats": {k: st[k] for k in ("n_lr_blocks", "n_dense_blocks", "max_rank", "compression_rate",
                                     "n_kernel_launches", "factor_flops", "factor_flops_executed", "ir_iterations",
                                     "quad_seconds", "aca_fallbacks", "aca_unconverged")},
    }
    for name, (d, s2, x) in results.items():
        rec = {"seconds": d, "unknowns_per_s": N / d, "ir_iterations": s2["ir_iterations"],
               # the truncation the factor used: the ACA tolerance unless set,
               # and no less than 1e-5 for the complex64 factor
               "factor_tolerance": (max(args.factor_tol or 1e-6, 1e-5) if name == "mixed" else 1e-6),
               "phases_s": {p: s2["t_" + p] for p in ("tree", "fill", "compress", "factor", "solve")},
               "rank_widths": "predicted" if name == "mixed" else "adaptive"}
        if gold is not None:
            rec["accuracy_vs_dense_oracle"] = accuracy(x.cpu().numpy(), gold["x"])
        if name != name0:
            rec["rooflines"] = phase_rooflines(s2, name, N)
        line.setdefault("pipelines", {})[name] = rec
    if gold is not None:
        line["accuracy"] = {name: line["pipelines"][name]["accuracy_vs_dense_oracle"]["rel_l2"] for name in results}
    if model is not None:
        line["rank_network"] = dict(train_info, compress=compress_modes(cbie, spec, model))
    if not args.no_dielectric:
        line["dielectric_sphere"] = dielectric(cbie, W, precs, names)
        line["dielectric_sphere"]["nm_aca_entries"] = nm_compress_modes(cbie, W)
    if not args.no_batch:
        line["ellipsoid_batch"] = ellipsoid_batch(cbie, W)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(spec, kh, pol)
    print(json.dumps(line))


def gemm_roofline(st, pipeline):
    """The dominant kernel: the batched complex GEMM of the H-LU and of the
    first (recorded) substitution, timed by HIP events on the library stream
    around every launch of the step; algorithmic flops (8 m n k per product,
    a leaf solve through an explicit inverse counted as the triangular solve
    it stands for, 4 n^2 k)."""
    peak = 157.3 if pipeline == "mixed" else 78.6      # MI355X dense MFMA FP32 / FP64, TFLOP/s
    sec = st["gemm_seconds"]
    achieved = st["gemm_flops_alg"] / sec / 1e12 if sec > 0 else None
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak if achieved else None, "traffic": gemm_traffic(pipeline),
            "kernel": "k_zgemm (batched complex GEMM, %s)" % ("complex64" if pipeline == "mixed" else "complex128"),
            "launches": st["gemm_launches"], "avg_launch_us": 1e6 * sec / max(st["gemm_launches"], 1),
            "flops_per_launch": st["gemm_flops_alg"] / max(st["gemm_launches"], 1),
            "executed_flops_per_launch": st["gemm_flops"] / max(st["gemm_launches"], 1),
            "algorithmic_bytes_per_launch": st["gemm_bytes_alg"] / max(st["gemm_launches"], 1),
            "executed_tflops": st["gemm_flops"] / sec / 1e12 if sec > 0 else None,
            "complex_product": ("three real products on 64x64 tiles, four on the others"
                                if pipeline == "mixed" and os.environ.get("CBIE_GEMM_3M", "1") != "0"
                                else "four real products"),
            "mfma_tflops": st["gemm_flops_mfma"] / sec / 1e12 if sec > 0 else None,
            "kernel_seconds": sec}


def phase_rooflines(st, pipeline, N):
    """Per-phase roofline of one step: near quadrature (FP64 VALU, the basis
    contraction's flops over the quadrature kernels' event time), far fill
    (HBM writes of the dense blocks over their kernel time), leaf LU (8/3 b^3
    per leaf over the leaf kernels' event time, against the vector peak of
    the factor precision), the GEMMs (above) and the solve (HBM: the bytes
    the substitutions and the refinement matvecs must read, over the solve
    stage's wall time)."""
    vec = 157.3 if pipeline == "mixed" else 78.6       # FP32 / FP64 vector peak, TFLOP/s
    out = {"k_zgemm": gemm_roofline(st, pipeline)}
    out["k_zgemm"].pop("traffic", None)
    if st["quad_seconds"] > 0:
        a = st["quad_flops"] / st["quad_seconds"] / 1e12
        out["near_quadrature"] = {"kernel": "k_quad", "bound": "alu", "achieved": a, "peak": 78.6,
                                  "unit": "TFLOP/s", "frac": a / 78.6, "points": st["quad_points"],
                                  "seconds": st["quad_seconds"]}
    if st["far_fill_seconds"] > 0:
        gb = 16.0 * st["dense_entries"] / st["far_fill_seconds"] / 1e9
        out["far_fill"] = {"kernel": "k_far_fill", "bound": "hbm", "achieved": gb, "peak": 8000.0, "unit": "GB/s",
                           "frac": gb / 8000.0, "bytes": 16.0 * st["dense_entries"], "seconds": st["far_fill_seconds"]}
    if st["leaf_lu_seconds"] > 0:
        a = st["leaf_lu_flops"] / st["leaf_lu_seconds"] / 1e12
        out["leaf_lu"] = {"kernel": "k_leaf_lu", "bound": "alu", "achieved": a, "peak": vec, "unit": "TFLOP/s",
                          "frac": a / vec, "launches": st["leaf_lu_launches"], "seconds": st["leaf_lu_seconds"]}
    it = st["ir_iterations"]
    op_bytes = 16.0 * (st["dense_entries"] + st["lr_entries"])
    # x = M b, then per sweep one matvec + one substitution, and the final check
    byt = (1 + it) * st["solve_factor_bytes"] + (it + 1) * op_bytes
    gb = byt / st["t_solve"] / 1e9
    out["solve"] = {"bound": "hbm", "achieved": gb, "peak": 8000.0, "unit": "GB/s", "frac": gb / 8000.0,
                    "bytes": byt, "substitutions": 1 + it, "matvecs": it + 1, "seconds": st["t_solve"]}
    return out


if __name__ == "__main__":
    main()
