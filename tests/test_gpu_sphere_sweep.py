"""The 20-wavelength-diameter PEC sphere of the paper's accuracy study
(Sec. IV-A, Table 1): radius 10 m at wavelength 1 m (ka = 20 pi), plane
wave along +z polarized along +x, 10 x 10 points per patch.

The paper compresses at ACA 1e-4.  Here ka = 20 pi lies close to an
interior resonance of the MFIE (the derivative of x j_1(x) is 0.016 there),
so the operator has a small singular value and the compression error is
amplified about a thousandfold: at 76,800 unknowns ACA 1e-4 leaves 1.2e-1
against the Mie series, ACA 1e-6 and 1e-8 both 1.49e-2 (the two solutions
agree to 1.4e-5), next to the table's 1.41e-2.  The test compresses at
1e-6, the tolerance of the other PEC workloads, so that the error measured
is the discretization's, the quantity the table reports.

The cube-sphere faces split s x s give exactly the table's four unknown
counts at q = 10: s = 6, 8, 10, 12 -> 216, 384, 600, 864 patches ->
43,200, 76,800, 120,000, 172,800 unknowns.  The H-LU solution (complex64
with FP64 refinement) is compared with the Mie series: relative L2 error of
the surface current, quadrature-weighted over the nodes.

The table's errors of the proposed solver (1.91e-1, 1.41e-2, 6.69e-3,
2.13e-3) fall by 13.5x, 2.1x and 3.1x from each column to the next, the
convergence of the discretization.  The test asserts that the error falls
at every step and stays within 3x of the table's: the paper states neither
its patching nor the norm of its error, so an exact match is not expected.
The 172,800-unknown case needs the factorization's storage-pressure
recompressions (its update columns would otherwise outgrow the GPU's
memory)."""
import numpy as np
import pytest

from oracle import geometry as G, mie, post
from synth import workloads as W

pytestmark = pytest.mark.gpu

TABLE1 = {43200: 1.91e-1, 76800: 1.41e-2, 120000: 6.69e-3, 172800: 2.13e-3}   # proposed solver


def test_twenty_wavelength_sphere_at_order_ten_against_mie():
    # s = 6 .. 12 at ACA 1e-6: about five minutes on one GPU
    import torch
    from paper_2408_17116_amd import cbie
    errs = {}
    for s in (6, 8, 10, 12):
        spec = W.ObjectSpec(axes=(10.0, 10.0, 10.0), center=(0.0, 0.0, 0.0), s=s, q=10, k0=2.0 * np.pi)
        N = spec.n_unknowns
        sv = cbie.Solver([spec])
        sv.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
        sv.fill()
        sv.compress(1e-6)
        sv.factor(cbie.PREC_C64_IR)
        kh, pol = W.axial_wave()
        b = sv.rhs_planewave(kh, pol)
        x, it = sv.solve(b, tol=1e-10, maxit=30)
        res = (torch.linalg.norm(sv.matvec(x) - b) / torch.linalg.norm(b)).item()
        st = sv.stats()
        sv.close()
        nd = G.build_nodes(spec)
        J = post.surface_current(nd, x.cpu().numpy()[:, 0])
        Jm = mie.pec_surface_current(spec.k0, 10.0, nd.r)
        errs[N] = post.weighted_rel_l2(nd, J, Jm)
        print(f"N {N} ({6 * s * s} patches, q 10): max rank {st['max_rank']}, CR {st['compression_rate']:.3f}, "
              f"fill {st['t_fill']:.2f} s, compress {st['t_compress']:.2f} s, factor {st['t_factor']:.2f} s, "
              f"solve {st['t_solve']:.2f} s ({it} sweeps), residual {res:.1e}; J vs Mie {errs[N]:.3e} "
              f"(Table 1: {TABLE1[N]:.2e})", flush=True)
        assert res < 1e-8
    ns = sorted(errs)
    for a, b in zip(ns, ns[1:]):
        assert errs[b] < errs[a], (a, b)
    for n in ns:
        assert errs[n] < 3.0 * TABLE1[n], n
