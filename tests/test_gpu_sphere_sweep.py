"""The 20-wavelength-diameter PEC sphere of the paper's accuracy study
(Sec. IV, Table 1): radius 10 m at wavelength 1 m (ka = 20 pi), ACA
tolerance 1e-4, plane wave along +z polarized along +x.  The H-LU solution
(complex64 with FP64 refinement) is compared with the Mie series: relative
L2 error of the surface current, quadrature-weighted over the nodes.

The paper uses 10 x 10 points per patch; the library takes q <= 8, and
q = 8 with more patches (cube-sphere faces split s x s) gives the same
numbers of unknowns for two of the table's four columns: 76,800 (s = 10,
patches 1.57 wavelengths across) and 172,800 (s = 15).  The errors are
above the paper's (6.1e-2 at 76,800 against its 1.41e-2).  Both sample
about 5.1 points per wavelength; at a fixed patch size the error grows with
the electrical size (the oracle's own dense solution with the same
1.57-wavelength patches: 2.7e-3 at ka = 4 pi, 7.3e-3 at ka = 8 pi), and the
higher order explains part of the gap, not all of it (the paper states
neither its patching nor its error norm).  The bound, 0.07, is a
regression bound above the measured 6.5e-2 (49,152) and 6.1e-2 (76,800),
not the paper's figure, which is printed beside the result.  The 172,800
case takes a few minutes and runs only with CBIE_LARGE_TESTS=1."""
import os

import numpy as np
import pytest

from oracle import geometry as G, mie, post
from synth import workloads as W

pytestmark = pytest.mark.gpu

KA = 20.0 * np.pi
PAPER = {76800: 1.41e-2, 172800: 2.13e-3}   # Table 1, proposed solver


@pytest.mark.parametrize("s", [8, 10, 15], ids=["N49152", "N76800", "N172800"])
def test_twenty_wavelength_sphere_against_mie(s):
    import torch
    from paper_2408_17116_amd import cbie
    if s == 15 and os.environ.get("CBIE_LARGE_TESTS") != "1":
        pytest.skip("172,800 unknowns: set CBIE_LARGE_TESTS=1")
    spec = W.ObjectSpec(axes=(10.0, 10.0, 10.0), center=(0.0, 0.0, 0.0), s=s, q=8, k0=2.0 * np.pi)
    N = spec.n_unknowns
    s_ = cbie.Solver([spec])
    s_.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
    s_.fill()
    s_.compress(1e-4)
    s_.factor(cbie.PREC_C64_IR)
    kh, pol = W.axial_wave()
    b = s_.rhs_planewave(kh, pol)
    x, it = s_.solve(b, tol=1e-10, maxit=30)
    res = (torch.linalg.norm(s_.matvec(x) - b) / torch.linalg.norm(b)).item()
    st = s_.stats()
    s_.close()
    nd = G.build_nodes(spec)
    J = post.surface_current(nd, x.cpu().numpy()[:, 0])
    Jm = mie.pec_surface_current(spec.k0, 10.0, nd.r)
    err = post.weighted_rel_l2(nd, J, Jm)
    print(f"N {N}: max rank {st['max_rank']}, CR {st['compression_rate']:.3f}, fill {st['t_fill']:.2f} s, "
          f"compress {st['t_compress']:.2f} s, factor {st['t_factor']:.2f} s, solve {st['t_solve']:.2f} s "
          f"({it} sweeps), residual {res:.1e}; J vs Mie {err:.3e} (paper {PAPER.get(N)})", flush=True)
    assert res < 1e-8
    assert err < 0.07
