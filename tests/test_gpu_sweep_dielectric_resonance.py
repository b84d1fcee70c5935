"""The dielectric sphere of the paper's N-Mueller resonance study (Sec. IV-B,
Fig. 7): diameter 4 exterior wavelengths (radius 2 m, wavelength 1 m,
ka = 4 pi), plane wave along +z polarized along +x, permittivity swept
through a sharp physical resonance near eps_d = 10.5082 (mu_d = 1).  The
paper uses 96 patches of 10 x 10 points (38,400 unknowns); here q = 8 on
150 patches gives the same count (an N-Mueller patch of 10 x 10 points
would not fit a 256-unknown leaf).  ACA 1e-6, complex64 H-LU.

Two refinements of the same factorization at every permittivity:
  - stationary FP64 refinement (cbie_solve, at most 30 sweeps);
  - GMRES-based refinement (cbie_solve_gmres: FP64 GMRES on A M, the
    factorization M as right preconditioner).
Both must reach a relative residual of 1e-10 against the stored FP64
operator at every permittivity, resonance included, and the factorization
time must not depend on the resonance (every factor time within 1.5x of the
fastest): the paper's point for a direct solver (Fig. 7).  The error of the
surface current against the Mie series is printed; near the resonance it
grows (the discrete model's resonance sits slightly off the sphere's), and
the dense oracle on the same discretization at eps 10.5074 shows the same
error (tests/test_gpu_fullsize_accuracy.py), so it is the discretization's,
not the solver's.
"""
import numpy as np
import pytest

from oracle import geometry as G, mie, muller as Mu, post
from synth import workloads as W

pytestmark = pytest.mark.gpu

EPS = (10.3, 10.5, 10.5074, 10.5082, 10.6, 10.7)


def test_resonance_sweep_of_the_four_wavelength_sphere():
    import torch
    from paper_2408_17116_amd import cbie
    kh, pol = W.axial_wave()
    rows = {}
    for eps in EPS:
        spec = W.ObjectSpec(axes=(2.0, 2.0, 2.0), center=(0.0, 0.0, 0.0), s=5, q=8, k0=2.0 * np.pi,
                            form=W.FORM_NMULLER, eps_r=eps, mu_r=1.0)
        assert spec.n_unknowns == 38400
        s = cbie.Solver([spec])
        s.build_tree(leaf_size=256, eta=1.0, near_delta=1.0)
        s.fill()
        s.compress(1e-6)
        s.factor(cbie.PREC_C64_IR)
        t_factor = s.stats()["t_factor"]
        b = s.rhs_planewave(kh, pol)
        x0, it0 = s.solve(b, tol=1e-10, maxit=30)
        res0 = (torch.linalg.norm(s.matvec(x0) - b) / torch.linalg.norm(b)).item()
        x, itg = s.solve_gmres(b, tol=1e-10, restart=40, maxit=400)
        res = (torch.linalg.norm(s.matvec(x) - b) / torch.linalg.norm(b)).item()
        t_gmres = s.stats()["t_solve"]
        s.close()
        nd = G.build_nodes(spec)
        J, M = Mu.currents(nd, x.cpu().numpy()[:, 0])
        Jm, Mm = mie.dielectric_surface_currents(spec.k0, 2.0, eps, 1.0, nd.r)
        eJ, eM = post.weighted_rel_l2(nd, J, Jm), post.weighted_rel_l2(nd, M, Mm)
        rows[eps] = (res, res0, eJ, t_factor)
        print(f"eps {eps}: factor {t_factor:.2f} s; stationary {it0} sweeps, residual {res0:.1e}; "
              f"GMRES {itg} steps in {t_gmres:.2f} s, residual {res:.1e}; J vs Mie {eJ:.3e}, M vs Mie {eM:.3e}",
              flush=True)
    for eps, (res, res0, eJ, tf) in rows.items():
        assert res <= 1.01e-10 and res0 <= 1.01e-10, eps
    tmin = min(r[3] for r in rows.values())
    assert all(r[3] <= 1.5 * tmin for r in rows.values())
