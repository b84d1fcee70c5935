"""Write oracle-only reference values for the GPU tests.

Calls nothing but the CPU oracle (oracle/) and the seeded workloads (synth/).
Output: tests/golden/sphere_2pi_q8.npz with the dense-oracle solution of the
PEC sphere r = 1 m, k = 2 pi, 24 patches, q = 8 (3072 unknowns) for the
axial plane wave (+z, x-polarised), its bistatic RCS in the phi = 0 and
phi = 90 degree planes at 181 angles, the Mie RCS and the Mie surface
current at the nodes.

    python tests/golden/make_golden.py [workers]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dense, geometry as G, mfie, mie, post  # noqa: E402
from synth import workloads as W  # noqa: E402


def main(workers=8):
    spec = W.sphere_pec_small()
    nd = G.build_nodes(spec)
    k = spec.k0
    t0 = time.time()
    A = mfie.dense_matrix(nd, k, workers=workers)
    t_fill = time.time() - t0
    kh, pol = W.axial_wave()
    b = mfie.rhs_planewave(nd, k, kh, pol)[:, 0]
    t0 = time.time()
    x = dense.solve(A, b)
    t_lu = time.time() - t0
    th = np.linspace(0.0, 180.0, 181)
    rcs_e = post.rcs(nd, k, x, post.plane_cut(th, 0.0))
    rcs_h = post.rcs(nd, k, x, post.plane_cut(th, 90.0))
    mie_e, mie_h = mie.pec_rcs(k, 1.0, np.deg2rad(th))
    J_mie = mie.pec_surface_current(k, 1.0, nd.r)
    cond = np.linalg.cond(A)
    out = os.path.join(HERE, "sphere_2pi_q8.npz")
    np.savez_compressed(out, x=x, b=b, theta=th, rcs_e=rcs_e, rcs_h=rcs_h, mie_e=mie_e, mie_h=mie_h,
                        J_mie=J_mie, cond=cond, t_fill=t_fill, t_lu=t_lu)
    J = post.surface_current(nd, x)
    print(f"wrote {out}: N={x.size} cond={cond:.2f} fill {t_fill:.1f}s LU {t_lu:.2f}s "
          f"|J-Jmie|/|Jmie|={post.weighted_rel_l2(nd, J, J_mie):.2e} "
          f"RCS_E err={np.linalg.norm(rcs_e - mie_e) / np.linalg.norm(mie_e):.2e}")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
