"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module holds *inputs only*: patch tables, material and wave parameters,
and the random numbers the method consumes (plane-wave directions, ellipsoid
shapes).  It contains none of the method's arithmetic: no geometry map, no
quadrature, no kernel.  Both the CPU oracle and the GPU path read these tables
and each computes everything else on its own.

Workloads mirror the paper's structure (Sec. IV): curved quadrilateral patches
covering a smooth closed surface, a tensor grid of q x q Chebyshev points per
patch, two tangential unknowns per point for the PEC MFIE (four for N-Mueller),
plane-wave incidence.  The paper's CAD models are not available; equiangular
cube-sphere spheres and ellipsoids stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

# Patch record: (face, i, j, s) on the equiangular cube sphere; face 0..5 is
# +x, -x, +y, -y, +z, -z; (i, j) indexes the s x s sub-squares of the face.
Patch = Tuple[int, int, int, int]

FORM_MFIE_PEC = 0
FORM_NMULLER = 1


@dataclass
class ObjectSpec:
    """One scatterer: an ellipsoid (sphere when all axes agree)."""
    axes: Tuple[float, float, float]
    center: Tuple[float, float, float]
    s: int                      # faces split s x s -> 6 s^2 patches
    q: int                      # Chebyshev points per patch direction
    k0: float                   # exterior wavenumber (rad/m), normalized units
    form: int = FORM_MFIE_PEC
    eps_r: complex = 1.0        # interior relative permittivity (N-Mueller)
    mu_r: complex = 1.0         # interior relative permeability (N-Mueller)

    @property
    def n_patches(self) -> int:
        return 6 * self.s * self.s

    @property
    def n_nodes(self) -> int:
        return self.n_patches * self.q * self.q

    @property
    def unknowns_per_node(self) -> int:
        return 2 if self.form == FORM_MFIE_PEC else 4

    @property
    def n_unknowns(self) -> int:
        return self.n_nodes * self.unknowns_per_node

    def patches(self) -> List[Patch]:
        return cube_sphere_patches(self.s)


def cube_sphere_patches(s: int) -> List[Patch]:
    """Patch order: face-major, then i (first face coordinate), then j."""
    return [(f, i, j, s) for f in range(6) for i in range(s) for j in range(s)]


def plane_waves(n: int, seed: int = 0):
    """Seeded incident plane waves: unit propagation directions drawn
    uniformly on the sphere (normalized standard-normal 3-vectors) and a unit
    polarization perpendicular to each: x-hat projected out of the direction,
    falling back to y-hat when the direction is within ~6 degrees of +-x.

    Returns (khat[n,3], pol[n,3]) float64.
    """
    rng = np.random.default_rng(seed)
    k = rng.standard_normal((n, 3))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    pol = np.empty_like(k)
    for w in range(n):
        ref = np.array([1.0, 0.0, 0.0])
        if np.linalg.norm(np.cross(ref, k[w])) < 0.1:
            ref = np.array([0.0, 1.0, 0.0])
        e = ref - np.dot(ref, k[w]) * k[w]
        pol[w] = e / np.linalg.norm(e)
    return k, pol


def axial_wave():
    """The paper's excitation: propagation +z, polarization +x (Sec. IV)."""
    return np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]])


# --------------------------------------------------------------------------
# Named workloads.
# --------------------------------------------------------------------------

def sphere_pec_small() -> ObjectSpec:
    """PEC sphere r = 1 m, k = 2 pi, 24 patches, q = 8: 3072 unknowns."""
    return ObjectSpec(axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), s=2, q=8,
                      k0=2.0 * math.pi)


def sphere_pec_ka20() -> ObjectSpec:
    """PEC sphere r = 1 m, ka = 20, 384 patches, q = 8: 49152 unknowns."""
    return ObjectSpec(axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), s=8, q=8,
                      k0=20.0)


def sphere_dielectric() -> ObjectSpec:
    """Dielectric sphere r = 1 m, eps_r = 16, ka = 5, 96 patches, q = 8."""
    return ObjectSpec(axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), s=4, q=8,
                      k0=5.0, form=FORM_NMULLER, eps_r=16.0, mu_r=1.0)


def ellipsoid_pec_large() -> ObjectSpec:
    """PEC ellipsoid semi-axes (8, 4, 2) m, ka = 40 on the long axis,
    1536 patches, q = 8: 196608 unknowns."""
    return ObjectSpec(axes=(8.0, 4.0, 2.0), center=(0.0, 0.0, 0.0), s=16, q=8,
                      k0=5.0)


def ellipsoid_batch(n: int = 64, seed: int = 0) -> List[ObjectSpec]:
    """Uneven batch of PEC ellipsoids: semi-axes ~ U[0.5, 2] m, ka ~ U[2, 12]
    on the longest semi-axis, faces split s ~ U{2..5}, q ~ U{6, 7, 8}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        axes = tuple(float(a) for a in rng.uniform(0.5, 2.0, size=3))
        ka = float(rng.uniform(2.0, 12.0))
        s = int(rng.integers(2, 6))
        q = int(rng.integers(6, 9))
        out.append(ObjectSpec(axes=axes, center=(0.0, 0.0, 0.0), s=s, q=q,
                              k0=ka / max(axes)))
    return out


def mlp_initial_weights(seed: int = 0) -> np.ndarray:
    """Seeded initial parameters of the 8-64-64-1 rank network in the
    library's packing (W1 64x8 row-major, b1, W2 64x64 row-major, b2, W3,
    b3), float32: He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((64, 8)) * math.sqrt(2.0 / 8)
    w2 = rng.standard_normal((64, 64)) * math.sqrt(2.0 / 64)
    w3 = rng.standard_normal(64) * math.sqrt(2.0 / 64)
    return np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3, np.zeros(1)]).astype(np.float32)


def tiny_sphere(s: int = 1, q: int = 4, k0: float = 1.0) -> ObjectSpec:
    """Small spheres for brute-force checks (6 s^2 patches)."""
    return ObjectSpec(axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), s=s, q=q,
                      k0=k0)


def sample_indices(n_total: int, n_sample: int, seed: int) -> np.ndarray:
    """Seeded sorted sample of row indices (for full-size residual checks)."""
    rng = np.random.default_rng(seed)
    n_sample = min(n_sample, n_total)
    return np.sort(rng.choice(n_total, size=n_sample, replace=False))


def random_complex(shape, seed: int) -> np.ndarray:
    """Seeded complex128 test vectors with standard-normal parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
