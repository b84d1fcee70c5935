"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module holds *inputs only*: patch tables, material and wave parameters,
and the random numbers the method consumes (plane-wave directions, ellipsoid
shapes).  It contains none of the method's arithmetic: no evaluation of a
patch map, no quadrature, no kernel.  Both the CPU oracle and the GPU path
read these tables and each computes everything else on its own.  The one
surface formula here makes input data: closed-form surfaces (a gnomonic
cube sphere, a torus) sampled at Chebyshev points and turned into the
coefficient tables of Chebyshev-interpolated patches, the form a CAD
surface would be handed over in.

Workloads mirror the paper's structure (Sec. IV): curved quadrilateral patches
covering a smooth closed surface, a tensor grid of q x q Chebyshev points per
patch, two tangential unknowns per point for the PEC MFIE (four for N-Mueller),
plane-wave incidence.  The paper's CAD models are not available; equiangular
cube-sphere spheres and ellipsoids stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# Patch record: (face, i, j, s) on the equiangular cube sphere; face 0..5 is
# +x, -x, +y, -y, +z, -z; (i, j) indexes the s x s sub-squares of the face.
Patch = Tuple[int, int, int, int]

FORM_MFIE_PEC = 0
FORM_NMULLER = 1
CHEB_FACE = 6          # patch record (CHEB_FACE, p, 0, 0): Chebyshev-interpolated patch p


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
    # Chebyshev-interpolated patches instead of the cube sphere: coeffs[p, c,
    # n, m] multiplies T_n(u) T_m(v) in coordinate c of r(u, v); axes, center
    # and s are then unused
    coeffs: Optional[np.ndarray] = None

    @property
    def n_patches(self) -> int:
        if self.coeffs is not None:
            return self.coeffs.shape[0]
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
        if self.coeffs is not None:
            return [(CHEB_FACE, p, 0, 0) for p in range(self.coeffs.shape[0])]
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


# --------------------------------------------------------------------------
# Chebyshev-interpolated patches (generic surface input).
# --------------------------------------------------------------------------

def cheb_fit(f, deg: int) -> np.ndarray:
    """Coefficients (3, deg + 1, deg + 1) of the tensor interpolant of the
    map f(u, v) -> (..., 3) at the deg + 1 Chebyshev points of the first
    kind per direction (numpy's Chebyshev Vandermonde matrix, inverted)."""
    x = np.cos(np.pi * (np.arange(deg + 1) + 0.5) / (deg + 1))
    V = np.polynomial.chebyshev.chebvander(x, deg)
    Vi = np.linalg.inv(V)
    U, Vg = np.meshgrid(x, x, indexing="ij")
    F = f(U, Vg)
    return np.einsum("nk,klc,ml->cnm", Vi, F, Vi)


# right-handed frames (outward axis, first and second face directions)
_GNOMONIC_FRAMES = np.array([
    [[1, 0, 0], [0, 1, 0], [0, 0, 1]], [[-1, 0, 0], [0, 0, 1], [0, 1, 0]],
    [[0, 1, 0], [0, 0, 1], [1, 0, 0]], [[0, -1, 0], [1, 0, 0], [0, 0, 1]],
    [[0, 0, 1], [1, 0, 0], [0, 1, 0]], [[0, 0, -1], [0, 1, 0], [1, 0, 0]]], dtype=float)


def gnomonic_sphere_cheb(s: int, q: int, k0: float, deg: int, radius: float = 1.0,
                         form: int = FORM_MFIE_PEC, eps_r: float = 1.0) -> ObjectSpec:
    """A sphere given as 6 s^2 Chebyshev-interpolated patches of degree deg:
    the gnomonic cube sphere (face point e_n + x e_1 + y e_2 with x, y
    uniform on the face, projected onto the sphere), a parametrization other
    than the library's equiangular one."""
    C = []
    for f in range(6):
        en, e1, e2 = _GNOMONIC_FRAMES[f]
        for i in range(s):
            for j in range(s):
                def r(u, v, i=i, j=j, en=en, e1=e1, e2=e2):
                    x = (2 * i + 1 + u) / s - 1.0
                    y = (2 * j + 1 + v) / s - 1.0
                    c = en + x[..., None] * e1 + y[..., None] * e2
                    return radius * c / np.linalg.norm(c, axis=-1, keepdims=True)
                C.append(cheb_fit(r, deg))
    return ObjectSpec(axes=(radius, radius, radius), center=(0.0, 0.0, 0.0), s=s, q=q, k0=k0,
                      form=form, eps_r=eps_r, coeffs=np.array(C))


def torus_cheb(n_theta: int, n_phi: int, q: int, k0: float, deg: int, R: float = 1.0,
               rho: float = 0.4) -> ObjectSpec:
    """A torus (major radius R, minor radius rho) as n_theta x n_phi
    Chebyshev-interpolated patches of degree deg: u runs along the major
    angle theta, v along the minor angle phi, so a_u x a_v points outward."""
    C = []
    for a in range(n_theta):
        for b in range(n_phi):
            def r(u, v, a=a, b=b):
                th = 2 * np.pi * (a + 0.5 * (u + 1)) / n_theta
                ph = 2 * np.pi * (b + 0.5 * (v + 1)) / n_phi
                w = R + rho * np.cos(ph)
                return np.stack([w * np.cos(th), w * np.sin(th), rho * np.sin(ph)], axis=-1)
            C.append(cheb_fit(r, deg))
    return ObjectSpec(axes=(R + rho, R + rho, rho), center=(0.0, 0.0, 0.0), s=0, q=q, k0=k0, coeffs=np.array(C))


def sample_indices(n_total: int, n_sample: int, seed: int) -> np.ndarray:
    """Seeded sorted sample of row indices (for full-size residual checks)."""
    rng = np.random.default_rng(seed)
    n_sample = min(n_sample, n_total)
    return np.sort(rng.choice(n_total, size=n_sample, replace=False))


def random_complex(shape, seed: int) -> np.ndarray:
    """Seeded complex128 test vectors with standard-normal parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
