"""The seeded synthetic workloads against the configurations they stand for:
sizes (patches, order, unknowns), electrical sizes and the ranges of the
batch, and determinism of every seeded generator."""
import numpy as np

from synth import workloads as W


def test_named_workloads_have_the_stated_sizes():
    cases = [
        (W.sphere_pec_small(), 24, 8, 3072, 2 * np.pi),          # r = 1, k = 2 pi
        (W.sphere_pec_ka20(), 384, 8, 49152, 20.0),               # r = 1, ka = 20
        (W.sphere_dielectric(), 96, 8, 24576, 5.0),               # r = 1, ka = 5, 4 unknowns per node
        (W.ellipsoid_pec_large(), 1536, 8, 196608, 40.0),         # long semi-axis 8, ka = 40
    ]
    for spec, patches, q, N, ka in cases:
        assert 6 * spec.s * spec.s == patches
        assert spec.q == q
        assert spec.n_unknowns == N
        assert abs(spec.k0 * max(spec.axes) - ka) < 1e-12
    d = W.sphere_dielectric()
    assert d.form == W.FORM_NMULLER and d.eps_r == 16.0 and d.mu_r == 1.0


def test_batch_ranges_and_total():
    objs = W.ellipsoid_batch(64, seed=0)
    assert len(objs) == 64
    assert sum(o.n_unknowns for o in objs) == 548208
    for o in objs:
        assert all(0.5 <= a <= 2.0 for a in o.axes)
        assert 2.0 <= o.k0 * max(o.axes) <= 12.0
        assert 24 <= 6 * o.s * o.s <= 150 and 6 <= o.q <= 8
        assert 1728 <= o.n_unknowns <= 19200


def test_seeded_generators_are_deterministic():
    a = W.ellipsoid_batch(8, seed=5)
    b = W.ellipsoid_batch(8, seed=5)
    assert [(o.axes, o.s, o.q, o.k0) for o in a] == [(o.axes, o.s, o.q, o.k0) for o in b]
    k1, p1 = W.plane_waves(16, seed=0)
    k2, p2 = W.plane_waves(16, seed=0)
    assert np.array_equal(k1, k2) and np.array_equal(p1, p2)
    assert np.allclose(np.linalg.norm(k1, axis=1), 1.0) and np.allclose(np.sum(k1 * p1, axis=1), 0.0)
    assert np.array_equal(W.random_complex((5, 3), seed=2), W.random_complex((5, 3), seed=2))
    assert np.array_equal(W.mlp_initial_weights(1), W.mlp_initial_weights(1))
