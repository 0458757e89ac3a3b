"""Pins of the oracle's off-grid evaluation of the volume potential and its gradient
(oracle/quad.py potential_at_points, the plain definition by adaptive quadrature).

* The closed-form gradient of the uniform-square potential against centred differences of
  the closed-form potential (the derivative algebra).
* A uniform density on an adaptive tree: u and grad u at arbitrary points (inside leaves, on
  leaf edges and corners, on the root's boundary, outside) equal the square closed forms.
* At leaf nodes, the adaptive quadrature equals the table-based direct sum (two independent
  quadratures of the same integrals).
* The gradient of a Gaussian source against Richardson-extrapolated centred differences of u at
  points away from leaf edges.
"""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import quad, tree
from workloads import gen


def _points(rng, n):
    p = rng.uniform(-1, 1, (n, 2))
    edges = np.array([[0.0, 0.3], [0.5, 0.5], [-0.25, -0.75], [1.0, 0.2], [-1.0, -1.0], [0.125, 1.0]])
    outside = np.array([[1.3, 0.4], [-0.2, -1.6]])
    return np.vstack([p, edges, outside])


def test_square_gradient_closed_form():
    rng = np.random.default_rng(1)
    x, y = rng.uniform(-2, 2, 40), rng.uniform(-2, 2, 40)
    gx, gy = cf.square_gradient(x, y, -1.0, 0.5, -0.25, 1.0)

    def fd(h, ax):
        ex = h if ax == 0 else 0.0
        ey = h if ax == 1 else 0.0
        return (cf.square_potential(x + ex, y + ey, -1.0, 0.5, -0.25, 1.0)
                - cf.square_potential(x - ex, y - ey, -1.0, 0.5, -0.25, 1.0)) / (2 * h)

    for ax, g in ((0, gx), (1, gy)):
        r = (4 * fd(5e-4, ax) - fd(1e-3, ax)) / 3  # Richardson
        assert np.max(np.abs(r - g)) < 1e-9


@pytest.mark.parametrize("seed", range(2))
def test_uniform_density_at_points(seed):
    w = gen.random_small_tree(seed, max_level=4, n_splits=6)
    T = tree.Tree(w.centres, w.levels)
    f = np.ones((w.n_leaves, 256))
    p = _points(np.random.default_rng(seed), 12)
    u, g = quad.potential_at_points(w.centres, T.halfw, f, p, grad=True)
    ue = cf.square_potential(p[:, 0], p[:, 1], -1, 1, -1, 1)
    gx, gy = cf.square_gradient(p[:, 0], p[:, 1], -1, 1, -1, 1)
    assert np.max(np.abs(u - ue)) < 1e-13
    assert np.max(np.abs(g[:, 0] - gx)) < 1e-11 and np.max(np.abs(g[:, 1] - gy)) < 1e-11


def test_points_at_leaf_nodes_match_tables():
    w = gen.random_small_tree(3, max_level=4, n_splits=5)
    T = tree.Tree(w.centres, w.levels)
    rng = np.random.default_rng(2)
    samples = [(int(rng.integers(w.n_leaves)), int(rng.integers(256))) for _ in range(20)]
    ref = quad.direct_potential(T, w.f, samples=samples)
    t = -np.cos((2 * np.arange(1, 17) - 1) * np.pi / 32)
    xy = np.array([[w.centres[a, 0] + T.halfw[a] * t[m % 16], w.centres[a, 1] + T.halfw[a] * t[m // 16]]
                   for a, m in samples])
    u = quad.potential_at_points(w.centres, T.halfw, w.f, xy)
    assert np.max(np.abs(u - ref)) < 1e-13 * np.max(np.abs(ref))


def test_gradient_matches_differences_of_u():
    w = gen.random_small_tree(5, max_level=4, n_splits=6)
    T = tree.Tree(w.centres, w.levels)
    rng = np.random.default_rng(4)
    p = rng.uniform(-0.95, 0.95, (60, 2))
    # keep points at least 2e-3 from every leaf edge (the second derivatives jump across edges)
    lo = w.centres - T.halfw[:, None]
    hi = w.centres + T.halfw[:, None]
    keep = []
    for q in p:
        inside = np.all((q >= lo) & (q <= hi), axis=1)
        a = int(np.argmax(inside))
        if np.min(np.abs(np.concatenate([q - lo[a], hi[a] - q]))) > 2e-3:
            keep.append(q)
    p = np.array(keep[:12])
    _, g = quad.potential_at_points(w.centres, T.halfw, w.f, p, grad=True)

    def fd(h, ax):
        e = np.zeros(2)
        e[ax] = h
        return (quad.potential_at_points(w.centres, T.halfw, w.f, p + e)
                - quad.potential_at_points(w.centres, T.halfw, w.f, p - e)) / (2 * h)

    for ax in (0, 1):
        r = (4 * fd(2.5e-4, ax) - fd(5e-4, ax)) / 3
        assert np.max(np.abs(r - g[:, ax])) < 1e-8 * np.max(np.abs(g))
