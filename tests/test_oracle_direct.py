"""Pins for the oracle's direct sum u = A f against analysis and exact invariances."""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import nodes, quad
from oracle.tree import Tree
from workloads import gen


def _node_xy(t, a):
    return nodes.leaf_nodes(t.centres[a], t.halfw[a])


def test_uniform_density_equals_square_closed_form():
    # f = 1 on every leaf of an adaptive tree: u is the potential of the uniform root square.
    w = gen.random_small_tree(2, max_level=4, n_splits=5)
    t = Tree(w.centres, w.levels)
    f = np.ones((t.n_leaves, 256))
    u = quad.direct_potential(t, f)
    for a in range(t.n_leaves):
        xy = _node_xy(t, a)
        ref = cf.square_potential(xy[:, 0], xy[:, 1], -1, 1, -1, 1)
        assert np.max(np.abs(u[a] - ref)) < 1e-14


def test_gaussian_closed_form_level4():
    # A narrow centred Gaussian (exterior tail below 1e-20) on a uniform level-4 tree: the
    # result differs from the closed form only by the leaf interpolation error of f.
    g = gen.Gaussians(np.array([[0.05, -0.03]]), np.array([0.1]), np.array([0.8]))
    w = gen.make_workload("gauss-l4", g, gen.uniform_tree(4))
    t = Tree(w.centres, w.levels)
    rng = np.random.default_rng(0)
    samples = [(int(a), int(m)) for a, m in zip(rng.integers(0, t.n_leaves, 48), rng.integers(0, 256, 48))]
    u = quad.direct_potential(t, w.f, samples)
    ref = []
    for a, m in samples:
        x, y = _node_xy(t, a)[m]
        ref.append(cf.gaussian_potential(x, y, 0.05, -0.03, 0.1, 0.8))
    ref = np.array(ref)
    assert np.max(np.abs(u - ref)) / np.max(np.abs(ref)) < 1e-11


def test_scaling_law_log_term():
    # Shrink a tree by lam = 1/2 into the lower-left quadrant (other quadrants: zero data).
    # Then u'(lam x + c) = lam^2 u(x) - (lam^2 / 2pi) log(lam) int f: exercises every log s term.
    w = gen.random_small_tree(1, max_level=3, n_splits=3)
    t = Tree(w.centres, w.levels)
    u = quad.direct_potential(t, w.f)
    cen2 = np.vstack([0.5 * w.centres - 0.5, [[0.5, -0.5], [-0.5, 0.5], [0.5, 0.5]]])
    lev2 = np.concatenate([w.levels + 1, [1, 1, 1]])
    f2 = np.vstack([w.f, np.zeros((3, 256))])
    t2 = Tree(cen2, lev2, check_balance=False)
    u2 = quad.direct_potential(t2, f2)[: t.n_leaves]
    mass = np.sum(w.f @ nodes.tensor_weights() * t.halfw ** 2)
    lam = 0.5
    ref = lam ** 2 * u - lam ** 2 / (2 * np.pi) * np.log(lam) * mass
    assert np.max(np.abs(u2 - ref)) / np.max(np.abs(ref)) < 1e-13


def test_refinement_invariance():
    # Splitting a leaf with exact polynomial prolongation leaves f_h unchanged, hence u at
    # all other leaves. The split leaf is chosen with no coarser neighbour.
    w = gen.random_small_tree(0, max_level=3, n_splits=3)
    t = Tree(w.centres, w.levels)
    u = quad.direct_potential(t, w.f)
    a = None
    for cand in range(t.n_leaves):
        if all(t.halfw[b] <= t.halfw[cand] for b, _ in t.adjacent_leaves(cand)):
            a = cand
            break
    assert a is not None
    c, s = t.centres[a], t.halfw[a]
    tt = nodes.cheb1_points()
    kids_c, kids_f = [], []
    for dy in (-0.5, 0.5):
        for dx in (-0.5, 0.5):
            cc = c + s * np.array([dx, dy])
            # child nodes in parent reference coordinates
            xq = dx + 0.5 * tt
            yq = dy + 0.5 * tt
            kids_c.append(cc)
            kids_f.append(nodes.interp_to_points(w.f[a], xq, yq).reshape(-1))
    keep = [b for b in range(t.n_leaves) if b != a]
    cen2 = np.vstack([t.centres[keep], kids_c])
    lev2 = np.concatenate([t.levels[keep], [t.levels[a] + 1] * 4])
    f2 = np.vstack([w.f[keep], kids_f])
    t2 = Tree(cen2, lev2)
    u2 = quad.direct_potential(t2, f2)[: len(keep)]
    assert np.max(np.abs(u2 - u[keep])) / np.max(np.abs(u)) < 1e-13


def test_rotation_invariance():
    # Rotate tree and data by 90 degrees: (x, y) -> (-y, x). Node (i, j) maps to (15-j, i).
    w = gen.random_small_tree(4, max_level=3, n_splits=3)
    t = Tree(w.centres, w.levels)
    u = quad.direct_potential(t, w.f)
    cen2 = np.stack([-w.centres[:, 1], w.centres[:, 0]], axis=1)
    idx = np.arange(256)
    i, j = idx % 16, idx // 16
    newpos = i * 16 + (15 - j)  # rotated node index of old node (i, j)
    f2 = np.zeros_like(w.f)
    f2[:, newpos] = w.f
    t2 = Tree(cen2, w.levels)
    u2 = quad.direct_potential(t2, f2)
    assert np.max(np.abs(u2[:, newpos] - u)) / np.max(np.abs(u)) < 1e-13
