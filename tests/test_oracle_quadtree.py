"""Pins of the quadtree oracle (Sec. 4.2.1, Alg. 2 with reading C6; 2:1 balance, C7).

* The Chebyshev transform recovers T_a(x) T_b(y) exactly, and is the inverse of evaluating a
  Chebyshev series at the nodes (NumPy's chebval).
* Polynomials of degree <= p - 3 in each variable have no tail: the root is a leaf.
* The dictionary-based balance equals the all-pairs version on random trees, and the result is
  balanced by brute force; balance only refines (every input leaf is covered).
* A built tree's leaves pass the tail test (or are forced), and each leaf's parent fails it.
* A Gaussian centred at the origin gives a tree symmetric under the square's symmetries.
"""
import numpy as np
import pytest

from oracle import quadtree as qt


def _cheb_T(n, t):
    return np.cos(n * np.arccos(np.clip(t, -1, 1)))


def test_transform_recovers_chebyshev_products():
    t = qt.cheb_points()
    X, Y = np.meshgrid(t, t, indexing="xy")
    for a, b in ((0, 0), (3, 7), (15, 2), (14, 15)):
        c = qt.coefficients(_cheb_T(a, X) * _cheb_T(b, Y))
        e = np.zeros((16, 16))
        e[b, a] = 1.0
        assert np.max(np.abs(c - e)) < 1e-14
    rng = np.random.default_rng(0)
    C = rng.standard_normal((16, 16))
    V = np.polynomial.chebyshev.chebval2d(X, Y, C.T)  # chebval2d(x, y, c) uses c[i(x), j(y)]
    assert np.max(np.abs(qt.coefficients(V) - C)) < 1e-13


def test_low_degree_polynomials_resolve_at_root():
    f = lambda p: 1.0 + p[:, 0] ** 13 - 3 * p[:, 0] * p[:, 1] ** 12 + p[:, 1] ** 5
    assert qt.tail(f(qt.box_nodes((0, 0, 0)))) < 1e-13
    assert qt.refine(f, 1e-11, 1.0) == [(0, 0, 0)]


def _random_leaves(seed, n_splits=12, max_level=6):
    rng = np.random.default_rng(seed)
    leaves = {(1, x, y) for x in (0, 1) for y in (0, 1)}
    for _ in range(n_splits):
        cand = sorted(k for k in leaves if k[0] < max_level)
        k = cand[int(rng.integers(len(cand)))]
        leaves.remove(k)
        leaves.update(qt.children(k))
    return leaves


@pytest.mark.parametrize("seed", range(6))
def test_balance_matches_brute_force(seed):
    raw = _random_leaves(seed)
    a, b = qt.balance(raw), qt.balance_brute(raw)
    assert a == b
    for x in a:
        for y in a:
            assert not (y[0] >= x[0] + 2 and qt._adjacent(x, y))
    for (l, x, y) in raw:  # every input leaf is covered by output leaves no coarser
        assert (l, x, y) in a or any(k[0] > l and (k[1] >> (k[0] - l), k[2] >> (k[0] - l)) == (x, y) for k in a)
    # the leaves tile the root
    assert sum(4.0 ** -k[0] for k in a) == pytest.approx(1.0, abs=1e-15)


def test_refined_tree_invariants():
    g = lambda p: np.exp(-((p[:, 0] - 0.3) ** 2 + (p[:, 1] + 0.2) ** 2) / (2 * 0.05 ** 2))
    leaves = qt.refine(g, 1e-10, 1.0, min_level=1, max_level=12)
    for k in leaves:
        assert qt.tail(g(qt.box_nodes(k))) <= 1e-10 or k[0] == 12
        if k[0] > 1:
            par = (k[0] - 1, k[1] >> 1, k[2] >> 1)
            assert qt.tail(g(qt.box_nodes(par))) > 1e-10
    assert sum(4.0 ** -k[0] for k in leaves) == pytest.approx(1.0, abs=1e-15)


def test_symmetric_source_gives_symmetric_tree():
    g = lambda p: np.exp(-(p[:, 0] ** 2 + p[:, 1] ** 2) / (2 * 0.08 ** 2))
    leaves = qt.build(g, 1e-10, 1.0)
    for (l, x, y) in leaves:
        n = (1 << l) - 1
        for k in ((l, n - x, y), (l, x, n - y), (l, y, x)):
            assert k in leaves
