"""Pins for the oracle's tree keys, validation and FMM lists (brute force on small trees)."""
import itertools

import numpy as np
import pytest

from oracle.tree import Tree, TreeError, _touch
from workloads import gen


def _anc_or_self(k):
    out = [k]
    while k[0] > 0:
        k = Tree.parent(k)
        out.append(k)
    return out


@pytest.mark.parametrize("seed", range(6))
def test_lists_cover_every_leaf_pair_exactly_once(seed):
    w = gen.random_small_tree(seed, max_level=5, n_splits=8)
    t = Tree(w.centres, w.levels)
    U, V, W, X = t.lists()
    vset = {(a, b) for a, bs in V.items() for b in bs}
    for ka in t.keys:
        for kb in t.keys:
            n = 0
            n += kb in U[ka]
            n += sum(c in W[ka] for c in _anc_or_self(kb))
            n += sum(kb in X.get(a2, []) for a2 in _anc_or_self(ka))
            n += sum((a2, b2) in vset for a2 in _anc_or_self(ka) for b2 in _anc_or_self(kb))
            assert n == 1, (ka, kb, n)


@pytest.mark.parametrize("seed", range(4))
def test_adjacency_matches_brute_force(seed):
    w = gen.random_small_tree(seed, max_level=5, n_splits=8)
    t = Tree(w.centres, w.levels)
    for ka in t.keys:
        brute = sorted(kb for kb in t.keys if kb != ka and _touch(ka, kb))
        assert t.adjacent_leaf_keys(ka) == brute


def test_relation_offsets_of_balanced_tree_are_the_33():
    from oracle import quad

    w = gen.random_small_tree(3, max_level=5, n_splits=10)
    t = Tree(w.centres, w.levels)
    for a in range(t.n_leaves):
        for b, rel in t.adjacent_leaves(a):
            assert quad.relation_index(*rel) >= 0


def test_validation_errors():
    c = np.array([[-0.5, -0.5], [0.5, -0.5], [-0.5, 0.5], [0.5, 0.5]])
    Tree(c, [1, 1, 1, 1])
    with pytest.raises(TreeError):
        Tree(c[:3], [1, 1, 1])  # gap
    with pytest.raises(TreeError):
        Tree(np.vstack([c, [[-0.75, -0.75]]]), [1, 1, 1, 1, 2])  # overlap
    with pytest.raises(TreeError):
        Tree(c + 0.01, [1, 1, 1, 1])  # off grid
    # unbalanced: one quadrant refined to level 3 next to level-1 leaves
    leaves = {(1, 1, 0), (1, 0, 1), (1, 1, 1)} | {(2, x, y) for x in (0, 1) for y in (0, 1)}
    leaves.remove((2, 1, 1))
    leaves |= {(3, x, y) for x in (2, 3) for y in (2, 3)}
    keys = sorted(leaves)
    cen = [(-1 + (2 * x + 1) * 2.0 ** -l, -1 + (2 * y + 1) * 2.0 ** -l) for l, x, y in keys]
    with pytest.raises(TreeError):
        Tree(cen, [k[0] for k in keys])
    Tree(cen, [k[0] for k in keys], check_balance=False)


def test_generator_trees_are_balanced_tilings():
    w = gen.config2(1)
    Tree(w.centres, w.levels)  # raises if not a balanced tiling
    assert w.n_leaves > 500
