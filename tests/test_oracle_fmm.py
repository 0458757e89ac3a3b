"""Pins for the oracle box code (fmm.py): agreement with the plain definition (direct sum),
convergence in the expansion order, and exactness of its transpose."""
import numpy as np
import pytest

from oracle import fmm, nodes, quad, tree
from oracle.tree import Tree
from workloads import gen


@pytest.fixture(scope="module")
def c1():
    w = gen.config1(0)
    t = Tree(w.centres, w.levels)
    return w, t, fmm.BoxCode(t)


def test_box_code_matches_direct_sum_config1(c1):
    w, t, bc = c1
    ud = quad.direct_potential(t, w.f)
    uf = bc.apply(w.f)
    assert np.max(np.abs(uf - ud)) / np.max(np.abs(ud)) < 2e-14


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_box_code_matches_direct_sum_adaptive(seed):
    w = gen.random_small_tree(seed, max_level=5, n_splits=7)
    t = Tree(w.centres, w.levels)
    bc = fmm.BoxCode(t)
    ud = quad.direct_potential(t, w.f)
    assert np.max(np.abs(bc.apply(w.f) - ud)) / np.max(np.abs(ud)) < 3e-14


def test_truncation_error_decays_with_order(c1):
    w, t, bc = c1
    ref = bc.apply(w.f)
    errs = []
    for P in (8, 16, 24):
        u = fmm.BoxCode(t, P=P).apply(w.f)
        errs.append(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-9


def test_transpose_dot_product(c1):
    w, t, bc = c1
    rng = np.random.default_rng(3)
    f = rng.standard_normal((t.n_leaves, 256))
    r = rng.standard_normal((t.n_leaves, 256))
    Af = bc.apply(f)
    Atr = bc.apply_adjoint(r)
    lhs = np.sum(Af * r)
    rhs = np.sum(f * Atr)
    # scale-free form of the test: relative to |Af| |r| (and |f| |A^T r|)
    assert abs(lhs - rhs) / (np.linalg.norm(Af) * np.linalg.norm(r)) < 1e-14
    assert abs(lhs - rhs) / (np.linalg.norm(f) * np.linalg.norm(Atr)) < 1e-14


def test_transpose_against_plain_definition():
    # <A_direct f, r> = <f, A_boxcode^T r>: ties the transpose to the plain definition.
    w = gen.random_small_tree(5, max_level=4, n_splits=5)
    t = Tree(w.centres, w.levels)
    bc = fmm.BoxCode(t)
    rng = np.random.default_rng(4)
    r = rng.standard_normal((t.n_leaves, 256))
    Af = quad.direct_potential(t, w.f)
    lhs = np.sum(Af * r)
    rhs = np.sum(w.f * bc.apply_adjoint(r))
    assert abs(lhs - rhs) / (np.linalg.norm(Af) * np.linalg.norm(r)) < 1e-14


def test_symmetry_in_quadrature_inner_product():
    # <A f, g>_W ~ <f, A g>_W for over-resolved smooth f, g (uniform depth 3, sigma >= 0.2):
    # the continuous operator is symmetric; the discrete one only to the quadrature error.
    gf = gen.Gaussians(np.array([[0.1, 0.2]]), np.array([0.25]), np.array([1.0]))
    gg = gen.Gaussians(np.array([[-0.3, 0.1]]), np.array([0.3]), np.array([-0.7]))
    wf = gen.make_workload("f", gf, gen.uniform_tree(3))
    wg = gen.make_workload("g", gg, gen.uniform_tree(3))
    t = Tree(wf.centres, wf.levels)
    bc = fmm.BoxCode(t)
    from oracle import nodes

    Wq = nodes.tensor_weights()[None, :] * (t.halfw ** 2)[:, None]
    a = np.sum(Wq * bc.apply(wf.f) * wg.f)
    b = np.sum(Wq * wf.f * bc.apply(wg.f))
    assert abs(a - b) / abs(a) < 1e-12


def test_config1_matches_gaussian_closed_form_minus_exterior_tail():
    # config 1 (uniform level 3, two Gaussians per seed, sigma in [0.1, 0.3], up to 9 % of a
    # source's mass outside the root): the box code against the whole-plane closed form minus
    # the exterior tail. At level 3 these widths are resolved to about 1e-15, so the difference
    # is rounding and truncation only (measured 2.1e-15 at worst over these seeds).
    from oracle import closed_forms as cf

    worst = 0.0
    for seed in (0, 3, 5, 6):
        w = gen.config1(seed)
        u = fmm.BoxCode(tree.Tree(w.centres, w.levels)).apply(w.f)
        rng = np.random.default_rng(2)
        for a, m in zip(rng.integers(0, w.n_leaves, 6), rng.integers(0, 256, 6)):
            x, y = nodes.leaf_nodes(w.centres[a], 2.0 ** -w.levels[a])[m]
            ref = sum(cf.gaussian_potential(x, y, cx, cy, s, A) - cf.gaussian_exterior_tail(x, y, cx, cy, s, A)
                      for (cx, cy), s, A in zip(w.src.centres, w.src.sigmas, w.src.amps))
            worst = max(worst, abs(u[a, m] - ref) / np.max(np.abs(u)))
    print("config 1 closed form: max rel err %.2e" % worst)
    assert worst <= 1e-13
