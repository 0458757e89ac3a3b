"""GPU parity of the off-grid evaluation (volpot_plan_points / volpot_apply_points): u and its
gradient at arbitrary points against the oracle's adaptive quadrature of the plain definition
(oracle/quad.py potential_at_points), max-norm relative error <= 1e-11 for u and for the
gradient. Cases: small adaptive trees at random points, points on leaf edges and corners and on
the root's boundary, points at leaf nodes (must agree with the leaf-node output), no points,
and the star-cut tree at the nodes of a curve inside it.
"""
import numpy as np
import pytest

from oracle import quad, tree
from tests.conftest import rel_max_err
from workloads import gen

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _run(device, w, pts, **kw):
    import torch

    from paper_2501_17967_amd import PointPlan

    print("points case: %d leaves, %d points %s" % (w.n_leaves, len(pts), kw), flush=True)
    plan = PointPlan(w.centres, w.levels, pts, **kw)
    f = torch.from_numpy(w.f).to(device)
    u, up, gp = plan.apply_points(f)
    torch.cuda.synchronize()
    return plan, u.cpu().numpy(), up.cpu().numpy(), gp.cpu().numpy()


def _oracle(w, pts):
    T = tree.Tree(w.centres, w.levels)
    return quad.potential_at_points(w.centres, T.halfw, w.f, pts, grad=True)


@pytest.mark.parametrize("seed", range(3))
def test_random_points_small_trees(device, seed):
    w = gen.random_small_tree(seed, max_level=5, n_splits=9)
    rng = np.random.default_rng(seed)
    pts = np.vstack([rng.uniform(-1, 1, (40, 2)),
                     [[0.5, 0.5], [0.0, -0.25], [1.0, 1.0], [-1.0, -1.0], [1.0, 0.3], [-0.6, 1.0], [0.25, 0.125]]])
    _, _, up, gp = _run(device, w, pts)
    u_o, g_o = _oracle(w, pts)
    assert rel_max_err(up, u_o) < TOL
    assert rel_max_err(gp, g_o) < TOL


def test_points_at_leaf_nodes_equal_node_output(device):
    w = gen.config1(0)
    t = -np.cos((2 * np.arange(1, 17) - 1) * np.pi / 32)
    rng = np.random.default_rng(1)
    sel = [(int(rng.integers(w.n_leaves)), int(rng.integers(256))) for _ in range(50)]
    s = 2.0 ** (-w.levels.astype(float))
    pts = np.array([[w.centres[a, 0] + s[a] * t[m % 16], w.centres[a, 1] + s[a] * t[m // 16]] for a, m in sel])
    _, u, up, _ = _run(device, w, pts)
    ref = np.array([u[a, m // 16, m % 16] if u.ndim == 3 else u.reshape(-1, 256)[a, m] for a, m in sel])
    assert np.max(np.abs(up - ref)) < 1e-13 * np.max(np.abs(u))


def test_no_points(device):
    w = gen.config1(0)
    _, u, up, gp = _run(device, w, np.zeros((0, 2)))
    assert up.shape == (0,) and gp.shape == (0, 2) and np.all(np.isfinite(u))


def test_star_tree_at_curve_nodes(device):
    w = gen.config3(0, lcut=8)
    c = gen.star_curve(n_panels=56, order=24, scale=0.95)
    plan, _, up, gp = _run(device, w, c.nodes)
    assert plan.info()["pairs_points"] > 9 * c.n_nodes
    idx = np.random.default_rng(2).choice(c.n_nodes, 120, replace=False)
    u_o, g_o = _oracle(w, c.nodes[idx])
    assert rel_max_err(up[idx], u_o) < TOL
    assert rel_max_err(gp[idx], g_o) < TOL


def test_points_close_to_leaf_edges(device):
    # points at 1e-6 .. 1e-14 from leaf edges and corners: the moment quadrature refines deep
    # towards the neighbouring leaves' edges
    w = gen.random_small_tree(4, max_level=5, n_splits=9)
    rng = np.random.default_rng(4)
    s = 2.0 ** (-w.levels.astype(float))
    pts = []
    for d in (1e-6, 1e-9, 1e-12, 1e-14):
        for a in rng.choice(w.n_leaves, 6, replace=False):
            cx, cy, h = w.centres[a, 0], w.centres[a, 1], s[a]
            pts.append([cx + h - d, cy + 0.3 * h])       # inside, near the right edge
            pts.append([cx - 0.7 * h, cy - h + d])       # inside, near the bottom edge
            pts.append([cx + h - d, cy + h - d])         # inside, near the top-right corner
    pts = np.clip(np.array(pts), -1.0, 1.0)
    _, _, up, gp = _run(device, w, pts)
    u_o, g_o = _oracle(w, pts)
    assert rel_max_err(up, u_o) < TOL
    assert rel_max_err(gp, g_o) < TOL


def test_points_within_rounding_of_edges_and_subsquare_corners(device):
    # points 1e-16 .. 1e-15 from leaf edges and corners (both sides) and from the corners of the
    # dyadic sub-squares the moment quadrature refines towards (offsets 1/2, 1/4, 1/32 of a
    # half-width): the deepest refinements the moment kernel makes, all on the GPU
    w = gen.random_small_tree(2, max_level=5, n_splits=9)
    rng = np.random.default_rng(6)
    s = 2.0 ** (-w.levels.astype(float))
    pts = []
    for d in (1e-15, 3e-16, 1e-16):
        for a in rng.choice(w.n_leaves, 4, replace=False):
            cx, cy, h = w.centres[a, 0], w.centres[a, 1], s[a]
            for sgn in (-1.0, 1.0):
                pts.append([cx + h + sgn * d, cy + 0.3 * h])          # across the right edge
                pts.append([cx - h + sgn * d, cy - h + sgn * d])      # across the bottom-left corner
            for frac in (0.5, 0.25, 1.0 / 32.0):
                pts.append([cx + frac * h - d, cy + frac * h - d])    # beside a sub-square corner
                pts.append([cx - frac * h + d, cy + 0.6 * h])         # beside a sub-square edge
    pts = np.clip(np.array(pts), -1.0, 1.0)
    _, _, up, gp = _run(device, w, pts)
    u_o, g_o = _oracle(w, pts)
    assert rel_max_err(up, u_o) < TOL
    assert rel_max_err(gp, g_o) < TOL
