"""GPU tests of the root-box option (volpot_options.root_centre / root_halfwidth, Sec. 4.2.1: the
root box B_0 holds the domain). With y = c + h eta and x = c + h xi, the log kernel gives
    u(x) = h^2 (u_ref(xi) - (1/2pi) ln h M),   M = sum_b s_b^2 sum_k W_k f_b,k,
where u_ref is the potential of the same nodal values on the reference tree ([-1,1]^2) and M their
integral there; the operator is A = h^2 (A_ref - (1/2pi) ln h 1 m^T) with m_(b,k) = s_b^2 W_k, so
the adjoint is A^T r = h^2 (A_ref^T r - (1/2pi) ln h m (1^T r)), and at points the gradient is
h grad_xi u_ref. The identity is exact; both sides round, so the bar is the method's 1e-11. The
layer potentials at physical curve nodes are checked against the oracle's direct sum.
"""
import numpy as np
import pytest

from oracle import layer as olayer
from oracle import nodes
from tests.conftest import rel_max_err
from workloads import gen

pytestmark = pytest.mark.gpu
TOL = 1e-11
C, H = np.array([0.3, -1.7]), 2.5


def _mass_vector(levels):
    return nodes.tensor_weights()[None, :] * (2.0 ** (-2 * np.asarray(levels, dtype=float)))[:, None]


def test_moved_and_scaled_root_forward_and_adjoint(device):
    import torch

    from paper_2501_17967_amd import Plan

    w = gen.config2(0)
    print("root case: config2 (%d leaves), centre %s, half-width %g" % (w.n_leaves, C, H), flush=True)
    r = np.random.default_rng(3).standard_normal(w.f.shape)
    f, rd = torch.from_numpy(w.f).to(device), torch.from_numpy(r).to(device)
    ref = Plan(w.centres, w.levels)
    u0, a0 = ref.apply(f).cpu().numpy(), ref.apply_adjoint(rd).cpu().numpy()
    ref.close()
    phys = Plan(C + H * w.centres, w.levels, root_centre=C, root_halfwidth=H)
    u1, a1 = phys.apply(f).cpu().numpy(), phys.apply_adjoint(rd).cpu().numpy()
    phys.close()
    m = _mass_vector(w.levels)
    k = np.log(H) / (2 * np.pi)
    assert rel_max_err(u1, H * H * (u0 - k * np.sum(m * w.f))) <= TOL
    assert rel_max_err(a1, H * H * (a0 - k * m * np.sum(r))) <= TOL


def test_forest_with_a_moved_root(device):
    import torch

    from paper_2501_17967_amd import Plan

    ws = [gen.random_small_tree(s, max_level=5, n_splits=8) for s in range(3)] + [gen.config1(1)]
    off = np.cumsum([0] + [x.n_leaves for x in ws])
    F = np.vstack([x.f for x in ws])
    Cc = np.vstack([x.centres for x in ws])
    Lv = np.concatenate([x.levels for x in ws])
    print("root case: forest of %d trees, half-width 0.125" % len(ws), flush=True)
    Fd = torch.from_numpy(F).to(device)
    ref = Plan(Cc, Lv, tree_offsets=off)
    u0 = ref.apply(Fd).cpu().numpy()
    ref.close()
    h, c = 0.125, np.array([-4.0, 7.5])
    phys = Plan(c + h * Cc, Lv, tree_offsets=off, root_centre=c, root_halfwidth=h, use_graph=True)
    u1 = phys.apply(Fd).cpu().numpy()
    phys.close()
    m = _mass_vector(Lv)
    k = np.log(h) / (2 * np.pi)
    for t in range(len(ws)):
        sl = slice(off[t], off[t + 1])
        assert rel_max_err(u1[sl], h * h * (u0[sl] - k * np.sum(m[sl] * F[sl]))) <= TOL, t


def test_points_with_a_moved_root(device):
    import torch

    from paper_2501_17967_amd import PointPlan

    w = gen.random_small_tree(4, max_level=5, n_splits=9)
    pts = np.random.default_rng(8).uniform(-1, 1, (40, 2))
    print("root case: %d points, centre %s, half-width %g" % (len(pts), C, H), flush=True)
    f = torch.from_numpy(w.f).to(device)
    ref = PointPlan(w.centres, w.levels, pts)
    _, p0, g0 = ref.apply_points(f)
    p0, g0 = p0.cpu().numpy(), g0.cpu().numpy()
    ref.close()
    phys = PointPlan(C + H * w.centres, w.levels, C + H * pts, root_centre=C, root_halfwidth=H)
    _, p1, g1 = phys.apply_points(f)
    p1, g1 = p1.cpu().numpy(), g1.cpu().numpy()
    phys.close()
    M = np.sum(_mass_vector(w.levels) * w.f)
    assert rel_max_err(p1, H * H * (p0 - np.log(H) / (2 * np.pi) * M)) <= TOL
    assert rel_max_err(g1, H * g0) <= TOL


def test_layer_potentials_with_a_moved_root(device):
    import torch

    from paper_2501_17967_amd import LayerPlan

    w = gen.random_small_tree(1, max_level=5, n_splits=9)
    c = gen.star_curve(n_panels=16, order=16, scale=0.9)
    y, wt = C + H * c.nodes, H * c.weights  # arc length scales with the curve
    print("root case: layer potentials, %d curve nodes, half-width %g" % (c.n_nodes, H), flush=True)
    lp = LayerPlan(C + H * w.centres, w.levels, y, wt, c.normals, root_centre=C, root_halfwidth=H)
    v = lp.apply(torch.from_numpy(c.sigma).to(device), torch.from_numpy(c.tau).to(device)).cpu().numpy()
    lp.close()
    targets = C + H * olayer.leaf_targets(w.centres, w.levels)
    ref = olayer.layer_potential(targets, y, wt, c.normals, c.sigma, c.tau)
    assert rel_max_err(v.reshape(-1), ref) <= TOL
