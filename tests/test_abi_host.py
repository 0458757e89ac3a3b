"""CPU-side checks of the C-ABI library: every declared symbol is exported, host validation
and error codes, and the host plan (lists, tables) against the oracle. No GPU calls."""
import os
import re

import numpy as np
import pytest

from oracle import nodes as onodes
from oracle import quad, tree
from workloads import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def vp():
    from paper_2501_17967_amd import volpot

    if not os.path.exists(volpot.LIB_PATH):
        from paper_2501_17967_amd import build

        build.build()
    volpot.lib()
    return volpot


def test_header_symbols_are_exported(vp):
    hdr = open(os.path.join(ROOT, "include", "volpot.h")).read()
    names = sorted(set(re.findall(r"\b(volpot_[a-z_]+)\s*\(", hdr)))
    assert len(names) >= 13
    L = vp.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(vp.EXPORTED) == names


def test_nodes_match_oracle_convention(vp):
    t, w = vp.nodes(16)
    assert np.max(np.abs(t - onodes.cheb1_points(16))) < 1e-15
    assert np.max(np.abs(w - onodes.fejer1_weights(16))) < 1e-15


def _tree_arrays(keys):
    keys = sorted(keys)
    cen = [(-1 + (2 * x + 1) * 2.0 ** -l, -1 + (2 * y + 1) * 2.0 ** -l) for l, x, y in keys]
    return np.array(cen), np.array([k[0] for k in keys], dtype=np.int32)


def test_validate_tree_status_codes(vp):
    c, l = _tree_arrays(gen.uniform_tree(2))
    assert vp.validate_tree(c, l) == (vp.OK, -1)
    rc, bad = vp.validate_tree(c[1:], l[1:])  # gap
    assert rc == vp.ERR_TREE
    c2 = c.copy()
    c2[3, 0] += 0.01  # off grid
    rc, bad = vp.validate_tree(c2, l)
    assert rc == vp.ERR_TREE and bad == 3
    c3 = np.vstack([c, [[-0.875, -0.875]]])  # overlap with a level-3 leaf
    l3 = np.concatenate([l, [3]])
    assert vp.validate_tree(c3, l3)[0] == vp.ERR_TREE
    # unbalanced: level 3 next to level 1
    leaves = {(1, 1, 0), (1, 0, 1), (1, 1, 1), (2, 0, 0), (2, 1, 0), (2, 0, 1)} | {(3, x, y) for x in (2, 3) for y in (2, 3)}
    c4, l4 = _tree_arrays(leaves)
    assert vp.validate_tree(c4, l4)[0] == vp.ERR_UNBALANCED
    l5 = l.copy()
    l5[0] = 31
    assert vp.validate_tree(c, l5)[0] in (vp.ERR_TREE, vp.ERR_UNSUPPORTED)
    c6 = c.copy()
    c6[0, 0] = np.nan
    assert vp.validate_tree(c6, l)[0] == vp.ERR_TREE
    assert vp.validate_tree(c, l, p=8)[0] == vp.ERR_UNSUPPORTED


def test_plan_errors(vp):
    c, l = _tree_arrays(gen.uniform_tree(1))
    with pytest.raises(vp.VolpotError) as e:
        vp.Plan(c, l, p=12, host_only=True)
    assert e.value.code == vp.ERR_UNSUPPORTED
    with pytest.raises(vp.VolpotError) as e:
        vp.Plan(c[:3], l[:3], host_only=True)
    assert e.value.code == vp.ERR_TREE


@pytest.fixture(scope="module")
def host_plan(vp):
    w = gen.config1(0)
    return vp.Plan(w.centres, w.levels, host_only=True)


def test_host_only_plan_refuses_apply(vp, host_plan):
    L = vp.lib()
    import ctypes

    rc = L.volpot_apply(host_plan._h, ctypes.c_void_p(16), ctypes.c_void_p(32), None)
    assert rc == vp.ERR_STATE


def test_near_tables_agree_with_oracle(vp, host_plan):
    # two independent quadratures (polar/graded in the library, subdivision in the oracle)
    OT = quad.near_tables()
    worst = 0.0
    for r in range(33):
        ro = quad.relation_index(*vp.near_relation(r))
        assert ro >= 0
        worst = max(worst, np.max(np.abs(host_plan.table(0, r) - OT[ro])))
    assert worst < 1e-14


def test_low_rank_near_factors_reproduce_oracle_tables(vp, host_plan):
    # the factors the near field applies for every relation but the self one: U_r has k_r
    # orthonormal columns (pivoted QR), the rest zero, and U_r V_r stays within the tables' own
    # quadrature error of the oracle's independently integrated tables. k_r is 48 for a corner
    # neighbour or a coarser one, 64 for an edge neighbour of the same size or finer
    OT = quad.near_tables()
    worst = 0.0
    for r in range(1, 33):
        U, V = host_plan.table(3, r), host_plan.table(4, r)
        k = int(np.sum(np.any(U != 0.0, axis=0)))
        dx, dy, rho = vp.near_relation(r)
        assert k == (48 if rho > 1 or (abs(dx) > 1 and abs(dy) > 1) else 64), (r, k)
        assert np.all(U[:, k:] == 0.0) and np.all(V[k:] == 0.0)
        assert np.max(np.abs(U[:, :k].T @ U[:, :k] - np.eye(k))) < 1e-13
        worst = max(worst, np.max(np.abs(U @ V - OT[quad.relation_index(*vp.near_relation(r))])))
    assert worst < 1e-14
    with pytest.raises(vp.VolpotError):
        host_plan.table(3, 0)  # the self relation is applied dense


@pytest.mark.parametrize("seed", range(2))
def test_pair_stages_take_every_adjacent_pair_once(vp, seed):
    # every adjacent pair other than a leaf with itself is one row of exactly one pair stage,
    # the one of its relation's rank, forward (V_r: the R factor, row i zero in its first i
    # pivot columns) and adjoint (U_r^T, dense); the plan's flops count the non-zeros
    w = gen.random_small_tree(seed, max_level=6, n_splits=14)
    T = tree.Tree(w.centres, w.levels)
    U = T.lists()[0]  # each leaf's adjacent leaves, itself included
    plan = vp.Plan(w.centres, w.levels, host_only=True)
    n_pairs = sum(len(v) - 1 for v in U.values())
    assert plan.info()["pairs_lowrank"] == n_pairs
    for adj, kind in ((False, "nearc"), (True, "adj_nearc")):
        got = 0
        for s in plan.stages(adj):
            if s["kind"] != kind:
                continue
            k = s["rows"]
            assert (s["name"].endswith("48")) == (k == 48) and k in (48, 64), s
            nnz = 256 * k if adj else 256 * k - k * (k - 1) // 2
            c = s["flops"] / (2.0 * nnz)
            assert abs(c - round(c)) < 1e-9, s
            got += int(round(c))
        assert got == n_pairs
    plan.close()


def test_s2m_and_l2t_reproduce_definitions(vp, host_plan):
    # S2M row 0 is the leaf mass weights W; rows 2, 3 (n = 1) are -int l_k eta_x, -int l_k eta_y
    W = onodes.tensor_weights()
    S = host_plan.table(1)
    assert np.max(np.abs(S[0] - W)) < 1e-15 and np.max(np.abs(S[1])) == 0.0
    gx, gw = np.polynomial.legendre.leggauss(32)
    L = onodes.lagrange_matrix(gx)
    m0, m1 = L @ gw, L @ (gw * gx)  # exact 1D moments of each L_i
    assert np.max(np.abs(S[2] + np.outer(m0, m1).reshape(-1))) < 1e-15  # index [j, i]
    assert np.max(np.abs(S[3] + np.outer(m1, m0).reshape(-1))) < 1e-15
    t = onodes.cheb1_points()
    X, Y = np.meshgrid(t, t, indexing="xy")
    Lt = host_plan.table(2)
    assert np.allclose(Lt[:, 0], -1 / (2 * np.pi)) and np.allclose(Lt[:, 2], -X.reshape(-1) / (2 * np.pi))


@pytest.mark.parametrize("seed", range(4))
def test_pair_counts_match_oracle_lists(vp, seed):
    w = gen.random_small_tree(seed, max_level=5, n_splits=9)
    T = tree.Tree(w.centres, w.levels)
    U, V, W, X = T.lists()
    inf = vp.Plan(w.centres, w.levels, host_only=True).info()
    assert inf["pairs_near"] == sum(len(v) for v in U.values())
    assert inf["pairs_v"] == sum(len(v) for v in V.values())
    assert inf["pairs_w"] == sum(len(v) for v in W.values())
    assert inf["pairs_x"] == sum(len(v) for v in X.values())


def test_forest_pair_counts_add_up(vp):
    ws = [gen.random_small_tree(s, max_level=4, n_splits=5) for s in range(3)]
    infs = [vp.Plan(w.centres, w.levels, host_only=True).info() for w in ws]
    off = np.cumsum([0] + [w.n_leaves for w in ws])
    f = vp.Plan(np.vstack([w.centres for w in ws]), np.concatenate([w.levels for w in ws]), tree_offsets=off,
                host_only=True).info()
    for k in ("pairs_near", "pairs_v", "pairs_w", "pairs_x", "n_boxes", "n_leaves"):
        assert f[k] == sum(i[k] for i in infs), k
    assert abs(f["flops_total"] - sum(i["flops_total"] for i in infs)) < 1e-6 * f["flops_total"]


@pytest.mark.parametrize("split_min", [0, 1, 3, -1])
def test_schedules_cover_stages(vp, split_min):
    # host-only plans schedule for a nominal 1024 resident blocks; the library checks each
    # schedule chunk by chunk when it builds it, these are the counts seen from outside
    w = gen.config2(0)
    plan = vp.Plan(w.centres, w.levels, host_only=True, split_min=split_min)
    for adj in (False, True):
        for s in plan.stages(adj):
            if s["n_tiles"] == 0:
                continue
            chunks = s["inner"] // s["kchunk"]  # k-chunks of the widest segment (one if factored)
            assert chunks * s["kchunk"] == s["inner"], s
            assert s["n_chunks"] <= s["n_segments"] * chunks, s
            # every tile here has at least one segment; its fixed cost counts as that many more
            units = s["n_chunks"] + s["n_tiles"] * chunks
            if split_min == -1:
                assert s["n_blocks"] == s["n_tiles"] and s["n_split_tiles"] == 0, s
            else:
                mu = split_min if split_min > 0 else chunks
                assert s["n_blocks"] == min(1024, -(-units // mu)), s
                # each boundary between consecutive blocks cuts at most one tile
                assert s["n_split_tiles"] <= s["n_blocks"] - 1 or s["n_split_tiles"] == 0, s
            assert s["flops_issued"] >= s["flops"] * (1 - 1e-12) or s["rows"] == 256 and s["kchunk"] == 16, s


def test_deterministic_plans_cut_no_tile(vp):
    # deterministic = 1: every tile belongs to one block (no arrival counters), whatever
    # split_min asks for
    w = gen.config2(0)
    for split_min in (0, 1):
        plan = vp.Plan(w.centres, w.levels, host_only=True, split_min=split_min, deterministic=True)
        for adj in (False, True):
            for s in plan.stages(adj):
                if s["n_tiles"]:
                    assert s["n_blocks"] == s["n_tiles"] and s["n_split_tiles"] == 0, s
        plan.close()


def test_overlap_launch_order(vp):
    # Dense near field: with overlap it is cut in two launches, each placed beside one far-field
    # chain (helper stream), and the leaf stage runs last. Low-rank near field: the leaf stage is
    # folded into its one launch, which runs last, and its two pair stages (V_r f~ / U_r^T u~ by
    # rank) run beside the chains. Every stage still comes after the stages it reads
    w = gen.config2(0)
    for dense in (True, False):
        for overlap in (0, 16):
            plan = vp.Plan(w.centres, w.levels, host_only=True, overlap=overlap, dense_near=dense)
            for adj, (head, up, near, far, down, tail) in (
                    (False, ("S2M", "M2M", "NEAR", ("FARV", "FARX"), "L2L", "LOCT")),
                    (True, ("AL2T", "AL2L", "ANEAR", ("AFARV", "AFARW"), "AM2M", "ALOCT"))):
                names = [s["name"] for s in plan.stages(adj)]
                helper = [s["name"] for s in plan.stages(adj) if s["helper"]]
                chains = [n for n in names if n.startswith(up + "[") or n.startswith(down + "[")]
                assert names[0] == head
                assert set(helper) == set(chains + ([far[1]] if dense else []))
                i_far = names.index(far[0])
                assert all(names.index(n) < i_far for n in names if n.startswith(up + "["))
                # S2L / M2T^T comes right after M2L, before the downward chain
                assert names.index(far[-1]) == i_far + 1
                assert all(names.index(n) > names.index(far[-1]) for n in names if n.startswith(down + "["))
                pre = [n for n in names if n.startswith(near + "C")]
                nears = [n for n in names if n.startswith(near) and n not in pre]
                if dense:
                    assert pre == [] and names[-1] == tail
                    if overlap:
                        assert nears == [near + "_A", near + "_B"]
                        assert names.index(near + "_A") < i_far < names.index(near + "_B") < len(names) - 1
                    else:
                        assert nears == [near]
                else:
                    assert nears == [near + "+" + tail] and names[-1] == nears[0] and tail not in names
                    # the rank-64 pair stage beside the upward chain, the rank-48 one beside the
                    # downward chain
                    assert pre == [near + "C", near + "C48"]
                    assert names.index(pre[0]) < i_far < names.index(far[-1]) < names.index(pre[1])
                    assert all(names.index(n) < names.index(pre[1]) for n in names if n.startswith(down + "["))
            plan.close()


# ---------------------------------------------------------------- layer potentials (host side)
def _circle_nodes(R, m, c=(0.0, 0.0)):
    th = 2 * np.pi * np.arange(m) / m
    y = np.stack([c[0] + R * np.cos(th), c[1] + R * np.sin(th)], axis=1)
    return y, np.full(m, 2 * np.pi * R / m), np.stack([np.cos(th), np.sin(th)], axis=1)


def _leaf_of_point(T, x, y):
    """The leaf holding (x, y): half-open boxes [lo, hi), the root's right / top edge included."""
    for l in range(T.max_level + 1):
        n = 1 << l
        ix = min(int(np.floor((x + 1.0) * n / 2.0)), n - 1)
        iy = min(int(np.floor((y + 1.0) * n / 2.0)), n - 1)
        if (l, ix, iy) in T.leaf_of:
            return (l, ix, iy)
    raise AssertionError("point not covered")


@pytest.mark.parametrize("seed", range(3))
def test_layer_plan_counts_match_oracle_lists(vp, seed):
    w = gen.random_small_tree(seed, max_level=5, n_splits=9)
    # a circle through box edges and corners (nodes at angles k pi / 2 sit on x = 0.5 or y = 0.5)
    y, wt, nrm = _circle_nodes(0.5, 64)
    c = gen.star_curve(n_panels=8, order=6, scale=0.6, seed=seed)
    y = np.vstack([y, c.nodes]); wt = np.concatenate([wt, c.weights]); nrm = np.vstack([nrm, c.normals])
    plan = vp.LayerPlan(w.centres, w.levels, y, wt, nrm, host_only=True)
    inf = plan.info()
    T = tree.Tree(w.centres, w.levels)
    U, V, W, X = T.lists()
    count = {}
    for (px, py) in y:
        k = _leaf_of_point(T, px, py)
        count[k] = count.get(k, 0) + 1
    active = set()
    for k in count:
        l, x, yy = k
        while True:
            active.add((l, x, yy))
            if l == 0:
                break
            l, x, yy = l - 1, x >> 1, yy >> 1
    assert inf["n_layer_nodes"] == len(y)
    assert inf["n_source_leaves"] == len(count)
    assert inf["n_active_boxes"] == len(active)
    assert inf["pairs_p2p"] == 256 * sum(count.get(b, 0) for a in U for b in U[a])
    assert inf["pairs_p2l"] == sum(count.get(a, 0) for cbox in X for a in X[cbox])
    names = [s["name"] for s in plan.stages(False)]
    assert plan.stages(True) == []
    assert names[0] == "P2M" and names[-2:] == ["LOCT", "P2P"]  # the direct sum adds onto LOCT
    assert not any(n in ("S2M", "NEAR", "FARX") for n in names)
    i_far = names.index("FARV")
    assert names.index("P2L") == i_far + 1
    p2p = [s for s in plan.stages(False) if s["name"] == "P2P"][0]
    assert p2p["n_tiles"] == sum(1 for a in U if any(count.get(b, 0) for b in U[a]))
    assert all(names.index(n) < i_far for n in names if n.startswith("M2M["))
    assert all(names.index(n) > i_far + 1 for n in names if n.startswith("L2L["))
    # only active boxes are multipole sources: M2L work is that of the active V pairs (each a
    # real 80 x 80 matrix with at least half its entries non-zero, plus one log term)
    farv = [s for s in plan.stages(False) if s["name"] == "FARV"]
    n_v_active = sum(1 for b in V for s in V[b] if s in active)
    if farv:
        assert 2 * 3200 * n_v_active <= farv[0]["flops"] <= 2 * (6400 + 1) * n_v_active


def test_layer_plan_errors(vp):
    w = gen.config1(0)
    y, wt, nrm = _circle_nodes(0.5, 16)
    for bad in ((1.5, 0.0), (np.nan, 0.0), (0.0, -1.000001)):
        yb = y.copy()
        yb[3] = bad
        with pytest.raises(vp.VolpotError) as e:
            vp.LayerPlan(w.centres, w.levels, yb, wt, nrm, host_only=True)
        assert e.value.code == vp.ERR_ARG
    nb = nrm.copy()
    nb[5, 1] = np.inf
    with pytest.raises(vp.VolpotError):
        vp.LayerPlan(w.centres, w.levels, y, wt, nb, host_only=True)
    with pytest.raises(ValueError):
        vp.LayerPlan(w.centres, w.levels, y, wt[:-1], nrm, host_only=True)
    # nodes on the root's edges and corners belong to the boxes inside; no nodes at all is valid
    edge = np.array([[1.0, 1.0], [-1.0, -1.0], [1.0, 0.0], [0.0, -1.0]])
    p = vp.LayerPlan(w.centres, w.levels, edge, np.ones(4), np.tile([[1.0, 0.0]], (4, 1)), host_only=True)
    assert p.info()["n_source_leaves"] == 4
    p0 = vp.LayerPlan(w.centres, w.levels, np.zeros((0, 2)), np.zeros(0), np.zeros((0, 2)), host_only=True)
    assert p0.info()["n_active_boxes"] == 0 and p0.info()["pairs_p2p"] == 0
    # host-only plans refuse to apply; the arguments are checked first (pointers never dereferenced)
    import ctypes
    L = vp.lib()
    a16, b16 = ctypes.c_void_p(256), ctypes.c_void_p(512)
    assert L.volpot_layer_apply(p._h, a16, a16, b16, None) == vp.ERR_STATE
    assert L.volpot_layer_apply(p._h, None, a16, b16, None) == vp.ERR_ARG
    assert L.volpot_layer_apply(p._h, a16, a16, ctypes.c_void_p(520 + 4), None) == vp.ERR_ARG
    assert L.volpot_apply(p._h, a16, b16, None) == vp.ERR_STATE
    assert L.volpot_layer_apply(p0._h, None, None, b16, None) == vp.ERR_STATE  # no nodes: no densities needed


# ---------------------------------------------------------------- evaluation points (host side)
def test_point_plan_counts_and_errors(vp):
    w = gen.random_small_tree(4, max_level=5, n_splits=8)
    rng = np.random.default_rng(0)
    pts = np.vstack([rng.uniform(-1, 1, (30, 2)), [[0.5, 0.5], [1.0, 1.0], [-1.0, 0.25], [0.0, 0.0]]])
    plan = vp.PointPlan(w.centres, w.levels, pts, host_only=True)
    inf = plan.info()
    T = tree.Tree(w.centres, w.levels)
    U, V, W, X = T.lists()
    assert inf["n_points"] == len(pts)
    assert inf["pairs_points"] == sum(len(U[_leaf_of_point(T, x, y)]) for x, y in pts)
    # it is a full volume plan
    assert [s["name"] for s in plan.stages(False)][0] == "S2M" and plan.stages(True)
    for bad in ((1.0000001, 0.0), (np.nan, 0.2)):
        with pytest.raises(vp.VolpotError) as e:
            vp.PointPlan(w.centres, w.levels, np.vstack([pts, [bad]]), host_only=True)
        assert e.value.code == vp.ERR_ARG
    assert vp.PointPlan(w.centres, w.levels, np.zeros((0, 2)), host_only=True).info()["pairs_points"] == 0


# ---------------------------------------------------------------- quadtree builder (host side)
def test_tree_builder_arguments(vp):
    import ctypes
    L = vp.lib()
    h = ctypes.c_void_p()
    assert L.volpot_tree_create(16, 0.0, 1.0, 0, 10, ctypes.byref(h)) == vp.ERR_ARG
    assert L.volpot_tree_create(16, 1e-10, 1.0, 5, 4, ctypes.byref(h)) == vp.ERR_ARG
    assert L.volpot_tree_create(12, 1e-10, 1.0, 0, 10, ctypes.byref(h)) == vp.ERR_UNSUPPORTED
    assert L.volpot_tree_create(16, 1e-10, 1.0, 13, 20, ctypes.byref(h)) == vp.ERR_UNSUPPORTED
    assert L.volpot_tree_create(16, 1e-10, 1.0, 3, 10, ctypes.byref(h)) == vp.OK
    n = ctypes.c_int64(0)
    assert L.volpot_tree_pending(h, ctypes.byref(n)) == vp.OK and n.value == 64  # the level-3 boxes
    assert L.volpot_tree_leaves(h, ctypes.byref(n), None, None) == vp.ERR_STATE  # boxes still pending
    L.volpot_tree_destroy(h)


def test_strip_plan_arguments(vp):
    import ctypes
    L = vp.lib()
    h = ctypes.c_void_p()
    g = np.zeros((4, 8, 2))
    p = g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.volpot_strip_plan(2, 8, p, p, 12, 10, ctypes.byref(h)) == vp.ERR_ARG   # too few panels
    assert L.volpot_strip_plan(4, 8, p, p, 3, 10, ctypes.byref(h)) == vp.ERR_ARG    # q too small
    assert L.volpot_strip_plan(4, 8, p, p, 32, 33, ctypes.byref(h)) == vp.ERR_ARG   # n_r too large
    # a strip of zero width (Gamma~ = Gamma): the interfaces have zero length, rejected on the host
    th = np.linspace(0, 2 * np.pi, 33)[:32].reshape(4, 8)
    g[...] = np.stack([np.cos(th), np.sin(th)], axis=2)
    assert L.volpot_strip_plan(4, 8, p, p, 12, 10, ctypes.byref(h)) == vp.ERR_ARG
    g[1, 2, 0] = np.nan
    assert L.volpot_strip_plan(4, 8, p, p, 12, 10, ctypes.byref(h)) == vp.ERR_ARG   # non-finite node


def test_root_box_option_maps_the_tree(vp):
    # a tree given in the caller's coordinates of a moved and scaled root box plans to the same
    # lists as the reference tree; an invalid half-width is rejected
    w = gen.config1(0)
    c, h = np.array([0.3, -1.7]), 2.5
    ref = vp.Plan(w.centres, w.levels, host_only=True).info()
    got = vp.Plan(c + h * w.centres, w.levels, host_only=True, root_centre=c, root_halfwidth=h).info()
    for k in ("n_leaves", "n_boxes", "pairs_near", "pairs_v", "pairs_w", "pairs_x", "flops_total"):
        assert got[k] == ref[k], k
    # the reference centres are off the moved root's grid
    with pytest.raises(vp.VolpotError) as e:
        vp.Plan(w.centres, w.levels, host_only=True, root_centre=c, root_halfwidth=h)
    assert e.value.code == vp.ERR_TREE
    for bad in (-1.0, float("inf"), float("nan")):
        with pytest.raises(vp.VolpotError) as e:
            vp.Plan(w.centres, w.levels, host_only=True, root_halfwidth=bad)
        assert e.value.code == vp.ERR_ARG


_TABLE_SCRIPT = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[3])
from paper_2501_17967_amd import volpot as vp
from workloads import gen
w = gen.config1(0)
p = vp.Plan(w.centres, w.levels, host_only=True, table_cache=sys.argv[1])
np.save(sys.argv[2], np.stack([p.table(0, r) for r in (0, 5, 20, 32)]))
"""


def test_corrupt_table_cache_is_rejected_and_rewritten(tmp_path):
    # the near tables are cached on disk with a magic, a shape header and a hash of the data; a
    # cache whose data or length do not match is not used: the tables are computed again (in a
    # fresh process, since a process computes them once) and the file rewritten
    import subprocess
    import sys

    cache = tmp_path / "cache"
    cache.mkdir()

    def run(tag):
        out = tmp_path / ("t_%s.npy" % tag)
        subprocess.run([sys.executable, "-c", _TABLE_SCRIPT, str(cache), str(out), ROOT], check=True, timeout=300)
        return np.load(out)

    ref = run("first")
    (f,) = list(cache.iterdir())
    good = f.read_bytes()
    assert good[:8] == b"VPNEAR01"
    bad = bytearray(good)
    bad[len(bad) // 2] ^= 0x40  # one flipped bit in the data
    f.write_bytes(bytes(bad))
    assert np.array_equal(run("flipped"), ref)
    assert f.read_bytes() == good
    f.write_bytes(good[: len(good) // 3])  # truncated
    assert np.array_equal(run("truncated"), ref)
    assert f.read_bytes() == good
