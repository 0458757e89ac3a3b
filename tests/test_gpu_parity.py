"""GPU parity: the HIP box code (through the C ABI) against the CPU oracle.

Tolerance: relative max-norm error <= 1e-11 (rel err = max|u_gpu - u_ref| / max|u_ref|), the
bar for the FP64 path. Both sides truncate expansions (GPU order 39, oracle order 50) far below
it; near tables come from two independent quadratures that agree to ~1e-16.
"""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import fmm, nodes, quad, tree
from workloads import gen

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def vp():
    from paper_2501_17967_amd import volpot

    volpot.lib()
    return volpot


def _gpu(torch_mod, a):
    return torch_mod.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _run(vp, torch_mod, w, adjoint_input=None, **kw):
    plan = vp.Plan(w.centres, w.levels, **kw)
    u = plan.apply(_gpu(torch_mod, w.f)).cpu().numpy()
    fb = None
    if adjoint_input is not None:
        fb = plan.apply_adjoint(_gpu(torch_mod, adjoint_input)).cpu().numpy()
    plan.close()
    return u, fb


# ------------------------------------------------------------------------ forward
def test_config1_forward_vs_direct_sum(vp, torch_mod):
    w = gen.config1(0)
    _say("case config1 seed 0 (64 leaves)")
    u, _ = _run(vp, torch_mod, w)
    ud = quad.direct_potential(tree.Tree(w.centres, w.levels), w.f)
    assert rel(u, ud) <= TOL


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_config1_seeds_vs_box_code_oracle(vp, torch_mod, seed):
    w = gen.config1(seed)
    _say("case config1 seed %d" % seed)
    r = np.random.default_rng(seed).standard_normal(w.f.shape)
    u, fb = _run(vp, torch_mod, w, adjoint_input=r)
    bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
    assert rel(u, bc.apply(w.f)) <= TOL
    assert rel(fb, bc.apply_adjoint(r)) <= TOL


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_random_adaptive_trees_forward_and_adjoint(vp, torch_mod, seed):
    # small random balanced trees in shuffled caller order: every list type, ragged tiles
    w = gen.random_small_tree(seed, max_level=6, n_splits=12)
    _say("case random tree seed %d (%d leaves)" % (seed, w.n_leaves))
    r = np.random.default_rng(10 + seed).standard_normal(w.f.shape)
    u, fb = _run(vp, torch_mod, w, adjoint_input=r)
    bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
    assert rel(u, bc.apply(w.f)) <= TOL
    assert rel(fb, bc.apply_adjoint(r)) <= TOL


def test_config2_forward_and_adjoint_vs_box_code_oracle(vp, torch_mod):
    w = gen.config2(0)
    _say("case config2 seed 0 (%d leaves)" % w.n_leaves)
    r = np.random.default_rng(7).standard_normal(w.f.shape)
    u, fb = _run(vp, torch_mod, w, adjoint_input=r)
    bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
    assert rel(u, bc.apply(w.f)) <= TOL
    assert rel(fb, bc.apply_adjoint(r)) <= TOL


def test_config2_forward_sampled_vs_direct_sum(vp, torch_mod):
    w = gen.config2(1)
    _say("case config2 seed 1 sampled direct (%d leaves)" % w.n_leaves)
    u, _ = _run(vp, torch_mod, w)
    rng = np.random.default_rng(3)
    samples = [(int(a), int(m)) for a, m in zip(rng.integers(0, w.n_leaves, 48), rng.integers(0, 256, 48))]
    ud = quad.direct_potential(tree.Tree(w.centres, w.levels), w.f, samples)
    ug = np.array([u[a, m] for a, m in samples])
    assert np.max(np.abs(ug - ud)) / np.max(np.abs(u)) <= TOL


def test_size_matched_config2_sampled_vs_direct_sum(vp, torch_mod):
    # the benchmark workload (about 20k leaves), in the launch configuration bench.py times
    w = gen.config2(0, size_matched=True)
    _say("case config2-sm seed 0 sampled direct (%d leaves)" % w.n_leaves)
    u, _ = _run(vp, torch_mod, w)
    rng = np.random.default_rng(5)
    samples = [(int(a), int(m)) for a, m in zip(rng.integers(0, w.n_leaves, 32), rng.integers(0, 256, 32))]
    ud = quad.direct_potential(tree.Tree(w.centres, w.levels), w.f, samples)
    ug = np.array([u[a, m] for a, m in samples])
    assert np.max(np.abs(ug - ud)) / np.max(np.abs(u)) <= TOL


@pytest.mark.parametrize("seed", [0, 3, 5, 6, 9])
def test_config1_against_gaussian_closed_form(vp, torch_mod, seed):
    # analysis check: the closed-form whole-plane potential minus the part of each Gaussian
    # outside the root (both pinned on the CPU). Widths 0.11-0.3 are resolved at level 3 to about
    # 1e-15, so the oracle box code meets the closed form to 2e-15 on these seeds; the GPU adds
    # its own rounding only.
    w = gen.config1(seed)
    u, _ = _run(vp, torch_mod, w)
    rng = np.random.default_rng(2)
    g = w.src
    errs = []
    for a, m in zip(rng.integers(0, w.n_leaves, 6), rng.integers(0, 256, 6)):
        x, y = nodes.leaf_nodes(w.centres[a], 2.0 ** -w.levels[a])[m]
        ref = 0.0
        for (cx, cy), s, A in zip(g.centres, g.sigmas, g.amps):
            ref += cf.gaussian_potential(x, y, cx, cy, s, A) - cf.gaussian_exterior_tail(x, y, cx, cy, s, A)
        errs.append(abs(u[a, m] - ref))
    err = max(errs) / np.max(np.abs(u))
    _say("case config1 seed %d closed form: max rel err %.2e (min sigma %.3f)" % (seed, err, g.sigmas.min()))
    assert err <= 1e-13


# ------------------------------------------------------------------------ invariants
def test_dot_product_transpose(vp, torch_mod):
    w = gen.config2(2)
    _say("case dot product config2 seed 2")
    plan = vp.Plan(w.centres, w.levels)
    rng = np.random.default_rng(4)
    f = rng.standard_normal(w.f.shape)
    r = rng.standard_normal(w.f.shape)
    Af = plan.apply(_gpu(torch_mod, f)).cpu().numpy()
    Atr = plan.apply_adjoint(_gpu(torch_mod, r)).cpu().numpy()
    plan.close()
    lhs, rhs = np.sum(Af * r), np.sum(f * Atr)
    assert abs(lhs - rhs) / (np.linalg.norm(Af) * np.linalg.norm(r)) < 1e-13


def test_bitwise_determinism(vp, torch_mod):
    w = gen.config2(0)
    _say("case determinism")
    plan = vp.Plan(w.centres, w.levels)
    f = _gpu(torch_mod, w.f)
    a = plan.apply(f).cpu().numpy()
    b = plan.apply(f).cpu().numpy()
    c = plan.apply_adjoint(f).cpu().numpy()
    d = plan.apply_adjoint(f).cpu().numpy()
    plan.close()
    assert np.array_equal(a, b) and np.array_equal(c, d)


def test_forest_equals_single_tree_applies(vp, torch_mod):
    ws = [gen.random_small_tree(s, max_level=5, n_splits=8) for s in range(4)] + [gen.config1(0)]
    _say("case forest of %d trees" % len(ws))
    off = np.cumsum([0] + [w.n_leaves for w in ws])
    F = np.vstack([w.f for w in ws])
    forest = vp.Plan(np.vstack([w.centres for w in ws]), np.concatenate([w.levels for w in ws]), tree_offsets=off)
    u = forest.apply(_gpu(torch_mod, F)).cpu().numpy()
    fb = forest.apply_adjoint(_gpu(torch_mod, F)).cpu().numpy()
    forest.close()
    # per target the relation order is the same in both plans; only the points where the
    # balanced schedule cuts a tile (and so the grouping of partial sums) differ
    for t, w in enumerate(ws):
        us, fs = _run(vp, torch_mod, w, adjoint_input=w.f)
        assert rel(u[off[t]:off[t + 1]], us) <= 1e-14
        assert rel(fb[off[t]:off[t + 1]], fs) <= 1e-14


@pytest.mark.parametrize("split_min", [1, 3])
def test_split_schedules_agree_and_repeat(vp, torch_mod, split_min):
    # split_min = 1 cuts almost every tile of every stage over several blocks, exercising the
    # partial-sum hand-off; the result must not depend on which block finishes last
    w = gen.config2(0)
    _say("case split schedule split_min=%d" % split_min)
    f = _gpu(torch_mod, w.f)
    base = vp.Plan(w.centres, w.levels)
    ref, refa = base.apply(f).cpu().numpy(), base.apply_adjoint(f).cpu().numpy()
    base.close()
    plan = vp.Plan(w.centres, w.levels, split_min=split_min)
    first = None
    for _ in range(4):
        u, ua = plan.apply(f).cpu().numpy(), plan.apply_adjoint(f).cpu().numpy()
        if first is None:
            first = (u, ua)
            assert rel(u, ref) <= 1e-14 and rel(ua, refa) <= 1e-14
        else:
            assert np.array_equal(u, first[0]) and np.array_equal(ua, first[1])
    plan.close()


@pytest.mark.parametrize("tile_leaf,tile_box,split_min,tile_leaf_exp,kchunk_leaf,overlap",
                         [(64, 64, 0, 64, 32, 16), (64, 16, 1, 32, 32, 16), (32, 32, 0, 64, 32, 8),
                          (32, 32, 1, 32, 32, 8), (32, 32, 0, 16, 16, 0), (64, 32, 1, 16, 16, 0),
                          (32, 16, 0, 16, 16, 16)])
def test_tile_shapes_vs_box_code_oracle(vp, torch_mod, tile_leaf, tile_box, split_min, tile_leaf_exp, kchunk_leaf,
                                        overlap):
    # 64-slot near-field tiles, near-field k-chunks of 16, and 32- and 64-slot tiles of the leaf
    # stages that read expansions run in instantiations of their own, with and without the
    # overlapped streams; every stage against the oracle, and repeat applies bitwise
    w = gen.config2(0)
    _say("case tile_leaf=%d tile_box=%d split_min=%d tile_leaf_exp=%d kchunk_leaf=%d overlap=%d (%d leaves)"
         % (tile_leaf, tile_box, split_min, tile_leaf_exp, kchunk_leaf, overlap, w.n_leaves))
    r = np.random.default_rng(29).standard_normal(w.f.shape)
    plan = vp.Plan(w.centres, w.levels, tile_leaf=tile_leaf, tile_box=tile_box, split_min=split_min,
                   tile_leaf_exp=tile_leaf_exp, kchunk_leaf=kchunk_leaf, overlap=overlap)
    f, rd = _gpu(torch_mod, w.f), _gpu(torch_mod, r)
    u, fb = plan.apply(f).cpu().numpy(), plan.apply_adjoint(rd).cpu().numpy()
    u2, fb2 = plan.apply(f).cpu().numpy(), plan.apply_adjoint(rd).cpu().numpy()
    plan.close()
    bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
    assert rel(u, bc.apply(w.f)) <= TOL
    assert rel(fb, bc.apply_adjoint(r)) <= TOL
    assert np.array_equal(u, u2) and np.array_equal(fb, fb2)


def test_deterministic_option_matches_default(vp, torch_mod):
    # no cut tiles (no atomics): the same map, another summation order; repeatable bit for bit
    w = gen.config3(0)
    _say("case deterministic option, %d leaves" % w.n_leaves)
    f = _gpu(torch_mod, w.f)
    r = _gpu(torch_mod, np.random.default_rng(5).standard_normal(w.f.shape))
    out = {}
    for det in (False, True):
        plan = vp.Plan(w.centres, w.levels, deterministic=det)
        assert all(s["n_split_tiles"] == 0 for s in plan.stages() + plan.stages(adjoint=True)) or not det
        u1, a1 = plan.apply(f).cpu().numpy(), plan.apply_adjoint(r).cpu().numpy()
        u2, a2 = plan.apply(f).cpu().numpy(), plan.apply_adjoint(r).cpu().numpy()
        assert np.array_equal(u1, u2) and np.array_equal(a1, a2)
        out[det] = (u1, a1)
        plan.close()
    assert rel(out[True][0], out[False][0]) <= 1e-14 and rel(out[True][1], out[False][1]) <= 1e-13


@pytest.mark.parametrize("overlap", [0, 16])
def test_low_rank_near_matches_dense_near(vp, torch_mod, overlap):
    # the default near field applies rank-64 factors of the non-self tables; dense_near applies
    # the 256 x 256 tables. Same map to the factors' accuracy, forward and adjoint, with the near
    # field in one launch or cut in two around the far field
    w = gen.config3(0)
    _say("case low-rank vs dense near field, overlap %d, %d leaves" % (overlap, w.n_leaves))
    f = _gpu(torch_mod, w.f)
    r = _gpu(torch_mod, np.random.default_rng(6).standard_normal(w.f.shape))
    out = {}
    for dense in (False, True):
        plan = vp.Plan(w.centres, w.levels, dense_near=dense, overlap=overlap)
        names = [s["name"] for s in plan.stages() + plan.stages(adjoint=True)]
        assert all(n in names for n in ("NEARC", "NEARC48", "ANEARC", "ANEARC48")) != dense
        assert (plan.info()["pairs_lowrank"] > 0) != dense
        out[dense] = (plan.apply(f).cpu().numpy(), plan.apply_adjoint(r).cpu().numpy())
        plan.close()
    assert rel(out[False][0], out[True][0]) <= 1e-13 and rel(out[False][1], out[True][1]) <= 1e-13


def test_graph_replays_match_eager(vp, torch_mod):
    w = gen.config2(0)
    _say("case graph replay")
    eager = vp.Plan(w.centres, w.levels)
    graph = vp.Plan(w.centres, w.levels, use_graph=True)
    f = _gpu(torch_mod, w.f)
    ref = eager.apply(f).cpu().numpy()
    refa = eager.apply_adjoint(f).cpu().numpy()
    out = torch_mod.empty_like(f)
    outa = torch_mod.empty_like(f)
    for rep in range(3):
        graph.apply(f, out=out)
        graph.apply_adjoint(f, out=outa)
        torch_mod.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref)
        assert np.array_equal(outa.cpu().numpy(), refa)
        eager.apply(f)  # eager work between replays
        torch_mod.cuda.synchronize()
    eager.close()
    graph.close()


def _deep_tree(depth, point=(0.0013, -0.0021)):
    leaves = {(1, x, y) for x in (0, 1) for y in (0, 1)}
    for lev in range(1, depth):
        k = (lev, int((point[0] + 1) / 2 * (1 << lev)), int((point[1] + 1) / 2 * (1 << lev)))
        leaves.remove(k)
        leaves |= {(lev + 1, 2 * k[1] + a, 2 * k[2] + b) for a in (0, 1) for b in (0, 1)}
        leaves = gen.balance(leaves)
    return leaves


@pytest.mark.parametrize("case", ["root", "level1", "deep12", "deep20"])
def test_edge_trees(vp, torch_mod, case):
    # root-only leaf (no far field), the four level-1 leaves, deep thin refinements
    leaves = {"root": {(0, 0, 0)}, "level1": gen.uniform_tree(1), "deep12": _deep_tree(12),
              "deep20": _deep_tree(20)}[case]
    g = gen.Gaussians(np.array([[0.01, -0.02], [0.0011, -0.002]]), np.array([0.3, 2e-4]), np.array([1.0, -0.5]))
    w = gen.make_workload("edge-" + case, g, leaves, shuffle_seed=3)
    _say("case edge tree %s: %d leaves, max level %d" % (case, w.n_leaves, w.levels.max()))
    r = np.random.default_rng(1).standard_normal(w.f.shape)
    u, fb = _run(vp, torch_mod, w, adjoint_input=r)
    bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
    assert rel(u, bc.apply(w.f)) <= TOL
    assert rel(fb, bc.apply_adjoint(r)) <= TOL


def test_zero_input_gives_zero(vp, torch_mod):
    w = gen.config1(0)
    plan = vp.Plan(w.centres, w.levels)
    z = torch_mod.zeros((w.n_leaves, 256), dtype=torch_mod.float64, device="cuda:0")
    assert float(plan.apply(z).abs().max()) == 0.0
    assert float(plan.apply_adjoint(z).abs().max()) == 0.0
    plan.close()


# ------------------------------------------------------------------------ autograd
def test_autograd_gradient_matches_finite_differences(vp, torch_mod):
    # J(f) = 1/2 sum W s^2 (A f - u_t)^2 on the config-2 tree; dJ/df through the adjoint kernels.
    # J is quadratic, so central differences are exact up to rounding: about 1e-16 |J| / h, which
    # the oracle measures at 2.3e-8 |dJ.d| at worst over these ten directions.
    from paper_2501_17967_amd import volume_potential

    w, f2, dirs = gen.config5(n_dirs=10)
    assert len(dirs) == 10
    _say("case autograd FD (%d leaves, %d directions)" % (w.n_leaves, len(dirs)))
    plan = vp.Plan(w.centres, w.levels)
    Wq = _gpu(torch_mod, nodes.tensor_weights()[None, :] * (2.0 ** (-2 * w.levels.astype(float)))[:, None])
    ut = plan.apply(_gpu(torch_mod, f2))

    def J(fv):
        return 0.5 * torch_mod.sum(Wq * (volume_potential(fv, plan) - ut) ** 2)

    f = _gpu(torch_mod, w.f).requires_grad_(True)
    j = J(f)
    (g,) = torch_mod.autograd.grad(j, f)
    h = 1e-6
    worst = 0.0
    for d in dirs:
        dt = _gpu(torch_mod, d)
        with torch_mod.no_grad():
            fd = float((J(f + h * dt) - J(f - h * dt)) / (2 * h))
        an = float(torch_mod.sum(g * dt))
        worst = max(worst, abs(fd - an) / abs(an))
    _say("  FD vs autograd: max rel diff %.2e" % worst)
    assert worst <= 1e-7
    # against the oracle's transpose, applied to the GPU's own residual: grad = A^T (W s^2 (A f - u_t))
    with torch_mod.no_grad():
        resid_gpu = (Wq * (plan.apply(f.detach()) - ut)).cpu().numpy()
    bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
    assert rel(g.cpu().numpy(), bc.apply_adjoint(resid_gpu)) <= TOL
    # and with the residual formed by the oracle's forward (the residual is a difference of two
    # potentials, so its relative rounding is larger than theirs)
    resid = Wq.cpu().numpy() * (bc.apply(w.f) - ut.cpu().numpy())
    assert rel(g.cpu().numpy(), bc.apply_adjoint(resid)) <= 1e-10
    plan.close()


def test_autograd_through_a_forest_plan(vp, torch_mod):
    # the batched adjoint: one objective over a 24-tree slice of the forest workload, dJ/df
    # through the forest plan's adjoint; each tree's gradient against the oracle's transpose of
    # that tree, and a forest-wide central difference along a seeded direction
    from paper_2501_17967_amd import volume_potential

    trees = gen.config4(0, n_trees=24)
    off = np.cumsum([0] + [t.n_leaves for t in trees])
    _say("case autograd through a forest of %d trees (%d leaves)" % (len(trees), off[-1]))
    C = np.vstack([t.centres for t in trees])
    L = np.concatenate([t.levels for t in trees])
    forest = vp.Plan(C, L, tree_offsets=off)
    Wq = _gpu(torch_mod, nodes.tensor_weights()[None, :] * (2.0 ** (-2 * L.astype(float)))[:, None])
    rng = np.random.default_rng(41)
    ut = forest.apply(_gpu(torch_mod, np.roll(np.vstack([t.f for t in trees]), 7, axis=0)))
    f = _gpu(torch_mod, np.vstack([t.f for t in trees])).requires_grad_(True)

    def J(fv):
        return 0.5 * torch_mod.sum(Wq * (volume_potential(fv, forest) - ut) ** 2)

    (g,) = torch_mod.autograd.grad(J(f), f)
    with torch_mod.no_grad():
        resid = (Wq * (forest.apply(f.detach()) - ut)).cpu().numpy()
    gn = g.cpu().numpy()
    for i, t in enumerate(trees):
        bc = fmm.BoxCode(tree.Tree(t.centres, t.levels))
        assert rel(gn[off[i]:off[i + 1]], bc.apply_adjoint(resid[off[i]:off[i + 1]])) <= TOL, i
    d = rng.standard_normal(gn.shape)
    d /= np.max(np.abs(d))
    dt = _gpu(torch_mod, d)
    # J is quadratic, so the central difference is exact for any step up to rounding, which is
    # about 1e-16 |J| / h: a step of 1e-3 keeps it far below the bar for a random direction
    h = 1e-3
    with torch_mod.no_grad():
        fd = float((J(f + h * dt) - J(f - h * dt)) / (2 * h))
    an = float(np.sum(gn * d))
    _say("  forest FD vs autograd: rel diff %.2e" % (abs(fd - an) / abs(an)))
    assert abs(fd - an) <= 1e-7 * abs(an)
    forest.close()


def test_autotune_picks_a_valid_shape_and_caches(vp, torch_mod, tmp_path):
    w = gen.config2(0)
    _say("case autotune config2 seed 0")
    cache = str(tmp_path / "tune.txt")
    with open(cache, "w") as fh:  # lines that hold no valid shape are ignored, never taken
        fh.write("garbage\n0123456789abcdef 32 32 0 0 16\n")
    best, ms = vp.autotune(w.centres, w.levels, cache=cache)
    assert best["tile_leaf"] in (32, 64) and best["tile_box"] in (16, 32, 64) and best["split_min"] in (0, 1, -1)
    assert best["tile_leaf_exp"] in (16, 32, 64) and best["kchunk_leaf"] in (16, 32)
    assert ms > 0
    again, ms2 = vp.autotune(w.centres, w.levels, cache=cache)  # answered from the cache file
    assert again == best and abs(ms2 - ms) <= 1e-6 * ms
    lines = open(cache).read().splitlines()
    assert len(lines) == 3
    # a corrupted entry for this very key (a tile size the library does not have) is not taken:
    # the shape is timed again and a valid line appended
    key = lines[-1].split()[0]
    cache2 = str(tmp_path / "tune2.txt")
    with open(cache2, "w") as fh:
        fh.write("%s 48 32 0 0 16 32 0.5\n%s 32 32 0 0 16\n" % (key, key))
    again2, _ = vp.autotune(w.centres, w.levels, cache=cache2)
    assert again2["tile_leaf"] in (32, 64) and again2["tile_leaf_exp"] in (16, 32, 64)
    lines2 = open(cache2).read().splitlines()
    assert len(lines2) == 3 and lines2[-1].split()[0] == key
    ref, _ = _run(vp, torch_mod, w)
    u, _ = _run(vp, torch_mod, w, **best)
    assert rel(u, ref) <= 1e-14


def test_config3_forward_and_adjoint_vs_box_code_oracle(vp, torch_mod):
    # 200 Gaussians cut off outside the star curve, cut boxes refined to level 8 (about 9k leaves)
    w = gen.config3(0)
    _say("case config3 seed 0 (%d leaves)" % w.n_leaves)
    rng = np.random.default_rng(11)
    r = rng.standard_normal(w.f.shape)
    u, fb = _run(vp, torch_mod, w, adjoint_input=r)
    bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
    assert rel(u, bc.apply(w.f)) <= TOL
    assert rel(fb, bc.apply_adjoint(r)) <= TOL


@pytest.mark.timeout(400)
def test_size_matched_config3_sampled_vs_direct_sum(vp, torch_mod):
    # star-cut source with cut boxes refined to level 13: about 170k leaves, 43M unknowns
    w = gen.config3(0, lcut=13)
    _say("case config3-sm (lcut 13, %d leaves)" % w.n_leaves)
    u, _ = _run(vp, torch_mod, w)
    rng = np.random.default_rng(13)
    samples = [(int(a), int(m)) for a, m in zip(rng.integers(0, w.n_leaves, 16), rng.integers(0, 256, 16))]
    ud = quad.direct_potential(tree.Tree(w.centres, w.levels), w.f, samples)
    ug = np.array([u[a, m] for a, m in samples])
    assert np.max(np.abs(ug - ud)) / np.max(np.abs(u)) <= TOL


@pytest.mark.timeout(600)
def test_config4_full_forest_graph_vs_single_trees_and_oracle(vp, torch_mod):
    # the whole batched workload: 256 uneven trees (1-40 Gaussians, min level 3) in one forest
    # plan, graph-captured, forward and adjoint, against every tree's own single-tree apply and,
    # for ten trees (the smallest and the largest among them), against the oracle.
    # Forest and single-tree plans sum the same terms; they group them differently where the
    # balanced schedule cuts a tile between blocks (partial sums), and where the two-level chains
    # pair other levels (a forest pairs levels from its deepest tree down). The difference is
    # rounding: 1e-14 relative for the forward output, and 1e-13 for the adjoint of a random
    # cotangent, whose sums cancel (|result| ~ sqrt(terms) |term|).
    trees = gen.config4(0, n_trees=256)
    off = np.cumsum([0] + [t.n_leaves for t in trees])
    _say("case config4 full forest of %d trees (%d leaves)" % (len(trees), off[-1]))
    F = np.vstack([t.f for t in trees])
    R = np.random.default_rng(17).standard_normal(F.shape)
    C = np.vstack([t.centres for t in trees])
    L = np.concatenate([t.levels for t in trees])
    Fd, Rd = _gpu(torch_mod, F), _gpu(torch_mod, R)

    def forest_out(**kw):
        forest = vp.Plan(C, L, tree_offsets=off, **kw)
        u, fb = torch_mod.empty_like(Fd), torch_mod.empty_like(Fd)
        for _ in range(3):  # with use_graph the second and third calls replay the captured graphs
            forest.apply(Fd, out=u)
            forest.apply_adjoint(Rd, out=fb)
        torch_mod.cuda.synchronize()
        forest.close()
        return u.cpu().numpy(), fb.cpu().numpy()

    def singles_out(**kw):
        u, fb = np.empty_like(F), np.empty_like(F)
        for i, t in enumerate(trees):
            plan = vp.Plan(t.centres, t.levels, **kw)
            u[off[i]:off[i + 1]] = plan.apply(Fd[off[i]:off[i + 1]]).cpu().numpy()
            fb[off[i]:off[i + 1]] = plan.apply_adjoint(Rd[off[i]:off[i + 1]]).cpu().numpy()
            plan.close()
        return u, fb

    u, fb = forest_out(use_graph=True)
    us, fs = singles_out()
    ef = max(rel(u[off[i]:off[i + 1]], us[off[i]:off[i + 1]]) for i in range(len(trees)))
    ea = max(rel(fb[off[i]:off[i + 1]], fs[off[i]:off[i + 1]]) for i in range(len(trees)))
    _say("  graph-replayed forest vs single-tree applies: max rel diff forward %.2e adjoint %.2e" % (ef, ea))
    assert ef <= 1e-14 and ea <= 1e-13
    sizes = np.array([t.n_leaves for t in trees])
    order = np.argsort(sizes, kind="stable")
    pick = sorted({int(order[0]), int(order[-1])} | {int(order[k]) for k in np.linspace(1, 254, 8).astype(int)})
    assert len(pick) == 10
    for i in pick:
        t = trees[i]
        bc = fmm.BoxCode(tree.Tree(t.centres, t.levels))
        ef = rel(u[off[i]:off[i + 1]], bc.apply(t.f))
        ea = rel(fb[off[i]:off[i + 1]], bc.apply_adjoint(R[off[i]:off[i + 1]]))
        _say("  tree %d (%d leaves): forward %.2e adjoint %.2e vs oracle" % (i, t.n_leaves, ef, ea))
        assert ef <= TOL and ea <= TOL, i


def test_size_matched_config2_forward_and_adjoint_vs_box_code_oracle(vp, torch_mod):
    # the benchmark workload in full, in the launch configuration bench.py times
    w = gen.config2(0, size_matched=True)
    _say("case config2-sm seed 0 full oracle (%d leaves)" % w.n_leaves)
    rng = np.random.default_rng(19)
    r = rng.standard_normal(w.f.shape)
    u, fb = _run(vp, torch_mod, w, adjoint_input=r)
    bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
    assert rel(u, bc.apply(w.f)) <= TOL
    assert rel(fb, bc.apply_adjoint(r)) <= TOL


def test_size_matched_config2_in_the_benchmark_launch_shape(vp, torch_mod):
    # the benchmark workload in full, in the shape bench.py times (tiles 32 / 32, two near-field
    # launches beside the far-field chains with 32 compute units left to them)
    w = gen.config2(0, size_matched=True)
    _say("case config2-sm seed 0 full oracle, overlap 32 (%d leaves)" % w.n_leaves)
    r = np.random.default_rng(31).standard_normal(w.f.shape)
    u, fb = _run(vp, torch_mod, w, adjoint_input=r, tile_leaf=32, tile_box=32, split_min=0, overlap=32)
    bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
    assert rel(u, bc.apply(w.f)) <= TOL
    assert rel(fb, bc.apply_adjoint(r)) <= TOL


@pytest.mark.parametrize("overlap", [8, 32])
def test_overlapped_streams_match_single_stream(vp, torch_mod, overlap):
    # near field in two launches beside the far-field chains on a second stream: the same
    # per-target sums, cut differently between blocks; repeated applies agree bit for bit
    w = gen.config2(1)
    _say("case overlapped streams, %d compute units left to the chains" % overlap)
    r = np.random.default_rng(23).standard_normal(w.f.shape)
    u1, f1 = _run(vp, torch_mod, w, adjoint_input=r)
    plan = vp.Plan(w.centres, w.levels, overlap=overlap)
    f, rd = _gpu(torch_mod, w.f), _gpu(torch_mod, r)
    u2, f2 = plan.apply(f).cpu().numpy(), plan.apply_adjoint(rd).cpu().numpy()
    u3, f3 = plan.apply(f).cpu().numpy(), plan.apply_adjoint(rd).cpu().numpy()
    plan.close()
    assert rel(u2, u1) <= 1e-14 and rel(f2, f1) <= 1e-14
    assert np.array_equal(u2, u3) and np.array_equal(f2, f3)


def test_graph_replays_with_overlap_match_eager(vp, torch_mod):
    # captured applies that fork to and join from the helper stream, replayed with other work
    # in between, against eager applies of a single-stream plan
    w = gen.config2(0)
    _say("case graph replay with overlap")
    f = _gpu(torch_mod, w.f)
    eager = vp.Plan(w.centres, w.levels)
    ref, refa = eager.apply(f).cpu().numpy(), eager.apply_adjoint(f).cpu().numpy()
    graph = vp.Plan(w.centres, w.levels, use_graph=True, overlap=32)
    out, outa = torch_mod.empty_like(f), torch_mod.empty_like(f)
    for rep in range(3):
        graph.apply(f, out=out)
        graph.apply_adjoint(f, out=outa)
        torch_mod.cuda.synchronize()
        assert rel(out.cpu().numpy(), ref) <= 1e-14 and rel(outa.cpu().numpy(), refa) <= 1e-14
        eager.apply(f)
        torch_mod.cuda.synchronize()
    eager.close()
    graph.close()
