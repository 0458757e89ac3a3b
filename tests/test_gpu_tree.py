"""GPU quadtree construction (volpot_tree_*) against the oracle builder (oracle/quadtree.py):
the balanced leaf sets must be identical (bit-exact integer result).

Both sides sample f in FP64 with NumPy at their own node coordinates and decide each box in FP64
(the Chebyshev transform in a different summation order). A decision can only differ when a
tail lies within a few units in the last place of eps * scale, which for these continuous
random sources does not happen; a mismatch would show as a different leaf set.
"""
import numpy as np
import pytest

from oracle import quadtree as qt
from workloads import gen

pytestmark = pytest.mark.gpu


def _gauss_f(g):
    def f(p):
        out = np.zeros(p.shape[0])
        for c, s, a in zip(g.centres, g.sigmas, g.amps):
            out += a * np.exp(-((p[:, 0] - c[0]) ** 2 + (p[:, 1] - c[1]) ** 2) / (2 * s * s))
        return out
    return f


def _gpu_build(f, eps, scale, min_level, max_level):
    import torch

    from paper_2501_17967_amd import build_tree

    def f_dev(nodes):
        return torch.from_numpy(f(nodes.cpu().numpy())).to(nodes.device)

    c, l = build_tree(f_dev, eps, scale, min_level, max_level)
    s = 2.0 ** (-l.astype(float))
    ix = np.round((c[:, 0] + 1) / (2 * s) - 0.5).astype(int)
    iy = np.round((c[:, 1] + 1) / (2 * s) - 0.5).astype(int)
    return {(int(a), int(b), int(d)) for a, b, d in zip(l, ix, iy)}, c, l


@pytest.mark.parametrize("seed,min_level", [(0, 0), (1, 0), (2, 4)])
def test_tree_matches_oracle(device, seed, min_level):
    rng = np.random.default_rng(seed)
    g = gen.sample_gaussians(rng, 6, -0.9, 0.9, 5e-3, 1e-1)
    f = _gauss_f(g)
    print("tree case: seed %d, min level %d" % (seed, min_level), flush=True)
    got, c, l = _gpu_build(f, 1e-10, g.scale, min_level, 14)
    ref = qt.build(f, 1e-10, g.scale, min_level, 14)
    assert got == set(ref)
    # the result is a valid plan input, and ordered by level, then y, then x
    from paper_2501_17967_amd import validate_tree
    assert validate_tree(c, l)[0] == 0
    keys = [(int(a), float(y), float(x)) for a, (x, y) in zip(l, c)]
    assert keys == sorted(keys)


def test_unresolvable_source_stops_at_max_level(device):
    # a discontinuous source never resolves along its jump: refinement stops at max_level
    f = lambda p: (p[:, 0] > 0.1234).astype(float)
    got, _, _ = _gpu_build(f, 1e-10, 1.0, 0, 7)
    assert got == set(qt.build(f, 1e-10, 1.0, 0, 7))
    assert max(k[0] for k in got) == 7


def test_polynomial_source_is_one_box(device):
    f = lambda p: 1.0 + p[:, 0] ** 3 * p[:, 1] ** 5
    got, _, _ = _gpu_build(f, 1e-12, 1.0, 0, 10)
    assert got == {(0, 0, 0)}


@pytest.mark.parametrize("centre", [(0.37, -0.61), (-0.999, 0.999)])
def test_deep_point_source_needs_many_balance_rounds(device, centre):
    # a near-singular source d^2 / (|x - c|^2 + d^2), d = 1e-5, refines down to level 18 around
    # one point (next to a corner of the root for the second case): the 2:1 balance ripples
    # outwards over many levels
    d2 = 1e-10
    f = lambda p: d2 / ((p[:, 0] - centre[0]) ** 2 + (p[:, 1] - centre[1]) ** 2 + d2)
    print("tree case: point source at %s" % (centre,), flush=True)
    got, c, l = _gpu_build(f, 1e-10, 1.0, 0, 24)
    ref = qt.build(f, 1e-10, 1.0, 0, 24)
    assert got == set(ref)
    assert max(k[0] for k in got) >= 15
    from paper_2501_17967_amd import validate_tree
    assert validate_tree(c, l)[0] == 0


def test_size_matched_tree_matches_the_generator(device):
    # the benchmark's size-matched 20-Gaussian tree (background level 7, about 17k leaves)
    rng = np.random.default_rng(0)
    g = gen.sample_gaussians(rng, 20, -0.9, 0.9, 1e-3, 1e-1)
    print("tree case: size-matched 20-Gaussian tree", flush=True)
    got, _, _ = _gpu_build(_gauss_f(g), 1e-11, g.scale, 7, 24)
    w = gen.config2(0, size_matched=True)
    s = 2.0 ** (-w.levels.astype(float))
    ref = {(int(a), int(x), int(y)) for a, x, y in zip(w.levels, np.round((w.centres[:, 0] + 1) / (2 * s) - 0.5),
                                                        np.round((w.centres[:, 1] + 1) / (2 * s) - 0.5))}
    assert got == ref
