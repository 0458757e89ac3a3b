"""GPU strip solve (volpot_strip_*, Sec. 4.3) against the strip oracle (dense assembly and direct
solve of the same collocation system) and against manufactured solutions.

Tolerances. Both sides solve the same discrete system in FP64 after equilibrating its rows (the
oracle divides every row by its 1-norm; the factored solve scales the PDE and derivative rows);
the row-scaled system has condition numbers of 1e2 .. 3e2 on these cases, and a replica of the
factored solve in host FP64 agrees with the oracle to 2e-14 .. 7e-14. The bar is the box code's,
1e-11 relative max-norm. At the 56-element, 24 x 16 size the oracle's dense solve takes tens of
seconds, so there the test checks what a backward-stable solve guarantees at any size: the
row-scaled backward error max_i |(A v - b)_i| / |A_i|_1 / |v|_inf against the oracle's assembled
matrix, bar 1e-12 (the host replica gives 2.5e-14), and a manufactured solution on a 56-element
annulus of the same resolution.
"""
import numpy as np
import pytest

from oracle import strip
from tests.conftest import rel_max_err
from workloads import gen

pytestmark = pytest.mark.gpu


def _annulus(n_panel, n_gl, R):
    s, _ = np.polynomial.legendre.leggauss(n_gl)
    h = np.pi / n_panel
    th = (2 * h * np.arange(n_panel))[:, None] + h * (s[None, :] + 1)
    return np.stack([R * np.cos(th), R * np.sin(th)], axis=2)


def _run(device, g, gt, f, q, n_r):
    import torch

    from paper_2501_17967_amd import StripPlan

    print("strip case: %d panels, q %d, n_r %d" % (g.shape[0], q, n_r), flush=True)
    sp = StripPlan(g, gt, q, n_r)
    fv = torch.from_numpy(f(sp.nodes.reshape(-1, 2))).to(device)
    v = sp.apply(fv)
    torch.cuda.synchronize()
    return sp, v.cpu().numpy()


def test_annulus_manufactured_and_oracle(device):
    from tests.test_oracle_strip import _manufactured

    a, b = 0.75, 0.9
    v_exact, f = _manufactured(a, b)
    g, gt = _annulus(12, 16, b), _annulus(12, 16, a)
    sp, v = _run(device, g, gt, f, 16, 10)
    ref, X = strip.solve(g, gt, f, q=16, n_r=10)
    assert np.max(np.abs(sp.nodes - X)) < 1e-14
    assert rel_max_err(v, ref) < 1e-11
    ve = v_exact(X.reshape(-1, 2)).reshape(v.shape)
    assert rel_max_err(v, ve) < 1e-11


@pytest.mark.parametrize("n_panel,q,n_r", [(16, 12, 8), (7, 16, 12), (24, 10, 16), (5, 8, 32), (9, 20, 4)])
def test_star_strip_vs_oracle(device, n_panel, q, n_r):
    # strip between the star and the star pulled inwards, a smooth f
    c_out = gen.star_curve(n_panels=n_panel, order=16, scale=1.0)
    c_in = gen.star_curve(n_panels=n_panel, order=16, scale=0.93)
    g = c_out.nodes.reshape(n_panel, 16, 2)
    gt = c_in.nodes.reshape(n_panel, 16, 2)
    f = lambda p: np.sin(3 * p[:, 0]) * np.exp(p[:, 1]) + 0.5
    _, v = _run(device, g, gt, f, q, n_r)
    ref, _ = strip.solve(g, gt, f, q=q, n_r=n_r)
    assert rel_max_err(v, ref) < 1e-11


def test_repeat_is_deterministic(device):
    import torch

    from paper_2501_17967_amd import StripPlan

    g, gt = _annulus(9, 16, 0.9), _annulus(9, 16, 0.8)
    sp = StripPlan(g, gt, 12, 10)
    f = torch.from_numpy(np.cos(sp.nodes[..., 0]) * sp.nodes[..., 1]).to(device)
    a = sp.apply(f).cpu().numpy()
    b = sp.apply(f).cpu().numpy()
    assert np.array_equal(a, b)


def test_full_size_backward_error(device):
    # the 56-element strip at 24 (along) x 16 (across), the size the benchmark times
    n = 56
    g = gen.star_curve(n_panels=n, order=16, scale=1.0).nodes.reshape(n, 16, 2)
    gt = gen.star_curve(n_panels=n, order=16, scale=0.93).nodes.reshape(n, 16, 2)
    f = lambda p: np.sin(3 * p[:, 0]) * np.exp(p[:, 1]) + 0.5
    sp, v = _run(device, g, gt, f, 24, 16)
    X = strip.element_grids(g, gt, 24, 16)
    assert np.max(np.abs(sp.nodes - X)) < 1e-14
    A, pde = strip.assemble(X)
    b = np.where(pde, f(X.reshape(-1, 2)), 0.0)
    x = v.reshape(-1)
    bwd = np.max(np.abs(A @ x - b) / np.abs(A).sum(axis=1)) / np.max(np.abs(x))
    assert bwd < 1e-12, bwd


def test_full_size_annulus_manufactured(device):
    from tests.test_oracle_strip import _manufactured

    a, b = 0.85, 0.9
    v_exact, f = _manufactured(a, b)
    g, gt = _annulus(56, 16, b), _annulus(56, 16, a)
    sp, v = _run(device, g, gt, f, 24, 16)
    ve = v_exact(sp.nodes.reshape(-1, 2)).reshape(v.shape)
    assert rel_max_err(v, ve) < 1e-11


def test_maximum_size_annulus(device):
    # the largest element the library takes: q = n_r = 32 (interior block 960 x 960, m = 30)
    from tests.test_oracle_strip import _manufactured

    a, b = 0.8, 0.9
    v_exact, f = _manufactured(a, b)
    g, gt = _annulus(4, 16, b), _annulus(4, 16, a)
    sp, v = _run(device, g, gt, f, 32, 32)
    ref, X = strip.solve(g, gt, f, q=32, n_r=32)
    assert rel_max_err(v, ref) < 1e-11
    assert rel_max_err(v, v_exact(X.reshape(-1, 2)).reshape(v.shape)) < 1e-11
