"""Pins for the oracle's near tables and log-kernel integrals (quad.py / _quad.c)."""
import numpy as np
import pytest
from scipy import integrate

from oracle import closed_forms as cf
from oracle import nodes, quad

T1 = nodes.cheb1_points()
XX, YY = np.meshgrid(T1, T1, indexing="xy")
XI = XX.reshape(-1)
ETA = YY.reshape(-1)


@pytest.fixture(scope="module")
def tables():
    return quad.near_tables()


def test_row_sums_equal_square_closed_form(tables):
    # sum_k T_r[m,k] * 1 is the potential of a uniform source on the source box, in target
    # half-widths, divided by rho^2 (the table integrates over the reference square).
    for r, (dx, dy, rho) in enumerate(quad.near_relations()):
        ref = cf.square_potential(XI, ETA, dx - rho, dx + rho, dy - rho, dy + rho) / rho ** 2
        assert np.max(np.abs(tables[r].sum(axis=1) - ref)) < 5e-15, (dx, dy, rho)


def _lag1(i, x):
    v = 1.0
    for j in range(16):
        if j != i:
            v *= (x - T1[j]) / (T1[i] - T1[j])
    return v


def _entry_by_quadpack(dx, dy, rho, m, k):
    xm, ym = XI[m], ETA[m]
    i, j = k % 16, k // 16
    # integrate over the physical source box in target units, then divide by rho^2
    g = lambda t, s: -np.log(np.hypot(xm - s, ym - t)) / (2 * np.pi) * _lag1(i, (s - dx) / rho) * _lag1(j, (t - dy) / rho)
    a1, b1, a2, b2 = dx - rho, dx + rho, dy - rho, dy + rho
    xs = sorted({a1, b1} | ({xm} if a1 < xm < b1 else set()))
    ys = sorted({a2, b2} | ({ym} if a2 < ym < b2 else set()))
    tot = 0.0
    for xa, xb in zip(xs[:-1], xs[1:]):
        for ya, yb in zip(ys[:-1], ys[1:]):
            tot += integrate.dblquad(g, xa, xb, ya, yb, epsabs=1e-15, epsrel=1e-12)[0]
    return tot / rho ** 2


@pytest.mark.parametrize("rel,m,k", [((0.0, 0.0, 1.0), 37, 200), ((2.0, 0.0, 1.0), 15, 16),
                                     ((-1.5, 0.5, 0.5), 16 * 7, 3), ((3.0, -3.0, 2.0), 15, 255),
                                     ((0.0, -2.0, 1.0), 5, 5 + 16)])
def test_single_entries_match_quadpack(tables, rel, m, k):
    r = quad.relation_index(*rel)
    ref = _entry_by_quadpack(*rel, m, k)
    assert abs(tables[r][m, k] - ref) < 2e-13 * max(1.0, abs(ref))


def _perm(fn):
    idx = np.arange(256)
    i, j = idx % 16, idx // 16
    i2, j2 = fn(i, j)
    return j2 * 16 + i2


def test_d4_symmetry_between_relations(tables):
    # reflections x->-x, y->-y and the swap x<->y map the geometry onto itself: the tables of
    # mapped relations are the originals with rows and columns permuted alike.
    ops = [
        (lambda i, j: (15 - i, j), lambda dx, dy: (-dx, dy)),
        (lambda i, j: (i, 15 - j), lambda dx, dy: (dx, -dy)),
        (lambda i, j: (j, i), lambda dx, dy: (dy, dx)),
    ]
    for pm, pd in ops:
        perm = _perm(pm)
        for r, (dx, dy, rho) in enumerate(quad.near_relations()):
            r2 = quad.relation_index(*pd(dx, dy), rho)
            assert r2 >= 0
            A = tables[r]
            B = tables[r2][np.ix_(perm, perm)]
            assert np.max(np.abs(A - B)) < 2e-15


def test_logint_far_point_is_point_mass_limit():
    # far away, int log|x0 - eta| l_k = W_k log|x0| + O(1/|x0|) (multipole expansion)
    x0 = np.array([[1e8, 3e8]])
    I = quad.logint(x0)[0]
    W = nodes.tensor_weights()
    assert np.max(np.abs(I - W * np.log(np.hypot(1e8, 3e8)))) < 1e-8
