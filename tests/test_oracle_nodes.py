"""Pins for the oracle's leaf node convention (first-kind Chebyshev points, Fejer-1 weights)."""
import numpy as np

from oracle import nodes


def test_points_ascending_interior():
    t = nodes.cheb1_points(16)
    assert np.all(np.diff(t) > 0)
    assert np.isclose(t[0], -np.cos(np.pi / 32)) and np.isclose(t[-1], np.cos(np.pi / 32))


def test_fejer_exact_on_polynomials():
    # Fejer's first rule on p points integrates every polynomial of degree < p exactly.
    t, w = nodes.cheb1_points(16), nodes.fejer1_weights(16)
    for k in range(16):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, t ** k) - exact) < 1e-15
    assert abs(w.sum() - 2.0) < 1e-15
    assert np.all(w > 0)


def test_weights_are_integrals_of_lagrange_basis():
    gx, gw = np.polynomial.legendre.leggauss(32)
    L = nodes.lagrange_matrix(gx)
    assert np.max(np.abs(L @ gw - nodes.fejer1_weights(16))) < 1e-15


def test_lagrange_interpolates_and_partitions_unity():
    t = nodes.cheb1_points(16)
    assert np.max(np.abs(nodes.lagrange_matrix(t) - np.eye(16))) < 1e-14
    x = np.linspace(-1.3, 1.3, 41)
    assert np.max(np.abs(nodes.lagrange_matrix(x).sum(axis=0) - 1.0)) < 1e-11


def test_barycentric_matches_product_formula():
    t = nodes.cheb1_points(16)
    lam = nodes.barycentric_weights(16)
    x = np.array([-0.93, -0.2, 0.0123, 0.77])
    num = lam[:, None] / (x[None, :] - t[:, None])
    bary = num / num.sum(axis=0)
    assert np.max(np.abs(bary - nodes.lagrange_matrix(x))) < 1e-13


def test_interp_reproduces_polynomials():
    t = nodes.cheb1_points(16)
    X, Y = np.meshgrid(t, t, indexing="xy")
    f = (X ** 3 * Y - 2 * Y ** 5 + X ** 15).reshape(-1)
    xq = np.array([-0.5, 0.1, 0.9])
    yq = np.array([0.3, -0.8])
    F = nodes.interp_to_points(f, xq, yq)
    XQ, YQ = np.meshgrid(xq, yq, indexing="xy")
    assert np.max(np.abs(F - (XQ ** 3 * YQ - 2 * YQ ** 5 + XQ ** 15))) < 1e-13
