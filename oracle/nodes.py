"""Leaf node convention (oracle side; test infrastructure only).

Sec. 4.2.1 ("Constructing a quadtree approximation to f") puts an order-p tensor
Chebyshev approximation of f on every leaf, with p = 16 in all the paper's examples.
The paper does not say which Chebyshev points carry the samples; we read it as p points
of the first kind per dimension (interior points, no shared-edge duplicates):

    t_i = -cos((2i - 1) pi / (2p)),  i = 1..p   (ascending)

and the tensor index m = j*p + i with the x index i fastest. The weights w_i are those
of the interpolatory rule on these points (Fejer's first rule), i.e. w_i = int L_i, the
integral over [-1,1] of the i-th Lagrange basis polynomial.

Everything here is written from those definitions: Lagrange polynomials by their product
formula, weights by Fejer's closed form. Pinned by tests/test_oracle_nodes.py
(exactness on polynomials of degree < p, agreement with NumPy's Legendre quadrature of
each L_i, partition of unity).
"""
import numpy as np

P_DEFAULT = 16


def cheb1_points(p=P_DEFAULT):
    """First-kind Chebyshev points on [-1,1], ascending."""
    i = np.arange(1, p + 1)
    return -np.cos((2 * i - 1) * np.pi / (2 * p))


def fejer1_weights(p=P_DEFAULT):
    """Fejer first-rule weights for the points of ``cheb1_points`` (same order).

    For x_k = cos(theta_k), theta_k = (2k-1) pi/(2p):
        w_k = (2/p) [1 - 2 sum_{j=1}^{floor(p/2)} cos(2 j theta_k) / (4 j^2 - 1)].
    The weights are symmetric, so the ascending reordering leaves them unchanged.
    """
    k = np.arange(1, p + 1)
    theta = (2 * k - 1) * np.pi / (2 * p)
    s = np.zeros(p)
    for j in range(1, p // 2 + 1):
        s += np.cos(2 * j * theta) / (4 * j * j - 1)
    w = (2.0 / p) * (1.0 - 2.0 * s)
    return w[::-1].copy()


def lagrange_matrix(x, p=P_DEFAULT):
    """L[i, q] = L_i(x_q) for the Lagrange basis on ``cheb1_points(p)`` (product formula)."""
    t = cheb1_points(p)
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    L = np.ones((p, x.size))
    for i in range(p):
        for j in range(p):
            if j != i:
                L[i] *= (x - t[j]) / (t[i] - t[j])
    return L


def barycentric_weights(p=P_DEFAULT):
    """lambda_i = 1 / prod_{j != i} (t_i - t_j)  (plain definition)."""
    t = cheb1_points(p)
    lam = np.ones(p)
    for i in range(p):
        for j in range(p):
            if j != i:
                lam[i] /= (t[i] - t[j])
    return lam


def tensor_weights(p=P_DEFAULT):
    """W[j*p + i] = w_i w_j : the integral over [-1,1]^2 of the tensor basis l_{j*p+i}."""
    w = fejer1_weights(p)
    return np.outer(w, w).reshape(-1)


def leaf_nodes(centre, halfwidth, p=P_DEFAULT):
    """Physical node coordinates of one leaf, shape (p*p, 2), x fastest."""
    t = cheb1_points(p)
    X, Y = np.meshgrid(t, t, indexing="xy")  # X[j, i] = t_i, Y[j, i] = t_j
    return np.stack([centre[0] + halfwidth * X.reshape(-1), centre[1] + halfwidth * Y.reshape(-1)], axis=1)


def interp_to_points(fvals, xq, yq, p=P_DEFAULT):
    """Evaluate the tensor interpolant of nodal values (p*p, x fastest) on the grid xq x yq.

    Returns F[b, a] = f_h(xq[a], yq[b]).
    """
    F = np.asarray(fvals).reshape(p, p)  # F[j, i]
    Lx = lagrange_matrix(xq, p)  # (p, na)
    Ly = lagrange_matrix(yq, p)  # (p, nb)
    return Ly.T @ F @ Lx
