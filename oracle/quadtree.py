"""Adaptive quadtree construction and 2:1 balance (oracle; test infrastructure only).

Sec. 4.2.1 (Alg. 2) builds the quadtree from a root box B_0 by splitting a box into four while
the order-p Chebyshev coefficients of f on it do not decay below the tolerance, and finishes
with a 2:1 balance so that neighbouring leaves differ by at most one level. The paper does not
fix the decay test; the reading used throughout (C6) is: a box is resolved when

    max { |c_nm| : n >= p - 2 or m >= p - 2 } <= eps * scale,

c_nm the tensor Chebyshev coefficients of the box's samples (n in y, m in x) and scale a global
magnitude of f supplied by the caller. Boxes above ``min_level`` are split unconditionally and
boxes at ``max_level`` are leaves. Balance: neighbours over edges and corners (C7).

Written from those definitions: the coefficients by the discrete Chebyshev transform of values
at the first-kind points, c_m = (2 - delta_m0)/p sum_i f(t_i) T_m(t_i), T_m(t) = cos(m arccos t);
the balance by splitting any leaf that has a neighbouring leaf two or more levels finer, until
none does. ``balance_brute`` checks every pair of leaves; ``balance`` finds neighbours through a
dictionary of keys and is pinned against the brute-force version on small trees.
Pinned by tests/test_oracle_quadtree.py.
"""
import numpy as np


def cheb_points(p=16):
    i = np.arange(1, p + 1)
    return -np.cos((2 * i - 1) * np.pi / (2 * p))


def transform_matrix(p=16):
    """D[m, i] = (2 - delta_m0)/p T_m(t_i): values at cheb_points -> Chebyshev coefficients."""
    t = cheb_points(p)
    D = np.empty((p, p))
    for m in range(p):
        for i in range(p):
            D[m, i] = (2.0 - (m == 0)) / p * np.cos(m * np.arccos(t[i]))
    return D


def coefficients(values, p=16):
    """c[n, m] of a box's samples values[j*p + i] = f(x_i, y_j) (x fastest)."""
    D = transform_matrix(p)
    V = np.asarray(values, dtype=np.float64).reshape(p, p)  # V[j, i]
    return D @ V @ D.T  # [n(y), m(x)]


def tail(values, p=16):
    c = np.abs(coefficients(values, p))
    return max(np.max(c[p - 2:, :]), np.max(c[:, p - 2:]))


def box_nodes(key, p=16):
    """(p*p, 2) node coordinates of box (l, ix, iy) on the root [-1,1]^2, x fastest."""
    l, ix, iy = key
    s = 2.0 ** (-l)
    cx, cy = -1.0 + (2 * ix + 1) * s, -1.0 + (2 * iy + 1) * s
    t = cheb_points(p)
    X, Y = np.meshgrid(t, t, indexing="xy")
    return np.stack([cx + s * X.reshape(-1), cy + s * Y.reshape(-1)], axis=1)


def children(key):
    l, x, y = key
    return [(l + 1, 2 * x + a, 2 * y + b) for b in (0, 1) for a in (0, 1)]


def refine(f, eps, scale, min_level=0, max_level=24, p=16):
    """Leaf keys of the adaptive tree (before balance). f maps an (n, 2) array of points to n
    values."""
    leaves = []
    pending = [(0, 0, 0)]
    while pending:
        nxt = []
        for k in pending:
            if k[0] < min_level:
                nxt.extend(children(k))
            elif k[0] >= max_level or tail(f(box_nodes(k, p)), p) <= eps * scale:
                leaves.append(k)
            else:
                nxt.extend(children(k))
        pending = nxt
    return leaves


def _adjacent(a, b):
    """Boxes a and b (keys) share an edge or a corner and neither contains the other."""
    (la, xa, ya), (lb, xb, yb) = a, b
    L = max(la, lb)
    ax0, ax1 = xa << (L - la), (xa + 1) << (L - la)
    ay0, ay1 = ya << (L - la), (ya + 1) << (L - la)
    bx0, bx1 = xb << (L - lb), (xb + 1) << (L - lb)
    by0, by1 = yb << (L - lb), (yb + 1) << (L - lb)
    touch = max(ax0, bx0) <= min(ax1, bx1) and max(ay0, by0) <= min(ay1, by1)
    overlap = max(ax0, bx0) < min(ax1, bx1) and max(ay0, by0) < min(ay1, by1)
    return touch and not overlap


def balance_brute(leaves):
    """Split until no two adjacent leaves differ by more than one level (all pairs checked)."""
    leaves = set(leaves)
    while True:
        bad = None
        for a in leaves:
            for b in leaves:
                if b[0] >= a[0] + 2 and _adjacent(a, b):
                    bad = a
                    break
            if bad:
                break
        if bad is None:
            return leaves
        leaves.remove(bad)
        leaves.update(children(bad))


def balance(leaves):
    """Same result as balance_brute: a leaf is split when some leaf two or more levels finer
    touches it. For each fine leaf the candidate coarse leaves are the ancestors-or-self of its
    eight neighbouring same-level boxes that are leaves."""
    leaves = set(leaves)
    changed = True
    while changed:
        changed = False
        for k in sorted(leaves, key=lambda q: -q[0]):
            if k not in leaves:
                continue
            l, x, y = k
            n = 1 << l
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if not (dx or dy) or not (0 <= x + dx < n and 0 <= y + dy < n):
                        continue
                    # the leaf covering the neighbouring box, if it is coarser
                    cl, cx, cy = l, x + dx, y + dy
                    while cl >= 0 and (cl, cx, cy) not in leaves:
                        cl, cx, cy = cl - 1, cx >> 1, cy >> 1
                    if cl >= 0 and cl <= l - 2:
                        leaves.remove((cl, cx, cy))
                        leaves.update(children((cl, cx, cy)))
                        changed = True
    return leaves


def build(f, eps, scale, min_level=0, max_level=24, p=16):
    """Balanced leaf keys (a set of (level, ix, iy))."""
    return balance(refine(f, eps, scale, min_level, max_level, p))
