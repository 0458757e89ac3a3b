"""Synthetic Gaussian-bump workloads on adaptive quadtrees.

The paper's examples resolve sums of Gaussians (the raindrop test solution, Sec. 5.1) and
200 random Gaussians with widely varying variances (the cell bleb, Sec. 5.4); their exact
geometries and data are not available, so these seeded stand-ins have the same structure.

Source:   f(y) = sum_g A_g exp(-|y - c_g|^2 / (2 sigma_g^2)), drawn from
          numpy.random.default_rng(seed) in the order: centres (K x 2), sigmas, amplitudes.
Tree:     start from the root [-1,1]^2; a box is split while its level is below
          ``min_level`` or while its order-p Chebyshev tail is above eps * sum_g |A_g|
          (the function-resolution criterion of Sec. 4.2.1 / Alg. 2, with "coefficients do
          not decay below eps" read as: the largest coefficient with i >= p-2 or j >= p-2
          is at most eps times the global scale). Then 2:1 balance over edges and corners.
Cut:      optionally f * chi(inside a star r < 0.7 (1 + 0.3 cos 5 theta)); boxes cut by the
          curve skip the tail test and are split down to ``lcut`` (mimicking the truncation-
          separation criterion); the zero-extended values are kept on cut boxes (Remark on
          keeping cut data, end of Sec. 4.2.1).
Nodes:    first-kind Chebyshev points, x index fastest (leaf data layout [leaf][j][i]).
"""
from dataclasses import dataclass, field

import numpy as np

P = 16


def _cheb_points(p=P):
    i = np.arange(1, p + 1)
    return -np.cos((2 * i - 1) * np.pi / (2 * p))


def _cheb_coeff_matrix(p=P):
    """D[n, i] with c = D v the Chebyshev coefficients of the interpolant of v at the points."""
    t = _cheb_points(p)
    theta = np.arccos(t)
    n = np.arange(p)
    D = (2.0 / p) * np.cos(np.outer(n, theta))
    D[0] *= 0.5
    return D


@dataclass
class Gaussians:
    centres: np.ndarray
    sigmas: np.ndarray
    amps: np.ndarray

    @property
    def scale(self):
        return float(np.sum(np.abs(self.amps)))


@dataclass
class Workload:
    name: str
    centres: np.ndarray  # (n, 2)
    levels: np.ndarray  # (n,) int32
    f: np.ndarray  # (n, 256) float64, x fastest
    src: Gaussians = None
    meta: dict = field(default_factory=dict)

    @property
    def n_leaves(self):
        return self.centres.shape[0]

    @property
    def unknowns(self):
        return self.n_leaves * P * P


def sample_gaussians(rng, K, c_lo, c_hi, s_lo, s_hi, log_sigma=True):
    c = rng.uniform(c_lo, c_hi, size=(K, 2))
    if log_sigma:
        s = np.exp(rng.uniform(np.log(s_lo), np.log(s_hi), size=K))
    else:
        s = rng.uniform(s_lo, s_hi, size=K)
    a = rng.uniform(-1.0, 1.0, size=K)
    return Gaussians(c, s, a)


def _box_nodes(keys_l, keys_x, keys_y, p=P):
    """Node coordinates for boxes given as arrays; returns X, Y of shape (n, p*p)."""
    t = _cheb_points(p)
    s = 2.0 ** (-keys_l.astype(np.float64))
    cx = -1.0 + (2 * keys_x + 1) * s
    cy = -1.0 + (2 * keys_y + 1) * s
    TX = np.tile(t, p)  # i fastest
    TY = np.repeat(t, p)
    X = cx[:, None] + s[:, None] * TX[None, :]
    Y = cy[:, None] + s[:, None] * TY[None, :]
    return X, Y


def eval_gaussians(g, X, Y, boxr=None, bcx=None, bcy=None):
    """f at points X, Y (any shape). If box radii/centres are given, skip Gaussians whose
    value on the box is below 1e-19 of their amplitude (exp(-43.7) ~ 1e-19)."""
    out = np.zeros_like(X)
    for c, s, a in zip(g.centres, g.sigmas, g.amps):
        if boxr is not None:
            d = np.hypot(bcx - c[0], bcy - c[1]) - boxr
            sel = (d < 9.35 * s).reshape(-1)
            if not np.any(sel):
                continue
            Xs, Ys = X[sel], Y[sel]
            out[sel] += a * np.exp(-((Xs - c[0]) ** 2 + (Ys - c[1]) ** 2) / (2 * s * s))
        else:
            out += a * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2 * s * s))
    return out


def star_inside(X, Y):
    r = np.hypot(X, Y)
    th = np.arctan2(Y, X)
    return r < 0.7 * (1.0 + 0.3 * np.cos(5 * th))


def _eval_boxes(g, L, IX, IY, cut):
    X, Y = _box_nodes(L, IX, IY)
    s = 2.0 ** (-L.astype(np.float64))
    cx = -1.0 + (2 * IX + 1) * s
    cy = -1.0 + (2 * IY + 1) * s
    F = eval_gaussians(g, X, Y, np.sqrt(2.0) * s[:, None], cx[:, None], cy[:, None])
    if cut:
        F = F * star_inside(X, Y)
    return F


def _tail(F, p=P):
    D = _cheb_coeff_matrix(p)
    Fb = F.reshape(-1, p, p)  # [box, j, i]
    C = np.matmul(np.matmul(D, Fb), D.T)  # C[b, n(y), m(x)] = sum_ji D[n, j] F[b, j, i] D[m, i]
    mask = np.zeros((p, p), dtype=bool)
    mask[p - 2:, :] = True
    mask[:, p - 2:] = True
    return np.max(np.abs(C[:, mask]), axis=1)


def _cut_status(L, IX, IY):
    """0 inside, 1 outside, 2 cut (nodes and corners on both sides)."""
    X, Y = _box_nodes(L, IX, IY)
    s = 2.0 ** (-L.astype(np.float64))
    cx = -1.0 + (2 * IX + 1) * s
    cy = -1.0 + (2 * IY + 1) * s
    corners_x = np.stack([cx - s, cx + s, cx - s, cx + s], axis=1)
    corners_y = np.stack([cy - s, cy - s, cy + s, cy + s], axis=1)
    ins = np.concatenate([star_inside(X, Y), star_inside(corners_x, corners_y)], axis=1)
    allin = ins.all(axis=1)
    allout = (~ins).all(axis=1)
    st = np.full(L.shape, 2)
    st[allin] = 0
    st[allout] = 1
    return st


def build_tree(g, eps=1e-11, min_level=0, max_level=24, cut=False, lcut=8):
    """Adaptive refinement from the root, then 2:1 balance. Returns a set of leaf keys."""
    tol = eps * g.scale
    leaves = set()
    L = np.array([0]); IX = np.array([0]); IY = np.array([0])
    while L.size:
        lev = int(L[0])
        split = np.zeros(L.shape, dtype=bool)
        if lev < min_level:
            split[:] = True
        elif lev < max_level:
            if cut:
                st = _cut_status(L, IX, IY)
                F = _eval_boxes(g, L, IX, IY, cut=True)
                tl = _tail(F)
                split = np.where(st == 2, lev < lcut, np.where(st == 0, tl > tol, False))
            else:
                F = _eval_boxes(g, L, IX, IY, cut=False)
                split = _tail(F) > tol
        for l, x, y in zip(L[~split], IX[~split], IY[~split]):
            leaves.add((int(l), int(x), int(y)))
        Ls, Xs, Ys = L[split], IX[split], IY[split]
        L = np.repeat(Ls + 1, 4)
        IX = (2 * np.repeat(Xs, 4) + np.tile([0, 1, 0, 1], Xs.size)).astype(np.int64)
        IY = (2 * np.repeat(Ys, 4) + np.tile([0, 0, 1, 1], Ys.size)).astype(np.int64)
    return balance(leaves)


def _pack(L, X, Y):
    return (np.asarray(L, np.int64) << 58) | (np.asarray(X, np.int64) << 29) | np.asarray(Y, np.int64)


def balance(leaves):
    """2:1 balance over edges and corners: split every leaf that a leaf two or more levels finer
    touches, until none does (the coarsest balanced refinement, which is unique). Vectorised:
    a neighbour box q of a level-l leaf is fine when q is a leaf, an internal box, or the child
    of a leaf; otherwise the leaf covering q is at level <= l - 2 and is split."""
    keys = np.array(sorted(leaves), dtype=np.int64).reshape(-1, 3)
    L, X, Y = keys[:, 0], keys[:, 1], keys[:, 2]
    offs = [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dx or dy]
    while True:
        leaf_k = np.sort(_pack(L, X, Y))
        # internal boxes: all proper ancestors of leaves
        anc = []
        l, x, y = L.copy(), X.copy(), Y.copy()
        while np.any(l > 0):
            m = l > 0
            l, x, y = l[m] - 1, x[m] >> 1, y[m] >> 1
            anc.append(_pack(l, x, y))
        inner_k = np.unique(np.concatenate(anc)) if anc else np.zeros(0, np.int64)

        def member(sorted_keys, k):
            if sorted_keys.size == 0:
                return np.zeros(k.shape, bool)
            i = np.minimum(np.searchsorted(sorted_keys, k), sorted_keys.size - 1)
            return sorted_keys[i] == k

        split = []
        for dx, dy in offs:
            qx, qy = X + dx, Y + dy
            n = np.left_shift(1, L)
            ok = (qx >= 0) & (qy >= 0) & (qx < n) & (qy < n)
            ql, qx, qy = L[ok], qx[ok], qy[ok]
            qk = _pack(ql, qx, qy)
            fine = member(leaf_k, qk) | member(inner_k, qk)
            fine |= (ql > 0) & member(leaf_k, _pack(np.maximum(ql - 1, 0), qx >> 1, qy >> 1))
            ql, qx, qy = ql[~fine], qx[~fine], qy[~fine]
            # the covering leaf, two or more levels coarser
            for d in range(2, int(ql.max()) + 1 if ql.size else 0):
                cl = ql - d
                live = cl >= 0
                ck = _pack(np.maximum(cl, 0), qx >> np.minimum(d, ql), qy >> np.minimum(d, ql))
                hit = live & member(leaf_k, ck)
                split.append(ck[hit])
                ql, qx, qy = ql[~hit], qx[~hit], qy[~hit]
                if ql.size == 0:
                    break
        sk = np.unique(np.concatenate(split)) if split else np.zeros(0, np.int64)
        if sk.size == 0:
            break
        k = _pack(L, X, Y)
        keep = ~member(sk, k)
        sl, sx, sy = sk >> 58, (sk >> 29) & ((1 << 29) - 1), sk & ((1 << 29) - 1)
        L = np.concatenate([L[keep], np.repeat(sl + 1, 4)])
        X = np.concatenate([X[keep], (2 * np.repeat(sx, 4) + np.tile([0, 1, 0, 1], sx.size))])
        Y = np.concatenate([Y[keep], (2 * np.repeat(sy, 4) + np.tile([0, 0, 1, 1], sy.size))])
    return {(int(a), int(b), int(c)) for a, b, c in zip(L, X, Y)}


def _order(leaves):
    """Deterministic caller order: by level, then Morton-free (y, x) raster."""
    return sorted(leaves, key=lambda k: (k[0], k[2], k[1]))


def make_workload(name, g, leaves, cut=False, shuffle_seed=None, meta=None):
    keys = _order(leaves)
    if shuffle_seed is not None:
        perm = np.random.default_rng(shuffle_seed).permutation(len(keys))
        keys = [keys[i] for i in perm]
    L = np.array([k[0] for k in keys], dtype=np.int64)
    IX = np.array([k[1] for k in keys], dtype=np.int64)
    IY = np.array([k[2] for k in keys], dtype=np.int64)
    s = 2.0 ** (-L.astype(np.float64))
    centres = np.stack([-1.0 + (2 * IX + 1) * s, -1.0 + (2 * IY + 1) * s], axis=1)
    F = _eval_boxes(g, L, IX, IY, cut=cut) if g is not None else np.zeros((len(keys), P * P))
    return Workload(name, centres, L.astype(np.int32), np.ascontiguousarray(F), g, meta or {})


def uniform_tree(level):
    n = 1 << level
    return {(level, x, y) for y in range(n) for x in range(n)}


def config1(seed=0):
    """Uniform depth-3 tree (64 leaves), f = 2 Gaussians, centres U[-0.5,0.5]^2, sigma U[0.1,0.3]."""
    rng = np.random.default_rng(seed)
    g = sample_gaussians(rng, 2, -0.5, 0.5, 0.1, 0.3, log_sigma=False)
    return make_workload("config1-uniform-l3-64", g, uniform_tree(3), meta={"seed": seed})


def config2(seed=0, size_matched=False, eps=1e-11):
    """20 Gaussians, sigma log-U[1e-3,1e-1], centres U[-0.9,0.9]^2, tail rule, 2:1 balanced.
    size_matched: background level 7 (16,384 leaves) under the same rule (about 20k leaves)."""
    rng = np.random.default_rng(seed)
    g = sample_gaussians(rng, 20, -0.9, 0.9, 1e-3, 1e-1)
    leaves = build_tree(g, eps=eps, min_level=7 if size_matched else 0)
    name = "config2-adaptive-20g" + ("-sm" if size_matched else "")
    return make_workload(name, g, leaves, meta={"seed": seed, "size_matched": size_matched})


def config3(seed=0, lcut=8, eps=1e-11):
    """200 Gaussians, sigma log-U[3e-4,5e-2], truncated outside a star; cut boxes to lcut."""
    rng = np.random.default_rng(seed)
    g = sample_gaussians(rng, 200, -0.9, 0.9, 3e-4, 5e-2)
    leaves = build_tree(g, eps=eps, cut=True, lcut=lcut)
    return make_workload("config3-star-200g-lcut%d" % lcut, g, leaves, cut=True,
                         meta={"seed": seed, "lcut": lcut})


def config4(seed=0, n_trees=256, max_leaves=8192):
    """A forest: per tree K ~ U{1..40} Gaussians (config-2 generator), min level 3."""
    children = np.random.SeedSequence(seed).spawn(n_trees)
    out = []
    for t, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        while True:
            K = int(rng.integers(1, 41))
            g = sample_gaussians(rng, K, -0.9, 0.9, 1e-3, 1e-1)
            leaves = build_tree(g, eps=1e-11, min_level=3)
            if len(leaves) <= max_leaves:
                break
        out.append(make_workload("config4-tree%d" % t, g, leaves, meta={"tree": t, "K": K}))
    return out


def config5(seed_f=0, seed_target=1, seed_dir=2, n_dirs=10):
    """Adjoint check on the config-2 tree: f from seed 0, a second 20-Gaussian source from seed 1
    sampled on the same tree, and n_dirs directions d ~ N(0,1) per unknown, scaled to
    max |d| = 1."""
    w = config2(seed_f)
    rng = np.random.default_rng(seed_target)
    g2 = sample_gaussians(rng, 20, -0.9, 0.9, 1e-3, 1e-1)
    L = w.levels.astype(np.int64)
    s = 2.0 ** (-L.astype(np.float64))
    IX = np.round((w.centres[:, 0] + 1) / (2 * s) - 0.5).astype(np.int64)
    IY = np.round((w.centres[:, 1] + 1) / (2 * s) - 0.5).astype(np.int64)
    f2 = _eval_boxes(g2, L, IX, IY, cut=False)
    rng_d = np.random.default_rng(seed_dir)
    dirs = rng_d.standard_normal((n_dirs, w.n_leaves, P * P))
    dirs /= np.max(np.abs(dirs), axis=(1, 2), keepdims=True)
    return w, f2, dirs


def random_small_tree(seed, max_level=4, n_splits=6):
    """A random 2:1-balanced tree with a handful of refinements (for brute-force tests)."""
    rng = np.random.default_rng(seed)
    leaves = {(1, x, y) for x in (0, 1) for y in (0, 1)}
    for _ in range(n_splits):
        cand = sorted(k for k in leaves if k[0] < max_level)
        k = cand[int(rng.integers(len(cand)))]
        leaves.remove(k)
        l, x, y = k
        leaves.update({(l + 1, 2 * x + a, 2 * y + b) for a in (0, 1) for b in (0, 1)})
        leaves = balance(leaves)
    g = sample_gaussians(rng, 3, -0.8, 0.8, 0.05, 0.4, log_sigma=True)
    return make_workload("random-small-%d" % seed, g, leaves, shuffle_seed=seed, meta={"seed": seed})


@dataclass
class Curve:
    """A closed curve cut into panels, each carrying Gauss-Legendre nodes: node positions,
    quadrature weights (arc length included), outward unit normals, and two seeded smooth
    densities (sigma, tau) on the nodes."""
    name: str
    nodes: np.ndarray    # (m, 2)
    weights: np.ndarray  # (m,)
    normals: np.ndarray  # (m, 2)
    sigma: np.ndarray    # (m,)
    tau: np.ndarray      # (m,)
    theta: np.ndarray    # (m,) curve parameter of each node
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return self.nodes.shape[0]


def star_curve(n_panels=128, order=24, scale=0.95, seed=0, n_modes=8):
    """The star r(theta) = scale * 0.7 (1 + 0.3 cos 5 theta) (the truncation curve of the
    200-Gaussian workload, pulled inwards by ``scale``), cut into n_panels equal parameter
    intervals with ``order`` Gauss-Legendre nodes each (counter-clockwise, outward normals).
    sigma and tau are random trigonometric series in theta with n_modes modes and
    coefficients decaying like 1/(1 + k), drawn from default_rng(seed): sigma first, then tau."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(0.0, 2.0 * np.pi, n_panels + 1)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    th = (mid[:, None] + half[:, None] * xg[None, :]).reshape(-1)
    wq = (half[:, None] * wg[None, :]).reshape(-1)
    R0, a, k = 0.7 * scale, 0.3, 5
    r = R0 * (1.0 + a * np.cos(k * th))
    dr = -R0 * a * k * np.sin(k * th)
    x, y = r * np.cos(th), r * np.sin(th)
    dx = dr * np.cos(th) - r * np.sin(th)
    dy = dr * np.sin(th) + r * np.cos(th)
    speed = np.hypot(dx, dy)
    normals = np.stack([dy / speed, -dx / speed], axis=1)
    rng = np.random.default_rng(seed)
    dens = []
    for _ in range(2):
        c = rng.standard_normal((2, n_modes + 1)) / (1.0 + np.arange(n_modes + 1))[None, :]
        kk = np.arange(n_modes + 1)[:, None]
        dens.append(c[0] @ np.cos(kk * th[None, :]) + c[1] @ np.sin(kk * th[None, :]))
    return Curve("star-curve-%dx%d" % (n_panels, order), np.stack([x, y], axis=1), wq * speed, normals,
                 dens[0], dens[1], th, meta={"n_panels": n_panels, "order": order, "scale": scale, "seed": seed})
