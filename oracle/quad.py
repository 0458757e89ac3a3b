"""Log-kernel leaf integrals, near tables and the direct sum (oracle; test infrastructure only).

The box code's result has a plain definition (Sec. 4.2, eq. (vbulk), with Omega_B the union
of leaves and f_h the leaf interpolants of Sec. 4.2.1):

    u(x_{a,m}) = sum_b int_{B_b} G(x_{a,m} - y) f_h(y) dy.

Writing y = c_b + s_b eta turns each leaf term into s_b^2 [ -(1/2pi) log(s_b) (W . f_b)
- (1/2pi) I(x0) . f_b ] with x0 = (x - c_b)/s_b and I_k(x0) = int log|x0 - eta| l_k(eta).
For a source leaf adjacent to the target leaf, x0 = (xi_m - d)/rho depends only on the node m,
the offset d of the source centre (in target half-widths) and the size ratio rho = s_b/s_a,
so the adjacent part is carried by 33 level-independent tables

    T_r[m, k] = -(1/2pi) int log|xi_m - d_r - rho_r eta| l_k(eta) d eta
              = -(1/2pi) [ log(rho_r) W_k + I_k((xi_m - d_r)/rho_r) ],

and A_{(a,m),(b,k)} = s_b^2 [ T_r[m,k] + kappa(s_a) W_k ],  kappa(s) = -(1/2pi) log s.

Relations (offsets in units of the target half-width; 2:1 balance with corners):
  self (0,0) rho 1; 8 colleagues (+-2|0, +-2|0) rho 1; 12 finer neighbours
  (+-1.5,+-0.5), (+-0.5,+-1.5), (+-1.5,+-1.5) rho 1/2; 12 coarser neighbours
  (+-3,+-1), (+-1,+-3), (+-3,+-3) rho 2.

``I`` is computed by the plain-C adaptive subdivision in ``_quad.c``. Pinned by
tests/test_oracle_quad.py: uniform-square closed form for the row sums of every table,
SciPy ``dblquad`` for single entries, D4 symmetry between relations, and the scaling law.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import nodes

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "_quad.c")
_LIB = os.path.join(_HERE, "_quad.so")
NQ = 24
_lib = None


def build(force=False):
    """Compile the oracle's C core with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load(p=nodes.P_DEFAULT):
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_longlong)
        lib.oq_init.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, dp, dp, ctypes.c_double]
        lib.oq_init.restype = ctypes.c_int
        lib.oq_logint.argtypes = [ctypes.c_int, dp, dp]
        lib.oq_direct_far.argtypes = [ctypes.c_int, dp, lp, lp, ctypes.c_int, dp, dp, dp, dp]
        lib.oq_direct_grad.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, dp]
        t = np.ascontiguousarray(nodes.cheb1_points(p))
        lam = np.ascontiguousarray(nodes.barycentric_weights(p))
        wt = np.ascontiguousarray(nodes.tensor_weights(p))
        gx, gw = np.polynomial.legendre.leggauss(NQ)
        gx = np.ascontiguousarray(gx)
        gw = np.ascontiguousarray(gw)
        rc = lib.oq_init(p, _dp(t), _dp(lam), _dp(wt), NQ, _dp(gx), _dp(gw), 2.5e-10)
        if rc != 0:
            raise RuntimeError("oq_init failed")
        lib._keep = (t, lam, wt, gx, gw)
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))


def logint(x0):
    """I(x0) for points x0 (n x 2): out[n, k] = int_{[-1,1]^2} log|x0 - eta| l_k(eta) d eta."""
    lib = _load()
    x0 = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).reshape(-1, 2))
    out = np.zeros((x0.shape[0], nodes.P_DEFAULT ** 2))
    lib.oq_logint(x0.shape[0], _dp(x0), _dp(out))
    return out


def near_relations():
    """The 33 adjacent-leaf relations as (dx, dy, rho), offsets in target half-widths."""
    rel = [(0.0, 0.0, 1.0)]
    for dy in (-2.0, 0.0, 2.0):
        for dx in (-2.0, 0.0, 2.0):
            if dx or dy:
                rel.append((dx, dy, 1.0))
    fine = []
    for sx in (-1, 1):
        for sy in (-1, 1):
            fine += [(1.5 * sx, 0.5 * sy), (0.5 * sx, 1.5 * sy), (1.5 * sx, 1.5 * sy)]
    rel += [(a, b, 0.5) for a, b in sorted(set(fine))]
    coarse = []
    for sx in (-1, 1):
        for sy in (-1, 1):
            coarse += [(3.0 * sx, 1.0 * sy), (1.0 * sx, 3.0 * sy), (3.0 * sx, 3.0 * sy)]
    rel += [(a, b, 2.0) for a, b in sorted(set(coarse))]
    assert len(rel) == 33
    return rel


def table(dx, dy, rho, p=nodes.P_DEFAULT):
    """T[m, k] for one relation (see module docstring)."""
    t = nodes.cheb1_points(p)
    X, Y = np.meshgrid(t, t, indexing="xy")
    xi = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    x0 = (xi - np.array([dx, dy])) / rho
    W = nodes.tensor_weights(p)
    return -(np.log(rho) * W[None, :] + logint(x0)) / (2.0 * np.pi)


_TABLES = None
_CACHE = os.path.join(_HERE, "_cache", "near_tables_p16_nq24_v1.npy")


def near_tables():
    """All 33 tables, shape (33, 256, 256), in the order of ``near_relations()``.

    Cached in oracle/_cache (written only by this function).
    """
    global _TABLES
    if _TABLES is None:
        if os.path.exists(_CACHE):
            arr = np.load(_CACHE, allow_pickle=False)
            if arr.shape == (33, 256, 256) and np.all(np.isfinite(arr)):
                _TABLES = arr
        if _TABLES is None:
            arr = np.stack([table(dx, dy, rho) for dx, dy, rho in near_relations()])
            os.makedirs(os.path.dirname(_CACHE), exist_ok=True)
            tmp = _CACHE + ".tmp%d.npy" % os.getpid()
            np.save(tmp, arr)
            os.replace(tmp, _CACHE)
            _TABLES = arr
    return _TABLES


def relation_index(dx, dy, rho):
    for r, (a, b, c) in enumerate(near_relations()):
        if a == dx and b == dy and c == rho:
            return r
    return -1


def direct_far(targets_xy, excl, centres, halfw, f):
    """sum over leaves not in excl[t] of int_{B_b} G(x_t - y) f_h(y) dy  (C, OpenMP)."""
    lib = _load()
    tx = np.ascontiguousarray(np.asarray(targets_xy, dtype=np.float64).reshape(-1, 2))
    nt = tx.shape[0]
    ptr = np.zeros(nt + 1, dtype=np.int64)
    for t, e in enumerate(excl):
        ptr[t + 1] = ptr[t] + len(e)
    idx = np.ascontiguousarray(np.concatenate([np.asarray(e, dtype=np.int64) for e in excl]) if ptr[-1] else np.zeros(1, np.int64))
    c = np.ascontiguousarray(centres, dtype=np.float64)
    h = np.ascontiguousarray(halfw, dtype=np.float64)
    ff = np.ascontiguousarray(f, dtype=np.float64).reshape(-1, nodes.P_DEFAULT ** 2)
    out = np.zeros(nt)
    lib.oq_direct_far(nt, _dp(tx), _lp(ptr), _lp(idx), c.shape[0], _dp(c), _dp(h), _dp(ff), _dp(out))
    return out


def direct_potential(tree, f, samples=None):
    """u = A f at leaf nodes by the plain definition (tables for adjacent leaves, adaptive
    quadrature for all others).

    tree: oracle.tree.Tree; f: (n_leaves, 256); samples: optional list of (leaf, node)
    pairs, default all. Returns u with shape (n_leaves, 256) or (len(samples),).
    """
    f = np.asarray(f, dtype=np.float64).reshape(tree.n_leaves, -1)
    Ts = near_tables()
    W = nodes.tensor_weights()
    full = samples is None
    if full:
        samples = [(a, m) for a in range(tree.n_leaves) for m in range(256)]
    samples = list(samples)
    adj = {}
    excl = []
    xy = np.empty((len(samples), 2))
    near = np.zeros(len(samples))
    t1 = nodes.cheb1_points()
    for n, (a, m) in enumerate(samples):
        if a not in adj:
            adj[a] = tree.adjacent_leaves(a)
        ca, sa = tree.centres[a], tree.halfw[a]
        i, j = m % 16, m // 16
        xy[n] = (ca[0] + sa * t1[i], ca[1] + sa * t1[j])
        ex = []
        kap = -np.log(sa) / (2 * np.pi)
        for b, (dx, dy, rho) in adj[a]:
            r = relation_index(dx, dy, rho)
            if r < 0:
                continue  # not a tabulated relation: leave it to adaptive quadrature
            sb = tree.halfw[b]
            near[n] += sb * sb * (Ts[r][m] @ f[b] + kap * (W @ f[b]))
            ex.append(b)
        excl.append(ex)
    far = direct_far(xy, excl, tree.centres, tree.halfw, f)
    u = near + far
    return u.reshape(tree.n_leaves, 256) if full else u


def potential_at_points(centres, halfw, f, xy, grad=False):
    """u(x) = sum_b int_{B_b} G(x - y) f_h(y) dy at arbitrary points x (n, 2) by the plain
    definition (adaptive quadrature over every leaf, no tables), and with grad=True also its
    gradient (n, 2) (the same sum with grad_x G = -(1/2pi) (x - y)/|x - y|^2)."""
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
    u = direct_far(xy, [[] for _ in range(xy.shape[0])], centres, halfw, f)
    if not grad:
        return u
    lib = _load()
    c = np.ascontiguousarray(centres, dtype=np.float64)
    h = np.ascontiguousarray(halfw, dtype=np.float64)
    ff = np.ascontiguousarray(f, dtype=np.float64).reshape(-1, nodes.P_DEFAULT ** 2)
    g = np.zeros((xy.shape[0], 2))
    lib.oq_direct_grad(xy.shape[0], _dp(xy), c.shape[0], _dp(c), _dp(h), _dp(ff), _dp(g))
    return u, g
