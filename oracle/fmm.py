"""CPU machine code with complex scaled expansions, and its exact transpose (oracle; tests only).

The paper evaluates the truncated volume potential (Sec. 4.2, eq. (vbulk)) with an adaptive box
code, i.e. an FMM specialised to tensor Chebyshev data on a quadtree (introduction and
Sec. 4.2, citing the box-code literature and the Greengard-Rokhlin FMM). This module writes
that method out plainly, stage by stage, in complex arithmetic with z = x + i y and
G = -(1/2pi) Re log z:

  near   u_a += sum_{b in U(a)} s_b^2 [T_r f_b + kappa(s_a) (W . f_b)]      (tables, quad.py)
  S2M    alpha_n = s_b^2 c_n int f^_b(eta) eta^n d eta,  c_0 = 1, c_n = -1/n
         (multipole phi(z) = alpha_0 log(z-c) + sum_n alpha_n (s/(z-c))^n)
  M2M    beta_0 = alpha_0,  beta_l = -alpha_0 z0^l / l + sum_{k=1}^{l} alpha_k 2^-k C(l-1,k-1) z0^{l-k}
         (z0 = child centre minus parent centre over the parent half-width)
  M2L    lambda_0 = alpha_0 [log s + log|d|] + sum_k alpha_k (-1)^k d^-k
         lambda_l = -alpha_0 / (l d^l) + sum_k alpha_k (-1)^k C(k+l-1, l) d^-(k+l)
         (local psi(z) = sum_l lambda_l ((z-c)/s)^l; d = source minus target centre over s)
  S2L    lambda_0 = s_b^2 int f^ [log s_a + log|d + rho eta|],  lambda_l = -(s_b^2/l) int f^ (d + rho eta)^-l
  L2L    mu_l = sum_{k>=l} lambda_k C(k,l) z0^{k-l} 2^-l
  L2T    u += -(1/2pi) Re sum_l lambda_l xi^l
  M2T    u += -(1/2pi) Re[alpha_0 (log s_a + log|xi - d|) + sum_k alpha_k rho^k (xi - d)^-k]

Only real parts reach u, so the imaginary part of every log is dropped (it only ever lands in
the imaginary part of constant terms). The transpose applies each stage's real transpose in
reverse order: for a complex-linear stage K it is K^H; for real-to-complex S it is Re(S^H .);
for complex-to-real Re(L .) it is L^H.

Expansion order ``P`` (default 50, i.e. 51 complex terms). Pinned by tests/test_oracle_fmm.py
against the direct sum of quad.py on small trees, by its own dot-product test, and by the
closed forms through quad.py.
"""
import math

import numpy as np

from . import nodes, quad
from .tree import Tree

NG = 48


def _binom(n, k):
    return float(math.comb(n, k)) if 0 <= k <= n else 0.0


class BoxCode:
    def __init__(self, tree: Tree, P=50):
        self.t = tree
        self.P = P
        self.Q = P + 1
        t = tree
        U, V, W, X = t.lists()
        self.U, self.V, self.W, self.X = U, V, W, X
        self.box_keys = sorted(t.boxes, key=lambda k: (k[0], k[2], k[1]))
        self.bidx = {k: i for i, k in enumerate(self.box_keys)}
        self.nb = len(self.box_keys)
        self.box_level = np.array([k[0] for k in self.box_keys])
        self.leaf_box = np.array([self.bidx[k] for k in t.keys])
        self.W_t = nodes.tensor_weights()
        gx, gw = np.polynomial.legendre.leggauss(NG)
        self.gx, self.gw = gx, gw
        self.Lg = nodes.lagrange_matrix(gx)  # (16, NG)
        # basis at the tensor Gauss points, BQ[q=(b*NG + a), k=(j*16+i)] * weights
        self.BQ = np.einsum("ia,jb->baji", self.Lg, self.Lg).reshape(NG * NG, 256)
        self.wq = np.outer(gw, gw).reshape(-1)  # index b*NG + a  (y index b)
        self.eta = (gx[None, :] + 1j * gx[:, None]).reshape(-1)  # eta[b*NG + a] = x_a + i y_b
        Q = self.Q
        # S2M (Q x 256)
        pw = self.eta[None, :] ** np.arange(Q)[:, None]
        c = np.array([1.0] + [-1.0 / n for n in range(1, Q)])
        self.S = c[:, None] * ((pw * self.wq[None, :]) @ self.BQ)
        # L2T (256 x Q)
        tt = nodes.cheb1_points()
        XX, YY = np.meshgrid(tt, tt, indexing="xy")
        self.xi = (XX + 1j * YY).reshape(-1)
        self.Lt = -(self.xi[:, None] ** np.arange(Q)[None, :]) / (2 * np.pi)
        self._m2l, self._s2l, self._m2t = {}, {}, {}
        self.Mq = {}
        self.Eq = {}
        for qx in (-0.5, 0.5):
            for qy in (-0.5, 0.5):
                z0 = complex(qx, qy)
                self.Mq[(qx, qy)] = self._m2m_matrix(z0)
                self.Eq[(qx, qy)] = self._l2l_matrix(z0)
        self.tables = quad.near_tables()
        self._build_pairs()

    # ------------------------------------------------------------------ matrices
    def _m2m_matrix(self, z0):
        Q = self.Q
        B = np.zeros((Q, Q), dtype=complex)
        B[0, 0] = 1.0
        for l in range(1, Q):
            B[l, 0] = -(z0 ** l) / l
            for k in range(1, l + 1):
                B[l, k] = 0.5 ** k * _binom(l - 1, k - 1) * z0 ** (l - k)
        return B

    def _l2l_matrix(self, z0):
        Q = self.Q
        E = np.zeros((Q, Q), dtype=complex)
        for l in range(Q):
            for k in range(l, Q):
                E[l, k] = _binom(k, l) * z0 ** (k - l) * 0.5 ** l
        return E

    def m2l_matrix(self, d):
        if d not in self._m2l:
            Q = self.Q
            dz = complex(*d)
            K = np.zeros((Q, Q), dtype=complex)
            K[0, 0] = np.log(abs(dz))
            for k in range(1, Q):
                K[0, k] = (-1) ** k * dz ** (-k)
            for l in range(1, Q):
                K[l, 0] = -1.0 / (l * dz ** l)
                for k in range(1, Q):
                    K[l, k] = (-1) ** k * _binom(k + l - 1, l) * dz ** (-(k + l))
            self._m2l[d] = K
        return self._m2l[d]

    def s2l_matrix(self, d, rho=2.0):
        if d not in self._s2l:
            Q = self.Q
            w = complex(*d) + rho * self.eta
            G = np.empty((Q, self.eta.size), dtype=complex)
            G[0] = np.log(np.abs(w))
            for l in range(1, Q):
                G[l] = -(w ** (-l)) / l
            self._s2l[d] = (G * self.wq[None, :]) @ self.BQ
        return self._s2l[d]

    def m2t_matrix(self, d, rho=0.5):
        if d not in self._m2t:
            Q = self.Q
            z = self.xi - complex(*d)
            M = np.empty((256, Q), dtype=complex)
            M[:, 0] = np.log(np.abs(z))
            for k in range(1, Q):
                M[:, k] = rho ** k * z ** (-k)
            self._m2t[d] = -M / (2 * np.pi)
        return self._m2t[d]

    # ------------------------------------------------------------------ pairs
    def _build_pairs(self):
        t = self.t
        cen = {k: t.box_centre(k) for k in self.box_keys}
        # near: (a, b, r)
        self.near = []
        for a in range(t.n_leaves):
            for b, (dx, dy, rho) in t.adjacent_leaves(a):
                r = quad.relation_index(dx, dy, rho)
                if r < 0:
                    raise ValueError("unbalanced adjacency in box code")
                self.near.append((a, b, r))
        # V: grouped by offset -> list of (tgt box, src box)
        self.vpairs = {}
        for k, srcs in self.V.items():
            s = 2.0 ** (-k[0])
            for c in srcs:
                d = tuple(np.round((cen[c] - cen[k]) / s, 12))
                self.vpairs.setdefault(d, []).append((self.bidx[k], self.bidx[c]))
        # X: target box k, source leaves (leaf index)
        self.xpairs = {}
        for k, srcs in self.X.items():
            s = 2.0 ** (-k[0])
            for c in srcs:
                d = tuple(np.round((cen[c] - cen[k]) / s, 12))
                self.xpairs.setdefault(d, []).append((self.bidx[k], t.leaf_of[c]))
        # W: target leaf, source box
        self.wpairs = {}
        for k, srcs in self.W.items():
            s = 2.0 ** (-k[0])
            for c in srcs:
                d = tuple(np.round((cen[c] - cen[k]) / s, 12))
                self.wpairs.setdefault(d, []).append((t.leaf_of[k], self.bidx[c]))
        # M2M / L2L: child -> parent by quadrant
        self.tree_pairs = {}
        for k in self.box_keys:
            if k[0] < 3:
                continue
            p = Tree.parent(k)
            sp = 2.0 ** (-p[0])
            q = tuple((cen[k] - cen[p]) / sp)
            self.tree_pairs.setdefault(k[0], {}).setdefault(q, []).append((self.bidx[k], self.bidx[p]))
        self.max_level = max(k[0] for k in self.box_keys)

    # ------------------------------------------------------------------ forward
    def apply(self, f):
        t = self.t
        f = np.asarray(f, dtype=np.float64).reshape(t.n_leaves, 256)
        Q = self.Q
        s2 = t.halfw ** 2
        u = np.zeros((t.n_leaves, 256))
        # near field
        kap = -np.log(t.halfw) / (2 * np.pi)
        mass = f @ self.W_t
        for a, b, r in self.near:
            u[a] += s2[b] * (self.tables[r] @ f[b] + kap[a] * mass[b])
        # S2M
        mp = np.zeros((self.nb, Q), dtype=complex)
        mp[self.leaf_box] = (s2[:, None] * f) @ self.S.T
        # M2M (levels max..3 push into parents at levels >= 2)
        for lev in range(self.max_level, 2, -1):
            for q, pairs in self.tree_pairs.get(lev, {}).items():
                ch = np.array([c for c, _ in pairs])
                par = np.array([p for _, p in pairs])
                np.add.at(mp, par, mp[ch] @ self.Mq[q].T)
        # downward
        loc = np.zeros((self.nb, Q), dtype=complex)
        lnS = -self.box_level * np.log(2.0)
        for d, pairs in self.vpairs.items():
            tg = np.array([a for a, _ in pairs])
            sr = np.array([b for _, b in pairs])
            contrib = mp[sr] @ self.m2l_matrix(d).T
            contrib[:, 0] += lnS[tg] * mp[sr, 0]
            np.add.at(loc, tg, contrib)
        for d, pairs in self.xpairs.items():
            tg = np.array([a for a, _ in pairs])
            sr = np.array([b for _, b in pairs])
            contrib = (s2[sr, None] * f[sr]) @ self.s2l_matrix(d).T
            contrib[:, 0] += lnS[tg] * s2[sr] * mass[sr]
            np.add.at(loc, tg, contrib)
        for lev in range(3, self.max_level + 1):
            for q, pairs in self.tree_pairs.get(lev, {}).items():
                ch = np.array([c for c, _ in pairs])
                par = np.array([p for _, p in pairs])
                loc[ch] += loc[par] @ self.Eq[q].T
        # L2T at leaves of level >= 2
        lv = t.levels >= 2
        u[lv] += np.real(loc[self.leaf_box[lv]] @ self.Lt.T)
        # M2T
        for d, pairs in self.wpairs.items():
            tg = np.array([a for a, _ in pairs])
            sr = np.array([b for _, b in pairs])
            contrib = np.real(mp[sr] @ self.m2t_matrix(d).T)
            contrib += (kap[tg] * np.real(mp[sr, 0]))[:, None]
            np.add.at(u, tg, contrib)
        return u

    # ------------------------------------------------------------------ transpose
    def apply_adjoint(self, ubar):
        t = self.t
        ubar = np.asarray(ubar, dtype=np.float64).reshape(t.n_leaves, 256)
        Q = self.Q
        s2 = t.halfw ** 2
        kap = -np.log(t.halfw) / (2 * np.pi)
        usum = ubar.sum(axis=1)
        fbar = np.zeros((t.n_leaves, 256))
        # near transpose
        for a, b, r in self.near:
            fbar[b] += s2[b] * (self.tables[r].T @ ubar[a] + kap[a] * usum[a] * self.W_t)
        mpb = np.zeros((self.nb, Q), dtype=complex)
        locb = np.zeros((self.nb, Q), dtype=complex)
        # M2T transpose
        for d, pairs in self.wpairs.items():
            tg = np.array([a for a, _ in pairs])
            sr = np.array([b for _, b in pairs])
            contrib = ubar[tg] @ np.conj(self.m2t_matrix(d))
            contrib[:, 0] += kap[tg] * usum[tg]
            np.add.at(mpb, sr, contrib)
        # L2T transpose
        lv = t.levels >= 2
        np.add.at(locb, self.leaf_box[lv], ubar[lv] @ np.conj(self.Lt))
        # L2L transpose (bottom-up)
        for lev in range(self.max_level, 2, -1):
            for q, pairs in self.tree_pairs.get(lev, {}).items():
                ch = np.array([c for c, _ in pairs])
                par = np.array([p for _, p in pairs])
                np.add.at(locb, par, locb[ch] @ np.conj(self.Eq[q]))
        lnS = -self.box_level * np.log(2.0)
        mass_bar = np.zeros(t.n_leaves)
        # S2L transpose
        for d, pairs in self.xpairs.items():
            tg = np.array([a for a, _ in pairs])
            sr = np.array([b for _, b in pairs])
            contrib = np.real(locb[tg] @ np.conj(self.s2l_matrix(d)))
            np.add.at(fbar, sr, s2[sr, None] * contrib)
            np.add.at(mass_bar, sr, lnS[tg] * s2[sr] * np.real(locb[tg, 0]))
        # M2L transpose
        for d, pairs in self.vpairs.items():
            tg = np.array([a for a, _ in pairs])
            sr = np.array([b for _, b in pairs])
            contrib = locb[tg] @ np.conj(self.m2l_matrix(d))
            contrib[:, 0] += lnS[tg] * locb[tg, 0]
            np.add.at(mpb, sr, contrib)
        # M2M transpose (top-down)
        for lev in range(3, self.max_level + 1):
            for q, pairs in self.tree_pairs.get(lev, {}).items():
                ch = np.array([c for c, _ in pairs])
                par = np.array([p for _, p in pairs])
                mpb[ch] += mpb[par] @ np.conj(self.Mq[q])
        # S2M transpose
        fbar += s2[:, None] * np.real(mpb[self.leaf_box] @ np.conj(self.S))
        fbar += np.outer(mass_bar, self.W_t)
        return fbar
