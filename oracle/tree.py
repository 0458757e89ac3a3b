"""Quadtree keys, validation and adaptive-FMM interaction lists (oracle; test infrastructure only).

The quadtree of Sec. 4.2.1 (Alg. 2) starts from a root box B_0 and splits boxes into four;
after construction it is 2:1 balanced, i.e. every leaf differs by at most one level from its
neighbours (end of Sec. 4.2.1). We read "neighbour" as sharing an edge or a corner. The root
is [-1,1]^2 at level 0; a level-l box has half-width s_l = 2^-l and integer key (l, ix, iy)
with centre (-1 + (2 ix + 1) s_l, -1 + (2 iy + 1) s_l).

The box code (Sec. 4.2, the paper cites the adaptive box-code and FMM literature for it)
needs the four interaction lists of the adaptive FMM, written here from their geometric
definitions:

  U(a), a leaf:  all leaves adjacent to a, a included (near field, exact tables);
  V(b), any box: children of the colleagues of b's parent that are not adjacent to b
                 (multipole-to-local);
  W(a), a leaf:  children of a's colleagues that are not adjacent to a (multipole evaluated
                 at a's nodes);
  X(b), any box: leaves c with b in W(c) (source data to b's local expansion).

Colleagues of a box are the same-level boxes adjacent to it. Every ordered pair of leaves must
be covered exactly once by these lists; tests/test_oracle_tree.py checks that by brute force.
"""
import numpy as np


def _touch(k1, k2):
    """Closed boxes intersect (share at least a point)."""
    l1, x1, y1 = k1
    l2, x2, y2 = k2
    L = max(l1, l2)
    a1, b1 = x1 << (L - l1), (x1 + 1) << (L - l1)
    a2, b2 = x2 << (L - l2), (x2 + 1) << (L - l2)
    c1, d1 = y1 << (L - l1), (y1 + 1) << (L - l1)
    c2, d2 = y2 << (L - l2), (y2 + 1) << (L - l2)
    return max(a1, a2) <= min(b1, b2) and max(c1, c2) <= min(d1, d2)


class TreeError(ValueError):
    pass


class Tree:
    """A set of leaves given by centres and levels; validates tiling and 2:1 balance."""

    def __init__(self, centres, levels, check_balance=True):
        centres = np.asarray(centres, dtype=np.float64).reshape(-1, 2)
        levels = np.asarray(levels, dtype=np.int64).reshape(-1)
        if centres.shape[0] != levels.shape[0] or centres.shape[0] == 0:
            raise TreeError("need matching, non-empty centres and levels")
        self.n_leaves = centres.shape[0]
        self.centres = centres.copy()
        self.levels = levels.copy()
        self.halfw = 2.0 ** (-levels.astype(np.float64))
        keys = []
        for (cx, cy), l in zip(centres, levels):
            if l < 0 or l > 40:
                raise TreeError("level out of range")
            s = 2.0 ** (-int(l))
            fx = (cx + 1.0) / (2.0 * s) - 0.5
            fy = (cy + 1.0) / (2.0 * s) - 0.5
            ix, iy = int(round(fx)), int(round(fy))
            if abs(fx - ix) > 1e-9 or abs(fy - iy) > 1e-9 or not (0 <= ix < (1 << int(l))) or not (0 <= iy < (1 << int(l))):
                raise TreeError("centre does not sit on the level grid")
            keys.append((int(l), ix, iy))
        self.keys = keys
        self.leaf_of = {}
        for i, k in enumerate(keys):
            if k in self.leaf_of:
                raise TreeError("duplicate leaf")
            self.leaf_of[k] = i
        # no leaf may be an ancestor of another; total area must be the root's
        L = max(k[0] for k in keys)
        area = 0
        for k in keys:
            area += 1 << (2 * (L - k[0]))
            l, x, y = k
            while l > 0:
                l, x, y = l - 1, x >> 1, y >> 1
                if (l, x, y) in self.leaf_of:
                    raise TreeError("leaves overlap")
        if area != 1 << (2 * L):
            raise TreeError("leaves do not tile the root")
        # all boxes (leaves and their ancestors)
        self.boxes = set()
        for k in keys:
            l, x, y = k
            while True:
                self.boxes.add((l, x, y))
                if l == 0:
                    break
                l, x, y = l - 1, x >> 1, y >> 1
        self.max_level = L
        if check_balance:
            self._check_balance()

    # ---------------------------------------------------------------- helpers
    def is_leaf(self, k):
        return k in self.leaf_of

    def exists(self, k):
        return k in self.boxes

    @staticmethod
    def children(k):
        l, x, y = k
        return [(l + 1, 2 * x + dx, 2 * y + dy) for dy in (0, 1) for dx in (0, 1)]

    @staticmethod
    def parent(k):
        l, x, y = k
        return (l - 1, x >> 1, y >> 1)

    def colleagues(self, k):
        l, x, y = k
        n = 1 << l
        out = []
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dx or dy) and 0 <= x + dx < n and 0 <= y + dy < n and (l, x + dx, y + dy) in self.boxes:
                    out.append((l, x + dx, y + dy))
        return out

    def box_centre(self, k):
        l, x, y = k
        s = 2.0 ** (-l)
        return np.array([-1.0 + (2 * x + 1) * s, -1.0 + (2 * y + 1) * s])

    def _leaves_touching_under(self, k, target):
        """Leaves inside box k (k exists) that touch box target."""
        if not _touch(k, target):
            return []
        if self.is_leaf(k):
            return [k]
        out = []
        for c in self.children(k):
            out += self._leaves_touching_under(c, target)
        return out

    def adjacent_leaf_keys(self, k):
        """Leaves adjacent to box k (sharing an edge or corner), k excluded."""
        l, x, y = k
        n = 1 << l
        found = set()
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if not (dx or dy):
                    continue
                nx, ny = x + dx, y + dy
                if not (0 <= nx < n and 0 <= ny < n):
                    continue
                q = (l, nx, ny)
                if q in self.boxes:
                    for leaf in self._leaves_touching_under(q, k):
                        found.add(leaf)
                else:  # covered by a coarser leaf
                    ql, qx, qy = q
                    while (ql, qx, qy) not in self.leaf_of:
                        ql, qx, qy = ql - 1, qx >> 1, qy >> 1
                    found.add((ql, qx, qy))
        return sorted(found)

    def _check_balance(self):
        for k in self.keys:
            for q in self.adjacent_leaf_keys(k):
                if abs(q[0] - k[0]) > 1:
                    raise TreeError("tree is not 2:1 balanced (edges and corners)")

    def adjacent_leaves(self, a):
        """[(b, (dx, dy, rho))] for leaves b adjacent to leaf a or equal to it; offsets of the
        centre of b from the centre of a in units of s_a, rho = s_b / s_a."""
        ka = self.keys[a]
        out = [(a, (0.0, 0.0, 1.0))]
        for q in self.adjacent_leaf_keys(ka):
            b = self.leaf_of[q]
            d = (self.centres[b] - self.centres[a]) / self.halfw[a]
            out.append((b, (float(d[0]), float(d[1]), float(self.halfw[b] / self.halfw[a]))))
        return out

    # ---------------------------------------------------------------- FMM lists
    def lists(self):
        """U, V, W, X as dicts keyed by box key, values lists of keys (U, W, X hold leaf keys
        for their sources; V holds box keys)."""
        U, V, W, X = {}, {}, {}, {}
        for k in self.keys:
            U[k] = [k] + self.adjacent_leaf_keys(k)
            w = []
            for c in self.colleagues(k):
                if self.is_leaf(c):
                    continue
                for ch in self.children(c):
                    if not _touch(ch, k):
                        w.append(ch)
            W[k] = w
        for k in self.boxes:
            if k[0] < 2:
                continue
            v = []
            for pc in self.colleagues(self.parent(k)) + [self.parent(k)]:
                if self.is_leaf(pc):
                    continue
                for ch in self.children(pc):
                    if ch != k and not _touch(ch, k):
                        v.append(ch)
            V[k] = v
        for a, ws in W.items():
            for c in ws:
                X.setdefault(c, []).append(a)
        return U, V, W, X
