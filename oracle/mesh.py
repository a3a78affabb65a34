"""Plain-Python mesh topology of the oracle (TEST INFRASTRUCTURE ONLY).

A forest of quadtrees/octrees on a brick of nt[0] x nt[1] (x nt[2]) trees
(Sec. 2.2).  A leaf is (level l, global integer coordinates G at level l);
its tree is G >> l and its anchor inside the tree is G - (tree << l).  Leaves
are ordered by tree id (t_x + n_x (t_y + n_y t_z)) and then by the Morton key
of the anchor scaled to a common resolution with x in the lowest bit, so that
the n-th leaf is the n-th block (Sec. 2.2).

Neighbour search, the ghost pattern (Sec. 2.6), 2:1 balance with corner
connectivity (Sec. 2.2) and the regrid map (Sec. 2.2) are written with plain
dictionaries and loops; the tests pin them against brute-force geometry.
"""
from __future__ import annotations

import itertools
import numpy as np

LMAX = 20  # resolution of the Morton keys


def morton(a, ndim):
    key = 0
    for bit in range(LMAX):
        for d in range(ndim):
            key |= ((a[d] >> bit) & 1) << (bit * ndim + d)
    return key


class Forest:
    def __init__(self, ndim, nt, periodic=(True, True, True), level=0):
        self.ndim = ndim
        self.nt = tuple(int(x) for x in nt[:ndim]) + (1,) * (3 - ndim)
        self.periodic = tuple(bool(p) for p in periodic[:3])
        leaves = []
        for t in itertools.product(*[range(self.nt[d] << level) for d in range(ndim)]):
            G = tuple(t) + (0,) * (3 - ndim)
            leaves.append((level, G))
        self.set_leaves(leaves)

    # ------------------------------------------------------------------ order
    def tree_id(self, l, G):
        t = [G[d] >> l for d in range(3)]
        return t[0] + self.nt[0] * (t[1] + self.nt[1] * t[2])

    def key(self, leaf):
        l, G = leaf
        t = [G[d] >> l for d in range(3)]
        a = [(G[d] - (t[d] << l)) << (LMAX - l) for d in range(3)]
        return (self.tree_id(l, G), morton(a, self.ndim))

    def set_leaves(self, leaves):
        self.leaves = sorted(leaves, key=self.key)
        self.index = {leaf: n for n, leaf in enumerate(self.leaves)}

    @property
    def nb(self):
        return len(self.leaves)

    def levels(self):
        return np.array([l for l, _ in self.leaves], dtype=np.int32)

    def export(self):
        """(level[nb], tree[nb], anchor[nb][3]) as int arrays."""
        lev = np.array([l for l, _ in self.leaves], dtype=np.int32)
        tree = np.array([self.tree_id(l, G) for l, G in self.leaves], dtype=np.int32)
        anc = np.array([[G[d] - ((G[d] >> l) << l) for d in range(3)] for l, G in self.leaves],
                       dtype=np.int32).reshape(-1, 3)
        return lev, tree, anc

    # ------------------------------------------------------------- geometry
    def extent(self, l, ax):
        return self.nt[ax] << l

    def shift(self, l, G, ax, step):
        """Coordinates of the level-l region next to G along ax, or None at a
        non-periodic domain boundary."""
        H = list(G)
        H[ax] += step
        E = self.extent(l, ax)
        if H[ax] < 0 or H[ax] >= E:
            if not self.periodic[ax]:
                return None
            H[ax] %= E
        return tuple(H)

    def tangential(self, ax):
        return [d for d in range(self.ndim) if d != ax]

    def children(self, l, G):
        """The 2^d children in child-id order bx + 2 by + 4 bz (Morton order)."""
        out = []
        for cid in range(1 << self.ndim):
            C = tuple(2 * G[d] + ((cid >> d) & 1) if d < self.ndim else 0 for d in range(3))
            out.append((l + 1, C))
        return out

    def covering(self, leafset, l, G):
        """The leaf of `leafset` that covers the level-l region G, if any is at
        level <= l; None if the region is subdivided further."""
        for lc in range(l, -1, -1):
            s = l - lc
            H = tuple(G[d] >> s for d in range(3))
            if (lc, H) in leafset:
                return (lc, H)
        return None

    # ------------------------------------------------------ neighbour search
    def face_neighbours(self, n, f):
        """Classify face f (= 2*axis + side, side 1 = +) of block n:
        ('srl', m) | ('coarse', m, h) | ('fine', [(m, h), ...]) | ('bc',)."""
        l, G = self.leaves[n]
        ax, side = f // 2, f % 2
        H = self.shift(l, G, ax, 1 if side else -1)
        if H is None:
            return ("bc",)
        if (l, H) in self.index:
            return ("srl", self.index[(l, H)])
        tang = self.tangential(ax)
        if l > 0:
            Hp = tuple(H[d] >> 1 for d in range(3))
            if (l - 1, Hp) in self.index:
                h = sum((G[t] & 1) << i for i, t in enumerate(tang))
                return ("coarse", self.index[(l - 1, Hp)], h)
        fine = []
        for h in range(1 << (self.ndim - 1)):
            C = [2 * H[d] for d in range(3)]
            C[ax] += 0 if side else 1
            for i, t in enumerate(tang):
                C[t] += (h >> i) & 1
            C = tuple(C)
            if (l + 1, C) not in self.index:
                raise ValueError(f"mesh not 2:1 balanced at block {n} face {f}")
            fine.append((self.index[(l + 1, C)], h))
        return ("fine", fine)

    # ---------------------------------------------------------- ghost pattern
    def pattern(self):
        """Ghost pattern of Sec. 2.6, grouped by face f and sorted by
        (receiving block, hanging offset):
          srl[f]  (a, b)             for f = +axis: b is a's +axis neighbour
          f2c[f]  (c, q, h, c2f_ix)  coarse c receives restricted data from q
          c2f[f]  (q, c, h)          fine q receives prolonged data from c
          bc[f]   (b,)               physical boundary faces
        Returned as flat int32 arrays plus CSR offsets over the 2*ndim faces."""
        nf = 2 * self.ndim
        srl = [[] for _ in range(nf)]
        f2c = [[] for _ in range(nf)]
        c2f = [[] for _ in range(nf)]
        bc = [[] for _ in range(nf)]
        for n in range(self.nb):
            for f in range(nf):
                kind = self.face_neighbours(n, f)
                if kind[0] == "srl":
                    if f % 2 == 1:
                        srl[f].append((n, kind[1]))
                elif kind[0] == "coarse":
                    c2f[f].append((n, kind[1], kind[2]))
                elif kind[0] == "fine":
                    for q, h in kind[1]:
                        f2c[f].append([n, q, h, -1])
                else:
                    bc[f].append((n,))
        c2f_off = np.cumsum([0] + [len(x) for x in c2f]).astype(np.int32)
        c2f_pos = {}
        for f in range(nf):
            for i, (q, c, h) in enumerate(c2f[f]):
                c2f_pos[(q, f)] = c2f_off[f] + i
        for f in range(nf):
            for rec in f2c[f]:
                rec[3] = c2f_pos[(rec[1], f ^ 1)]

        def flat(lists, width):
            rows = [r for lst in lists for r in lst]
            arr = np.array(rows, dtype=np.int32).reshape(-1, width) if rows else np.zeros((0, width), np.int32)
            off = np.cumsum([0] + [len(x) for x in lists]).astype(np.int32)
            return arr, off

        out = {}
        out["srl"], out["srl_off"] = flat(srl, 2)
        out["f2c"], out["f2c_off"] = flat(f2c, 4)
        out["c2f"], out["c2f_off"] = flat(c2f, 3)
        out["bc"], out["bc_off"] = flat(bc, 1)
        return out

    # ------------------------------------------------------------ 2:1 balance
    def offsets(self):
        return [o for o in itertools.product(*[(-1, 0, 1)] * self.ndim) if any(o)]

    def wrap(self, l, G):
        H = list(G)
        for d in range(self.ndim):
            E = self.extent(l, d)
            if H[d] < 0 or H[d] >= E:
                if not self.periodic[d]:
                    return None
                H[d] %= E
        return tuple(H)

    def balance(self, leafset):
        """Refine the coarser leaf of any face/edge/corner-adjacent pair whose
        levels differ by more than one, until no such pair is left."""
        leafset = set(leafset)
        while True:
            refine = set()
            for (l, G) in leafset:
                if l < 2:
                    continue
                for o in self.offsets():
                    H = self.wrap(l, tuple(G[d] + (o[d] if d < self.ndim else 0) for d in range(3)))
                    if H is None:
                        continue
                    cov = self.covering(leafset, l, H)
                    if cov is not None and cov[0] < l - 1:
                        refine.add(cov)
            if not refine:
                return leafset
            for leaf in refine:
                leafset.remove(leaf)
                leafset.update(self.children(*leaf))

    def parent_fits(self, leafset, lp, Gp):
        """True when every leaf touching the level-lp region Gp has level
        <= lp + 1 (checked on cells of level lp + 2 along the contact)."""
        for o in self.offsets():
            R = self.wrap(lp, tuple(Gp[d] + (o[d] if d < self.ndim else 0) for d in range(3)))
            if R is None:
                continue
            ranges = []
            for d in range(3):
                if d >= self.ndim:
                    ranges.append([0])
                elif o[d] == 1:
                    ranges.append([0])
                elif o[d] == -1:
                    ranges.append([3])
                else:
                    ranges.append([0, 1, 2, 3])
            for sub in itertools.product(*ranges):
                C = tuple(4 * R[d] + sub[d] if d < self.ndim else 0 for d in range(3))
                cov = self.covering(leafset, lp + 2, C)
                if cov is None or cov[0] > lp + 1:
                    return False
        return True

    def regrid(self, flags, lmin, lmax):
        """Adapt the mesh to per-block flags (+1 refine, -1 derefine, 0 keep):
        refine flagged leaves below lmax, balance, then coarsen every complete
        family of old leaves that are all flagged -1, lie above lmin and whose
        parent stays within one level of every leaf it touches.  Returns the
        remap lists (op, src, arg) of the new blocks: op 0 copy old block src,
        op 1 prolong child arg of old block src, op 2 restrict old children
        src .. src + 2^d - 1.  Returns None (mesh unchanged) when nothing
        changes."""
        old = list(self.leaves)
        old_index = dict(self.index)
        flags = np.asarray(flags)
        cur = set()
        for (leaf, fl) in zip(old, flags):
            if fl > 0 and leaf[0] < lmax:
                cur.update(self.children(*leaf))
            else:
                cur.add(leaf)
        cur = self.balance(cur)
        minus = {leaf for leaf, fl in zip(old, flags) if fl < 0}
        fams = {}
        for (l, G) in cur:
            if l > lmin and (l, G) in minus:
                P = (l - 1, tuple(G[d] >> 1 for d in range(3)))
                fams.setdefault(P, []).append((l, G))
        merge = []
        for P, kids in fams.items():
            if len(kids) == (1 << self.ndim) and self.parent_fits(cur, *P):
                merge.append(P)
        for P in merge:
            for k in self.children(*P):
                cur.remove(k)
            cur.add(P)
        new = sorted(cur, key=self.key)
        if new == old:
            return None
        op, src, arg = [], [], []
        for (l, G) in new:
            if (l, G) in old_index:
                op.append(0); src.append(old_index[(l, G)]); arg.append(0)
                continue
            P = (l - 1, tuple(G[d] >> 1 for d in range(3)))
            if l > 0 and P in old_index:
                cid = sum((G[d] & 1) << d for d in range(self.ndim))
                op.append(1); src.append(old_index[P]); arg.append(cid)
                continue
            kids = self.children(l, G)
            if all(k in old_index for k in kids):
                first = old_index[kids[0]]
                assert all(old_index[k] == first + i for i, k in enumerate(kids))
                op.append(2); src.append(first); arg.append(0)
                continue
            raise AssertionError("new leaf is more than one level from the old mesh")
        self.set_leaves(new)
        return (np.array(op, np.int32), np.array(src, np.int32), np.array(arg, np.int32))

    # ------------------------------------------------------------ cell centres
    def cell_centres(self, N, tree_size, origin=(0.0, 0.0, 0.0)):
        """Cell-centre coordinates [nb][ndim][N^ndim] (i fastest)."""
        out = np.zeros((self.nb, self.ndim) + (N,) * self.ndim)
        idx = np.arange(N) + 0.5
        for n, (l, G) in enumerate(self.leaves):
            dx = tree_size / (N << l)
            for d in range(self.ndim):
                c = origin[d] + (G[d] * N + idx) * dx
                shape = [1] * self.ndim
                shape[self.ndim - 1 - d] = N
                out[n, d] = np.broadcast_to(c.reshape(shape), (N,) * self.ndim)
        return out
