"""Mesh topology for the oracle: leaves, faces and sub-entities.

TEST INFRASTRUCTURE: the FP64 CPU oracle (see oracle/__init__.py).

Geometry (Sec. 2): the domain is [0,1]^d tiled by axis-aligned square/cube
leaves of a forest of quadtrees/octrees over an n_base^d grid; T_kappa is the
affine map of [0,1]^d onto the leaf. All adjacency is decided in integer
coordinates at the finest scale N = n_base * 2^Lmax; "quarter units" (4x the
finest unit) give integer coordinates to points strictly inside finest cells.

Faces (Sec. 2, skeleton Gamma): every positive-measure intersection of two
leaf sides, plus every leaf side on the domain boundary. A coarse side met by
several finer leaves therefore contributes one face per fine neighbour.
Faces are found here by hashing every unit (finest-scale) piece of every leaf
side and grouping the pieces by the pair of leaves they separate.

Sub-entities: a leaf has 3^d sub-entities (vertices, edges, faces, interior),
labelled by t in {0,1,2}^d (0 = lower side, 1 = open interval, 2 = upper side
in each dimension). An entity is *hanging* when its relative interior lies in
the relative interior of a strictly larger sub-entity of another leaf (Sec.
3.2.1: a hanging vertex lies inside an element of which it is not a vertex);
its *master* is the largest such container.
"""
from __future__ import annotations

import itertools
from collections import defaultdict

import numpy as np


def types(dim):
    """All t in {0,1,2}^dim, ordered by sum t_m 3^m (dimension 0 fastest)."""
    out = []
    for idx in range(3 ** dim):
        t, r = [], idx
        for _ in range(dim):
            t.append(r % 3)
            r //= 3
        out.append(tuple(t))
    return out


class Mesh:
    def __init__(self, m):
        self.dim = d = int(m["dim"])
        self.n_base = int(m["n_base"])
        self.level = np.asarray(m["level"], dtype=np.int64)
        self.anchor = np.asarray(m["anchor"], dtype=np.int64).reshape(-1, d)
        self.p = np.asarray(m["degree"], dtype=np.int64)
        self.k = np.asarray(m["kcoef"], dtype=np.float64)
        self.ne = len(self.level)
        self.L = int(self.level.max())
        self.N = self.n_base * 2 ** self.L
        self.size = 2 ** (self.L - self.level)              # finest units
        self.lo = self.anchor * self.size[:, None]
        self.hi = self.lo + self.size[:, None]
        self.h = self.size / self.N
        self.nd = (self.p + 1) ** d
        self.off = np.concatenate([[0], np.cumsum(self.nd)])
        self.ndof = int(self.off[-1])
        self.lookup = {}
        for e in range(self.ne):
            key = (int(self.level[e]), tuple(int(a) for a in self.anchor[e]))
            if key in self.lookup:
                raise ValueError("duplicate leaf")
            self.lookup[key] = e
        self._validate()
        self.faces = self._build_faces()
        self._ent = None

    # ------------------------------------------------------------------ basics
    def _validate(self):
        d = self.dim
        for e in range(self.ne):
            lev = int(self.level[e])
            if lev < 0 or np.any(self.anchor[e] < 0) or np.any(
                    self.anchor[e] >= self.n_base * 2 ** lev):
                raise ValueError("leaf outside the domain")
            if not (1 <= self.p[e] <= 8) or not (self.k[e] > 0):
                raise ValueError("bad degree or coefficient")
            for l in range(lev):
                a = tuple(int(x) >> (lev - l) for x in self.anchor[e])
                if (l, a) in self.lookup:
                    raise ValueError("overlapping leaves")
        if int(np.sum(self.size.astype(object) ** d)) != self.N ** d:
            raise ValueError("leaves do not tile the domain")

    def locate(self, y4):
        """Leaf containing the point y4 (quarter units, strictly inside a
        finest cell), or -1 outside the domain."""
        for c in y4:
            if c < 0 or c >= 4 * self.N:
                return -1
        for l in range(self.L + 1):
            s4 = 4 * 2 ** (self.L - l)
            e = self.lookup.get((l, tuple(int(c) // s4 for c in y4)))
            if e is not None:
                return e
        raise RuntimeError("point not covered")

    def dofs(self, e):
        return np.arange(self.off[e], self.off[e + 1])

    def node_index(self, e):
        """Multi-indices (i_0,...,i_{d-1}) of the element's nodes, dimension 0
        fastest, in DOF order."""
        n = int(self.p[e]) + 1
        idx = np.indices((n,) * self.dim).reshape(self.dim, -1)[::-1].T
        return idx  # row r = (i_0, i_1, ...) with i_0 fastest

    # ------------------------------------------------------------------- faces
    def _build_faces(self):
        d = self.dim
        units = defaultdict(list)
        for e in range(self.ne):
            s = int(self.size[e])
            for m in range(d):
                tdims = [t for t in range(d) if t != m]
                for side in (0, 1):
                    c = int(self.lo[e, m]) + side * s
                    for off in itertools.product(range(s), repeat=d - 1):
                        tc = tuple(int(self.lo[e, t]) + o for t, o in zip(tdims, off))
                        units[(m, c, tc)].append((e, side))
        groups = defaultdict(list)
        for (m, c, tc), lst in units.items():
            if len(lst) == 1:
                e, side = lst[0]
                if c not in (0, self.N):
                    raise ValueError("interior side piece without neighbour")
                groups[("b", m, e, side)].append(tc)
            elif len(lst) == 2:
                (e1, s1), (e2, s2) = lst
                if s1 == s2:
                    raise ValueError("inconsistent sides")
                em, ep = (e1, e2) if s1 == 1 else (e2, e1)
                groups[("i", m, em, ep)].append(tc)
            else:
                raise ValueError("side piece shared by more than two leaves")
        faces = []
        for key, tcs in groups.items():
            tcs = np.array(tcs)
            kind, m = key[0], key[1]
            tdims = [t for t in range(d) if t != m]
            flo = np.zeros(d, dtype=np.int64)
            fhi = np.zeros(d, dtype=np.int64)
            for j, t in enumerate(tdims):
                flo[t] = tcs[:, j].min()
                fhi[t] = tcs[:, j].max() + 1
            area = int(np.prod([fhi[t] - flo[t] for t in tdims])) if d > 1 else 1
            assert area == len(tcs)
            if kind == "b":
                _, m, e, side = key
                c = int(self.lo[e, m]) + side * int(self.size[e])
                flo[m] = fhi[m] = c
                faces.append(dict(m=m, em=e, ep=-1, side=side, lo=flo, hi=fhi))
            else:
                _, m, em, ep = key
                c = int(self.hi[em, m])
                flo[m] = fhi[m] = c
                faces.append(dict(m=m, em=em, ep=ep, side=1, lo=flo, hi=fhi))
        faces.sort(key=lambda f: (f["em"], f["m"], f["side"], f["ep"]))
        return faces

    # ---------------------------------------------------------------- entities
    def sub_entity(self, e, t):
        """Geometry key of sub-entity t of leaf e: per dim (lo4, hi4) in
        quarter units; lo4 == hi4 in a degenerate dimension."""
        key = []
        for m in range(self.dim):
            lo4, hi4 = 4 * int(self.lo[e, m]), 4 * int(self.hi[e, m])
            key.append((lo4, lo4) if t[m] == 0 else (hi4, hi4) if t[m] == 2 else (lo4, hi4))
        return tuple(key)

    @staticmethod
    def ent_dim(key):
        return sum(1 for lo, hi in key if hi > lo)

    @staticmethod
    def ent_contains(big, small):
        return all(b[0] <= s[0] and s[1] <= b[1] for b, s in zip(big, small))

    def leaf_type_at(self, e, y4):
        """Type t of the sub-entity of leaf e whose relative interior holds the
        point y4 (which must lie in the closure of e)."""
        t = []
        for m in range(self.dim):
            if y4[m] == 4 * self.lo[e, m]:
                t.append(0)
            elif y4[m] == 4 * self.hi[e, m]:
                t.append(2)
            else:
                t.append(1)
        return tuple(t)

    def leaves_at(self, y4):
        """Leaves whose closure holds y4 (any point in quarter units)."""
        deg = [m for m in range(self.dim) if y4[m] % 4 == 0]
        found = []
        for signs in itertools.product((-1, 1), repeat=len(deg)):
            y = list(y4)
            for m, s in zip(deg, signs):
                y[m] += s
            e = self.locate(y)
            if e >= 0 and e not in found:
                found.append(e)
        return found

    def samples(self, key):
        """Points of the entity's relative interior, one per finest cell it
        covers (quarter units)."""
        axes = []
        for lo, hi in key:
            if hi > lo:
                axes.append(range(lo + 2, hi, 4))
            else:
                axes.append([lo])
        return list(itertools.product(*axes))

    def touching(self, key):
        """[(leaf, sample point, type of the leaf's sub-entity there)] over all
        leaves touching the entity's relative interior."""
        out = []
        for y in self.samples(key):
            for e in self.leaves_at(y):
                out.append((e, y, self.leaf_type_at(e, y)))
        return out

    def on_boundary(self, key):
        return any(lo == hi and lo in (0, 4 * self.N) for lo, hi in key)

    def entities(self):
        """Entity table: for every distinct sub-entity geometry: hanging flag,
        master (non-hanging container) and minimum-rule degree."""
        if self._ent is not None:
            return self._ent
        d = self.dim
        T = types(d)
        ent = {}
        for e in range(self.ne):
            for t in T:
                key = self.sub_entity(e, t)
                if key not in ent:
                    ent[key] = dict(dim=self.ent_dim(key), owner=e, t=t)
        # hanging / master: look at the leaves around one interior point
        for key, info in ent.items():
            y0 = tuple(lo + 2 if hi > lo else lo for lo, hi in key)
            best = None
            for e in self.leaves_at(y0):
                tau = self.sub_entity(e, self.leaf_type_at(e, y0))
                if tau != key and self.ent_contains(tau, key):
                    vol = np.prod([max(hi - lo, 1) for lo, hi in tau])
                    rank = (self.ent_dim(tau), vol)
                    if best is None or rank > best[0]:
                        best = (rank, tau)
            info["hanging"] = best is not None
            info["master"] = best[1] if best is not None else key
        for key, info in ent.items():
            if info["hanging"] and ent[info["master"]]["hanging"]:
                raise RuntimeError("master entity is itself hanging")
        # minimum-rule degrees, from the top dimension down
        for key, info in ent.items():
            if info["dim"] == d:
                info["deg"] = int(self.p[info["owner"]])
        for k in range(d - 1, -1, -1):
            for key, info in ent.items():
                if info["dim"] != k or info["hanging"]:
                    continue
                vals = []
                for e, y, tau in self.touching(key):
                    vals.append(int(self.p[e]))
                    for tp in T:
                        if tp == tau:
                            continue
                        if all(a == b or (b != 1 and a == 1) for a, b in zip(tp, tau)):
                            k2 = self.sub_entity(e, tp)
                            if not ent[k2]["hanging"]:
                                vals.append(ent[k2]["deg"])
                info["deg"] = min(vals)
        self._ent = ent
        return ent

    def resolve(self, key):
        """Non-hanging entity that carries the conforming function on `key`."""
        info = self.entities()[key]
        return info["master"] if info["hanging"] else key
