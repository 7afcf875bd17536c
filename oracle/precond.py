"""Additive subspace-correction preconditioner of the oracle (Sec. 3).

TEST INFRASTRUCTURE: the FP64 CPU oracle (see oracle/__init__.py).

B = B_J + B_E + P V(A~_C) P^T   (Sec. 3.1 with W_i = V_j, V_e, V_C; eq. TB;
                                 Sec. 3.4 and Sec. 4.1)
  B_J  point Jacobi on the one-dimensional spaces V_j (eq. VB-subspaces),
  B_E  exact solves with the diagonal blocks A[V_e, V_e],
  P    conforming prolongation V_C -> V_h (natural injection, Sec. 3.4),
  V    one algebraic-multigrid V-cycle on the low-order-refined conforming
       matrix A~_C = P^T A~ P (Sec. 3.4, Prop. lor-conditioning).

Readings of the paper used here (each is stated where it is used):
  * V_C = V_h intersected with H^1_0 (homogeneous Dirichlet data), built with
    the minimum rule of Sec. 3.2.1 generalised to every entity dimension.
  * V_J rules J1-J4 (Sec. 3.3, Lemmas regular-vertex, conf-edge, no-hp and
    Remark cases), with "edge" = element side mapped to its master.
  * V_e = connected components of the seed-and-grow relation of Sec. 3.3
    (2D); in 3D the growth stays inside the seed's master face, so the
    spaces are face-sized and may overlap (face_spaces).
  * The multigrid method is a project-defined smoothed-aggregation AMG
    (the paper uses BoomerAMG without stating its settings).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla

from . import dg
from .gl import gl_nodes, lagrange
from .mesh import types


# ----------------------------------------------------------- conforming space
def conforming_numbering(mesh):
    """Column numbering of V_C: leaves in input order, sub-entities of each
    leaf in type order; each non-hanging entity not on the boundary gets the
    (deg-1)^k interior nodes of its GL^deg grid (lowest open dimension
    fastest) the first time it is met."""
    ent = mesh.entities()
    num = {}
    ncols = 0
    for e in range(mesh.ne):
        for t in types(mesh.dim):
            key = mesh.sub_entity(e, t)
            info = ent[key]
            if info["hanging"] or key in num or mesh.on_boundary(key):
                continue
            num[key] = ncols
            ncols += (info["deg"] - 1) ** info["dim"]
    return num, ncols


class _Conf:
    def __init__(self, mesh):
        self.mesh = mesh
        self.ent = mesh.entities()
        self.num, self.ncols = conforming_numbering(mesh)
        self.cache = {}

    def open_dims(self, key):
        return [m for m, (lo, hi) in enumerate(key) if hi > lo]

    def eval_rows(self, key, pts):
        """Values of the conforming function carried by non-hanging entity
        `key` at points pts (list of per-dim (base, scale, xref) triples,
        coordinate = base + scale*xref in finest units): sparse matrix
        (len(pts) x ncols)."""
        C = self.coef(key)
        deg = self.ent[key]["deg"]
        nodes = gl_nodes(deg) if deg >= 1 else None
        O = self.open_dims(key)
        L = np.ones((len(pts), (deg + 1) ** len(O)))
        for j, m in enumerate(O):
            lo, hi = key[m][0] // 4, key[m][1] // 4
            S = hi - lo
            r = np.array([((pt[m][0] - lo) + pt[m][1] * pt[m][2]) / S for pt in pts])
            Lm = lagrange(nodes, r)
            idx = (np.arange((deg + 1) ** len(O)) // (deg + 1) ** j) % (deg + 1)
            L *= Lm[:, idx]
        return sp.csr_matrix(L) @ C

    def coef(self, key):
        """C_E: conforming-function values at every node of the GL^deg grid on
        the closure of E, as a sparse matrix (grid nodes x ncols)."""
        if key in self.cache:
            return self.cache[key]
        info = self.ent[key]
        assert not info["hanging"]
        deg = info["deg"]
        O = self.open_dims(key)
        k = len(O)
        nodes = gl_nodes(deg) if k > 0 else None
        ngrid = (deg + 1) ** k
        bnd = self.mesh.on_boundary(key)
        rows = []
        for g in range(ngrid):
            j = [(g // (deg + 1) ** a) % (deg + 1) for a in range(k)]
            if all(1 <= jj <= deg - 1 for jj in j):
                if bnd:
                    rows.append(sp.csr_matrix((1, self.ncols)))
                else:
                    li = 0
                    for a in reversed(range(k)):
                        li = li * (deg - 1) + (j[a] - 1)
                    rows.append(sp.csr_matrix(([1.0], ([0], [self.num[key] + li])),
                                              shape=(1, self.ncols)))
                continue
            # boundary node of the grid: it lies on a lower sub-entity beta
            beta = list(key)
            pt = []
            for m in range(self.mesh.dim):
                lo, hi = key[m]
                if hi > lo:
                    a = O.index(m)
                    if j[a] == 0:
                        beta[m] = (lo, lo)
                    elif j[a] == deg:
                        beta[m] = (hi, hi)
                    pt.append((lo // 4, (hi - lo) // 4, float(nodes[j[a]])))
                else:
                    pt.append((lo // 4, 0, 0.0))
            M = self.mesh.resolve(tuple(beta))
            rows.append(self.eval_rows(M, [pt]))
        C = sp.vstack(rows).tocsr() if rows else sp.csr_matrix((0, self.ncols))
        self.cache[key] = C
        return C


def prolongation(mesh):
    """P: V_C -> V_h (Sec. 3.4): row (K,i) holds the conforming function's
    value at the GL node xi_{K,i}. Returns (P as CSR, ncols)."""
    cf = _Conf(mesh)
    blocks = []
    for e in range(mesh.ne):
        p = int(mesh.p[e])
        nodes = gl_nodes(p)
        ni = mesh.node_index(e)
        rows = [None] * len(ni)
        groups = {}
        for r, i in enumerate(ni):
            t = tuple(0 if a == 0 else 2 if a == p else 1 for a in i)
            groups.setdefault(t, []).append(r)
        for t, rs in groups.items():
            M = mesh.resolve(mesh.sub_entity(e, t))
            pts = [[(int(mesh.lo[e, m]), int(mesh.size[e]), float(nodes[ni[r, m]]))
                    for m in range(mesh.dim)] for r in rs]
            R = cf.eval_rows(M, pts)
            for a, r in enumerate(rs):
                rows[r] = R[a]
        blocks.append(sp.vstack(rows))
    P = sp.vstack(blocks).tocsr()
    P.eliminate_zeros()
    return P, cf.ncols


# ------------------------------------------------------------------ labels
def _side_types(dim, t):
    """Side (codim-1) types of a leaf whose closure holds sub-entity t."""
    out = []
    for m in range(dim):
        if t[m] != 1:
            out.append(tuple(t[m] if j == m else 1 for j in range(dim)))
    return out


def labels(mesh, remark_relax=False):
    """Boolean arrays (inJ, inN) over DG DOFs (Sec. 3.3).

    A DOF at node xi on the boundary of K is in V_J iff
      J1 xi is a regular (non-hanging) vertex;
      J2 xi is interior to a conforming side whose neighbours share one degree;
      J3 some side of K through xi, mapped to its master, has a closure that
         touches no hp-hanging entity (a hanging entity of dimension <= d-2
         whose touching leaves have more than one degree: in 2D the
         hp-vertices of Sec. 3.2.1);
      J4 (Remark cases; optional, off by default) some side of K through xi
         maps to a master side whose coarse leaf's degree is at most every
         finer neighbour's degree. The paper reports this relaxation as an
         observation that its estimates do not imply; with it, the condition
         number grows with the penalty on meshes with three refinement levels,
         so it is not used unless asked for.
    Every other element-boundary DOF is in N = V_B minus V_J."""
    d = mesh.dim
    ent = mesh.entities()
    touch_cache = {}

    def touching(key):
        if key not in touch_cache:
            touch_cache[key] = mesh.touching(key)
        return touch_cache[key]

    not_hp_free = set()
    for key, info in ent.items():
        if not info["hanging"] or info["dim"] > d - 2:
            continue
        tch = touching(key)
        if len({int(mesh.p[e]) for e, _, _ in tch}) <= 1:
            continue
        for e, _, tau in tch:
            for ts in _side_types(d, tau):
                not_hp_free.add(mesh.resolve(mesh.sub_entity(e, ts)))

    side_cls = {}

    def side_class(E):
        if E not in side_cls:
            tch = touching(E)
            full = sorted({e for e, _, tau in tch if mesh.sub_entity(e, tau) == E})
            others = sorted({e for e, _, tau in tch if mesh.sub_entity(e, tau) != E})
            ps = {int(mesh.p[e]) for e in full + others}
            conf = len(others) == 0
            coarse_le = (not conf) and len(full) == 1 and \
                int(mesh.p[full[0]]) <= min(int(mesh.p[e]) for e in others)
            side_cls[E] = (conf, len(ps) == 1, coarse_le)
        return side_cls[E]

    inJ = np.zeros(mesh.ndof, dtype=bool)
    inN = np.zeros(mesh.ndof, dtype=bool)
    for e in range(mesh.ne):
        p = int(mesh.p[e])
        ni = mesh.node_index(e)
        base = int(mesh.off[e])
        for r, i in enumerate(ni):
            t = tuple(0 if a == 0 else 2 if a == p else 1 for a in i)
            if all(x == 1 for x in t):
                continue
            key = mesh.sub_entity(e, t)
            info = ent[key]
            j = False
            if info["dim"] == 0 and not info["hanging"]:
                j = True                                            # J1
            elif info["dim"] == d - 1 and not info["hanging"]:
                conf, uni, _ = side_class(key)
                j = conf and uni                                    # J2
            if not j:
                for ts in _side_types(d, t):
                    E = mesh.resolve(mesh.sub_entity(e, ts))
                    if E not in not_hp_free:
                        j = True                                    # J3
                        break
                    if remark_relax:
                        conf, _, cle = side_class(E)
                        if cle:
                            j = True                                # J4
                            break
            if j:
                inJ[base + r] = True
            else:
                inN[base + r] = True
    return inJ, inN


def edge_spaces(mesh, inN):
    """V_e (Sec. 3.3), 2D: two N-DOFs are related when both have a nonzero
    trace on a common face (so [[phi]].[[psi]] is not identically zero
    there); the V_e are the connected components. Returned as sorted DOF
    arrays, ordered by their smallest DOF."""
    parent = {}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for g in np.nonzero(inN)[0]:
        parent[int(g)] = int(g)
    for members in _face_members(mesh, inN):
        for a in members[1:]:
            ra, rb = find(a), find(members[0])
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    comps = {}
    for g in parent:
        comps.setdefault(find(g), []).append(g)
    out = [np.array(sorted(v), dtype=np.int64) for v in comps.values()]
    out.sort(key=lambda a: a[0])
    return out


def _face_members(mesh, inN):
    """Per face of the skeleton: the N-DOFs of its two sides (one on the
    boundary) whose basis function has a nonzero trace there, i.e. whose node
    lies on the element's side that contains the face."""
    out = []
    for f in mesh.faces:
        m = f["m"]
        sides = [(f["em"], 1), (f["ep"], 0)] if f["ep"] >= 0 else [(f["em"], f["side"])]
        members = []
        for e, upper in sides:
            p = int(mesh.p[e])
            ni = mesh.node_index(e)
            sel = ni[:, m] == (p if upper else 0)
            g = mesh.dofs(e)[sel]
            members.extend(int(x) for x in g if inN[x])
        out.append(members)
    return out


def face_spaces(mesh, inN):
    """V_e in 3D (the paper treats 2D only): the seed-and-grow process of
    Sec. 3.3 with growth kept inside the seed's master face. The seed of a
    face piece e holds the N-DOFs whose node lies on e; a function joins when
    its jump meets the jump of a member on a face piece of the same master
    face (the full side of the coarser of the two leaves, or the common side
    of two equal leaves, or a boundary side). The fixed point is the set of
    N-DOFs with a nonzero trace on any piece of that master face, from every
    leaf on either side of it. Spaces of different master faces overlap on
    shared element edges and vertices; B_E sums their exact block solves.
    (Unrestricted growth joins about two thirds of V_B into one space on
    random 3D hp meshes.) Returned as sorted DOF arrays, duplicates removed,
    ordered lexicographically."""
    groups = {}
    for f, members in zip(mesh.faces, _face_members(mesh, inN)):
        m = f["m"]
        if f["ep"] >= 0:
            em, ep = f["em"], f["ep"]
            key = (em, m, 1) if mesh.size[em] >= mesh.size[ep] else (ep, m, 0)
        else:
            key = (f["em"], m, f["side"])
        groups.setdefault(key, set()).update(members)
    out = sorted({tuple(sorted(v)) for v in groups.values() if v})
    return [np.array(b, dtype=np.int64) for b in out]


# --------------------------------------------------------------------- LOR
def lor_elem(mesh, e):
    """A~_K (Sec. 3.4): bilinear (Q1) stiffness on the Cartesian sub-grid whose
    vertices are the GL nodes of K, times k_K. Each sub-cell is an axis box
    with sides D_m; its Q1 matrix is sum_m (prod_{m'!=m} D_m')/D_m times
    (k1 in dim m, m1 in the others), k1 = [[1,-1],[-1,1]],
    m1 = [[1/3,1/6],[1/6,1/3]]."""
    d, p = mesh.dim, int(mesh.p[e])
    x = gl_nodes(p) * mesh.h[e]
    n = p + 1
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    m1 = np.array([[1.0 / 3, 1.0 / 6], [1.0 / 6, 1.0 / 3]])
    A = np.zeros((n ** d, n ** d))
    verts = list(itertools.product((0, 1), repeat=d))   # v[m] per dim
    for c in itertools.product(range(p), repeat=d):
        D = [x[c[m] + 1] - x[c[m]] for m in range(d)]
        gidx = [sum((c[m] + v[m]) * n ** m for m in range(d)) for v in verts]
        Kc = np.zeros((len(verts), len(verts)))
        for m in range(d):
            coef = np.prod([D[j] for j in range(d) if j != m]) / D[m]
            for a, va in enumerate(verts):
                for b, vb in enumerate(verts):
                    t = coef
                    for j in range(d):
                        t *= (k1 if j == m else m1)[va[j], vb[j]]
                    Kc[a, b] += t
        A[np.ix_(gidx, gidx)] += Kc
    return mesh.k[e] * A


def lor_matrix(mesh):
    return sp.block_diag([lor_elem(mesh, e) for e in range(mesh.ne)], format="csr")


def broken_stiffness(mesh):
    """A^ (Sec. 3.4): block diagonal matrix of int_K k grad u . grad v."""
    return sp.block_diag([dg.elem_matrix(mesh, e) for e in range(mesh.ne)], format="csr")


# ------------------------------------------------------------- AMG (project)
THETA = 0.04
THETAS = (0.04, 0.02, 0.01, 0.005, 0.0)   # retried in order when a level stalls
TIE = 1e-10


def aggregate(A, theta=None):
    """Three-phase greedy aggregation in natural row order.
    Strength: j in S_i iff j != i and |a_ij| >= THETA sqrt(a_ii a_jj).
    Phase 1: a free row whose strong neighbours are all free forms {i} + S_i.
    Phase 2: a free row joins the phase-1 aggregate of its strongest
             phase-1-aggregated neighbour (|a_ij| within relative TIE of the
             maximum count as ties; ties go to the lowest aggregate id).
    Phase 3: a still free row forms {i} + its free strong neighbours."""
    theta = THETA if theta is None else theta
    A = A.tocsr()
    n = A.shape[0]
    dg_ = A.diagonal()
    strong = []
    for i in range(n):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        s = [(int(j), abs(v)) for j, v in zip(cols, vals)
             if j != i and abs(v) >= theta * np.sqrt(dg_[i] * dg_[j])]
        strong.append(s)
    agg = -np.ones(n, dtype=np.int64)
    na = 0
    for i in range(n):
        if agg[i] >= 0:
            continue
        if all(agg[j] < 0 for j, _ in strong[i]):
            agg[i] = na
            for j, _ in strong[i]:
                agg[j] = na
            na += 1
    p1 = agg.copy()
    for i in range(n):
        if p1[i] >= 0:
            continue
        cand = [(a, p1[j]) for j, a in strong[i] if p1[j] >= 0]
        if cand:
            amax = max(a for a, _ in cand)
            agg[i] = min(g for a, g in cand if a >= amax * (1.0 - TIE))
    for i in range(n):
        if agg[i] >= 0:
            continue
        agg[i] = na
        for j, _ in strong[i]:
            if agg[j] < 0:
                agg[j] = na
        na += 1
    return agg, na


def filtered(A, theta):
    """Filtered matrix of smoothed aggregation: weak off-diagonal entries
    (|a_ij| < theta sqrt(a_ii a_jj)) are dropped and added to the diagonal,
    so row sums are kept."""
    A = A.tocsr()
    n = A.shape[0]
    d = A.diagonal()
    rows, cols, vals = [], [], []
    lump = np.zeros(n)
    for i in range(n):
        for q in range(A.indptr[i], A.indptr[i + 1]):
            j, v = int(A.indices[q]), A.data[q]
            if j == i or abs(v) >= theta * np.sqrt(d[i] * d[j]):
                rows.append(i)
                cols.append(j)
                vals.append(v)
            else:
                lump[i] += v
    F = sp.csr_matrix((vals, (rows, cols)), shape=A.shape) + sp.diags(lump)
    return F.tocsr()


class AMG:
    """Smoothed aggregation with a filtered smoother:
    P_l = (I - w D_F^{-1} A_F) P^_l, P^ the 0/1 aggregate indicator, A_F the
    filtered matrix (rows whose filtered diagonal is at most 1e-8 a_ii, e.g. a
    structural zero from a zero row sum, are not smoothed), w = (4/3)/rho, rho = max_i sum_j |a^F_ij| / a^F_ii;
    A_{l+1} = P_l^T A_l P_l. A level that would keep more than 0.4 of its
    rows is retried with theta = 0.02, 0.01, 0.005 and 0 (every connection
    strong); if it still stalls, or at n <= 256 or 12 levels, coarsening
    stops. Coarsest level: dense
    Cholesky. Smoother: l1-Jacobi (d_i = sum_j |a_ij|), one pre- and one
    post-sweep from a zero initial guess. The V(1,1) cycle is symmetric."""

    def __init__(self, A, max_levels=12, min_rows=256, max_ratio=0.4):
        self.A = [A.tocsr()]
        self.P = []
        self.aggs = []
        while True:
            Al = self.A[-1]
            n = Al.shape[0]
            if n <= min_rows or len(self.A) >= max_levels:
                break
            for theta in THETAS:
                agg, na = aggregate(Al, theta)
                if na <= max_ratio * n:
                    break
            if na > max_ratio * n:
                break
            Ph = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, na))
            F = filtered(Al, theta)
            d = F.diagonal()
            ok = d > 1e-8 * Al.diagonal()     # zero row sums lump to a structural 0
            dinv = np.where(ok, 1.0 / np.where(ok, d, 1.0), 0.0)
            rho = np.max(np.asarray(abs(F).sum(axis=1)).ravel() * dinv)
            w = (4.0 / 3.0) / rho
            Pl = (Ph - w * sp.diags(dinv) @ F @ Ph).tocsr()
            Pl.eliminate_zeros()
            Ac = (Pl.T @ Al @ Pl).tocsr()
            self.P.append(Pl)
            self.aggs.append(agg)
            self.A.append(Ac)
        self.l1 = [np.asarray(abs(Al).sum(axis=1)).ravel() for Al in self.A]
        Ac = self.A[-1].toarray()
        self.chol = sla.cho_factor(Ac, lower=True) if Ac.shape[0] > 0 else None

    def vcycle(self, b, l=0):
        if l == len(self.A) - 1:
            return sla.cho_solve(self.chol, b) if self.chol is not None else b * 0
        A, dinv = self.A[l], 1.0 / self.l1[l]
        x = dinv * b
        r = b - A @ x
        x = x + self.P[l] @ self.vcycle(self.P[l].T @ r, l + 1)
        x = x + dinv * (b - A @ x)
        return x


# ---------------------------------------------------------- preconditioner
class Preconditioner:
    """B = B_J + B_E + P T_C P^T. variant 'full' (B_B + B_C), 'jb' (point
    Jacobi on all of V_B plus B_C, the simplified preconditioner of Sec. 4.1);
    coarse 'amg' (one V-cycle on A~_C), 'lor-exact' (A~_C^{-1}) or
    'exact' (A_C^{-1} with A_C = P^T A^ P)."""

    def __init__(self, mesh, opts, variant="full", coarse="amg", remark_relax=False,
                 max_block=0):
        self.mesh, self.opts = mesh, opts
        self.diag = dg.diagonal(mesh, opts)
        self.inJ, self.inN = labels(mesh, remark_relax)
        if variant == "jb":
            self.inJ = self.inJ | self.inN
            self.inN = np.zeros_like(self.inN)
        self.blocks = (edge_spaces if mesh.dim == 2 else face_spaces)(mesh, self.inN)
        if max_block > 0:
            # project option: a space larger than max_block gets no block
            # solve; N-DOFs left in no block are handled by point Jacobi
            self.blocks = [b for b in self.blocks if len(b) <= max_block]
            covered = np.zeros(mesh.ndof, dtype=bool)
            for b in self.blocks:
                covered[b] = True
            moved = self.inN & ~covered
            self.inJ |= moved
            self.inN &= ~moved
        self.dinvJ = np.where(self.inJ, 1.0 / self.diag, 0.0)
        self.binv = [np.linalg.inv(dg.submatrix(mesh, opts, b)) for b in self.blocks]
        self.P, self.nc = prolongation(mesh)
        self.Atil = lor_matrix(mesh)
        self.AC_lor = (self.P.T @ self.Atil @ self.P).tocsr()
        self.coarse = coarse
        if coarse == "amg":
            self.amg = AMG(self.AC_lor)
        elif coarse == "lor-exact":
            self._fact = sla.cho_factor(self.AC_lor.toarray())
        else:
            AC = (self.P.T @ broken_stiffness(mesh) @ self.P).toarray()
            self._fact = sla.cho_factor(AC)

    def TC(self, rc):
        if self.coarse == "amg":
            return self.amg.vcycle(rc)
        return sla.cho_solve(self._fact, rc)

    def apply_parts(self, r):
        zJ = self.dinvJ * r
        zE = np.zeros_like(r)
        for idx, Bi in zip(self.blocks, self.binv):
            zE[idx] += Bi @ r[idx]
        rc = self.P.T @ r
        ec = self.TC(rc)
        zC = self.P @ ec
        return zJ, zE, rc, ec, zC

    def apply(self, r):
        zJ, zE, _, _, zC = self.apply_parts(np.asarray(r, dtype=float))
        return zJ + zE + zC
