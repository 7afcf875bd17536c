"""Exact rational brute-force assembly of the SIPG / BR2 matrices on tiny
meshes with degrees 1 and 2 (whose Gauss-Lobatto nodes 0, 1/2, 1 are
rational). Used only as a pin for the oracle: it shares no code with it.

Every basis function is an explicit polynomial with Fraction coefficients;
every entry is the exact integral of the defining integrand (Sec. 2, bilinear
form; Sec. 4.4, BR2 lifting) over boxes and face rectangles found here by a
pairwise search over leaf sides.
"""
from __future__ import annotations

import itertools
from fractions import Fraction as Fr

import numpy as np

GL = {1: [Fr(0), Fr(1)], 2: [Fr(0), Fr(1, 2), Fr(1)]}


class Poly:
    """Polynomial in d variables: dict {exponent tuple: Fraction}."""

    def __init__(self, d, terms=None):
        self.d = d
        self.t = dict(terms or {})

    def __mul__(self, o):
        if not isinstance(o, Poly):
            return Poly(self.d, {k: v * o for k, v in self.t.items()})
        out = {}
        for k1, v1 in self.t.items():
            for k2, v2 in o.t.items():
                k = tuple(a + b for a, b in zip(k1, k2))
                out[k] = out.get(k, 0) + v1 * v2
        return Poly(self.d, out)

    __rmul__ = __mul__

    def __add__(self, o):
        out = dict(self.t)
        for k, v in o.t.items():
            out[k] = out.get(k, 0) + v
        return Poly(self.d, out)

    def __neg__(self):
        return self * Fr(-1)

    def __sub__(self, o):
        return self + (-o)

    def deriv(self, m):
        out = {}
        for k, v in self.t.items():
            if k[m] > 0:
                k2 = list(k)
                k2[m] -= 1
                out[tuple(k2)] = out.get(tuple(k2), 0) + v * k[m]
        return Poly(self.d, out)

    def restrict(self, m, c):
        """Substitute x_m = c (the exponent of x_m becomes 0)."""
        out = {}
        for k, v in self.t.items():
            k2 = list(k)
            e = k2[m]
            k2[m] = 0
            out[tuple(k2)] = out.get(tuple(k2), 0) + v * c ** e
        return Poly(self.d, {k: v for k, v in out.items() if v != 0})

    def integrate_box(self, lo, hi):
        """Exact integral over prod [lo_m, hi_m]; a degenerate dimension
        (lo == hi) is evaluated at that coordinate instead."""
        s = Fr(0)
        for k, v in self.t.items():
            term = v
            for m in range(self.d):
                a, b = lo[m], hi[m]
                if a == b:
                    term *= a ** k[m]
                else:
                    term *= (b ** (k[m] + 1) - a ** (k[m] + 1)) / (k[m] + 1)
            s += term
        return s


def lagrange_1d(d, m, nodes, i, x0, h):
    """l_i((x_m - x0)/h) as a Poly in d variables."""
    p = Poly(d, {tuple([0] * d): Fr(1)})
    for j, xj in enumerate(nodes):
        if j == i:
            continue
        e = [0] * d
        e[m] = 1
        # ((x - x0)/h - xj) / (xi - xj)
        c = Fr(1) / (nodes[i] - xj)
        lin = Poly(d, {tuple(e): c / h, tuple([0] * d): c * (-x0 / h - xj)})
        p = p * lin
    return p


class ExactMesh:
    def __init__(self, mdict):
        self.d = d = mdict["dim"]
        nb = mdict["n_base"]
        self.elems = []
        for lev, a, p, k in zip(mdict["level"], mdict["anchor"], mdict["degree"], mdict["kcoef"]):
            h = Fr(1, nb * 2 ** int(lev))
            lo = [int(x) * h for x in a]
            self.elems.append(dict(lo=lo, hi=[x + h for x in lo], h=h, p=int(p),
                                   k=Fr(k).limit_denominator(10 ** 6)))
        self.basis = []
        self.off = [0]
        for E in self.elems:
            nodes = GL[E["p"]]
            n = E["p"] + 1
            funcs = []
            for idx in range(n ** d):
                mi = [(idx // n ** m) % n for m in range(d)]
                f = Poly(d, {tuple([0] * d): Fr(1)})
                for m in range(d):
                    f = f * lagrange_1d(d, m, nodes, mi[m], E["lo"][m], E["h"])
                funcs.append(f)
            self.basis.append(funcs)
            self.off.append(self.off[-1] + len(funcs))
        self.n = self.off[-1]

    def faces(self):
        """(normal dim m, lo, hi, minus elem, plus elem or None, outward sign
        for boundary) for every positive-measure side intersection."""
        d = self.d
        out = []
        E = self.elems
        for a in range(len(E)):
            for m in range(d):
                for side in (0, 1):
                    c = E[a]["hi"][m] if side else E[a]["lo"][m]
                    if c in (0, 1) and (c == 1) == bool(side):
                        lo = list(E[a]["lo"])
                        hi = list(E[a]["hi"])
                        lo[m] = hi[m] = c
                        out.append((m, lo, hi, a, None, 1 if side else -1))
                        continue
                    if side == 0:
                        continue                     # interior faces from the minus side
                    for b in range(len(E)):
                        if E[b]["lo"][m] != c:
                            continue
                        lo, hi, ok = [], [], True
                        for t in range(d):
                            if t == m:
                                lo.append(c)
                                hi.append(c)
                                continue
                            l = max(E[a]["lo"][t], E[b]["lo"][t])
                            u = min(E[a]["hi"][t], E[b]["hi"][t])
                            if u <= l:
                                ok = False
                                break
                            lo.append(l)
                            hi.append(u)
                        if ok:
                            out.append((m, lo, hi, a, b, 0))
        return out

    def mass(self, a):
        B = self.basis[a]
        E = self.elems[a]
        return [[(B[i] * B[j]).integrate_box(E["lo"], E["hi"]) for j in range(len(B))]
                for i in range(len(B))]


def _solve_fr(M, rhs):
    """Exact Gaussian elimination; rhs is a list of columns."""
    n = len(M)
    A = [list(row) + [c[i] for c in rhs] for i, row in enumerate(M)]
    for i in range(n):
        piv = next(r for r in range(i, n) if A[r][i] != 0)
        A[i], A[piv] = A[piv], A[i]
        inv = 1 / A[i][i]
        A[i] = [v * inv for v in A[i]]
        for r in range(n):
            if r != i and A[r][i] != 0:
                f = A[r][i]
                A[r] = [vr - f * vi for vr, vi in zip(A[r], A[i])]
    return [[A[i][n + j] for i in range(n)] for j in range(len(rhs))]


def assemble(mdict, form="sipg", eta=Fr(1), rule=0):
    """Exact matrix as a float64 array (entries computed in rationals)."""
    X = ExactMesh(mdict)
    d = X.d
    A = [[Fr(0)] * X.n for _ in range(X.n)]
    for a, E in enumerate(X.elems):
        B = X.basis[a]
        G = [[f.deriv(m) for m in range(d)] for f in B]
        for i in range(len(B)):
            for j in range(len(B)):
                s = Fr(0)
                for m in range(d):
                    s += (G[i][m] * G[j][m]).integrate_box(E["lo"], E["hi"])
                A[X.off[a] + i][X.off[a] + j] += E["k"] * s
    faces = X.faces()
    if form == "br2" and eta <= 0:
        cnt = [0] * len(X.elems)
        for f in faces:
            cnt[f[3]] += 1
            if f[4] is not None:
                cnt[f[4]] += 1
        eta = Fr(1 + max(cnt))
    minv = {}
    for (m, lo, hi, a, b, sgn) in faces:
        Ea = X.elems[a]
        if b is None:
            sides = [(a, Fr(sgn))]
            pe, he, ke = Ea["p"], Ea["h"], Ea["k"]
            avg = Fr(1)
        else:
            Eb = X.elems[b]
            sides = [(a, Fr(1)), (b, Fr(-1))]   # jump = u_a - u_b along +e_m
            pe, he, ke = max(Ea["p"], Eb["p"]), min(Ea["h"], Eb["h"]), max(Ea["k"], Eb["k"])
            avg = Fr(1, 2)
        sig = eta * ke * (Fr(pe + 1) ** 2 if rule == 0 else Fr(pe) ** 2) / he
        # test/trial functions on the face: (global index, value poly,
        # jump coefficient along e_m, k * d/dx_m poly)
        fn = []
        for e, jc in sides:
            for i, f in enumerate(X.basis[e]):
                fr = f.restrict(m, lo[m])
                if not fr.t and not f.deriv(m).restrict(m, lo[m]).t:
                    continue                 # no trace and no normal derivative
                fn.append((X.off[e] + i, fr, jc,
                           f.deriv(m).restrict(m, lo[m]) * X.elems[e]["k"]))
        for gi, fi, ji, di in fn:
            for gj, fj, jj, dj in fn:
                # -{k du}.[[v]] - {k dv}.[[u]] (+ sigma [[u]].[[v]])
                s = -(avg * dj * fi * ji).integrate_box(lo, hi) \
                    - (avg * di * fj * jj).integrate_box(lo, hi)
                if form == "sipg":
                    s += sig * (fi * fj * ji * jj).integrate_box(lo, hi)
                A[gi][gj] += s
        if form == "br2":
            c2 = Fr(1, 4) if b is not None else Fr(1)
            for e, _ in sides:
                if e not in minv:
                    minv[e] = X.mass(e)
                Be = X.basis[e]
                # g_e(u)_r = int_face [[u]].e_m phi_{e,r} for every trial u
                g = {}
                Br = [f.restrict(m, lo[m]) for f in Be]
                for gj, fj, jj, _ in fn:
                    g[gj] = [(fj * jj * Br[r]).integrate_box(lo, hi) for r in range(len(Be))]
                keys = list(g)
                sol = _solve_fr(minv[e], [g[k] for k in keys])
                for ii, gi in enumerate(keys):
                    for jj2, gj in enumerate(keys):
                        v = sum(x * y for x, y in zip(g[gi], sol[jj2]))
                        A[gi][gj] += c2 * eta * ke * v
    return np.array([[float(v) for v in row] for row in A])
