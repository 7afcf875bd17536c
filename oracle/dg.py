"""DG operator of the oracle: SIPG and BR2 forms for -div(k grad u) = f with
homogeneous Dirichlet conditions imposed weakly.

TEST INFRASTRUCTURE: the FP64 CPU oracle (see oracle/__init__.py).

Bilinear form (Sec. 2, eq. fe-problem and the form after it), with the
piecewise-constant coefficient k of Sec. 4.3 entering as
  A(u,v) = sum_K int_K k grad u . grad v
         - int_Gamma {k grad u} . [[v]] - int_Gamma {k grad v} . [[u]]
         + int_Gamma sigma [[u]] . [[v]]
with {w} = (w^- + w^+)/2 and [[w]] = w^- n^- + w^+ n^+ (Sec. 2). On a boundary
face {w} is the one-sided trace and [[w]] = w n.
Penalty (Sec. 2): sigma = eta * k_e * pi(p_e) / h_e with p_e the larger and
h_e the smaller of the two neighbours' degree and size, k_e the larger
coefficient; pi(p) = (p+1)^2 (rule 0) or p^2 (rule 1, the paper's choice).
BR2 (Sec. 4.4): the sigma term is replaced by
  sum_e eta * k_e * int_Omega r_e([[u]]) . r_e([[v]]),
  int_Omega r_e(phi) . tau = - int_e phi . {tau}   for all tau in [V_h]^d.
With n^- = e_m the lifting lives in component m only, and on a neighbour K it
is r = -c M_K^{-1} g_K with g_K,i = int_e J_u phi_{K,i}, c = 1/2 on interior
faces (c = 1 on the boundary), so the term is sum_K c^2 g_K(u)^T M_K^{-1} g_K(v).

All integrals are exact: element integrals with (p+1)^d Gauss points, face
integrals with (max p + 1)^(d-1) Gauss points on the face itself, where the
traces of both neighbours are evaluated at the physical quadrature points.
"""
from __future__ import annotations

import numpy as np

from .gl import gauss, gl_nodes, lagrange, lagrange_deriv, mass1d, stiff1d


class Opts:
    def __init__(self, form="sipg", penalty_rule=0, eta=1.0):
        assert form in ("sipg", "br2")
        self.form = form
        self.penalty_rule = penalty_rule
        self.eta = eta


def br2_eta(mesh, opts):
    """BR2 penalty: the given eta, or (eta <= 0) 1 + the largest number of
    faces (sub-faces and boundary faces included) of any element."""
    if opts.eta > 0:
        return opts.eta
    cnt = np.zeros(mesh.ne, dtype=np.int64)
    for f in mesh.faces:
        cnt[f["em"]] += 1
        if f["ep"] >= 0:
            cnt[f["ep"]] += 1
    return 1.0 + float(cnt.max())


def _pi(p, rule):
    return (p + 1.0) ** 2 if rule == 0 else float(p) ** 2


def penalty(mesh, opts, f):
    em, ep = f["em"], f["ep"]
    if ep < 0:
        pe, he, ke = mesh.p[em], mesh.h[em], mesh.k[em]
    else:
        pe = max(mesh.p[em], mesh.p[ep])
        he = min(mesh.h[em], mesh.h[ep])
        ke = max(mesh.k[em], mesh.k[ep])
    return opts.eta * ke * _pi(pe, opts.penalty_rule) / he


def _kron_apply(mats, x, dim):
    """Apply kron over dimensions (mats[m] acts on index i_m, i_0 fastest)."""
    n = mats[0].shape[1]
    X = x.reshape((n,) * dim)          # axes (i_{d-1}, ..., i_0)
    for m in range(dim):
        ax = dim - 1 - m
        X = np.moveaxis(np.tensordot(mats[m], X, axes=([1], [ax])), 0, ax)
    return X.reshape(-1)


def elem_apply(mesh, e, x):
    """Volume term y_K = k h^{d-2} sum_m (K in dim m, M elsewhere) x_K."""
    d, p = mesh.dim, int(mesh.p[e])
    M, K = mass1d(p), stiff1d(p)
    y = np.zeros_like(x)
    for m in range(d):
        y += _kron_apply([K if j == m else M for j in range(d)], x, d)
    return mesh.k[e] * mesh.h[e] ** (d - 2) * y


def elem_matrix(mesh, e):
    """Volume block by explicit quadrature of grad phi_i . grad phi_j."""
    d, p = mesh.dim, int(mesh.p[e])
    nodes = gl_nodes(p)
    xq, wq = gauss(p + 1)
    B1, G1 = lagrange(nodes, xq), lagrange_deriv(nodes, xq)
    qi = np.indices((p + 1,) * d).reshape(d, -1)[::-1].T  # quad multi-index
    ni = mesh.node_index(e)
    h = mesh.h[e]
    W = np.prod(wq[qi], axis=1) * h ** d
    A = np.zeros((len(ni), len(ni)))
    for m in range(d):
        G = np.ones((len(qi), len(ni)))
        for j in range(d):
            T = (G1 / h) if j == m else B1
            G *= T[qi[:, j]][:, ni[:, j]]
        A += G.T @ (W[:, None] * G)
    return mesh.k[e] * A


def elem_mass_matrix(mesh, e):
    d, p = mesh.dim, int(mesh.p[e])
    M = mass1d(p)
    ni = mesh.node_index(e)
    A = np.ones((len(ni), len(ni)))
    for j in range(d):
        A *= M[ni[:, j]][:, ni[:, j]]
    return A * mesh.h[e] ** d


def mass_apply(mesh, e, x):
    d, p = mesh.dim, int(mesh.p[e])
    M = mass1d(p)
    return mesh.h[e] ** d * _kron_apply([M] * d, x, d)


def mass_inv_apply(mesh, e, x):
    d, p = mesh.dim, int(mesh.p[e])
    Mi = np.linalg.inv(mass1d(p))
    return mesh.h[e] ** (-d) * _kron_apply([Mi] * d, x, d)


def face_eval(mesh, f):
    """Quadrature on face f and the traces of each neighbour's basis there.

    Returns W (quadrature weights times face measure) and, per side, (e, V, Dn)
    with V[Q,i] = phi_i(x_Q) and Dn[Q,i] = d phi_i / d x_m (x_Q), m the face
    normal dimension (derivative along +e_m, not along the outward normal)."""
    d, m = mesh.dim, f["m"]
    tdims = [t for t in range(d) if t != m]
    sides = [f["em"]] + ([f["ep"]] if f["ep"] >= 0 else [])
    q = int(max(mesh.p[e] for e in sides)) + 1
    xg, wg = gauss(q)
    qi = np.indices((q,) * (d - 1)).reshape(d - 1, -1)[::-1].T if d > 1 else np.zeros((1, 0), int)
    nQ = len(qi)
    W = np.ones(nQ)
    X = np.zeros((nQ, d))              # physical points, finest units
    for j, t in enumerate(tdims):
        a, b = f["lo"][t], f["hi"][t]
        X[:, t] = a + (b - a) * xg[qi[:, j]]
        W *= wg[qi[:, j]] * (b - a) / mesh.N
    X[:, m] = f["lo"][m]
    out = []
    for e in sides:
        p = int(mesh.p[e])
        nodes = gl_nodes(p)
        ni = mesh.node_index(e)
        h = mesh.h[e]
        V = np.ones((nQ, len(ni)))
        Dn = np.ones((nQ, len(ni)))
        for t in range(d):
            if t == m:
                r = np.full(nQ, 1.0 if X[0, m] == mesh.hi[e, m] else 0.0)
            else:
                a, s = mesh.lo[e, t], mesh.size[e]
                r = (X[:, t] - a) / s
            Lt = lagrange(nodes, r)
            V *= Lt[:, ni[:, t]]
            if t == m:
                Dn *= (lagrange_deriv(nodes, r) / h)[:, ni[:, t]]
            else:
                Dn *= Lt[:, ni[:, t]]
        out.append((e, V, Dn))
    return W, out


def face_matrix(mesh, opts, f, eta_br2=None):
    """(dofs, block) of the face terms of face f (explicit quadrature; BR2
    lifting by an explicit dense solve with the element mass matrix)."""
    W, sides = face_eval(mesh, f)
    sig = penalty(mesh, opts, f)
    if f["ep"] >= 0:
        (em, Vm, Dm), (ep, Vp, Dp) = sides
        Ju = np.hstack([Vm, -Vp])
        Fu = 0.5 * np.hstack([mesh.k[em] * Dm, mesh.k[ep] * Dp])
        dofs = np.concatenate([mesh.dofs(em), mesh.dofs(ep)])
        c2 = 0.25
        lifts = [(em, Vm), (ep, Vp)]
        ke = max(mesh.k[em], mesh.k[ep])
    else:
        (e, V, Dm), = sides
        sgn = 1.0 if f["side"] == 1 else -1.0
        Ju = sgn * V                      # [[u]] . e_m
        Fu = mesh.k[e] * Dm               # {k du/dx_m}
        dofs = mesh.dofs(e)
        c2 = 1.0
        lifts = [(e, V)]
        ke = mesh.k[e]
    B = -Ju.T @ (W[:, None] * Fu) - Fu.T @ (W[:, None] * Ju)
    if opts.form == "sipg":
        B += sig * Ju.T @ (W[:, None] * Ju)
    else:
        eta = eta_br2 if eta_br2 is not None else br2_eta(mesh, opts)
        for e, Ve in lifts:
            G = Ve.T @ (W[:, None] * Ju)
            B += c2 * eta * ke * G.T @ np.linalg.solve(elem_mass_matrix(mesh, e), G)
    return dofs, B


def assemble_dense(mesh, opts):
    A = np.zeros((mesh.ndof, mesh.ndof))
    for e in range(mesh.ne):
        i = mesh.dofs(e)
        A[np.ix_(i, i)] += elem_matrix(mesh, e)
    eta = br2_eta(mesh, opts) if opts.form == "br2" else None
    for f in mesh.faces:
        i, B = face_matrix(mesh, opts, f, eta)
        A[np.ix_(i, i)] += B
    return A


def assemble_sparse(mesh, opts):
    import scipy.sparse as sp
    rows, cols, vals = [], [], []

    def add(i, B):
        rows.append(np.repeat(i, len(i)))
        cols.append(np.tile(i, len(i)))
        vals.append(B.reshape(-1))
    for e in range(mesh.ne):
        add(mesh.dofs(e), elem_matrix(mesh, e))
    eta = br2_eta(mesh, opts) if opts.form == "br2" else None
    for f in mesh.faces:
        add(*face_matrix(mesh, opts, f, eta))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mesh.ndof, mesh.ndof)).tocsr()
    A.sum_duplicates()
    return A


def _face_action(mesh, opts, f, x, eta_br2):
    """Face terms applied to x: returns [(dofs, contribution), ...]."""
    W, sides = face_eval(mesh, f)
    sig = penalty(mesh, opts, f)
    if f["ep"] >= 0:
        (em, Vm, Dm), (ep, Vp, Dp) = sides
        xm, xp = x[mesh.dofs(em)], x[mesh.dofs(ep)]
        km, kp = mesh.k[em], mesh.k[ep]
        jmp = Vm @ xm - Vp @ xp
        flx = 0.5 * (km * (Dm @ xm) + kp * (Dp @ xp))
        if opts.form == "sipg":
            pen = sig * jmp
        else:
            ke = max(km, kp)
            pen = np.zeros_like(jmp)
            for e, Ve in ((em, Vm), (ep, Vp)):
                pen += 0.25 * eta_br2 * ke * (Ve @ mass_inv_apply(mesh, e, Ve.T @ (W * jmp)))
        ym = -Vm.T @ (W * flx) - 0.5 * km * (Dm.T @ (W * jmp)) + Vm.T @ (W * pen)
        yp = Vp.T @ (W * flx) - 0.5 * kp * (Dp.T @ (W * jmp)) - Vp.T @ (W * pen)
        return [(mesh.dofs(em), ym), (mesh.dofs(ep), yp)]
    (e, V, Dm), = sides
    xe = x[mesh.dofs(e)]
    sgn = 1.0 if f["side"] == 1 else -1.0
    k = mesh.k[e]
    jmp = sgn * (V @ xe)
    flx = k * (Dm @ xe)
    if opts.form == "sipg":
        pen = sig * jmp
    else:
        pen = eta_br2 * k * (V @ mass_inv_apply(mesh, e, V.T @ (W * jmp)))
    ye = sgn * (-V.T @ (W * flx) + V.T @ (W * pen)) - k * (Dm.T @ (W * jmp))
    return [(mesh.dofs(e), ye)]


def apply(mesh, opts, x, elems=None):
    """y = A x, element by element and face by face. With `elems` given, only
    the rows of those elements are computed (others are left zero)."""
    x = np.asarray(x, dtype=float)
    y = np.zeros(mesh.ndof)
    sel = np.ones(mesh.ne, dtype=bool) if elems is None else np.isin(np.arange(mesh.ne), elems)
    eta = br2_eta(mesh, opts) if opts.form == "br2" else None
    for e in np.nonzero(sel)[0]:
        i = mesh.dofs(e)
        y[i] += elem_apply(mesh, e, x[i])
    for f in mesh.faces:
        if not (sel[f["em"]] or (f["ep"] >= 0 and sel[f["ep"]])):
            continue
        for i, c in _face_action(mesh, opts, f, x, eta):
            y[i] += c
    if elems is not None:
        mask = np.zeros(mesh.ndof, dtype=bool)
        for e in elems:
            mask[mesh.dofs(e)] = True
        y[~mask] = 0.0
    return y


def diagonal(mesh, opts):
    """diag(A) from the element and face blocks, without forming them."""
    d = mesh.dim
    diag = np.zeros(mesh.ndof)
    for e in range(mesh.ne):
        p = int(mesh.p[e])
        M, K = np.diag(mass1d(p)), np.diag(stiff1d(p))
        ni = mesh.node_index(e)
        s = np.zeros(len(ni))
        for m in range(d):
            t = np.ones(len(ni))
            for j in range(d):
                t *= (K if j == m else M)[ni[:, j]]
            s += t
        diag[mesh.dofs(e)] += mesh.k[e] * mesh.h[e] ** (d - 2) * s
    eta = br2_eta(mesh, opts) if opts.form == "br2" else None
    for f in mesh.faces:
        i, dB = _face_diag(mesh, opts, f, eta)
        diag[i] += dB
    return diag


def _face_parts(mesh, opts, f):
    W, sides = face_eval(mesh, f)
    if f["ep"] >= 0:
        (em, Vm, Dm), (ep, Vp, Dp) = sides
        Ju = np.hstack([Vm, -Vp])
        Fu = 0.5 * np.hstack([mesh.k[em] * Dm, mesh.k[ep] * Dp])
        dofs = np.concatenate([mesh.dofs(em), mesh.dofs(ep)])
        return W, Ju, Fu, dofs, 0.25, [(em, Vm), (ep, Vp)], max(mesh.k[em], mesh.k[ep])
    (e, V, Dm), = sides
    sgn = 1.0 if f["side"] == 1 else -1.0
    return W, sgn * V, mesh.k[e] * Dm, mesh.dofs(e), 1.0, [(e, V)], mesh.k[e]


def _face_diag(mesh, opts, f, eta_br2):
    W, Ju, Fu, dofs, c2, lifts, ke = _face_parts(mesh, opts, f)
    dB = -2.0 * np.sum(W[:, None] * Ju * Fu, axis=0)
    if opts.form == "sipg":
        dB += penalty(mesh, opts, f) * np.sum(W[:, None] * Ju * Ju, axis=0)
    else:
        for e, Ve in lifts:
            G = Ve.T @ (W[:, None] * Ju)
            MiG = np.column_stack([mass_inv_apply(mesh, e, G[:, c]) for c in range(G.shape[1])])
            dB += c2 * eta_br2 * ke * np.sum(G * MiG, axis=0)
    return dofs, dB


def submatrix(mesh, opts, dofs):
    """A[dofs, dofs] (dense) from the element and face blocks that touch the
    given DOFs."""
    dofs = np.asarray(dofs)
    pos = {int(g): i for i, g in enumerate(dofs)}
    elem_of = np.searchsorted(mesh.off, dofs, side="right") - 1
    elems = set(int(e) for e in elem_of)
    S = np.zeros((len(dofs), len(dofs)))
    eta = br2_eta(mesh, opts) if opts.form == "br2" else None
    for e in elems:
        loc = [j for j, g in enumerate(mesh.dofs(e)) if int(g) in pos]
        idx = [pos[int(mesh.dofs(e)[j])] for j in loc]
        Ae = elem_matrix(mesh, e)
        S[np.ix_(idx, idx)] += Ae[np.ix_(loc, loc)]
    for f in mesh.faces:
        if f["em"] not in elems and not (f["ep"] >= 0 and f["ep"] in elems):
            continue
        W, Ju, Fu, fd, c2, lifts, ke = _face_parts(mesh, opts, f)
        loc = [j for j, g in enumerate(fd) if int(g) in pos]
        if not loc:
            continue
        idx = [pos[int(fd[j])] for j in loc]
        J, F = Ju[:, loc], Fu[:, loc]
        B = -J.T @ (W[:, None] * F) - F.T @ (W[:, None] * J)
        if opts.form == "sipg":
            B += penalty(mesh, opts, f) * J.T @ (W[:, None] * J)
        else:
            for e, Ve in lifts:
                G = Ve.T @ (W[:, None] * J)
                MiG = np.column_stack([mass_inv_apply(mesh, e, G[:, c]) for c in range(G.shape[1])])
                B += c2 * eta * ke * G.T @ MiG
        S[np.ix_(idx, idx)] += B
    return S


def rhs(mesh, fvals):
    """b = M I_h f (Sec. 2, eq. fe-problem, with f given by its GL nodal
    values; exact element mass matrices)."""
    fvals = np.asarray(fvals, dtype=float)
    b = np.zeros(mesh.ndof)
    for e in range(mesh.ne):
        i = mesh.dofs(e)
        b[i] = mass_apply(mesh, e, fvals[i])
    return b


def node_coords(mesh):
    """Physical coordinates of every DG node, shape (ndof, d)."""
    X = np.zeros((mesh.ndof, mesh.dim))
    for e in range(mesh.ne):
        nodes = gl_nodes(int(mesh.p[e]))
        ni = mesh.node_index(e)
        for m in range(mesh.dim):
            X[mesh.dofs(e), m] = (mesh.lo[e, m] + mesh.size[e] * nodes[ni[:, m]]) / mesh.N
    return X
