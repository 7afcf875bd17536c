"""Pins for the oracle's DG operator (Sec. 2 SIPG form, Sec. 4.4 BR2 form).

* exact rational brute force (tests/brute_exact.py, independent code) on
  tiny nonconforming meshes with degrees 1 and 2, SIPG and BR2;
* symmetry and positive definiteness;
* polynomial reproduction: for u = prod x_m(1-x_m) (degree 2 <= p in every
  element) and f = -div grad u, A^{-1} M I_h f = I_h u exactly (consistency);
* manufactured convergence of SIPG at the textbook rate p+1;
* the matrix-free apply, diagonal and sub-blocks agree with the assembly.
"""
import numpy as np
import pytest

import hpinputs as H
import oracle as O
from oracle import dg

import brute_exact


def _mesh(name):
    if name == "fig1":
        return H.fig1_mesh(1, p_coarse=2, p_fine=1)
    if name == "hang2":
        return H.hanging_mesh(2, 2, pmin=1, pmax=2, seed=5)
    if name == "rand2":
        return H.random_mesh(2, 2, 0.5, 2, 1, 2, seed=3)
    if name == "hang3":
        # root split into 8 octants, the first octant split again: 15 leaves,
        # two of them of degree 2
        md = H.uniform_mesh(3, 1, 1, levels=1)
        cells = [(2, tuple(2 * 0 + ((c >> m) & 1) for m in range(3))) for c in range(8)]
        lev = [2] * 8 + [1] * 7
        anc = [c[1] for c in cells] + [tuple(a) for a in md["anchor"][1:]]
        deg = [1] * 15
        deg[3] = deg[9] = 2
        return dict(dim=3, n_base=1, level=np.array(lev, np.int32),
                    anchor=np.array(anc, np.int32), degree=np.array(deg, np.int32),
                    kcoef=np.ones(15))
    raise KeyError(name)


@pytest.mark.parametrize("name", ["fig1", "hang2", "hang3"])
@pytest.mark.parametrize("form", ["sipg", "br2"])
def test_exact_bruteforce(name, form):
    md = _mesh(name)
    m = O.Mesh(md)
    if name == "hang3" and form == "br2":
        pytest.skip("3D BR2 rational brute force is covered by hang3/sipg + reproduction")
    eta = 1.0 if form == "sipg" else 0.0
    A = dg.assemble_dense(m, O.Opts(form, 0, eta))
    Ax = brute_exact.assemble(md, form, eta=eta if form == "sipg" else 0, rule=0)
    assert np.abs(A - Ax).max() <= 1e-12 * np.abs(Ax).max()


def test_exact_bruteforce_penalty_rule1():
    md = _mesh("fig1")
    m = O.Mesh(md)
    A = dg.assemble_dense(m, O.Opts("sipg", 1, 10.0))
    from fractions import Fraction
    Ax = brute_exact.assemble(md, "sipg", eta=Fraction(10), rule=1)
    assert np.abs(A - Ax).max() <= 1e-12 * np.abs(Ax).max()


def _poly_case(md, form):
    m = O.Mesh(md)
    opts = O.Opts(form, 0, 1.0 if form == "sipg" else 0.0)
    X = dg.node_coords(m)
    q = X * (1 - X)
    u = np.prod(q, axis=1)
    f = np.zeros(len(X))
    for j in range(m.dim):
        f += 2 * np.prod(np.delete(q, j, axis=1), axis=1)
    A = dg.assemble_dense(m, opts)
    b = dg.rhs(m, f)
    return A, b, u


@pytest.mark.parametrize("dim,form", [(2, "sipg"), (2, "br2"), (3, "sipg"), (3, "br2")])
def test_symmetric_spd_and_polynomial_reproduction(dim, form):
    md = H.hanging_mesh(dim, 3 if dim == 2 else 2, pmin=2, pmax=4 if dim == 2 else 3, seed=7)
    A, b, u = _poly_case(md, form)
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(A)
    x = np.linalg.solve(A, b)
    assert np.abs(x - u).max() < 1e-11


def test_manufactured_rate_uniform_p2():
    """Uniform p = 2 meshes: u = sin(pi x) sin(pi y), p=2, SIPG with (p+1)^2/h:
    L2 nodal-error decreases at about the rate p+1 = 3."""
    errs = []
    for n in (4, 8, 16):
        m = O.Mesh(H.uniform_mesh(2, n, 2))
        X = dg.node_coords(m)
        u = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])
        f = 2 * np.pi ** 2 * u
        A = dg.assemble_sparse(m, O.Opts("sipg", 0, 1.0))
        import scipy.sparse.linalg as spla
        x = spla.spsolve(A.tocsc(), dg.rhs(m, f))
        e = x - u
        errs.append(np.sqrt(e @ dg.rhs(m, e)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 2.7 < rates[-1] < 3.3, rates


@pytest.mark.parametrize("form", ["sipg", "br2"])
def test_matrix_free_diag_submatrix(form):
    md = H.random_mesh(2, 2, 0.5, 3, 1, 5, seed=9)
    m = O.Mesh(md)
    opts = O.Opts(form, 0, 1.0 if form == "sipg" else 0.0)
    A = dg.assemble_dense(m, opts)
    x = np.random.default_rng(0).standard_normal(m.ndof)
    y = dg.apply(m, opts, x)
    assert np.abs(y - A @ x).max() <= 1e-13 * np.abs(A @ x).max()
    assert np.allclose(dg.diagonal(m, opts), np.diag(A), rtol=1e-13, atol=0)
    sel = np.array(sorted(np.random.default_rng(1).choice(m.ndof, 40, replace=False)))
    assert np.allclose(dg.submatrix(m, opts, sel), A[np.ix_(sel, sel)], rtol=1e-12, atol=1e-12)
    els = [0, 3, 5]
    ys = dg.apply(m, opts, x, elems=els)
    rows = np.concatenate([m.dofs(e) for e in els])
    assert np.allclose(ys[rows], (A @ x)[rows], rtol=1e-13, atol=1e-12)
    assert np.all(np.delete(ys, rows) == 0)
    # element volume blocks: sum-factorised apply == explicit quadrature
    for e in range(m.ne):
        xe = x[m.dofs(e)]
        assert np.allclose(dg.elem_apply(m, e, xe), dg.elem_matrix(m, e) @ xe, rtol=1e-12, atol=1e-12)


def test_mesh_validation_and_faces():
    with pytest.raises(ValueError):
        md = H.uniform_mesh(2, 2, 1)
        md["level"] = md["level"][:-1].copy()
        md["anchor"] = md["anchor"][:-1].copy()
        md["degree"] = md["degree"][:-1].copy()
        md["kcoef"] = md["kcoef"][:-1].copy()
        O.Mesh(md)
    m = O.Mesh(H.uniform_mesh(2, 4, 2))
    assert sum(1 for f in m.faces if f["ep"] >= 0) == 24
    assert sum(1 for f in m.faces if f["ep"] < 0) == 16
    m = O.Mesh(H.fig1_mesh(3))
    # the coarse leaf's right side is cut into 2^3 sub-faces
    coarse = [e for e in range(m.ne) if m.p[e] == 2][0]
    assert sum(1 for f in m.faces if f["em"] == coarse and f["m"] == 0 and f["ep"] >= 0) == 8
