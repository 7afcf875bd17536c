"""CPU tests of the native library: it loads, exports every symbol the
header declares, validates meshes, and its host-side setup (built with
host_only=1, no GPU touched) matches the oracle: diagonal, V_J/N labels
(bit-exact), V_e blocks (bit-exact), conforming prolongation P, LOR matrix
A~_C and the AMG hierarchy sizes."""
import ctypes
import os
import re

import numpy as np
import pytest

import hpinputs as H
import oracle as O
from oracle import dg, precond

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
G = pytest.importorskip("paper_2009_01287_amd")


def _lib_or_skip():
    try:
        return G.lib()
    except ImportError as e:
        pytest.fail(str(e))


def test_library_exports_header_symbols():
    L = _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "hpdg.h")).read()
    names = sorted(set(re.findall(r"\b(hpdg_[A-Za-z_]+)\s*\(", hdr)))
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(G.SYMBOLS)


def test_mesh_validation_errors():
    _lib_or_skip()
    md = H.uniform_mesh(2, 2, 2)
    bad = dict(md, level=md["level"][:-1], anchor=md["anchor"][:-1], degree=md["degree"][:-1],
               kcoef=md["kcoef"][:-1])
    with pytest.raises(G.HpdgError) as ei:
        G.Mesh(bad)
    assert ei.value.code == -1
    with pytest.raises(G.HpdgError):
        G.Mesh(dict(md, degree=np.array([1, 2, 9, 1], np.int32)))
    with pytest.raises(G.HpdgError):
        G.Mesh(dict(md, kcoef=np.array([1, 1, -1, 1.0])))
    empty = dict(md, level=md["level"][:0], anchor=md["anchor"][:0], degree=md["degree"][:0],
                 kcoef=md["kcoef"][:0])
    with pytest.raises(G.HpdgError) as ei:
        G.Mesh(empty)
    assert ei.value.code == -1
    m = G.Mesh(H.fig1_mesh(3))
    assert m.max_level_jump == 3
    assert m.nface == len(O.Mesh(H.fig1_mesh(3)).faces)


def test_operator_calls_rejected_when_host_only():
    _lib_or_skip()
    op = G.Operator(G.Mesh(H.uniform_mesh(2, 2, 1)), host_only=True)
    L = G.lib()
    code = L.hpdg_apply_A(op.h, ctypes.c_void_p(8), ctypes.c_void_p(16), 1, None)
    assert code == -6


CASES = [
    ("fig1", lambda: H.fig1_mesh(3), "sipg", 1.0, 0),
    ("hang2", lambda: H.hanging_mesh(2, 3, seed=3), "sipg", 1.0, 0),
    ("rand2", lambda: H.random_mesh(2, 4, 0.3, 3, 1, 8, seed=11), "sipg", 1.0, 0),
    ("rand2br2", lambda: H.random_mesh(2, 3, 0.4, 2, 1, 6, seed=12), "br2", 0.0, 0),
    ("rand3", lambda: H.random_mesh(3, 2, 0.4, 1, 1, 3, seed=5), "sipg", 1.0, 0),
    ("rand3k", lambda: H.random_mesh(3, 2, 0.4, 2, 1, 4, seed=5, k_logrange=(-2, 2)), "br2", 0.0, 128),
    ("hang3br2", lambda: H.hanging_mesh(3, 2, seed=2), "br2", 0.0, 0),
]


@pytest.mark.parametrize("name,mk,form,eta,cap", CASES, ids=[c[0] for c in CASES])
def test_host_setup_matches_oracle(name, mk, form, eta, cap):
    _lib_or_skip()
    md = mk()
    m = O.Mesh(md)
    opts = O.Opts(form, 0, eta)
    op = G.Operator(G.Mesh(md), form=form, eta=eta, host_only=True, max_block=cap)
    dO = dg.diagonal(m, opts)
    assert np.abs(op.diag() - dO).max() <= 1e-13 * np.abs(dO).max()
    pc = precond.Preconditioner(m, opts, max_block=cap)
    lab = np.where(pc.inJ, 1, np.where(pc.inN, 2, 0)).astype(np.int8)
    assert np.array_equal(op.labels(), lab)
    bo = pc.blocks
    bg = op.blocks()
    assert len(bo) == len(bg) and all(np.array_equal(a, b) for a, b in zip(bo, bg))
    # exact V_e solves: the stored inverses times the oracle's A[V_e, V_e]
    for b, Binv in zip(bo, op.block_inverses()):
        Ab = dg.submatrix(m, opts, b)
        assert np.abs(Binv @ Ab - np.eye(len(b))).max() <= 1e-9, name
    P, nc = precond.prolongation(m)
    PG = op.prolongation()
    assert PG.shape == P.shape
    assert abs(P - PG).max() <= 1e-13
    AC = (P.T @ precond.lor_matrix(m) @ P).tocsr()
    assert abs(AC - op.lor_conforming()).max() <= 1e-13 * abs(AC).max()
    amg = precond.AMG(AC)
    assert [a.shape[0] for a in amg.A] == op.amg_levels()
    for l, Al in enumerate(amg.A):
        assert abs(op._csr(op.export(100 + l)) - Al).max() <= 1e-12 * abs(Al).max()
        if l < len(amg.P):
            assert np.array_equal(op.export(300 + l).view(np.int64), amg.aggs[l])
            assert abs(op._csr(op.export(200 + l)) - amg.P[l]).max() <= 1e-11


def test_no_prec_operator_host():
    _lib_or_skip()
    md = H.random_mesh(2, 3, 0.3, 2, 1, 5, seed=21)
    m = G.Mesh(md)
    full = G.Operator(m, host_only=True)
    bare = G.Operator(m, host_only=True, no_prec=True)
    assert bare.device_bytes() < full.device_bytes()
    s = bare.summary()
    assert s["ndof"] == m.ndof and s["amg_levels"] == 0 and s["nblocks"] == 0


@pytest.mark.parametrize("dim,nb", [(3, 2), (3, 4), (2, 12)])
def test_setup_threads_do_not_change_results(dim, nb):
    """The row-parallel setup products and the prolongation built on element
    ranges (each with its own memo of entity rows) give bitwise the same host
    data with one thread and with several; the larger meshes have enough
    elements for several ranges."""
    _lib_or_skip()
    md = H.random_mesh(dim, nb, 0.4, 2, 1, 4, seed=5, k_logrange=(-2, 2))
    m = G.Mesh(md)
    if nb > 2:
        assert len(md["degree"]) >= 256
    a = G.Operator(m, form="br2", eta=0.0, host_only=True, max_block=128, setup_threads=1)
    b = G.Operator(m, form="br2", eta=0.0, host_only=True, max_block=128, setup_threads=4)
    for what in (0, 1, 2, 3, 4, 6, 8):
        assert np.array_equal(a.export(what), b.export(what)), what
    for l in range(len(a.amg_levels())):
        assert np.array_equal(a.export(100 + l), b.export(100 + l))


def test_penalty_study_mesh():
    """The penalty-study mesh: one refinement sweep, degrees 5..8, the
    coefficient 1 or 20 by the parity of the base cell's number (inherited)."""
    import hpinputs as H
    m = H.penalty_study_mesh()
    assert set(np.unique(m["level"])) <= {0, 1}
    assert m["degree"].min() >= 5 and m["degree"].max() <= 8
    base = m["anchor"] >> m["level"][:, None]
    idx = base[:, 0] + 16 * base[:, 1]
    assert np.array_equal(m["kcoef"], np.where(idx % 2 == 0, 1.0, 20.0))
    # every base cell is covered once: 1 leaf at level 0 or 4 at level 1
    area = np.where(m["level"] == 0, 4, 1)
    assert area.sum() == 4 * 16 * 16
    assert np.array_equal(H.penalty_study_mesh()["degree"], m["degree"])   # seeded


def _faces_touch(a, b, dim):
    """Leaves a, b = (level, anchor) share a face piece of positive measure
    (exact rational arithmetic on the unit cube)."""
    from fractions import Fraction as F
    la, aa = a
    lb, ab = b
    for m in range(dim):
        a0, a1 = F(aa[m], 2 ** la), F(aa[m] + 1, 2 ** la)
        b0, b1 = F(ab[m], 2 ** lb), F(ab[m] + 1, 2 ** lb)
        if a1 == b0 or b1 == a0:
            ok = True
            for t in range(dim):
                if t == m:
                    continue
                c0, c1 = F(aa[t], 2 ** la), F(aa[t] + 1, 2 ** la)
                d0, d1 = F(ab[t], 2 ** lb), F(ab[t] + 1, 2 ** lb)
                ok &= max(c0, d0) < min(c1, d1)
            if ok:
                return True
    return False


def test_random_refinement_one_irregular():
    """The 1-irregular limit: no two face neighbours differ by more than one
    level (brute force over all pairs), the leaves tile the domain, and the
    unlimited mesh of the same recipe does have larger jumps."""
    import hpinputs as H
    for one in (True, False):
        m = H.random_refinement_mesh(3, 3, one_irregular=one, seed=7)
        leaves = [(int(l), tuple(int(v) for v in a)) for l, a in zip(m["level"], m["anchor"])]
        assert sum(4.0 ** -l for l, _ in leaves) == pytest.approx(9.0)     # 3 x 3 base cells
        jump = 0
        for i in range(len(leaves)):
            for j in range(i + 1, len(leaves)):
                if _faces_touch(leaves[i], leaves[j], 2):
                    jump = max(jump, abs(leaves[i][0] - leaves[j][0]))
        if one:
            assert jump <= 1
        else:
            assert jump >= 2
    g = G.Mesh(H.random_refinement_mesh(3, 3, one_irregular=True, seed=7))
    assert g.max_level_jump <= 1
