"""Seeded synthetic inputs for the hp-DG solver: leaf lists of randomly refined
quadtree/octree meshes, per-element degrees and coefficients, and nodal
right-hand sides.

This module holds no arithmetic of the discretisation or of the solver: it only
draws random numbers and lists leaves. Both the FP64 oracle and the GPU library
consume its output, so the two sides see identical inputs.

The random-refinement recipe stands in for the paper's random-refinement test
(Sec. 4.3): elements are marked for refinement at random, refinement is applied
level by level without limiting irregularity, and degrees are drawn after the
final mesh is known. The paper's own initial mesh, coefficient pattern and
right-hand side are not available, so the sizes below are synthetic.

Mesh description (shared convention)
------------------------------------
A mesh is a dict with
  dim      2 or 3
  n_base   base grid is n_base^dim cells on [0,1]^dim
  level    int32[n]   refinement level of each leaf (0 = base cell)
  anchor   int32[n,dim] lower corner in units of 1/(n_base*2^level)
  degree   int32[n]   polynomial degree p of each leaf
  kcoef    float64[n] piecewise-constant diffusion coefficient k > 0
Leaves are listed base cell by base cell (x fastest), and inside a base cell in
depth-first order with children in lexicographic (x fastest) order.
"""
from __future__ import annotations

import math
import numpy as np

__all__ = [
    "CONFIGS", "uniform_mesh", "random_mesh", "fig1_mesh", "hanging_mesh",
    "ndof", "gaussian_rhs", "config_mesh", "config_rhs", "serving_stream",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _children(level, anchor, dim):
    """Children of a cell in lexicographic order, x fastest."""
    out = []
    for c in range(2 ** dim):
        a = tuple(2 * anchor[m] + ((c >> m) & 1) for m in range(dim))
        out.append((level + 1, a))
    return out


def _base_cells(dim, n_base):
    cells = []
    for idx in range(n_base ** dim):
        a = []
        r = idx
        for _ in range(dim):
            a.append(r % n_base)
            r //= n_base
        cells.append((0, tuple(a)))
    return cells


def _pack(dim, n_base, cells, degree, kcoef):
    n = len(cells)
    level = np.array([c[0] for c in cells], dtype=np.int32)
    anchor = np.array([c[1] for c in cells], dtype=np.int32).reshape(n, dim)
    return dict(dim=dim, n_base=n_base, level=level, anchor=anchor,
                degree=np.asarray(degree, dtype=np.int32).reshape(n),
                kcoef=np.asarray(kcoef, dtype=np.float64).reshape(n))


def uniform_mesh(dim, n_base, p=2, k=1.0, levels=0):
    """Uniform mesh: every base cell refined `levels` times."""
    cells = _base_cells(dim, n_base)
    for _ in range(levels):
        cells = [ch for c in cells for ch in _children(c[0], c[1], dim)]
    n = len(cells)
    return _pack(dim, n_base, cells, np.full(n, p), np.full(n, k))


def random_mesh(dim, n_base, q, lmax, pmin, pmax, seed, k_seed=None,
                k_logrange=None, p_seed=None):
    """Random refinement: sweep levels 0..lmax-1; at sweep l every leaf of level
    l is split into 2^dim children iff a uniform draw is below q. Degrees are
    drawn uniformly in {pmin..pmax} after the mesh is final. If k_logrange =
    (a, b) is given, every base cell gets k = 10^U(a,b) (its own stream
    k_seed), inherited by all its descendants; otherwise k = 1."""
    rng = _rng(seed)
    base = _base_cells(dim, n_base)
    cells = [(c[0], c[1], i) for i, c in enumerate(base)]  # remember base id
    for l in range(lmax):
        u = rng.random(len(cells))
        nxt = []
        for (lev, a, b), ui in zip(cells, u):
            if lev == l and ui < q:
                nxt.extend((cl, ca, b) for cl, ca in _children(lev, a, dim))
            else:
                nxt.append((lev, a, b))
        cells = nxt
    prng = rng if p_seed is None else _rng(p_seed)
    degree = prng.integers(pmin, pmax + 1, size=len(cells))
    if k_logrange is not None:
        krng = _rng(seed + 1 if k_seed is None else k_seed)
        kb = 10.0 ** krng.uniform(k_logrange[0], k_logrange[1], size=len(base))
        kcoef = np.array([kb[c[2]] for c in cells])
    else:
        kcoef = np.ones(len(cells))
    return _pack(dim, n_base, [(c[0], c[1]) for c in cells], degree, kcoef)


def fig1_mesh(n_levels, p_coarse=2, p_fine=1):
    """Fig. 1 family on [0,1]^2 (n_base=1): the lower-left quarter is one
    coarse leaf of degree p_coarse; the cells of the lower-right quarter that
    touch the line x=1/2 are refined down to level n_levels+1, which stacks
    2^n_levels fine leaves along the coarse leaf's right side. All other
    leaves have degree p_fine."""
    assert n_levels >= 1
    cells = []

    def rec(level, a):
        h = 0.5 ** level
        touches = a[0] * h == 0.5 and a[1] * h < 0.5
        if level == 0 or (level < n_levels + 1 and touches):
            for cl, ca in _children(level, a, 2):
                rec(cl, ca)
        else:
            cells.append((level, a))
    rec(0, (0, 0))
    deg = [p_coarse if (lev == 1 and a == (0, 0)) else p_fine
           for lev, a in cells]
    return _pack(2, 1, cells, deg, np.ones(len(cells)))


def hanging_mesh(dim, depth, p=None, seed=0, pmin=1, pmax=3):
    """Small strongly irregular mesh: n_base=2; the first base cell is refined
    `depth` times towards its corner at the domain centre, giving a chain of
    level jumps against the unrefined base cells. Degrees are random in
    {pmin..pmax} (stream `seed`) unless p is given."""
    cells = []

    def rec(level, a, d):
        corner = all(a[m] == 2 ** level - 1 for m in range(dim))
        if d > 0 and corner:
            for cl, ca in _children(level, a, dim):
                rec(cl, ca, d - 1)
        else:
            cells.append((level, a))
    for lev, a in _base_cells(dim, 2):
        if a == tuple([0] * dim):
            rec(0, a, depth)
        else:
            cells.append((lev, a))
    n = len(cells)
    deg = (_rng(seed).integers(pmin, pmax + 1, size=n) if p is None
           else np.full(n, p))
    return _pack(dim, 2, cells, deg, np.ones(n))


def ndof(mesh) -> int:
    return int(np.sum((mesh["degree"].astype(np.int64) + 1) ** mesh["dim"]))


def gaussian_rhs(n, seed, nrhs=1):
    """i.i.d. N(0,1) nodal values; shape (n,) or RHS-interleaved (n, nrhs)."""
    g = _rng(seed).standard_normal(n * nrhs)
    return g if nrhs == 1 else g.reshape(n, nrhs)


# Named workloads. Sizes are the expected values of the generator.
CONFIGS = {
    1: dict(name="uniform2d_4x4_p2", dim=2, form="sipg", penalty_rule=0,
            eta=1.0, rtol=1e-10, prec_fp32=0, nrhs=1),
    2: dict(name="random2d_32x32_q0.3_L3_p1-8", dim=2, form="sipg",
            penalty_rule=0, eta=1.0, rtol=1e-8, prec_fp32=0, nrhs=1,
            mesh_seed=1002, rhs_seed=2002),
    3: dict(name="random3d_16^3_q0.2_L2_p1-6_br2", dim=3, form="br2",
            penalty_rule=0, eta=0.0, rtol=1e-8, prec_fp32=1, nrhs=1,
            mesh_seed=1003, rhs_seed=2003, k_seed=3003),
    4: dict(name="random2d_32x32_64rhs", dim=2, form="sipg",
            penalty_rule=0, eta=1.0, rtol=1e-8, prec_fp32=1, nrhs=64,
            mesh_seed=1002, rhs_seed=2004),
}


def penalty_study_mesh(n_base=16, seed=1262, pmin=5, pmax=8):
    """Mesh of the penalty-dependence study: one sweep of random refinement
    (each base cell split with probability 0.5), degrees drawn uniformly in
    {pmin..pmax}, and a piecewise constant coefficient k in {1, 20} set by the
    parity of the base cell's index (a numbering of the initial coarse mesh),
    inherited by its children."""
    m = random_mesh(2, n_base, 0.5, 1, pmin, pmax, seed)
    base = m["anchor"] >> m["level"][:, None]          # base cell of every leaf
    idx = base[:, 0] + n_base * base[:, 1]
    m["kcoef"] = np.where(idx % 2 == 0, 1.0, 20.0)
    return m


def _balance_1irregular(cells, dim):
    """Refine leaves until any two leaves sharing a face (a piece of positive
    measure) differ by at most one level (a 1-irregular mesh). Leaves are
    (level, anchor); refinement only ever splits the coarser leaf of a
    violating pair, so the result contains every refinement of the input."""
    while True:
        n = len(cells)
        lev = np.array([c[0] for c in cells], dtype=np.int64)
        anc = np.array([c[1] for c in cells], dtype=np.int64).reshape(n, dim)
        fine = int(lev.max())
        size = np.left_shift(1, fine - lev)                 # cell size at the finest level
        lo = anc * size[:, None]
        hi = lo + size[:, None]
        split = np.zeros(n, dtype=bool)
        for m in range(dim):
            # pairs (i, j) with hi_i == lo_j in direction m and overlapping
            # (positive measure) in the other directions
            touch = hi[:, m][:, None] == lo[:, m][None, :]
            for t in range(dim):
                if t == m:
                    continue
                touch &= (lo[:, t][:, None] < hi[:, t][None, :]) & (lo[:, t][None, :] < hi[:, t][:, None])
            ii, jj = np.nonzero(touch)
            d = lev[ii] - lev[jj]
            split[jj[d > 1]] = True                         # j coarser by more than one level
            split[ii[d < -1]] = True
        if not split.any():
            return cells
        nxt = []
        for c, sp in zip(cells, split):
            if sp:
                nxt.extend((cl, ca, c[2]) for cl, ca in _children(c[0], c[1], dim))
            else:
                nxt.append(c)
        cells = nxt


def random_refinement_mesh(n_base, rounds, uniform=0, q=0.5, one_irregular=False, seed=1198,
                           pmin=2, pmax=6, dim=2):
    """Mesh of the random-refinement study: `rounds` rounds in which every
    current leaf is split with probability q (optionally followed by the
    refinements that make the mesh 1-irregular), then `uniform` uniform
    refinements, then degrees drawn uniformly in {pmin..pmax}; coefficient 1
    or 20 by the parity of the base cell's number, inherited by the children."""
    rng = _rng(seed)
    cells = [(c[0], c[1], i) for i, c in enumerate(_base_cells(dim, n_base))]
    for _ in range(rounds):
        u = rng.random(len(cells))
        nxt = []
        for (lev, a, b), ui in zip(cells, u):
            if ui < q:
                nxt.extend((cl, ca, b) for cl, ca in _children(lev, a, dim))
            else:
                nxt.append((lev, a, b))
        cells = nxt
        if one_irregular:
            cells = _balance_1irregular(cells, dim)
    for _ in range(uniform):
        cells = [(cl, ca, c[2]) for c in cells for cl, ca in _children(c[0], c[1], dim)]
    degree = rng.integers(pmin, pmax + 1, size=len(cells))
    kcoef = np.array([1.0 if c[2] % 2 == 0 else 20.0 for c in cells])
    return _pack(dim, n_base, [(c[0], c[1]) for c in cells], degree, kcoef)


def config_mesh(cfg: int, scale: int = 1):
    """Mesh of a named workload. scale > 1 divides n_base (small variants of
    the same recipe for tests)."""
    if cfg == 1:
        return uniform_mesh(2, max(1, 4 // scale), p=2)
    if cfg in (2, 4):
        return random_mesh(2, max(1, 32 // scale), 0.3, 3, 1, 8, seed=1002)
    if cfg == 3:
        return random_mesh(3, max(1, 16 // scale), 0.2, 2, 1, 6, seed=1003,
                           k_seed=3003, k_logrange=(-2.0, 2.0))
    raise ValueError(cfg)


def config_rhs(cfg: int, n: int):
    c = CONFIGS[cfg]
    return gaussian_rhs(n, c["rhs_seed"], c["nrhs"])


def serving_stream(n_requests=2000, seed=5005, rate=None, dof_lo=1e3,
                   dof_hi=2e5):
    """Request stream: Poisson arrivals (times in seconds, rate in requests/s;
    rate None gives arrival time 0 for all), dim 2 or 3 (50/50), target DOF
    count log-uniform in [dof_lo, dof_hi], degrees U{1..8}, SIPG or BR2
    (50/50). Each request carries its own mesh seed."""
    rng = _rng(seed)
    reqs = []
    t = 0.0
    for i in range(n_requests):
        if rate:
            t += rng.exponential(1.0 / rate)
        dim = int(rng.integers(2, 4))
        target = math.exp(rng.uniform(math.log(dof_lo), math.log(dof_hi)))
        form = "sipg" if rng.random() < 0.5 else "br2"
        reqs.append(dict(id=i, t_arrive=t, dim=dim, target_dofs=target,
                         form=form, mesh_seed=int(rng.integers(1, 2**31)),
                         rhs_seed=int(rng.integers(1, 2**31))))
    return reqs


def request_mesh(req):
    """Mesh for one serving request: the 2D or 3D random-refinement recipe
    with n_base chosen so the expected DOF count is near the target."""
    dim = req["dim"]
    if dim == 2:
        q, lmax, e_dof = 0.3, 3, 35.5          # E[(p+1)^2], p ~ U{1..8}
    else:
        q, lmax, e_dof = 0.2, 2, 253.0         # E[(p+1)^3], p ~ U{1..8}
    e_leaves = 1.0
    for _ in range(lmax):
        e_leaves = (1 - q) + q * (2 ** dim) * e_leaves
    nb = max(1, int(round((req["target_dofs"] / (e_leaves * e_dof)) ** (1.0 / dim))))
    return random_mesh(dim, nb, q, lmax, 1, 8, seed=req["mesh_seed"])
