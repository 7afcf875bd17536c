"""One-dimensional Gauss-Lobatto nodal basis and exact 1D matrices (oracle).

TEST INFRASTRUCTURE: the FP64 CPU oracle. Only tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the GPU library never does.

Sec. 2.2: on the reference interval [0,1] the nodal points of degree p are the
p+1 Gauss-Lobatto points (the endpoints and the roots of the derivative of the
Legendre polynomial P_p, mapped from [-1,1]). The basis is the Lagrange basis
on those points. All integrals are exact: products of two degree-p
polynomials are integrated with a (p+1)-point Gauss-Legendre rule.
"""
from __future__ import annotations

import functools
import numpy as np
from numpy.polynomial import legendre as npleg


@functools.lru_cache(maxsize=None)
def gl_nodes(p: int) -> np.ndarray:
    """Gauss-Lobatto nodes of degree p on [0,1] (Sec. 2.2)."""
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    dc = npleg.legder(c)              # coefficients of P_p'
    ddc = npleg.legder(dc)            # P_p''
    r = np.sort(npleg.legroots(dc).real)
    for _ in range(4):                # Newton polish on P_p'(x) = 0
        r = r - npleg.legval(r, dc) / npleg.legval(r, ddc)
    x = np.concatenate([[-1.0], r, [1.0]])
    x = 0.5 * (x - x[::-1])           # enforce exact symmetry about 0
    out = 0.5 * (x + 1.0)
    out[0], out[-1] = 0.0, 1.0
    return out


@functools.lru_cache(maxsize=None)
def gauss(q: int):
    """q-point Gauss-Legendre rule on [0,1]: (points, weights)."""
    x, w = npleg.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange(nodes, x) -> np.ndarray:
    """L[k, i] = l_i(x_k), Lagrange basis on `nodes`, product formula."""
    nodes = np.asarray(nodes, dtype=float)
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = len(nodes)
    L = np.ones((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                L[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return L


def lagrange_deriv(nodes, x) -> np.ndarray:
    """D[k, i] = l_i'(x_k), derivative of the product formula."""
    nodes = np.asarray(nodes, dtype=float)
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            t = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    t *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += t
    return D


@functools.lru_cache(maxsize=None)
def mass1d(p: int) -> np.ndarray:
    """M_ij = int_0^1 l_i l_j (exact, (p+1)-point Gauss)."""
    xq, wq = gauss(p + 1)
    B = lagrange(gl_nodes(p), xq)
    return B.T @ (wq[:, None] * B)


@functools.lru_cache(maxsize=None)
def stiff1d(p: int) -> np.ndarray:
    """K_ij = int_0^1 l_i' l_j' (exact)."""
    xq, wq = gauss(p + 1)
    G = lagrange_deriv(gl_nodes(p), xq)
    return G.T @ (wq[:, None] * G)


def gl_weights(p: int) -> np.ndarray:
    """Gauss-Lobatto quadrature weights on [0,1] (integrals of the basis)."""
    return mass1d(p).sum(axis=0)
