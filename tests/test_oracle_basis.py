"""Pins for the oracle's 1D Gauss-Lobatto tables (Sec. 2.2) against closed
forms stored in tests/golden/gl_closed_forms.json and against exactness."""
import json
import math
import os

import numpy as np
import pytest

from oracle import gl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "gl_closed_forms.json")))


def _ev(s):
    return float(eval(s, {"sqrt": math.sqrt}))


@pytest.mark.parametrize("p", ["1", "2", "3", "4"])
def test_nodes_closed_form(p):
    ref = [_ev(s) for s in GOLD["nodes"][p]]
    assert np.allclose(gl.gl_nodes(int(p)), ref, atol=1e-15, rtol=0)


@pytest.mark.parametrize("p", ["2", "3", "4"])
def test_weights_closed_form(p):
    ref = [_ev(s) for s in GOLD["weights"][p]]
    assert np.allclose(gl.gl_weights(int(p)), ref, atol=1e-15, rtol=0)


@pytest.mark.parametrize("p", ["1", "2"])
def test_mass_stiffness_closed_form(p):
    M = np.array([[_ev(s) for s in r] for r in GOLD["mass"][p]])
    K = np.array([[_ev(s) for s in r] for r in GOLD["stiffness"][p]])
    assert np.allclose(gl.mass1d(int(p)), M, atol=1e-15)
    assert np.allclose(gl.stiff1d(int(p)), K, atol=1e-14)


@pytest.mark.parametrize("p", range(1, 9))
def test_gl_exactness_and_invariants(p):
    """GL quadrature is exact to degree 2p-1; K annihilates constants;
    the mass matrix integrates 1 to 1; nodes are symmetric; Lagrange basis
    is a partition of unity and interpolates."""
    x = gl.gl_nodes(p)
    w = gl.gl_weights(p)
    for k in range(2 * p):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-13
    assert np.allclose(gl.stiff1d(p).sum(axis=1), 0, atol=1e-12)
    assert abs(gl.mass1d(p).sum() - 1.0) < 1e-14
    assert np.allclose(x, 1 - x[::-1], atol=1e-16)
    L = gl.lagrange(x, np.linspace(0, 1, 17))
    assert np.allclose(L.sum(axis=1), 1, atol=1e-12)
    assert np.allclose(gl.lagrange(x, x), np.eye(p + 1), atol=1e-14)
    D = gl.lagrange_deriv(x, np.linspace(0, 1, 7))
    assert np.allclose(D.sum(axis=1), 0, atol=1e-10)
    # derivative of x^k interpolant is exact for k <= p
    t = np.linspace(0, 1, 7)
    for k in range(1, p + 1):
        assert np.allclose(D @ x ** k, k * t ** (k - 1), atol=1e-10)
