"""Pins of the oracle's element library and quadrature rules (CPU only).

The T10 shape functions and gradients are printed separately in App. A of the
paper; each is checked against the paper's node table (golden fixture) and
against the other by finite differences, so a mistyped coefficient in either
fails.  The quadrature rules (not printed in the paper) are pinned by exact
integration of monomials against closed forms.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "t10_nodes.txt")
GOLD_Q27 = os.path.join(os.path.dirname(__file__), "golden", "q27_nodes.txt")


def t10_table():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        tok = line.split()
        vals = [float(Fraction(t)) for t in tok[1:]]
        rows.append(vals)
    a = np.array(rows)
    return a[:, :4], a[:, 4:]


H8_NODES = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [1, 1, -1],
                     [-1, -1, 1], [1, -1, 1], [-1, 1, 1], [1, 1, 1]], dtype=float)


def q27_table():
    """(i, j, k) and parent coordinates of the Q27 nodes (App. A node table)."""
    rows = [list(map(int, line.split()[1:])) for line in open(GOLD_Q27)
            if line.strip() and not line.startswith("#")]
    a = np.array(rows)
    return a[:, :3], a[:, 3:].astype(float)


def nodes(elem):
    return {O.T10: lambda: t10_table()[1], O.H8: lambda: H8_NODES, O.Q27: lambda: q27_table()[1]}[elem]()


def rand_pts(elem, n, rng):
    if elem == O.T10:
        p = rng.dirichlet(np.ones(4), n)[:, 1:]
    else:
        p = rng.uniform(-1, 1, (n, 3))
    return p


def test_t10_barycentric_columns_match_parent():
    L, xi = t10_table()
    # L1 = 1 - xi - eta - zeta, L2..L4 = xi, eta, zeta (App. A, barycentric mapping)
    assert np.allclose(L[:, 1:], xi)
    assert np.allclose(L[:, 0], 1 - xi.sum(axis=1))


@pytest.mark.parametrize("elem", [O.T10, O.H8, O.Q27])
def test_kronecker_property(elem):
    X = nodes(elem)
    S = np.array([O.shape(elem, p) for p in X])
    assert np.array_equal(S, np.eye(len(X)))


@pytest.mark.parametrize("elem", [O.T10, O.H8, O.Q27])
def test_partition_of_unity_and_gradient_sum(elem):
    rng = np.random.default_rng(1)
    for p in rand_pts(elem, 50, rng):
        assert abs(O.shape(elem, p).sum() - 1) < 1e-14
        assert np.abs(O.dshape(elem, p).sum(axis=0)).max() < 1e-13


@pytest.mark.parametrize("elem", [O.T10, O.H8, O.Q27])
def test_gradient_table_is_derivative_of_shape_table(elem):
    rng = np.random.default_rng(2)
    h = 1e-6
    for p in rand_pts(elem, 20, rng):
        G = O.dshape(elem, p)
        Gfd = np.zeros_like(G)
        for k in range(3):
            e = np.zeros(3); e[k] = h
            Gfd[:, k] = (O.shape(elem, p + e) - O.shape(elem, p - e)) / (2 * h)
        assert np.abs(G - Gfd).max() < 1e-8


@pytest.mark.parametrize("elem", [O.T10, O.H8, O.Q27])
def test_linear_completeness(elem):
    # sum_a xi_a (ds_a/dxi)^T = I and sum_a s_a xi_a = xi: an affine map is reproduced
    X = nodes(elem)
    rng = np.random.default_rng(3)
    for p in rand_pts(elem, 20, rng):
        G = O.dshape(elem, p)
        assert np.abs(X.T @ G - np.eye(3)).max() < 1e-13
        assert np.abs(O.shape(elem, p) @ X - p).max() < 1e-14


def test_t10_quadratic_completeness():
    # any quadratic polynomial is reproduced by the 10 quadratic Lagrange functions
    X = nodes(O.T10)
    rng = np.random.default_rng(4)
    c = rng.standard_normal(10)

    def q(p):
        x, y, z = p
        return c @ np.array([1, x, y, z, x * x, y * y, z * z, x * y, y * z, x * z])

    vals = np.array([q(p) for p in X])
    for p in rand_pts(O.T10, 20, rng):
        assert abs(O.shape(O.T10, p) @ vals - q(p)) < 1e-13


def _tet_monomial(a, b, c):
    # integral of xi^a eta^b zeta^c over the unit tetrahedron (Dirichlet integral)
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)


def _cube_monomial(a, b, c):
    f = lambda n: 0.0 if n % 2 else 2.0 / (n + 1)
    return f(a) * f(b) * f(c)


def test_t10_rule_exact_to_degree_3_not_4():
    xi, w = O.quadrature(O.T10)
    assert len(w) == 5
    assert abs(w.sum() - 1 / 6) < 1e-16
    for a in range(4):
        for b in range(4 - a):
            for c in range(4 - a - b):
                q = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
                assert abs(q - _tet_monomial(a, b, c)) < 1e-16
    q4 = np.sum(w * xi[:, 0] ** 4)
    assert abs(q4 - _tet_monomial(4, 0, 0)) > 1e-6


def test_h8_rule_exact_per_axis_to_degree_3():
    xi, w = O.quadrature(O.H8)
    assert len(w) == 8 and abs(w.sum() - 8) < 1e-14
    for a in range(4):
        for b in range(4):
            for c in range(4):
                q = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
                assert abs(q - _cube_monomial(a, b, c)) < 1e-14
    q4 = np.sum(w * xi[:, 0] ** 4)
    assert abs(q4 - _cube_monomial(4, 0, 0)) > 1e-3


def test_q27_table_is_lexicographic_and_tensor_product():
    """The node table orders (i, j, k) with i fastest, at parent coordinates
    i - 1 etc.; every shape function is the product of the 1-D quadratic
    Lagrange polynomials of its indices (App. A: tensor product basis)."""
    ijk, xi = q27_table()
    assert np.array_equal(ijk[:, 0] + 3 * ijk[:, 1] + 9 * ijk[:, 2], np.arange(27))
    assert np.array_equal(xi, ijk - 1)
    L = [lambda s: s * (s - 1) / 2, lambda s: 1 - s * s, lambda s: s * (s + 1) / 2]
    rng = np.random.default_rng(5)
    for p in rng.uniform(-1, 1, (10, 3)):
        ref = np.array([L[i](p[0]) * L[j](p[1]) * L[k](p[2]) for i, j, k in ijk])
        assert np.abs(O.shape(O.Q27, p) - ref).max() < 1e-15


def test_q27_triquadratic_completeness():
    """Every polynomial of degree <= 2 in each coordinate separately is
    reproduced by the 27 functions (and so is its gradient)."""
    X = nodes(O.Q27)
    rng = np.random.default_rng(6)
    c = rng.standard_normal((3, 3, 3))

    def f(p):
        return sum(c[a, b, d] * p[0] ** a * p[1] ** b * p[2] ** d for a in range(3) for b in range(3) for d in range(3))

    def grad(p):
        g = np.zeros(3)
        for a in range(3):
            for b in range(3):
                for d in range(3):
                    g[0] += c[a, b, d] * (a * p[0] ** max(a - 1, 0) if a else 0) * p[1] ** b * p[2] ** d
                    g[1] += c[a, b, d] * p[0] ** a * (b * p[1] ** max(b - 1, 0) if b else 0) * p[2] ** d
                    g[2] += c[a, b, d] * p[0] ** a * p[1] ** b * (d * p[2] ** max(d - 1, 0) if d else 0)
        return g

    vals = np.array([f(p) for p in X])
    for p in rng.uniform(-1, 1, (20, 3)):
        assert abs(O.shape(O.Q27, p) @ vals - f(p)) < 1e-12
        assert np.abs(O.dshape(O.Q27, p).T @ vals - grad(p)).max() < 1e-12


def test_q27_rule_is_gauss_3x3x3_exact_per_axis_to_degree_5():
    xi, w = O.quadrature(O.Q27)
    assert len(w) == 27 and abs(w.sum() - 8) < 1e-14 and np.all(w > 0)
    for a in range(6):
        for b in range(6):
            for c in range(6):
                q = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
                assert abs(q - _cube_monomial(a, b, c)) < 1e-14
    assert abs(np.sum(w * xi[:, 0] ** 6) - _cube_monomial(6, 0, 0)) > 1e-3
    # the mass rule of Q27 is the same rule (exact for degree 4 per axis)
    xm, wm = O.mass_rule(O.Q27)
    assert np.array_equal(xm, xi) and np.array_equal(wm, w)
