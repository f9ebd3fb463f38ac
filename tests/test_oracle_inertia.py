"""Pins of the oracle's inertia and step functions (Sec. 4.1 consistent mass,
Sec. 7 backward-Euler residual and its velocity derivative), against what
the mathematics fixes: the exactness degree of the mass rule, the exact
Gram integrals of the shape functions on straight-sided elements, the mass
of a rigid translation, symmetry and definiteness, the special cases that
reduce the residual to one of its terms, central differences of the
residual, and quadratic convergence of the exact Newton step."""
import copy
from math import factorial

import numpy as np
import pytest

import oracle as O
import synth
from _util import rel


def test_mass_rule_t10_exact_to_degree_five_not_six():
    xi, w = O.mass_rule(synth.T10)
    assert xi.shape == (15, 3) and np.all(w > 0)
    # barycentric coordinates of every point are positive (interior points)
    assert np.all(xi > 0) and np.all(xi.sum(axis=1) < 1)
    exact = lambda i, j, k: factorial(i) * factorial(j) * factorial(k) / factorial(i + j + k + 3)
    worst6 = 0.0
    for d in range(7):
        for i in range(d + 1):
            for j in range(d + 1 - i):
                k = d - i - j
                q = float((w * xi[:, 0] ** i * xi[:, 1] ** j * xi[:, 2] ** k).sum())
                e = abs(q - exact(i, j, k)) / exact(i, j, k)
                if d <= 5:
                    assert e <= 1e-14, (i, j, k, e)
                else:
                    worst6 = max(worst6, e)
    assert worst6 > 1e-3


def test_mass_rule_h8_is_gauss_2x2x2():
    xi, w = O.mass_rule(synth.H8)
    assert xi.shape == (8, 3) and np.allclose(w, 1.0)
    for i in range(4):
        exact = 2.0 / (i + 1) if i % 2 == 0 else 0.0
        assert abs(float((w * xi[:, 0] ** i).sum()) / 4.0 - exact) <= 1e-14
    assert abs(float((w * xi[:, 0] ** 4).sum()) / 4.0 - 2.0 / 5.0) > 1e-3


def _monomials(elem):
    if elem == synth.T10:
        return [(i, j, k) for i in range(3) for j in range(3) for k in range(3) if i + j + k <= 2]
    if elem == synth.Q27:
        return [(i, j, k) for i in range(3) for j in range(3) for k in range(3)]
    return [(i, j, k) for i in range(2) for j in range(2) for k in range(2)]


def _shape_coefficients(elem):
    """Coefficients of every shape function in the monomial basis, recovered
    by interpolating the oracle's shape functions at random points (they are
    polynomials of that basis, so the fit is exact to rounding)."""
    mono = _monomials(elem)
    rng = np.random.default_rng(0)
    pts = rng.uniform(0.0, 0.3, (40, 3)) if elem == synth.T10 else rng.uniform(-1, 1, (40, 3))
    V = np.array([[p[0] ** i * p[1] ** j * p[2] ** k for (i, j, k) in mono] for p in pts])
    S = np.array([O.shape(elem, p) for p in pts])
    coef, *_ = np.linalg.lstsq(V, S, rcond=None)
    assert np.abs(V @ coef - S).max() <= 1e-13
    return mono, coef   # coef[m][a]


def _exact_gram(elem):
    """int s_a s_b over the parent element, exactly from monomial integrals."""
    mono, coef = _shape_coefficients(elem)
    if elem == synth.T10:
        integ = lambda i, j, k: factorial(i) * factorial(j) * factorial(k) / factorial(i + j + k + 3)
    else:
        one = lambda i: 2.0 / (i + 1) if i % 2 == 0 else 0.0
        integ = lambda i, j, k: one(i) * one(j) * one(k)
    n = coef.shape[1]
    G = np.zeros((n, n))
    for m1, (a1, b1, c1) in enumerate(mono):
        for m2, (a2, b2, c2) in enumerate(mono):
            G += np.outer(coef[m1], coef[m2]) * integ(a1 + a2, b1 + b2, c1 + c2)
    return G


@pytest.mark.parametrize("elem", [synth.T10, synth.H8, synth.Q27], ids=["T10", "H8", "Q27"])
def test_element_mass_equals_exact_gram_matrix_on_affine_element(elem):
    """For an affine parent-to-reference map u = A xi + b, m_ij = rho det A
    int s_i s_j dxi exactly; the rule is exact for the degree-4 (T10) or
    degree-2-per-direction (H8) integrand."""
    rng = np.random.default_rng(1)
    A = np.eye(3) * 0.02 + rng.uniform(-0.004, 0.004, (3, 3))
    b = rng.uniform(-1, 1, 3)
    if elem == synth.T10:
        nodes = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [.5, 0, 0], [.5, .5, 0], [0, .5, 0],
                          [0, 0, .5], [.5, 0, .5], [0, .5, .5]], float)
    elif elem == synth.Q27:
        nodes = np.array([[i - 1, j - 1, k - 1] for k in range(3) for j in range(3) for i in range(3)], float)
    else:
        nodes = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [1, 1, -1], [-1, -1, 1], [1, -1, 1],
                          [-1, 1, 1], [1, 1, 1]], float)
    Xe = (nodes @ A.T + b).T
    rho = 7800.0
    M = O.element_mass(elem, rho, Xe)
    G = _exact_gram(elem) * rho * np.linalg.det(A)
    assert np.abs(M - G).max() <= 1e-13 * np.abs(G).max()
    assert np.allclose(M, M.T, rtol=0, atol=1e-15 * np.abs(M).max())
    assert np.linalg.eigvalsh(M).min() > 0


def _box(elem, n=(3, 2, 2), cell=0.02, curved=False, seed=2):
    rng = np.random.default_rng(seed)
    size = tuple(k * cell for k in n)
    X, conn = {synth.T10: synth.box_t10, synth.H8: synth.box_h8, synth.Q27: synth.box_q27}[elem](*n, size=size)
    if curved:
        X = synth.curve_midside_t10(X, conn, 0.08, rng) if elem == synth.T10 else X + rng.uniform(
            -0.03 * cell, 0.03 * cell, X.shape)
    return X, conn, size


@pytest.mark.parametrize("elem", [synth.T10, synth.H8, synth.Q27], ids=["T10", "H8", "Q27"])
def test_mass_of_rigid_translation_is_rho_v(elem):
    """u = c at every node: sum_i (M u)_i = rho V c, the body's mass times c
    (the shape functions sum to one, Sec. 4.1)."""
    X, conn, size = _box(elem)
    rho = 1200.0
    blk = synth.Block(elem, synth.NH, conn, np.zeros(5), rho=rho)
    c = np.array([0.3, -1.2, 2.0])
    y = O.mass_action(X, [blk], np.repeat(c[:, None], X.shape[1], axis=1))
    V = size[0] * size[1] * size[2]
    assert np.abs(y.sum(axis=1) - rho * V * c).max() <= 1e-13 * rho * V * np.abs(c).max()
    # every row sum is positive for the positive-weight rule of H8 (lumped
    # masses); T10 corner rows are negative for the consistent mass
    if elem == synth.H8:
        assert np.all(y[0] / c[0] > 0)


@pytest.mark.parametrize("elem", [synth.T10, synth.H8, synth.Q27], ids=["T10", "H8", "Q27"])
def test_assembled_mass_symmetric_positive_definite(elem):
    X, conn, _ = _box(elem, curved=True)
    blk = synth.Block(elem, synth.SVK, conn, np.zeros(5), rho=900.0)
    n = X.shape[1]
    M = np.zeros((n, n))
    for j in range(n):
        u = np.zeros((3, n)); u[0, j] = 1.0
        M[:, j] = O.mass_action(X, [blk], u)[0]
        # components do not couple (M_e = [m_ij I_3])
        assert np.all(O.mass_action(X, [blk], u)[1:] == 0)
    assert np.abs(M - M.T).max() <= 1e-15 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 1e-8 * np.abs(M).max()


def _step_problem(elem, law, damped, seed=3, rho=1100.0):
    rng = np.random.default_rng(seed)
    X, conn, _ = _box(elem, curved=True, seed=seed)
    th = {synth.SVK: np.array([5.769e6, 3.846e6, 0.0, 1e4, 3e3]),
          synth.NH: np.array([1.7e6, 0.0, 1.72667e7, 1e4, 3e3]),
          synth.MR: np.array([1.2e6, 0.45e6, 1.72667e7, 1e4, 3e3])}[law].copy()
    if not damped:
        th[3:] = 0
    blk = synth.Block(elem, law, conn, th, damped=damped, rho=rho)
    blk.theta_e = th[:, None] * rng.uniform(0.5, 2.0, (5, conn.shape[0]))
    q_n = synth.sinusoidal_state(X, 0.03, rng)
    v_n = rng.normal(0, 0.3, X.shape)
    v = v_n + rng.normal(0, 0.3, X.shape)
    f_ext = rng.normal(0, 10.0, X.shape)
    return X, blk, q_n, v_n, v, f_ext


@pytest.mark.parametrize("damped", [False, True], ids=["el", "KV"])
def test_residual_reduces_to_its_terms(damped):
    X, blk, q_n, v_n, v, f_ext = _step_problem(synth.T10, synth.NH, damped)
    h = 1e-3
    # no material stiffness or damping: g = M (v - v_n) / h - f_ext
    b0 = copy.copy(blk); b0.theta_e = np.zeros_like(blk.theta_e)
    g = O.step_residual(X, [b0], q_n, v_n, v, h, f_ext)
    ref = O.mass_action(X, [blk], v - v_n) / h - f_ext
    assert rel(g, ref) <= 1e-14
    # no mass: g = f_int(q_n + h v, v) - f_ext
    b1 = copy.copy(blk); b1.rho = 0.0
    g = O.step_residual(X, [b1], q_n, v_n, v, h, f_ext)
    q = O.step_positions(h, v, q_n)
    ref = O.internal_force(X, [b1], q, v if damped else None) - f_ext
    assert rel(g, ref) <= 1e-14
    # the step map: v = 0 leaves q = q_n exactly
    g = O.step_residual(X, [b1], q_n, v_n, np.zeros_like(v), h)
    assert np.array_equal(g, O.internal_force(X, [b1], q_n, np.zeros_like(v) if damped else None))


@pytest.mark.parametrize("law", [synth.SVK, synth.NH, synth.MR], ids=["SVK", "NH", "MR"])
@pytest.mark.parametrize("damped", [False, True], ids=["el", "KV"])
@pytest.mark.parametrize("elem", [synth.T10, synth.H8], ids=["T10", "H8"])
def test_newton_operator_is_derivative_of_residual(elem, law, damped):
    """(M/h + hK + C) dv against central differences of g in v, and against
    the assembled matrix of the same blocks."""
    X, blk, q_n, v_n, v, f_ext = _step_problem(elem, law, damped, seed=4)
    h = 2e-3
    rng = np.random.default_rng(5)
    dv = rng.normal(0, 1.0, X.shape)
    y = O.newton_operator(X, [blk], q_n, v, h, dv)
    eps = 1e-5
    fd = (O.step_residual(X, [blk], q_n, v_n, v + eps * dv, h, f_ext)
          - O.step_residual(X, [blk], q_n, v_n, v - eps * dv, h, f_ext)) / (2 * eps)
    assert rel(fd, y) <= 1e-7, rel(fd, y)
    A = O.newton_matrix(X, [blk], q_n, v, h)
    assert rel((A @ dv.ravel()).reshape(dv.shape), y) <= 1e-13


@pytest.mark.parametrize("damped", [False, True], ids=["el", "KV"])
def test_exact_newton_steps_converge_quadratically(damped):
    """Exact Newton steps from the predictor v = v_n: the consistent
    linearisation gives a reduction that accelerates step by step (each
    residual about the square of the previous one) down to rounding."""
    X, blk, q_n, v_n, v, f_ext = _step_problem(synth.T10, synth.NH, damped, seed=6)
    h = 1e-4
    norms = []
    vk = v_n.copy()
    for it in range(4):
        v1, dv, g = O.newton_step(X, [blk], q_n, v_n, vk, h, f_ext)
        norms.append(np.abs(g).max())
        vk = v1
    norms.append(np.abs(O.step_residual(X, [blk], q_n, v_n, vk, h, f_ext)).max())
    assert norms[1] <= 0.1 * norms[0]
    assert norms[2] <= 0.01 * norms[1]
    assert norms[3] <= 1e-4 * norms[2]
    assert norms[4] <= 1e-9 * norms[0]
