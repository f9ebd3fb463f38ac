"""Pins of the oracle's constitutive laws, internal force, energy, tangent,
adjoint and tangent products against what the paper and the mathematics fix
(CPU only).  Each check is chosen so that a plausible slip in the oracle (a
dropped term, a wrong sign, a transposed operand, a wrong weight or Jacobian)
breaks at least one of them.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle as O
import synth

LAWS = {
    "SVK": (O.SVK, np.array([5.769e6, 3.846e6, 0.0, 1.0e4, 3.0e3])),
    "NH": (O.NH, np.array([1.7e6, 0.0, 1.72667e7, 1.0e4, 3.0e3])),
    "MR": (O.MR, np.array([1.2e6, 0.45e6, 1.72667e7, 1.0e4, 3.0e3])),
}


def blk(elem, law, conn, theta, damped):
    return SimpleNamespace(elem=elem, law=law, conn=np.ascontiguousarray(conn, np.int32),
                           theta=np.asarray(theta, float), theta_e=None, damped=damped)


def small_mesh(elem, n=(2, 2, 2), size=(0.2, 0.16, 0.12)):
    if elem == O.T10:
        return synth.box_t10(*n, size=size)
    if elem == O.Q27:
        return synth.box_q27(*n, size=size)
    return synth.box_h8(*n, size=size)


def single_element(elem, rng, curved=False):
    """One element with a random well-shaped reference geometry."""
    if elem == O.T10:
        A = np.eye(3) * 0.1 + rng.uniform(-0.02, 0.02, (3, 3))
        xi = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1],
                       [.5, 0, 0], [.5, .5, 0], [0, .5, 0], [0, 0, .5], [.5, 0, .5], [0, .5, .5]])
    elif elem == O.Q27:
        A = np.eye(3) * 0.05 + rng.uniform(-0.01, 0.01, (3, 3))
        xi = np.array([[i - 1, j - 1, k - 1] for k in range(3) for j in range(3) for i in range(3)], float)
    else:
        A = np.eye(3) * 0.05 + rng.uniform(-0.01, 0.01, (3, 3))
        xi = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [1, 1, -1],
                       [-1, -1, 1], [1, -1, 1], [-1, 1, 1], [1, 1, 1]], float)
    assert np.linalg.det(A) > 0
    X = (A @ xi.T) + rng.uniform(-1, 1, (3, 1))
    if curved:
        k0 = 4 if elem == O.T10 else 0
        X[:, k0:] += rng.uniform(-0.004, 0.004, (3, X.shape[1] - k0))
    conn = np.arange(X.shape[1], dtype=np.int32)[None, :]
    return np.ascontiguousarray(X), conn


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def deformed(X, rng, scale=0.05):
    L = (X.max(axis=1) - X.min(axis=1)).max()
    return X + rng.normal(0, scale * L / 4, X.shape)


# ---------------------------------------------------------------- stresses

@pytest.mark.parametrize("law", list(LAWS))
def test_stress_is_energy_derivative(law):
    """P = d psi / dF (Sec. 3.2) and the viscous part P_v = F dphi/dEdot
    seen as the power identity P_v : Fdot_dir = d phi/d Fdot (Sec. 3.1):
    central differences of the densities in random directions."""
    lid, th = LAWS[law]
    rng = np.random.default_rng(10)
    for _ in range(10):
        F = np.eye(3) + rng.uniform(-0.3, 0.3, (3, 3))
        Fd = rng.uniform(-2, 2, (3, 3))
        Pe = O.stress(lid, th, F, Fd, damped=False)
        P = O.stress(lid, th, F, Fd, damped=True)
        D = rng.standard_normal((3, 3))
        h = 1e-6
        psi_p, _ = O.density(lid, th, F + h * D, Fd, damped=False)
        psi_m, _ = O.density(lid, th, F - h * D, Fd, damped=False)
        fd = (psi_p - psi_m) / (2 * h)
        assert abs(np.sum(Pe * D) - fd) <= 1e-7 * np.abs(Pe).max() * np.abs(D).max() * 9
        # phi is quadratic in Fdot: d phi/d Fdot [D] = (F S_v) : D exactly
        _, phi_p = O.density(lid, th, F, Fd + D, damped=True)
        _, phi_m = O.density(lid, th, F, Fd - D, damped=True)
        Pv = P - Pe
        assert abs(np.sum(Pv * D) - (phi_p - phi_m) / 2) <= 1e-9 * np.abs(Pv).max() * 9 * np.abs(D).max()


def _diag_closed_form(law, th, a, b, c):
    """d psi / d(stretch) for F = diag(a, b, c), differentiated by hand."""
    J = a * b * c
    st = np.array([a, b, c])
    if law == "SVK":
        lam, mu = th[0], th[1]
        E = 0.5 * (st ** 2 - 1)
        return st * (lam * E.sum() + 2 * mu * E)
    mu10, mu01, k = th[0], (0.0 if law == "NH" else th[1]), th[2]
    I1 = (st ** 2).sum()
    I2 = a * a * b * b + b * b * c * c + c * c * a * a
    others2 = I1 - st ** 2
    return (2 * mu10 * J ** (-2 / 3) * (st - I1 / (3 * st))
            + 2 * mu01 * J ** (-4 / 3) * (st * others2 - 2 * I2 / (3 * st))
            + k * (J - 1) * J / st)


@pytest.mark.parametrize("law", list(LAWS))
def test_stress_closed_form_uniform_stretch(law):
    lid, th = LAWS[law]
    for st in [(1.01, 0.995, 1.003), (1.3, 0.8, 1.1), (0.7, 0.9, 1.2)]:
        P = O.stress(lid, th, np.diag(st), damped=False)
        ref = _diag_closed_form(law, th, *st)
        assert rel(np.diag(P), ref) < 1e-13
        assert np.abs(P - np.diag(np.diag(P))).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("law", list(LAWS))
def test_stress_zero_under_rotation(law):
    lid, th = LAWS[law]
    rng = np.random.default_rng(11)
    R = synth.random_rotation(rng)
    W = rng.standard_normal((3, 3)); W = W - W.T
    P = O.stress(lid, th, R, W @ R, damped=True)   # Fdot = W F: rigid spin
    assert np.abs(P).max() < 1e-15 * th[:3].max() * 10


# ---------------------------------------------------------------- mesh level

@pytest.mark.parametrize("elem", [O.T10, O.H8, O.Q27])
@pytest.mark.parametrize("law", list(LAWS))
def test_reference_state_and_rigid_motion_give_zero_force(elem, law):
    lid, th = LAWS[law]
    X, conn = small_mesh(elem)
    b = [blk(elem, lid, conn, th, True)]
    rng = np.random.default_rng(12)
    scale = th[:3].max() * 0.2 ** 2
    f0 = O.internal_force(X, b, X, np.zeros_like(X))
    assert np.abs(f0).max() < 1e-9 * scale
    R = synth.random_rotation(rng)
    t = rng.standard_normal(3)
    x = R @ X + t[:, None]
    W = rng.standard_normal((3, 3)); W = W - W.T
    v = W @ (x - x.mean(axis=1, keepdims=True)) + rng.standard_normal(3)[:, None]
    f = O.internal_force(X, b, x, v)
    assert np.abs(f).max() < 1e-9 * scale


@pytest.mark.parametrize("elem", [O.T10, O.H8, O.Q27])
@pytest.mark.parametrize("law", list(LAWS))
def test_objectivity_balance_and_angular_momentum(elem, law):
    lid, th = LAWS[law]
    X, conn = small_mesh(elem)
    b = [blk(elem, lid, conn, th, True)]
    rng = np.random.default_rng(13)
    x = deformed(X, rng)
    v = rng.normal(0, 0.5, X.shape)
    f = O.internal_force(X, b, x, v)
    R = synth.random_rotation(rng)
    fr = O.internal_force(X, b, R @ x + rng.standard_normal(3)[:, None], R @ v)
    assert rel(fr, R @ f) < 1e-12
    # sum_a f_a = 0 (sum of gradients of a partition of unity vanishes)
    assert np.abs(f.sum(axis=1)).max() < 1e-13 * np.abs(f).sum(axis=1).max()
    # sum_a x_a x f_a = 0 (P F^T = F S F^T is symmetric, Sec. 3.1)
    m = np.cross(x.T, f.T).sum(axis=0)
    assert np.abs(m).max() < 1e-13 * (np.linalg.norm(x, axis=0) * np.linalg.norm(f, axis=0)).sum()


@pytest.mark.parametrize("elem,curved", [(O.T10, False), (O.T10, True), (O.H8, False), (O.Q27, False)])
@pytest.mark.parametrize("law", list(LAWS))
def test_patch_test_uniform_deformation(elem, law, curved):
    """x = A X, v = B X: F = A and Fdot = B at every point, so interior nodes
    carry no force and sum_a f_a X_a^T = P(A, B) times the body volume."""
    lid, th = LAWS[law]
    X, conn = small_mesh(elem, n=(3, 2, 2), size=(0.3, 0.2, 0.2))
    if curved:
        X = synth.curve_midside_t10(X, conn, 0.1, np.random.default_rng(5))
        # keep the boundary straight so the volume stays 0.3*0.2*0.2
        bnd = np.zeros(X.shape[1], bool)
        X0, _ = small_mesh(elem, n=(3, 2, 2), size=(0.3, 0.2, 0.2))
        for k, L in enumerate((0.3, 0.2, 0.2)):
            bnd |= np.isclose(X0[k], 0) | np.isclose(X0[k], L)
        X[:, bnd] = X0[:, bnd]
    b = [blk(elem, lid, conn, th, True)]
    rng = np.random.default_rng(14)
    A = np.eye(3) + rng.uniform(-0.1, 0.1, (3, 3))
    B = rng.uniform(-1, 1, (3, 3))
    f = O.internal_force(X, b, A @ X, B @ X)
    P = O.stress(lid, th, A, B, damped=True)
    V = 0.3 * 0.2 * 0.2
    assert rel(f @ X.T, P * V) < 1e-12
    X0, _ = small_mesh(elem, n=(3, 2, 2), size=(0.3, 0.2, 0.2))
    interior = np.ones(X.shape[1], bool)
    for k, L in enumerate((0.3, 0.2, 0.2)):
        interior &= ~(np.isclose(X0[k], 0) | np.isclose(X0[k], L))
    assert interior.sum() > 0
    assert np.abs(f[:, interior]).max() < 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("law", ["SVK", "NH", "MR"])
def test_patch_closed_form_stretch(law):
    """Uniform stretch diag(1.01, 0.995, 1.003): the assembled moment
    sum_a f_a X_a^T equals the hand-derived closed-form stress times volume."""
    lid, th = LAWS[law]
    X, conn = small_mesh(O.T10, n=(2, 2, 2), size=(0.2, 0.2, 0.2))
    st = (1.01, 0.995, 1.003)
    b = [blk(O.T10, lid, conn, th, False)]
    f = O.internal_force(X, b, np.diag(st) @ X)
    ref = np.diag(_diag_closed_form(law, th, *st)) * 0.008
    assert rel(f @ X.T, ref) < 1e-12


@pytest.mark.parametrize("elem,curved", [(O.T10, False), (O.T10, True), (O.H8, False), (O.H8, True),
                                         (O.Q27, True)])
@pytest.mark.parametrize("law", list(LAWS))
def test_force_is_energy_gradient(elem, law, curved):
    """f_i = d/de_i int psi dV (App. C, internal force by definition):
    central differences of the discrete energy Pi_h on one element."""
    lid, th = LAWS[law]
    rng = np.random.default_rng(15)
    X, conn = single_element(elem, rng, curved=curved)
    b = [blk(elem, lid, conn, th, False)]
    x = deformed(X, rng, 0.15)
    f = O.internal_force(X, b, x)
    fd = np.zeros_like(x)
    h = 1e-6 * 0.1
    for i in range(3):
        for a in range(x.shape[1]):
            xp = x.copy(); xp[i, a] += h
            xm = x.copy(); xm[i, a] -= h
            fd[i, a] = (O.energy(X, b, xp)[0] - O.energy(X, b, xm)[0]) / (2 * h)
    assert rel(f, fd) < 1e-7


@pytest.mark.parametrize("elem", [O.T10, O.H8])
def test_viscous_force_is_dissipation_gradient_and_power(elem):
    """f_v = d Phi_h / dv (Phi_h quadratic in v, so differences are exact),
    and v . f_v = sum w J_p D = 2 Phi_h with D = S_v : Edot (Sec. 3.2.3)."""
    rng = np.random.default_rng(16)
    X, conn = small_mesh(elem, n=(2, 1, 1), size=(0.2, 0.1, 0.1))
    th = np.array([0.0, 0.0, 0.0, 1.0e4, 2.0e3])
    b = [blk(elem, O.SVK, conn, th, True)]
    x = deformed(X, rng, 0.1)
    v = rng.normal(0, 1, X.shape)
    fv = O.internal_force(X, b, x, v)          # elastic parameters are zero
    fd = np.zeros_like(v)
    for i in range(3):
        for a in range(v.shape[1]):
            vp = v.copy(); vp[i, a] += 1.0
            vm = v.copy(); vm[i, a] -= 1.0
            fd[i, a] = (O.energy(X, b, x, vp)[1] - O.energy(X, b, x, vm)[1]) / 2.0
    assert rel(fv, fd) < 1e-9
    Phi = O.energy(X, b, x, v)[1]
    assert abs(np.sum(v * fv) - 2 * Phi) < 1e-12 * abs(2 * Phi)
    if elem == O.H8:     # positive weights: dissipation is non-negative
        assert Phi > 0 and np.sum(v * fv) > 0


@pytest.mark.parametrize("law", list(LAWS))
def test_linear_in_parameters(law):
    lid, th = LAWS[law]
    X, conn = small_mesh(O.T10, n=(1, 1, 1), size=(0.1, 0.1, 0.1))
    rng = np.random.default_rng(17)
    x = deformed(X, rng); v = rng.normal(0, 1, X.shape)
    f1 = O.internal_force(X, [blk(O.T10, lid, conn, th, True)], x, v)
    f2 = O.internal_force(X, [blk(O.T10, lid, conn, 2 * th, True)], x, v)
    assert rel(f2, 2 * f1) < 1e-15


def test_inverted_reference_element_is_rejected():
    X, conn = small_mesh(O.T10, n=(1, 1, 1), size=(0.1, 0.1, 0.1))
    bad = conn.copy()
    # mirror the first element: swap corners 2<->3 and the mid-edge nodes that follow them
    for i, j in [(1, 2), (4, 6), (8, 9)]:
        bad[0, [i, j]] = bad[0, [j, i]]
    with pytest.raises(RuntimeError, match="-3"):
        O.internal_force(X, [blk(O.T10, O.SVK, bad, LAWS["SVK"][1], False)], X)


# ---------------------------------------------------------------- tangents

@pytest.mark.parametrize("elem,curved", [(O.T10, False), (O.T10, True), (O.H8, True), (O.Q27, True)])
@pytest.mark.parametrize("law", list(LAWS))
def test_element_tangent_matches_differences(elem, law, curved):
    """Paper's closed-form SVK and Mooney-Rivlin tangents (App. C) plus the
    derived Kelvin-Voigt blocks against central differences of f."""
    lid, th = LAWS[law]
    rng = np.random.default_rng(18)
    X, conn = single_element(elem, rng, curved=curved)
    x = deformed(X, rng, 0.15)
    v = rng.normal(0, 2, X.shape)
    b = [blk(elem, lid, conn, th, True)]
    K, Cv = O.element_tangent(elem, lid, th, X, x, v, damped=True)
    n = X.shape[1]
    Kfd = np.zeros_like(K); Cfd = np.zeros_like(Cv)
    h = 1e-6 * 0.1
    for a in range(n):
        for s in range(3):
            xp = x.copy(); xp[s, a] += h
            xm = x.copy(); xm[s, a] -= h
            col = (O.internal_force(X, b, xp, v) - O.internal_force(X, b, xm, v)) / (2 * h)
            Kfd[:, 3 * a + s] = col.T.ravel()
            vp = v.copy(); vp[s, a] += 1.0
            vm = v.copy(); vm[s, a] -= 1.0
            col = (O.internal_force(X, b, x, vp) - O.internal_force(X, b, x, vm)) / 2.0
            Cfd[:, 3 * a + s] = col.T.ravel()
    assert rel(K, Kfd) < 1e-7
    assert rel(Cv, Cfd) < 1e-9


@pytest.mark.parametrize("law", list(LAWS))
def test_hyperelastic_tangent_is_symmetric(law):
    lid, th = LAWS[law]
    rng = np.random.default_rng(19)
    X, conn = single_element(O.T10, rng, curved=True)
    x = deformed(X, rng, 0.2)
    K, Cv = O.element_tangent(O.T10, lid, th, X, x, None, damped=False)
    assert np.abs(K - K.T).max() < 1e-12 * np.abs(K).max()


@pytest.mark.parametrize("elem", [O.T10, O.H8, O.Q27])
@pytest.mark.parametrize("law", list(LAWS))
def test_assembled_vjp_jvp(elem, law):
    """Adjoint and tangent products on a small mesh: w.(K dx + C dv) equals
    gx.dx + gv.dv, the JVP matches differences of f, and gtheta matches
    exact differences in each parameter row (f is linear in each)."""
    lid, th = LAWS[law]
    X, conn = small_mesh(elem, n=(2, 2, 1) if elem != O.Q27 else (3, 1, 1), size=(0.2, 0.2, 0.1))
    rng = np.random.default_rng(20)
    ne = conn.shape[0]
    th_e = th[:, None] * rng.uniform(0.5, 2.0, (5, ne))
    b = SimpleNamespace(elem=elem, law=lid, conn=conn, theta=th, theta_e=th_e, damped=True)
    x = deformed(X, rng, 0.1); v = rng.normal(0, 1, X.shape)
    w = rng.standard_normal(X.shape); dx = rng.standard_normal(X.shape) * 0.01
    dv = rng.standard_normal(X.shape)
    gx, gv, gt = O.vjp(X, [b], x, v, w)
    df = O.jvp(X, [b], x, v, dx, dv)
    lhs = np.sum(w * df); rhs = np.sum(gx * dx) + np.sum(gv * dv)
    assert abs(lhs - rhs) < 1e-12 * (np.abs(w * df).sum())
    h = 1e-6
    fp = O.internal_force(X, [b], x + h * dx, v + h * dv)
    fm = O.internal_force(X, [b], x - h * dx, v - h * dv)
    assert rel(df, (fp - fm) / (2 * h)) < 1e-7
    f0 = O.internal_force(X, [b], x, v)
    unused = {O.SVK: [2], O.NH: [1], O.MR: []}[lid]
    for p in range(5):
        if p in unused:
            assert np.all(gt[p] == 0)
            continue
        for e in rng.choice(ne, 3, replace=False):
            t2 = th_e.copy(); t2[p, e] += 0.5 * th_e[p, e]
            b2 = SimpleNamespace(**{**b.__dict__, "theta_e": t2})
            f2 = O.internal_force(X, [b2], x, v)
            ref = np.sum(w * (f2 - f0)) / (0.5 * th_e[p, e])
            assert abs(gt[p, e] - ref) < 1e-8 * max(abs(ref), 1e-300) + 1e-10 * np.abs(w * f0).sum() / th_e[p, e]


# ---------------------------------------------------------------- inverted points

def _brute_inverted(elem, X, conn, x):
    """Points with det F <= 0, from the sign of det(dx/dxi) / det(dX/dxi) where
    both Jacobians are central differences of the interpolated maps
    sum_a x_a s_a(xi) (exact for the quadratic T10 and trilinear H8 maps up
    to rounding); uses only the shape functions and the rule's points."""
    xi, w = O.quadrature(elem)
    h = 1e-2
    n, mn = 0, np.inf
    for e in range(conn.shape[0]):
        xe, Xe = x[:, conn[e]], X[:, conn[e]]
        for q in range(len(w)):
            D, DX = np.empty((3, 3)), np.empty((3, 3))
            for k in range(3):
                p = np.array(xi[q], float); p[k] += h
                m = np.array(xi[q], float); m[k] -= h
                ds = (O.shape(elem, p) - O.shape(elem, m)) / (2 * h)
                D[:, k], DX[:, k] = xe @ ds, Xe @ ds
            d = np.linalg.det(D) / np.linalg.det(DX)
            n += int(d <= 0)
            mn = min(mn, abs(d))
    return n, mn


@pytest.mark.parametrize("elem", [O.T10, O.H8, O.Q27])
def test_inverted_point_count(elem):
    if elem == O.T10:
        X, conn = synth.box_t10(4, 2, 2, size=(0.4, 0.2, 0.2))
    elif elem == O.Q27:
        X, conn = synth.box_q27(3, 2, 2, size=(0.3, 0.2, 0.2))
    else:
        X, conn = synth.box_h8(4, 3, 2, size=(0.4, 0.3, 0.2))
    b = blk(elem, O.SVK, conn, LAWS["SVK"][1], False)
    n_qp = conn.shape[0] * len(O.quadrature(elem)[1])
    # reference state and a rigid motion: none; a reflection or a collapse: all
    assert O.count_inverted(X, [b], X)[0] == 0
    R = synth.random_rotation(np.random.default_rng(3))
    assert O.count_inverted(X, [b], R @ X + 0.3)[0] == 0
    assert O.count_inverted(X, [b], X * np.array([[1.0], [1.0], [-1.0]]))[0] == n_qp
    assert O.count_inverted(X, [b], np.zeros_like(X))[0] == n_qp
    # tangled: a mixed count, equal to the brute-force sign count
    seed, sigma = {O.T10: (1, 0.04), O.H8: (0, 0.04), O.Q27: (3, 0.025)}[elem]
    x = X + np.random.default_rng(seed).normal(0, sigma, X.shape)
    n, mn = O.count_inverted(X, [b], x)
    nb, mnb = _brute_inverted(elem, X, conn, x)
    assert 0 < n < n_qp
    assert n == nb
    assert mn > 1e-3 and abs(mn - mnb) < 1e-9


# ---------------------------------------------------------- position offsets

@pytest.mark.parametrize("elem", [O.T10, O.H8])
def test_results_depend_only_on_position_differences(elem):
    # The kinematics use positions only through differences of an element's
    # nodes (the parent gradients sum to zero, App. A), and the oracle forms
    # those differences before any product.  With coordinates on a grid of
    # 2^-40 m and a translation by powers of two, every translated
    # coordinate is exact and so is every difference: all outputs must be
    # bitwise equal.  A literal F = N H on coordinates of order 1000 m would
    # lose about eleven digits here.
    rng = np.random.default_rng(41)
    q = 2.0 ** -40
    X, conn = small_mesh(elem, n=(3, 2, 2), size=(0.03, 0.02, 0.02))
    X = np.round(X / q) * q
    x = np.round(deformed(X, rng, 0.02) / q) * q
    v = rng.normal(0, 0.1, X.shape)
    w = rng.standard_normal(X.shape)
    dx = rng.standard_normal(X.shape) * 1e-3
    T = np.array([[1024.0], [-2048.0], [512.0]])
    assert np.array_equal((X + T) - T, X) and np.array_equal((x + T) - T, x)
    for law, th in LAWS.values():
        b = [blk(elem, law, conn, th, True)]
        for fn in (lambda XX, xx: O.internal_force(XX, b, xx, v),
                   lambda XX, xx: O.vjp(XX, b, xx, v, w),
                   lambda XX, xx: O.jvp(XX, b, xx, v, dx, None),
                   lambda XX, xx: O.count_inverted(XX, b, xx)):
            a0, a1 = fn(X, x), fn(X + T, x + T)
            for u, t in zip(a0 if isinstance(a0, tuple) else (a0,), a1 if isinstance(a1, tuple) else (a1,)):
                assert np.array_equal(np.asarray(u), np.asarray(t))
