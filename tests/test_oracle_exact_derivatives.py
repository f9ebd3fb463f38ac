"""The oracle against 60-digit evaluations that take no stress formula from
it (CPU only): the elastic stress is the derivative of the strain energy
(Sec. 3.2.1, 3.2.2), formed by exact differentiation with dual numbers, the
viscous stress F S_v(Edot) (Sec. 3.2.3), and the element force the rule's
sum of w_q J_p P h_a (Sec. 4.3, 6).  A second level of dual numbers gives
the tangent product K dx + C dv without differencing, and one such product
per unit direction the whole element Jacobian, whose transpose applied to w
is the adjoint.  The consistent mass (Sec. 4.1) from its own transcription
of each mass rule gives the step residual and, through the same dual
numbers, the Newton operator (Sec. 7); the revolute joint's values and
transpose scatter (Sec. 2.2, App. B.1) follow from its defining rows, the
Jacobian again by exact differentiation.  Every element type (T10, H8, Q27)
and every law (Saint Venant-Kirchhoff, Mooney-Rivlin, Neo-Hookean, with and
without Kelvin-Voigt damping) on one curved element, offset by tens of element
sizes, under a rotation and strains of a few per cent.  60 digits leave
the reference exact far below FP64 rounding, so what the bars measure is
the oracle's own rounding.  The force is a difference of terms larger than
itself by about the inverse strain times the bulk-to-shear ratio (some
10^3 here), so its FP64 evaluation is good to a few hundred units of
rounding: the bar is BAR = 2e-13 of each array's norm.  A planted mistake
(a parameter off by 1e-9 of itself, a dropped term, a transposed operand)
moves the oracle by 1e-10 or more.
"""
import decimal
import os
from types import SimpleNamespace

import numpy as np
import pytest

import oracle as O

D = decimal.Decimal
CTX = decimal.Context(prec=60)
GOLD = os.path.join(os.path.dirname(__file__), "golden")
BAR = 2e-13
JBAR = 1e-12


class Dual:
    """a + b e with e^2 = 0.  The parts may themselves be duals, so that
    two levels give a directional derivative of a derivative."""
    __slots__ = ("a", "b")

    def __init__(self, a, b=0):
        self.a, self.b = a, b

    @staticmethod
    def lift(o):
        return o if isinstance(o, Dual) else Dual(o)

    def __add__(self, o):
        o = Dual.lift(o)
        return Dual(self.a + o.a, self.b + o.b)

    __radd__ = __add__

    def __sub__(self, o):
        o = Dual.lift(o)
        return Dual(self.a - o.a, self.b - o.b)

    def __rsub__(self, o):
        return Dual.lift(o) - self

    def __neg__(self):
        return Dual(-self.a, -self.b)

    def __mul__(self, o):
        o = Dual.lift(o)
        return Dual(self.a * o.a, self.a * o.b + self.b * o.a)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = Dual.lift(o)
        q = self.a / o.a
        return Dual(q, (self.b - q * o.b) / o.a)

    def __rtruediv__(self, o):
        return Dual.lift(o) / self

    def __pow__(self, p):   # a real exponent p (not a dual)
        return Dual(self.a ** p, p * self.a ** (p - 1) * self.b)


def eps(x):
    """The e part of a dual (0 for a plain number)."""
    return x.b if isinstance(x, Dual) else 0


def real(x):
    return x.a if isinstance(x, Dual) else x


def dec(t):
    return D(repr(float(t)))   # every FP64 value is a short exact decimal at 60 digits


# ------------------------------------------------------------------ elements

def t10_rule():
    """Parent gradients (10 x 3) and weights at the 5 points (App. A.1: the
    node table's barycentric columns; corner L_i (2 L_i - 1), mid-edge
    4 L_i L_j; the rule's weights -4/5 and 9/20 of the volume 1/6)."""
    bary = []
    for line in open(os.path.join(GOLD, "t10_nodes.txt")):
        if line.startswith("#") or not line.strip():
            continue
        bary.append([D(t) if "/" not in t else D(int(t.split("/")[0])) / D(int(t.split("/")[1]))
                     for t in line.split()[1:5]])
    dL = [(-1, -1, -1), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    pts = [([D(1) / 4] * 4, D(-4) / 5 / 6)]
    for m in range(4):
        L = [D(1) / 6] * 4
        L[m] = D(1) / 2
        pts.append((L, D(9) / 20 / 6))
    rule = []
    for L, w in pts:
        G = []
        for node in bary:
            nz = [i for i in range(4) if node[i] != 0]
            if len(nz) == 1:
                i = nz[0]
                G.append([(4 * L[i] - 1) * dL[i][k] for k in range(3)])
            else:
                i, j = nz
                G.append([4 * (L[i] * dL[j][k] + L[j] * dL[i][k]) for k in range(3)])
        rule.append((G, w))
    return rule, [[float(t) for t in row] for row in bary]


def h8_rule():
    """Trilinear hexahedron on [-1, 1]^3, nodes lexicographic with i fastest
    (n = i + 2 j + 4 k), 2 x 2 x 2 Gauss (points +-1/sqrt 3, weights 1)."""
    nodes = [(-1 + 2 * i, -1 + 2 * j, -1 + 2 * k) for k in range(2) for j in range(2) for i in range(2)]
    g = 1 / D(3).sqrt()
    rule = []
    for pz in (-g, g):
        for py in (-g, g):
            for px in (-g, g):
                p = (px, py, pz)
                G = []
                for n in nodes:
                    f = [1 + n[d] * p[d] for d in range(3)]
                    G.append([n[0] * f[1] * f[2] / 8, f[0] * n[1] * f[2] / 8, f[0] * f[1] * n[2] / 8])
                rule.append((G, D(1)))
    return rule, nodes


def q27_rule():
    """The 27-node hexahedron (App. A, node table from the golden file):
    products of the 1-D quadratic Lagrange polynomials on {-1, 0, 1},
    3 x 3 x 3 Gauss (points 0, +-sqrt(3/5), weights 8/9, 5/9)."""
    ijk, nodes = [], []
    for line in open(os.path.join(GOLD, "q27_nodes.txt")):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        ijk.append(tuple(int(s) for s in t[1:4]))
        nodes.append(tuple(int(s) for s in t[4:7]))

    def lag(s):      # values and derivatives of the three 1-D polynomials at s
        return ([s * (s - 1) / 2, 1 - s * s, s * (s + 1) / 2], [s - D(1) / 2, -2 * s, s + D(1) / 2])

    g = (D(3) / 5).sqrt()
    gp = [(-g, D(5) / 9), (D(0), D(8) / 9), (g, D(5) / 9)]
    rule = []
    for pz, wz in gp:
        for py, wy in gp:
            for px, wx in gp:
                Lx, dx = lag(px)
                Ly, dy = lag(py)
                Lz, dz = lag(pz)
                G = [[dx[i] * Ly[j] * Lz[k], Lx[i] * dy[j] * Lz[k], Lx[i] * Ly[j] * dz[k]] for i, j, k in ijk]
                rule.append((G, wx * wy * wz))
    return rule, nodes


RULES = {O.T10: t10_rule, O.H8: h8_rule, O.Q27: q27_rule}


# ------------------------------------------------------------- 3x3 algebra

def mat(a, b):
    return [[sum((a[i][k] * b[k][j] for k in range(len(b))), D(0)) for j in range(len(b[0]))] for i in range(len(a))]


def tr(a):
    return [[a[j][i] for j in range(len(a))] for i in range(len(a[0]))]


def det3(a):
    return (a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
            + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]))


def inv3(a):
    d = det3(a)
    c = [[a[(j + 1) % 3][(i + 1) % 3] * a[(j + 2) % 3][(i + 2) % 3] - a[(j + 1) % 3][(i + 2) % 3] * a[(j + 2) % 3][(i + 1) % 3]
          for j in range(3)] for i in range(3)]
    return [[c[i][j] / d for j in range(3)] for i in range(3)]


def trace(a):
    return a[0][0] + a[1][1] + a[2][2]


def ddot(a, b):
    return sum((a[i][j] * b[i][j] for i in range(3) for j in range(3)), D(0))


# --------------------------------------------------------------------- laws

def psi(law, th, F):
    """Strain energy per reference volume.  SVK (Sec. 3.2.1):
    lambda/2 (tr E)^2 + mu E:E with E = (F^T F - I)/2.  Mooney-Rivlin
    (Sec. 3.2.2): mu10 (J^(-2/3) I1 - 3) + mu01 (J^(-4/3) I2 - 3)
    + k/2 (J - 1)^2, Neo-Hookean with mu01 = 0."""
    C = mat(tr(F), F)
    if law == O.SVK:
        E = [[(C[i][j] - (1 if i == j else 0)) / 2 for j in range(3)] for i in range(3)]
        return th[0] / 2 * trace(E) * trace(E) + th[1] * ddot(E, E)
    J = det3(F)
    I1 = trace(C)
    W = th[0] * (J ** (D(-2) / 3) * I1 - 3) + th[2] / 2 * (J - 1) * (J - 1)
    if law == O.MR:
        I2 = (I1 * I1 - ddot(C, C)) / 2
        W = W + th[1] * (J ** (D(-4) / 3) * I2 - 3)
    return W


def stress(law, th, damped, F, Fd):
    """P = dPsi/dF (each entry the e part of Psi at F + e E_ij) plus the
    viscous F S_v, S_v = 2 mu_v Edot + lambda_v tr(Edot) I, Edot = sym(F^T Fdot)."""
    P = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            Fe = [[Dual(F[r][c], 1 if (r, c) == (i, j) else 0) for c in range(3)] for r in range(3)]
            P[i][j] = eps(psi(law, th, Fe))
    if damped:
        A = mat(tr(F), Fd)
        Ed = [[(A[i][j] + A[j][i]) / 2 for j in range(3)] for i in range(3)]
        t = trace(Ed)
        Sv = [[2 * th[3] * Ed[i][j] + (th[4] * t if i == j else 0) for j in range(3)] for i in range(3)]
        Pv = mat(F, Sv)
        P = [[P[i][j] + Pv[i][j] for j in range(3)] for i in range(3)]
    return P


def element_force(elem, law, th, damped, X, x, v):
    """f[a][i] = sum_q w_q det J_q (P(F_q, Fdot_q) h_a(q))_i with J = X G,
    h = G J^{-1}, F = x h, Fdot = v h (Sec. 2.1, 4.3, 6).  X, x, v: 3 x nen."""
    rule, _ = RULES[elem]()
    nen = len(rule[0][0])
    f = [[D(0)] * 3 for _ in range(nen)]
    for G, w in rule:
        J = mat(X, G)
        H = mat(G, inv3(J))
        F = mat(x, H)
        Fd = mat(v, H)
        P = stress(law, th, damped, F, Fd)
        c = w * det3(J)
        for a in range(nen):
            for i in range(3):
                f[a][i] = f[a][i] + c * sum((P[i][m] * H[a][m] for m in range(3)), D(0))
    return f


# ------------------------------------------------------------------ set-up

LAWS = {
    "SVK+KV": (O.SVK, [5.769e6, 3.846e6, 0.0, 1.0e4, 3.0e3], True),
    "MR+KV": (O.MR, [1.2e6, 0.45e6, 1.72667e7, 1.0e4, 3.0e3], True),
    "NH": (O.NH, [1.7e6, 0.0, 1.72667e7, 0.0, 0.0], False),
}


def curved_element(elem, seed):
    """A 1 cm element under a random affine map, offset by tens of element
    sizes, its nodes moved by a few per cent of its size; current positions
    a small strain, a rotation and a translation away; random velocities."""
    rng = np.random.default_rng(seed)
    _, nodes = RULES[elem]()
    if elem == O.T10:
        P = np.array([[n[1], n[2], n[3]] for n in nodes])          # barycentric L2..L4
    else:
        P = (np.array(nodes, float) + 1.0) / 2.0
    A = np.eye(3) * 0.01 + rng.uniform(-0.002, 0.002, (3, 3))
    X = (P @ A.T).T + np.array([[0.37], [-0.21], [0.55]])
    X += rng.uniform(-3e-4, 3e-4, X.shape)
    c, s = np.cos(0.3), np.sin(0.3)
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    x = R @ X + rng.normal(0, 6e-4, X.shape) + np.array([[0.2], [0.1], [-0.3]])
    v = rng.normal(0, 0.5, X.shape)
    return X, x, v


def block(elem, law, th, damped):
    nen = O.nen(elem)
    return SimpleNamespace(elem=elem, law=law, conn=np.arange(nen, dtype=np.int32)[None, :],
                           theta=np.asarray(th, float), theta_e=None, damped=damped)


def to_dec(a):
    return [[dec(t) for t in row] for row in a]


def as_array(f):
    return np.array([[float(real(t)) for t in row] for row in f]).T     # 3 x nen


def rel(a, b):
    return np.linalg.norm(np.asarray(a, float) - np.asarray(b, float)) / np.linalg.norm(np.asarray(b, float))


CASES = [(e, l) for e in (O.T10, O.H8, O.Q27) for l in LAWS]
IDS = [f"{ {O.T10: 'T10', O.H8: 'H8', O.Q27: 'Q27'}[e]}-{l}" for e, l in CASES]


@pytest.mark.parametrize("elem,lawname", CASES, ids=IDS)
def test_force_against_the_energy_derivative(elem, lawname):
    law, th, damped = LAWS[lawname]
    X, x, v = curved_element(elem, 60 + elem)
    with decimal.localcontext(CTX):
        f = element_force(elem, law, [dec(t) for t in th], damped, to_dec(X), to_dec(x), to_dec(v))
        ex = as_array(f)
    got = O.internal_force(X, [block(elem, law, th, damped)], x, v if damped else None)
    assert rel(got, ex) <= BAR, rel(got, ex)


def directional(elem, law, th, damped, X, x, v, dx, dv):
    """K dx + C dv: the e part of the force at (x + e dx, v + e dv)."""
    xe = [[Dual(x[i][a], dx[i][a]) for a in range(len(x[0]))] for i in range(3)]
    ve = [[Dual(v[i][a], dv[i][a]) for a in range(len(v[0]))] for i in range(3)]
    return [[eps(t) for t in row] for row in element_force(elem, law, th, damped, X, xe, ve)]


@pytest.mark.parametrize("elem,lawname", [(O.T10, "MR+KV"), (O.H8, "SVK+KV"), (O.Q27, "NH")],
                         ids=["T10-MR+KV", "H8-SVK+KV", "Q27-NH"])
def test_tangent_product_against_exact_directional_derivative(elem, lawname):
    law, th, damped = LAWS[lawname]
    X, x, v = curved_element(elem, 70 + elem)
    rng = np.random.default_rng(71 + elem)
    dx, dv = rng.normal(0, 1e-3, X.shape), rng.normal(0, 1.0, X.shape)
    with decimal.localcontext(CTX):
        thd = [dec(t) for t in th]
        ex = as_array(directional(elem, law, thd, damped, to_dec(X), to_dec(x), to_dec(v), to_dec(dx), to_dec(dv)))
    got = O.jvp(X, [block(elem, law, th, damped)], x, v, dx, dv if damped else np.zeros_like(dv))
    assert rel(got, ex) <= BAR, rel(got, ex)


@pytest.mark.parametrize("elem,lawname", [(O.T10, "MR+KV"), (O.H8, "NH")], ids=["T10-MR+KV", "H8-NH"])
def test_adjoint_against_the_exact_element_jacobian(elem, lawname):
    """gx = K^T w and gv = C^T w from every column K e_j, C e_j; gtheta_p =
    w . f(theta = e_p) (the stress is linear in each parameter)."""
    law, th, damped = LAWS[lawname]
    X, x, v = curved_element(elem, 80 + elem)
    nen = X.shape[1]
    w = np.random.default_rng(81 + elem).normal(0, 1, X.shape)
    gx = np.zeros_like(X)
    gv = np.zeros_like(X)
    gt = np.zeros(5)
    with decimal.localcontext(CTX):
        thd = [dec(t) for t in th]
        Xd, xd, vd, wd = to_dec(X), to_dec(x), to_dec(v), to_dec(w)
        zero = [[D(0)] * nen for _ in range(3)]
        for field in ((0, 1) if damped else (0,)):
            for i in range(3):
                for a in range(nen):
                    e = [[D(1) if (r, c) == (i, a) else D(0) for c in range(nen)] for r in range(3)]
                    col = directional(elem, law, thd, damped, Xd, xd, vd, e if field == 0 else zero,
                                      e if field == 1 else zero)
                    s = sum((wd[r][b] * col[b][r] for r in range(3) for b in range(nen)), D(0))
                    (gx if field == 0 else gv)[i, a] = float(s)
        for p in range(5):
            if (p == 1 and law == O.NH) or (p >= 3 and not damped):
                continue
            unit = [D(1) if q == p else D(0) for q in range(5)]
            f = element_force(elem, law, unit, damped, Xd, xd, vd)
            gt[p] = float(sum((wd[r][b] * f[b][r] for r in range(3) for b in range(nen)), D(0)))
    rx, rv, rt = O.vjp(X, [block(elem, law, th, damped)], x, v, w)
    assert rel(rx, gx) <= BAR, rel(rx, gx)
    if damped:
        assert rel(rv, gv) <= BAR, rel(rv, gv)
    else:
        assert not np.any(rv)
    for p in range(5):
        # rows of parameters the law does not use are exactly zero
        if gt[p] == 0:
            assert rt[p, 0] == 0, (p, rt[p, 0])
        else:
            assert abs(rt[p, 0] - gt[p]) <= BAR * abs(gt[p]), (p, rt[p, 0], gt[p])


# ------------------------------------------- inertia and the step (Sec. 4.1, 7)

def mass_points(elem):
    """(shape values, parent gradients, weight) at the points of the mass
    rule.  T10: the 15-point degree-5 rule on the tetrahedron, barycentric
    orbits the centroid (weight 16/135), (a, a, a, 1 - 3a) for
    a = (7 -+ sqrt 15)/34 (weights (2665 +- 14 sqrt 15)/37800) and
    (b, b, 1/2 - b, 1/2 - b) for b = (5 - sqrt 15)/20 (weight 10/189), all
    times the volume 1/6.  H8 and Q27: their Gauss rules (as for the force)."""
    r15 = D(15).sqrt()
    if elem == O.T10:
        _, bary = t10_rule()
        bary = [[D(repr(t)) for t in row] for row in bary]
        pts = [([D(1) / 4] * 4, D(16) / 135)]
        for a, w in (((7 - r15) / 34, (2665 + 14 * r15) / 37800), ((7 + r15) / 34, (2665 - 14 * r15) / 37800)):
            for m in range(4):
                L = [a] * 4
                L[m] = 1 - 3 * a
                pts.append((L, w))
        b = (5 - r15) / 20
        for i in range(4):
            for j in range(i + 1, 4):
                L = [D(1) / 2 - b] * 4
                L[i] = L[j] = b
                pts.append((L, D(10) / 189))
        dL = [(-1, -1, -1), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
        out = []
        for L, w in pts:
            s, G = [], []
            for node in bary:
                nz = [i for i in range(4) if node[i] != 0]
                if len(nz) == 1:
                    i = nz[0]
                    s.append(L[i] * (2 * L[i] - 1))
                    G.append([(4 * L[i] - 1) * dL[i][k] for k in range(3)])
                else:
                    i, j = nz
                    s.append(4 * L[i] * L[j])
                    G.append([4 * (L[i] * dL[j][k] + L[j] * dL[i][k]) for k in range(3)])
            out.append((s, G, w / 6, L))
        return out
    rule, nodes = RULES[elem]()
    out = []
    if elem == O.H8:
        g = 1 / D(3).sqrt()
        pts = [(px, py, pz) for pz in (-g, g) for py in (-g, g) for px in (-g, g)]
        for (G, w), p in zip(rule, pts):
            s = [(1 + n[0] * p[0]) * (1 + n[1] * p[1]) * (1 + n[2] * p[2]) / 8 for n in nodes]
            out.append((s, G, w, p))
        return out
    g = (D(3) / 5).sqrt()
    gp = [-g, D(0), g]
    ijk = [(n[0] + 1, n[1] + 1, n[2] + 1) for n in nodes]
    lag = lambda t: [t * (t - 1) / 2, 1 - t * t, t * (t + 1) / 2]
    pts = [(px, py, pz) for pz in gp for py in gp for px in gp]
    for (G, w), p in zip(rule, pts):
        Lx, Ly, Lz = lag(p[0]), lag(p[1]), lag(p[2])
        s = [Lx[i] * Ly[j] * Lz[k] for i, j, k in ijk]
        out.append((s, G, w, p))
    return out


def test_t10_mass_rule_is_exact_to_degree_five():
    """The transcription of the 15-point rule used below integrates every
    monomial of degree <= 5 over the unit tetrahedron exactly
    (i! j! k! / (i + j + k + 3)!), which fixes its orbits and weights."""
    from math import factorial
    with decimal.localcontext(CTX):
        pts = mass_points(O.T10)
        assert len(pts) == 15
        for i in range(6):
            for j in range(6 - i):
                for k in range(6 - i - j):
                    q = sum((w * L[1] ** i * L[2] ** j * L[3] ** k for _, _, w, L in pts), D(0))
                    ex = D(factorial(i) * factorial(j) * factorial(k)) / D(factorial(i + j + k + 3))
                    assert abs(q - ex) < D("1e-50"), (i, j, k)


def element_mass(elem, rho, X):
    """m_ab = rho sum_q w_q s_a s_b det J_q (Sec. 4.1) with the mass rule."""
    pts = mass_points(elem)
    nen = len(pts[0][0])
    M = [[D(0)] * nen for _ in range(nen)]
    for s, G, w, _ in pts:
        c = rho * w * det3(mat(X, G))
        for a in range(nen):
            for b in range(nen):
                M[a][b] = M[a][b] + c * s[a] * s[b]
    return M


def step_residual(elem, law, th, damped, rho, X, qn, vn, v, h):
    """g(v) = M (v - v_n) / h + f_int(q_n + h v, v) (Sec. 7, no constraints,
    f_ext = 0)."""
    nen = len(X[0])
    x = [[qn[i][a] + h * v[i][a] for a in range(nen)] for i in range(3)]
    f = element_force(elem, law, th, damped, X, x, v)
    M = element_mass(elem, rho, X)
    return [[f[a][i] + sum((M[a][b] * (v[i][b] - vn[i][b]) for b in range(nen)), D(0)) / h
             for i in range(3)] for a in range(nen)]


def grid(a, step):
    return np.round(np.asarray(a) / step) * step


@pytest.mark.parametrize("elem,lawname", [(O.T10, "MR+KV"), (O.H8, "NH"), (O.Q27, "SVK+KV")],
                         ids=["T10-MR+KV", "H8-NH", "Q27-SVK+KV"])
def test_step_residual_and_newton_operator_against_exact_evaluation(elem, lawname):
    """The step residual against its 60-digit evaluation, and the Newton
    operator (M/h + h K + C) dv against the exact derivative of that
    evaluation along dv.  The inputs make q = q_n + h v, v - v_n and the
    division by h exact in FP64 (h = 2^-13, q_n on a 2^-40 m grid, v and v_n
    on a 2^-20 m/s grid), so both sides see the same positions."""
    law, th, damped = LAWS[lawname]
    X, x, _ = curved_element(elem, 90 + elem)
    rng = np.random.default_rng(91 + elem)
    h, rho = 2.0 ** -13, 1100.0
    qn = grid(x, 2.0 ** -40)
    v = grid(rng.normal(0, 0.3, X.shape), 2.0 ** -20)
    vn = grid(v + rng.normal(0, 0.3, X.shape), 2.0 ** -20)
    dv = rng.normal(0, 1.0, X.shape)
    assert np.array_equal((qn + h * v) - h * v, qn)
    blk = block(elem, law, th, damped)
    blk.rho = rho
    with decimal.localcontext(CTX):
        thd = [dec(t) for t in th]
        Xd, qd, vd, vnd, dvd = to_dec(X), to_dec(qn), to_dec(v), to_dec(vn), to_dec(dv)
        hd, rd = dec(h), dec(rho)
        g = as_array(step_residual(elem, law, thd, damped, rd, Xd, qd, vnd, vd, hd))
        ve = [[Dual(vd[i][a], dvd[i][a]) for a in range(len(vd[0]))] for i in range(3)]
        ge = step_residual(elem, law, thd, damped, rd, Xd, qd, vnd, ve, hd)
        y = np.array([[float(eps(t)) for t in row] for row in ge]).T
    got = O.step_residual(X, [blk], qn, vn, v, h)
    assert rel(got, g) <= BAR, rel(got, g)
    op = O.newton_operator(X, [blk], qn, v, h, dv)
    assert rel(op, y) <= BAR, rel(op, y)


# ------------------------------------------------ the revolute joint (Sec. 2.2)

def shape_exact(elem, xi):
    """Shape values at parent point xi: T10 corner L_i (2 L_i - 1), mid-edge
    4 L_i L_j with L = (1 - xi - eta - zeta, xi, eta, zeta); H8 trilinear;
    Q27 products of the 1-D quadratic Lagrange polynomials."""
    if elem == O.T10:
        _, bary = t10_rule()
        L = [1 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]]
        s = []
        for node in bary:
            nz = [i for i in range(4) if node[i] != 0]
            s.append(L[nz[0]] * (2 * L[nz[0]] - 1) if len(nz) == 1 else 4 * L[nz[0]] * L[nz[1]])
        return s
    _, nodes = RULES[elem]()
    if elem == O.H8:
        return [(1 + n[0] * xi[0]) * (1 + n[1] * xi[1]) * (1 + n[2] * xi[2]) / 8 for n in nodes]
    lag = lambda t: [t * (t - 1) / 2, 1 - t * t, t * (t + 1) / 2]
    Lx, Ly, Lz = lag(xi[0]), lag(xi[1]), lag(xi[2])
    return [Lx[n[0] + 1] * Ly[n[1] + 1] * Lz[n[2] + 1] for n in nodes]


def joint_values_exact(Xd, qd, pts):
    """Row-normalised revolute values W c (Sec. 2.2, App. B.1): c = (r_R - r_P,
    a.b_1 - f_1, a.b_2 - f_2), a = r_Q - r_P, b_j = r_{S,T} - r_R, f_j and the
    DP1 weights 1 / sqrt(|a_0|^2 + |b_j0|^2) from the reference positions."""
    def positions(y):
        r = {}
        for key, (elem, nodes, xi) in pts.items():
            s = shape_exact(elem, [dec(t) for t in xi])
            r[key] = [sum((s[a] * y[i][n] for a, n in enumerate(nodes)), D(0)) for i in range(3)]
        return r
    dot = lambda u, v: u[0] * v[0] + u[1] * v[1] + u[2] * v[2]
    sub = lambda u, v: [u[i] - v[i] for i in range(3)]
    r0, r = positions(Xd), positions(qd)
    a0, b10, b20 = sub(r0["Q"], r0["P"]), sub(r0["S"], r0["R"]), sub(r0["T"], r0["R"])
    a, b1, b2 = sub(r["Q"], r["P"]), sub(r["S"], r["R"]), sub(r["T"], r["R"])
    w1 = 1 / (dot(a0, a0) + dot(b10, b10)).sqrt()
    w2 = 1 / (dot(a0, a0) + dot(b20, b20)).sqrt()
    d = sub(r["R"], r["P"])
    return [d[0], d[1], d[2], w1 * (dot(a, b1) - dot(a0, b10)), w2 * (dot(a, b2) - dot(a0, b20))]


def test_revolute_joint_values_and_scatter_against_exact_evaluation():
    """The five points in elements of all three types, a configuration that
    violates the joint by about a millimetre: values against the 60-digit
    evaluation, and the scatter h C^T (lambda + rho c) with each column of
    C the exact derivative of the values along one nodal coordinate.  The
    rows are differences of point positions some 50 times longer than the
    fibres between them, and the DP1 rows products of two such differences
    less their reference value (a condition of 10^3-10^4), so FP64 gives
    them to 1e-13-1e-12: the bar here is JBAR = 1e-12.  The mistakes this
    is meant to catch (a wrong weight, sign, block or factor) move them by
    0.1 or more."""
    rng = np.random.default_rng(95)
    nodes_of = {}
    X = np.zeros((3, 0))
    for elem, seed in ((O.T10, 96), (O.H8, 97), (O.Q27, 98)):
        Xe, _, _ = curved_element(elem, seed)
        nodes_of[elem] = list(range(X.shape[1], X.shape[1] + Xe.shape[1]))
        X = np.hstack([X, Xe])
    c, s = np.cos(0.2), np.sin(0.2)
    R = np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    q = R @ X + rng.normal(0, 1e-3, X.shape)
    t10_xi = lambda: (lambda u: u / (u.sum() + rng.uniform(0.2, 1.0)))(rng.uniform(0.05, 1.0, 3))
    cube_xi = lambda: rng.uniform(-0.9, 0.9, 3)
    pts = {"P": (O.T10, nodes_of[O.T10], t10_xi()), "Q": (O.H8, nodes_of[O.H8], cube_xi()),
           "R": (O.Q27, nodes_of[O.Q27], cube_xi()), "S": (O.T10, nodes_of[O.T10], t10_xi()),
           "T": (O.H8, nodes_of[O.H8], cube_xi())}
    lam = rng.normal(0, 1, 5)
    rho, h = 1e4, 1e-3
    n = X.shape[1]
    with decimal.localcontext(CTX):
        Xd, qd = to_dec(X), to_dec(q)
        cv = joint_values_exact(Xd, qd, pts)
        eta = [dec(lam[k]) + dec(rho) * cv[k] for k in range(5)]
        g = np.zeros((3, n))
        for i in range(3):
            for m in range(n):
                qe = [[Dual(qd[r][a], 1 if (r, a) == (i, m) else 0) for a in range(n)] for r in range(3)]
                col = joint_values_exact(Xd, qe, pts)
                g[i, m] = float(dec(h) * sum((eta[k] * eps(col[k]) for k in range(5)), D(0)))
        cvf = np.array([float(t) for t in cv])
    from oracle import constraints as OC
    joint = {k: (e, nd, xi) for k, (e, nd, xi) in pts.items()}
    got = OC.revolute_values(X, q, [joint])[0]
    assert rel(got, cvf) <= JBAR, rel(got, cvf)
    gs = OC.revolute_scatter(X, q, [joint], lam, rho, h)
    assert rel(gs, g) <= JBAR, rel(gs, g)
