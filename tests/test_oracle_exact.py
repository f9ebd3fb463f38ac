"""The oracle's FP64 rounding error on one curved T10 element, against an
evaluation of the same kinematics and laws without rounding (CPU only).

The T10 shape functions (App. A, from the node table's barycentric columns)
and the 5-point rule (weights -4/5 and 9/20 of the parent volume 1/6) are
rational, so for Saint Venant-Kirchhoff with Kelvin-Voigt damping the element
force is a rational function of the (exactly representable) inputs and is
evaluated exactly with fractions.  Neo-Hookean needs J^(-2/3): it is
evaluated with 60-digit decimals.  The oracle must agree to within a few
units of FP64 rounding: it forms every position relative to the element's
first node, so its products carry no cancellation of the element's offset.
"""
import decimal
import os
from fractions import Fraction
from types import SimpleNamespace

import numpy as np

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "t10_nodes.txt")


def t10_barycentric():
    """Barycentric coordinates (L1..L4) of the ten nodes, as fractions."""
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([Fraction(t) for t in line.split()[1:5]])
    return rows


# d L_i / d(xi, eta, zeta) with L1 = 1 - xi - eta - zeta, L2..L4 = xi, eta, zeta
DL = [(-1, -1, -1), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def shape_gradients(L):
    """Parent gradients of the ten shape functions at barycentric point L:
    corner i: L_i (2 L_i - 1), mid-edge (i, j): 4 L_i L_j."""
    G = []
    for node in t10_barycentric():
        nz = [i for i in range(4) if node[i] != 0]
        if len(nz) == 1:
            i = nz[0]
            G.append([(4 * L[i] - 1) * DL[i][k] for k in range(3)])
        else:
            i, j = nz
            G.append([4 * (L[i] * DL[j][k] + L[j] * DL[i][k]) for k in range(3)])
    return G


def keast5():
    """The 5-point rule on the parent tetrahedron: (barycentric point, weight)."""
    q = [([Fraction(1, 4)] * 4, Fraction(-4, 5) / 6)]
    for m in range(4):
        L = [Fraction(1, 6)] * 4
        L[m] = Fraction(1, 2)
        q.append((L, Fraction(9, 20) / 6))
    return q


def mat(a, b):
    return [[sum(a[i][k] * b[k][j] for k in range(len(b))) for j in range(len(b[0]))] for i in range(len(a))]


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


def element_force_exact(X, x, v, stress, scal):
    """f[a] (10 x 3) = sum_q w_q det J P(F, Fdot) h_a with h = G J^{-1},
    J = X G, F = x h, Fdot = v h (Sec. 2.1, 4.3, 6); X, x, v: 3 x 10 lists of
    fractions; stress(scal, F, Fdot) returns P; the weight, det J and the
    gradients pass through scal (the identity for fractions, a conversion
    for decimals)."""
    f = [[0, 0, 0] for _ in range(10)]
    for L, w in keast5():
        G = shape_gradients(L)
        J = mat(X, G)
        dJ = det3(J)
        H = mat(G, inv3(J))
        F, Fd = mat(x, H), mat(v, H)
        P = stress(scal, F, Fd)
        c = scal(w * dJ)
        Hs = [[scal(H[a][m]) for m in range(3)] for a in range(10)]
        for a in range(10):
            for i in range(3):
                f[a][i] += c * sum(P[i][m] * Hs[a][m] for m in range(3))
    return f


def svk_kv(lam, mu, mu_v, lam_v):
    """P = F (S + S_v), S = lam tr(E) I + 2 mu E, E = (F^T F - I)/2,
    S_v = lam_v tr(Edot) I + 2 mu_v Edot, Edot = sym(F^T Fdot) (Sec. 3.2.1, 3.2.3)."""
    def stress(scal, F, Fd):
        C = mat(tr(F), F)
        E = [[(C[i][j] - (1 if i == j else 0)) / 2 for j in range(3)] for i in range(3)]
        A = mat(tr(F), Fd)
        Ed = [[(A[i][j] + A[j][i]) / 2 for j in range(3)] for i in range(3)]
        tE, tEd = E[0][0] + E[1][1] + E[2][2], Ed[0][0] + Ed[1][1] + Ed[2][2]
        S = [[2 * mu * E[i][j] + 2 * mu_v * Ed[i][j] + ((lam * tE + lam_v * tEd) if i == j else 0) for j in range(3)]
             for i in range(3)]
        return mat(F, S)
    return stress


def nh(mu10, k):
    """P = 2 mu10 J^(-2/3) (F - I1/3 F^{-T}) + k (J - 1) J F^{-T} (Sec. 3.2.2
    with mu01 = 0), in decimals."""
    def stress(scal, F, Fd):
        Fd_ = [[scal(F[i][j]) for j in range(3)] for i in range(3)]
        J = det3(Fd_)
        FiT = tr(inv3(Fd_))
        I1 = sum(Fd_[i][j] * Fd_[i][j] for i in range(3) for j in range(3))
        J23 = J ** (decimal.Decimal(-2) / decimal.Decimal(3))
        a = 2 * scal(mu10) * J23
        b = -a * I1 / 3 + scal(k) * (J - 1) * J
        return [[a * Fd_[i][j] + b * FiT[i][j] for j in range(3)] for i in range(3)]
    return stress


def curved_element(rng):
    A = np.eye(3) * 0.01 + rng.uniform(-0.002, 0.002, (3, 3))
    xi = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1],
                   [.5, 0, 0], [.5, .5, 0], [0, .5, 0], [0, 0, .5], [.5, 0, .5], [0, .5, .5]])
    X = (xi @ A.T).T + np.array([[0.37], [-0.21], [0.55]])      # an offset of tens of element sizes
    X[:, 4:] += rng.uniform(-4e-4, 4e-4, (3, 6))                  # curved edges
    x = X + rng.normal(0, 3e-4, X.shape) + np.array([[0.2], [0.1], [-0.3]])
    v = rng.normal(0, 0.5, X.shape)
    return X, x, v


def frac(a):
    return [[Fraction(float(t)) for t in row] for row in a]


def rel(a, b):
    return np.linalg.norm(np.asarray(a, float) - np.asarray(b, float)) / np.linalg.norm(np.asarray(b, float))


def oracle_force(X, x, v, law, theta, damped):
    b = SimpleNamespace(elem=O.T10, law=law, conn=np.arange(10, dtype=np.int32)[None, :],
                        theta=np.asarray(theta, float), theta_e=None, damped=damped)
    return O.internal_force(X, [b], x, v if damped else None)


def test_svk_kelvin_voigt_force_against_exact_rational_evaluation():
    rng = np.random.default_rng(41)
    X, x, v = curved_element(rng)
    lam, mu, mu_v, lam_v = 5.769e6, 3.846e6, 1.0e4, 3.0e3
    ref = element_force_exact(frac(X), frac(x), frac(v),
                              svk_kv(Fraction(lam), Fraction(mu), Fraction(mu_v), Fraction(lam_v)), lambda t: t)
    f = oracle_force(X, x, v, O.SVK, [lam, mu, 0.0, mu_v, lam_v], True)
    ex = np.array([[float(t) for t in ref[a]] for a in range(10)]).T
    err = rel(f, ex)
    assert err <= 1e-14, err
    # the sum of an element's nodal forces vanishes exactly in the exact
    # evaluation (the parent gradients sum to zero at every point)
    assert all(sum(ref[a][i] for a in range(10)) == 0 for i in range(3))


def test_neo_hookean_force_against_60_digit_evaluation():
    rng = np.random.default_rng(43)
    X, x, v = curved_element(rng)
    mu10, k = 1.7e6, 1.72667e7
    ctx = decimal.Context(prec=60)
    with decimal.localcontext(ctx):
        def scal(t):
            t = Fraction(t)
            return decimal.Decimal(t.numerator) / decimal.Decimal(t.denominator)
        ref = element_force_exact(frac(X), frac(x), frac(v), nh(mu10, k), scal)
        ex = np.array([[float(t) for t in ref[a]] for a in range(10)]).T
    f = oracle_force(X, x, v, O.NH, [mu10, 0.0, k, 0.0, 0.0], False)
    err = rel(f, ex)
    assert err <= 1e-14, err
