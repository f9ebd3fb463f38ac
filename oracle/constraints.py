"""Bilateral joint constraints of the oracle (test infrastructure only):
the revolute joint of Sec. 2.2 built from three coordinate-difference (CD)
rows and two dot-product-1 (DP1) rows, with the constant row weights of
App. B.1, its Jacobian and the transpose scatter that inserts it into the
step residual.  Plain numpy, written from the paper; shares nothing with
the GPU library.

A material point is (element type, the hosting element's node ids in the
element's node order, parent coordinates xi).  Its current position is the
point evaluation r = N(t) s(xi) over the element's nodes (Sec. 2.1), and its
first variation is delta r = sum_i s_i(xi) delta e_i, so the Jacobian block
of any row that depends on r through a vector d is d^T (s^T (x) I_3)
(Sec. 2.2).

Revolute joint with points P, Q on body b and R, S, T on body c:
  a = r_Q - r_P,  b_1 = r_S - r_R,  b_2 = r_T - r_R,
  c = [e_x.(r_R - r_P), e_y.(r_R - r_P), e_z.(r_R - r_P),
       a.b_1 - f_1, a.b_2 - f_2],   f_j = a_0 . b_j0 (reference configuration),
  row weights w = (1, 1, 1, 1/sqrt(|a_0|^2 + |b_10|^2), 1/sqrt(|a_0|^2 + |b_20|^2)),
  c_hat = W c, C_hat = W dc/dq; the residual receives h C_hat^T (lambda + rho c_hat).
"""
from __future__ import annotations

import numpy as np

from .oracle import shape

POINTS = ("P", "Q", "R", "S", "T")


def point_position(q, point):
    """r = sum_i s_i(xi) q_i over the hosting element's nodes (Sec. 2.1)."""
    elem, nodes, xi = point
    s = shape(elem, np.asarray(xi, dtype=np.float64))
    return q[:, np.asarray(nodes)] @ s


def _directions(q, joint):
    r = {k: point_position(q, joint[k]) for k in POINTS}
    return r, r["Q"] - r["P"], r["S"] - r["R"], r["T"] - r["R"]


def reference_data(X, joint):
    """(f_1, f_2) and the five row weights from the reference configuration."""
    _, a0, b10, b20 = _directions(X, joint)
    f = np.array([a0 @ b10, a0 @ b20])
    w = np.array([1.0, 1.0, 1.0, 1.0 / np.sqrt(a0 @ a0 + b10 @ b10), 1.0 / np.sqrt(a0 @ a0 + b20 @ b20)])
    return f, w


def revolute_values(X, q, joints):
    """Row-normalised constraint values c_hat, [n_joints][5]."""
    out = np.zeros((len(joints), 5))
    for j, jt in enumerate(joints):
        f, w = reference_data(X, jt)
        r, a, b1, b2 = _directions(q, jt)
        d = r["R"] - r["P"]
        c = np.array([d[0], d[1], d[2], a @ b1 - f[0], a @ b2 - f[1]])
        out[j] = w * c
    return out


def revolute_jacobian(X, q, joints):
    """Row-normalised Jacobian C_hat = W dc/dq as a dense [5 n_joints][3 n]
    array (row 5 j + k, column c n + node: the [3][n] layout)."""
    n = q.shape[1]
    J = np.zeros((5 * len(joints), 3 * n))
    ex = np.eye(3)
    for j, jt in enumerate(joints):
        _, w = reference_data(X, jt)
        r, a, b1, b2 = _directions(q, jt)
        # d c_k / d r_X for every row k and point X (Sec. 2.2 blocks)
        d = {k: np.zeros((5, 3)) for k in POINTS}
        for k in range(3):
            d["P"][k] = -ex[k]
            d["R"][k] = ex[k]
        d["P"][3], d["Q"][3], d["R"][3], d["S"][3] = -b1, b1, -a, a
        d["P"][4], d["Q"][4], d["R"][4], d["T"][4] = -b2, b2, -a, a
        for key in POINTS:
            elem, nodes, xi = jt[key]
            s = shape(elem, np.asarray(xi, dtype=np.float64))
            for i, node in enumerate(nodes):
                for c in range(3):
                    J[5 * j:5 * j + 5, c * n + node] += w * d[key][:, c] * s[i]
    return J


def revolute_scatter(X, q, joints, lam=None, rho=0.0, h=1.0):
    """h C_hat^T (lambda + rho c_hat) as [3][n] (Sec. 2.2 residual insertion)."""
    c = revolute_values(X, q, joints).ravel()
    eta = (np.zeros_like(c) if lam is None else np.asarray(lam, dtype=np.float64).ravel()) + rho * c
    J = revolute_jacobian(X, q, joints)
    return (h * (J.T @ eta)).reshape(3, q.shape[1])


def revolute_scatter_local(X, q, joints, lam=None, rho=0.0, h=1.0):
    """revolute_scatter evaluated joint by joint on the joint's own nodes
    (the same formulas; the dense Jacobian of a large mesh would not fit)."""
    out = np.zeros_like(q, dtype=np.float64)
    lam = None if lam is None else np.asarray(lam, dtype=np.float64).reshape(len(joints), 5)
    for j, jt in enumerate(joints):
        nodes = sorted({int(n) for k in POINTS for n in jt[k][1]})
        loc = {n: i for i, n in enumerate(nodes)}
        jl = {k: (jt[k][0], [loc[int(n)] for n in jt[k][1]], jt[k][2]) for k in POINTS}
        g = revolute_scatter(X[:, nodes], q[:, nodes], [jl], None if lam is None else lam[j:j + 1], rho, h)
        out[:, nodes] += g
    return out
