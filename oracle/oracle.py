"""ctypes wrapper of the C oracle (test infrastructure only).

Blocks are any objects with attributes ``elem``, ``law``, ``damped``, ``conn``
([n_elem][nen] int32) and either ``theta_e`` ([5][n_elem]) or ``theta`` ([5]).
Nodal arrays are [3][n_nodes] float64.  Multi-block meshes are evaluated block
by block and summed into one nodal vector, in block order.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
T10, H8, Q27 = 0, 1, 2
SVK, MR, NH = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.oracle_nen.argtypes = [C.c_int]
        L.oracle_quadrature.argtypes = [C.c_int, _dp, _dp]
        L.oracle_shape.argtypes = [C.c_int, _dp, _dp]
        L.oracle_dshape.argtypes = [C.c_int, _dp, _dp]
        L.oracle_stress.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.oracle_density.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp]
        mesh = [C.c_int, C.c_int, C.c_int, C.c_int64, _dp, C.c_int64, _ip, _dp]
        L.oracle_internal_force.argtypes = mesh + [_dp, _dp, _dp]
        L.oracle_energy.argtypes = mesh + [_dp, _dp, _dp, _dp]
        L.oracle_vjp.argtypes = mesh + [_dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_internal_force_par.argtypes = mesh + [_dp, _dp, _dp, C.c_int]
        L.oracle_vjp_par.argtypes = mesh + [_dp, _dp, _dp, _dp, _dp, _dp, C.c_int]
        L.oracle_jvp.argtypes = mesh + [_dp, _dp, _dp, _dp, _dp]
        L.oracle_element_tangent.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_count_inverted.argtypes = [C.c_int, C.c_int64, _dp, C.c_int64, _ip, _dp,
                                             C.POINTER(C.c_int64), _dp]
        L.oracle_mass_rule.argtypes = [C.c_int, _dp, _dp]
        L.oracle_element_mass.argtypes = [C.c_int, C.c_double, _dp, _dp]
        L.oracle_mass_action.argtypes = [C.c_int, C.c_int64, _dp, C.c_int64, _ip, C.c_double, _dp, _dp]
        L.oracle_step_residual.argtypes = mesh + [C.c_double, _dp, _dp, _dp, C.c_double, _dp]
        L.oracle_newton_operator.argtypes = mesh + [C.c_double, _dp, _dp, C.c_double, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def nen(elem):
    return lib().oracle_nen(elem)


def quadrature(elem):
    xi = np.zeros((27, 3)); w = np.zeros(27)
    nq = lib().oracle_quadrature(elem, _d(xi), _d(w))
    return xi[:nq].copy(), w[:nq].copy()


def shape(elem, xi):
    s = np.zeros(nen(elem)); p = _f64(xi)
    lib().oracle_shape(elem, _d(p), _d(s))
    return s


def dshape(elem, xi):
    G = np.zeros((nen(elem), 3)); p = _f64(xi)
    lib().oracle_dshape(elem, _d(p), _d(G))
    return G


def stress(law, theta, F, Fd=None, damped=None):
    """P = P_e(F) + F S_v(Edot) at one point; theta is [5]."""
    th = _f64(theta); F = _f64(F)
    Fd = np.zeros((3, 3)) if Fd is None else _f64(Fd)
    if damped is None:
        damped = bool(th[3] != 0 or th[4] != 0)
    P = np.zeros((3, 3))
    lib().oracle_stress(law, int(damped), _d(th), _d(F), _d(Fd), _d(P))
    return P


def density(law, theta, F, Fd=None, damped=None):
    th = _f64(theta); F = _f64(F)
    Fd = np.zeros((3, 3)) if Fd is None else _f64(Fd)
    if damped is None:
        damped = bool(th[3] != 0 or th[4] != 0)
    psi = C.c_double(); phi = C.c_double()
    lib().oracle_density(law, int(damped), _d(th), _d(F), _d(Fd), C.byref(psi), C.byref(phi))
    return psi.value, phi.value


def _theta_e(b):
    te = getattr(b, "theta_e", None)
    if te is None:
        te = np.repeat(np.asarray(b.theta, np.float64)[:, None], b.conn.shape[0], axis=1)
    return np.ascontiguousarray(te, dtype=np.float64)


def _mesh_args(b, X):
    conn = np.ascontiguousarray(b.conn, dtype=np.int32)
    th = _theta_e(b)
    return ([b.elem, b.law, int(b.damped), X.shape[1], _d(X), conn.shape[0],
             conn.ctypes.data_as(_ip), _d(th)], (conn, th))


def internal_force(X, blocks, x, v=None):
    """Assembled f_int [3][n_nodes] (Sec. 4.3), blocks summed in order."""
    X = _f64(X); x = _f64(x); v = _f64(v)
    f = np.zeros_like(X)
    for b in blocks:
        args, keep = _mesh_args(b, X)
        _check(lib().oracle_internal_force(*args, _d(x), _d(v), _d(f)), "internal_force")
    return f


def internal_force_par(X, blocks, x, v=None, threads=1):
    """internal_force with each block's elements split over ``threads``
    OpenMP threads (private buffers added in thread order)."""
    X = _f64(X); x = _f64(x); v = _f64(v)
    f = np.zeros_like(X)
    for b in blocks:
        args, keep = _mesh_args(b, X)
        _check(lib().oracle_internal_force_par(*args, _d(x), _d(v), _d(f), int(threads)), "internal_force_par")
    return f


def vjp_par(X, blocks, x, v, w, want_gx=True, want_gv=True, want_gtheta=True, threads=1):
    """vjp with each block's elements split over ``threads`` OpenMP threads."""
    X = _f64(X); x = _f64(x); v = _f64(v); w = _f64(w)
    gx = np.zeros_like(X) if want_gx else None
    gv = np.zeros_like(X) if want_gv else None
    gts = []
    for b in blocks:
        args, keep = _mesh_args(b, X)
        gt = np.zeros((5, b.conn.shape[0])) if want_gtheta else None
        _check(lib().oracle_vjp_par(*args, _d(x), _d(v), _d(w), _d(gx), _d(gv), _d(gt), int(threads)), "vjp_par")
        gts.append(gt)
    gtheta = np.concatenate(gts, axis=1) if want_gtheta else None
    return gx, gv, gtheta


def energy(X, blocks, x, v=None):
    """(Pi_h, Phi_h): discrete elastic energy and dissipation potential."""
    X = _f64(X); x = _f64(x); v = _f64(v)
    Pi = C.c_double(0.0); Phi = C.c_double(0.0)
    for b in blocks:
        args, keep = _mesh_args(b, X)
        _check(lib().oracle_energy(*args, _d(x), _d(v), C.byref(Pi), C.byref(Phi)), "energy")
    return Pi.value, Phi.value


def vjp(X, blocks, x, v, w, want_gx=True, want_gv=True, want_gtheta=True):
    """(gx, gv, gtheta) with gtheta [5][n_elem_total] in block order."""
    X = _f64(X); x = _f64(x); v = _f64(v); w = _f64(w)
    gx = np.zeros_like(X) if want_gx else None
    gv = np.zeros_like(X) if want_gv else None
    gts = []
    for b in blocks:
        args, keep = _mesh_args(b, X)
        gt = np.zeros((5, b.conn.shape[0])) if want_gtheta else None
        _check(lib().oracle_vjp(*args, _d(x), _d(v), _d(w), _d(gx), _d(gv), _d(gt)), "vjp")
        gts.append(gt)
    gtheta = np.concatenate(gts, axis=1) if want_gtheta else None
    return gx, gv, gtheta


def jvp(X, blocks, x, v, dx=None, dv=None):
    """df = K dx + C dv, assembled [3][n_nodes]."""
    X = _f64(X); x = _f64(x); v = _f64(v); dx = _f64(dx); dv = _f64(dv)
    df = np.zeros_like(X)
    for b in blocks:
        args, keep = _mesh_args(b, X)
        _check(lib().oracle_jvp(*args, _d(x), _d(v), _d(dx), _d(dv), _d(df)), "jvp")
    return df


def count_inverted(X, blocks, x):
    """(number of quadrature points with det F <= 0, smallest |det F| met)."""
    X = _f64(X); x = _f64(x)
    n = C.c_int64(0)
    mn = C.c_double(float("inf"))
    for b in blocks:
        conn = np.ascontiguousarray(b.conn, dtype=np.int32)
        _check(lib().oracle_count_inverted(b.elem, X.shape[1], _d(X), conn.shape[0], conn.ctypes.data_as(_ip),
                                           _d(x), C.byref(n), C.byref(mn)), "count_inverted")
    return n.value, mn.value


def element_tangent(elem, law, theta, Xe, xe, ve=None, damped=None):
    """(K^e, C^e), each [3*nen][3*nen]; Xe, xe, ve are [3][nen]."""
    th = _f64(theta)
    if damped is None:
        damped = bool(th[3] != 0 or th[4] != 0)
    n3 = 3 * nen(elem)
    K = np.zeros((n3, n3)); Cv = np.zeros((n3, n3))
    _check(lib().oracle_element_tangent(elem, law, int(damped), _d(th), _d(_f64(Xe)), _d(_f64(xe)),
                                        _d(_f64(ve)), _d(K), _d(Cv)), "element_tangent")
    return K, Cv


def incident_elements(conn, nodes):
    """Indices of elements touching any of ``nodes`` (for sampled parity)."""
    mask = np.zeros(int(conn.max()) + 1, dtype=bool)
    mask[np.asarray(nodes)] = True
    return np.nonzero(mask[conn].any(axis=1))[0]


# ---------------------------------------------------------------- inertia and the step (Sec. 4.1, Sec. 7)

def mass_rule(elem):
    """(points [nq][3], weights [nq]) of the rule used for the mass integrals."""
    xi = np.zeros((27, 3)); w = np.zeros(27)
    nq = lib().oracle_mass_rule(elem, _d(xi), _d(w))
    return xi[:nq].copy(), w[:nq].copy()


def element_mass(elem, rho, Xe):
    """[nen][nen] element mass m_ij = int rho s_i s_j dV_r; Xe is [3][nen]."""
    n = nen(elem)
    M = np.zeros((n, n))
    _check(lib().oracle_element_mass(elem, float(rho), _d(_f64(Xe)), _d(M)), "element_mass")
    return M


def _rho(b):
    return float(getattr(b, "rho", 0.0) or 0.0)


def mass_action(X, blocks, u):
    """y = M u (assembled consistent mass, blocks summed in order)."""
    X = _f64(X); u = _f64(u)
    y = np.zeros_like(X)
    for b in blocks:
        conn = np.ascontiguousarray(b.conn, dtype=np.int32)
        _check(lib().oracle_mass_action(b.elem, X.shape[1], _d(X), conn.shape[0], conn.ctypes.data_as(_ip),
                                        _rho(b), _d(u), _d(y)), "mass_action")
    return y


def step_residual(X, blocks, q_n, v_n, v, h, f_ext=None):
    """g(v) = M (v - v_n)/h + f_int(q_n + h v, v) - f_ext (Sec. 7, no constraints)."""
    X = _f64(X); q_n = _f64(q_n); v_n = _f64(v_n); v = _f64(v)
    g = np.zeros_like(X)
    for b in blocks:
        args, keep = _mesh_args(b, X)
        _check(lib().oracle_step_residual(*args, _rho(b), _d(q_n), _d(v_n), _d(v), float(h), _d(g)), "step_residual")
    if f_ext is not None:
        g -= _f64(f_ext)
    return g


def newton_operator(X, blocks, q_n, v, h, dv):
    """(M/h + h K + C) dv at q = q_n + h v: the velocity derivative of g."""
    X = _f64(X); q_n = _f64(q_n); v = _f64(v); dv = _f64(dv)
    y = np.zeros_like(X)
    for b in blocks:
        args, keep = _mesh_args(b, X)
        _check(lib().oracle_newton_operator(*args, _rho(b), _d(q_n), _d(v), float(h), _d(dv), _d(y)),
               "newton_operator")
    return y


def newton_matrix(X, blocks, q_n, v, h):
    """The assembled (M/h + h K + C) as a scipy CSR matrix over the 3n
    unknowns ordered [3][n_nodes] (component-major), from the element
    blocks: the same operator newton_operator applies."""
    import scipy.sparse as sp
    X = _f64(X); q_n = _f64(q_n); v = _f64(v)
    n = X.shape[1]
    q = np.empty_like(q_n)
    # the step map with one rounding per entry, as the C oracle forms it
    q[...] = step_positions(h, v, q_n)
    rows, cols, vals = [], [], []
    for b in blocks:
        th = _theta_e(b)
        conn = np.ascontiguousarray(b.conn, dtype=np.int32)
        nn = conn.shape[1]
        for e in range(conn.shape[0]):
            c = conn[e]
            Ke, Ce = element_tangent(b.elem, b.law, th[:, e], X[:, c], q[:, c], v[:, c] if b.damped else None,
                                     damped=bool(b.damped))
            Me = element_mass(b.elem, _rho(b), X[:, c])
            A = h * Ke + Ce + np.kron(Me, np.eye(3)) / h
            gi = np.array([k * n + c[a] for a in range(nn) for k in range(3)])
            rows.append(np.repeat(gi, 3 * nn)); cols.append(np.tile(gi, 3 * nn)); vals.append(A.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * n, 3 * n))


def step_positions(a, x, y):
    """a * x + y with one rounding per entry (exact product via Dekker's
    splitting, then a correctly rounded sum of two terms)."""
    from fractions import Fraction
    out = np.empty_like(y)
    xf, yf = x.ravel(), y.ravel()
    o = out.ravel()
    fa = Fraction(a)
    for i in range(xf.size):
        o[i] = float(fa * Fraction(xf[i]) + Fraction(yf[i]))
    return out


def newton_step(X, blocks, q_n, v_n, v, h, f_ext=None):
    """One exact Newton step of g(v) = 0: dv = -(M/h + hK + C)^{-1} g(v)
    (direct sparse solve); returns (v + dv, dv, g)."""
    import scipy.sparse.linalg as spla
    g = step_residual(X, blocks, q_n, v_n, v, h, f_ext)
    A = newton_matrix(X, blocks, q_n, v, h)
    dv = -spla.spsolve(A.tocsc(), g.ravel()).reshape(g.shape)
    return v + dv, dv, g
