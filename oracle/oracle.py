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
T10, H8 = 0, 1
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
        L.oracle_jvp.argtypes = mesh + [_dp, _dp, _dp, _dp, _dp]
        L.oracle_element_tangent.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_count_inverted.argtypes = [C.c_int, C.c_int64, _dp, C.c_int64, _ip, _dp,
                                             C.POINTER(C.c_int64), _dp]
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
    xi = np.zeros((8, 3)); w = np.zeros(8)
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
