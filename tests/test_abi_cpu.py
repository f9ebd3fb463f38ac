"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects bad arguments on the host before any device work."""
import copy
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from paper_2602_17002_amd import _lib
from paper_2602_17002_amd._lib import Block

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tlfea.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tlfea_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tlfea_create_mesh", "tlfea_internal_force", "tlfea_internal_force_vjp", "tlfea_tangent_jvp",
              "tlfea_destroy_mesh", "tlfea_last_error"):
        assert n in names
    assert set(names) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def _create(X, blocks, flags=0, n_nodes=None):
    L = _lib.lib()
    arr = (Block * max(1, len(blocks)))()
    keep = []
    for i, b in enumerate(blocks):
        conn = np.ascontiguousarray(b["conn"], dtype=np.int32) if b.get("conn") is not None else None
        keep.append(conn)
        arr[i].elem = b.get("elem", 0)
        arr[i].law = b.get("law", 0)
        arr[i].n_elem = b.get("n_elem", 0 if conn is None else conn.shape[0])
        arr[i].conn = conn.ctypes.data_as(C.POINTER(C.c_int32)) if conn is not None else C.POINTER(C.c_int32)()
        for p, val in enumerate(b.get("theta", [1.0, 1.0, 1.0, 0.0, 0.0])):
            arr[i].theta[p] = val
        arr[i].damped = b.get("damped", 0)
        arr[i].tile_elems = b.get("tile_elems", 0)
        arr[i].rho = b.get("rho", 0.0)
        arr[i].reserved = b.get("reserved", 0)
        nq = b.get("nq", None)
        for name in ("qp_w", "dsdxi"):
            t = b.get(name)
            if t is not None:
                t = np.ascontiguousarray(t, dtype=np.float64)
                keep.append(t)
                setattr(arr[i], name, t.ctypes.data_as(C.POINTER(C.c_double)))
                nq = t.shape[0] if nq is None else nq
        arr[i].nq = nq or 0
    X = np.ascontiguousarray(X, dtype=np.float64)
    h = C.c_void_p()
    n = X.shape[1] if n_nodes is None else n_nodes
    st = L.tlfea_create_mesh(n, X.ctypes.data_as(C.POINTER(C.c_double)), len(blocks), arr, flags, None,
                             C.byref(h))
    return st, h, L.tlfea_last_error().decode()


@pytest.fixture(scope="module")
def box():
    return synth.box_t10(2, 1, 1, size=(0.2, 0.1, 0.1))


def test_node_id_out_of_range(box):
    X, conn = box
    c = conn.copy(); c[3, 2] = X.shape[1]
    st, h, msg = _create(X, [dict(conn=c)])
    assert st == -2 and not h.value and "outside" in msg


def test_negative_node_id(box):
    X, conn = box
    c = conn.copy(); c[0, 0] = -1
    assert _create(X, [dict(conn=c)])[0] == -2


def test_repeated_node_in_element(box):
    X, conn = box
    c = conn.copy(); c[1, 3] = c[1, 0]
    st, _, msg = _create(X, [dict(conn=c)])
    assert st == -2 and "repeats" in msg


def test_inverted_reference_element(box):
    X, conn = box
    c = conn.copy()
    for i, j in [(1, 2), (4, 6), (8, 9)]:
        c[5, [i, j]] = c[5, [j, i]]
    st, _, msg = _create(X, [dict(conn=c)])
    assert st == -3 and "element 5" in msg


def test_bad_enums_flags_and_sizes(box):
    X, conn = box
    assert _create(X, [dict(conn=conn, elem=7)])[0] == -1
    assert _create(X, [dict(conn=conn, law=9)])[0] == -1
    assert _create(X, [dict(conn=conn)], flags=64)[0] == -1
    assert _create(X, [dict(conn=conn, tile_elems=100)])[0] == -1
    assert _create(X, [dict(conn=None, n_elem=3)])[0] == -1
    assert _create(X, [dict(conn=conn, n_elem=-1)])[0] == -2
    assert _create(X, [dict(conn=conn, theta=[np.nan, 1, 1, 0, 0])])[0] == -1
    Xn = X.copy(); Xn[1, 4] = np.inf
    assert _create(Xn, [dict(conn=conn)])[0] == -1
    assert _create(X, [dict(conn=conn)], n_nodes=-5)[0] == -2


def test_wrong_element_type_for_connectivity_width(box):
    # H8 connectivity read as T10 would run past the row: sizes are checked
    X, conn = synth.box_h8(2, 2, 2)
    st, _, msg = _create(X, [dict(conn=conn[:, :8], elem=1)])
    assert st in (0, -5, -4)   # valid H8 input; only the device step can fail here


def test_compute_calls_reject_null_mesh():
    L = _lib.lib()
    assert L.tlfea_internal_force(None, None, None, None, None, None) == -1
    assert L.tlfea_internal_force_vjp(None, None, None, None, None, None, None, None, None) == -1
    assert L.tlfea_tangent_jvp(None, None, None, None, None, None, None, None, None) == -1
    assert L.tlfea_count_inverted(None, None, None, None) == -1
    assert L.tlfea_get_mesh_info(None, None) == -1
    assert L.tlfea_set_profiling(None, 1) == -1
    L.tlfea_destroy_mesh(None)   # no-op


def test_python_wrapper_raises_typed_error(box):
    from paper_2602_17002_amd import Mesh, TlfeaError
    X, conn = box
    blk = synth.Block(synth.T10, synth.SVK, conn.copy(), np.array([1.0, 1.0, 0, 0, 0]))
    blk.conn[0, 0] = 10 ** 6
    with pytest.raises(TlfeaError) as ei:
        Mesh(X, [blk])
    assert ei.value.status == -2


def test_header_is_plain_c(tmp_path):
    """include/tlfea.h compiles as C99 on its own (no C++ or torch types)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include <stddef.h>\n#include "tlfea.h"\n'
                   "int use(tlfea_mesh *m, const double *x, double *f, void *s)\n"
                   "{ tlfea_block b = {TLFEA_T10, TLFEA_NH, 0, NULL, {1, 0, 1, 0, 0}, 0, 0, 0, 0, NULL, NULL, 0.0};\n"
                   "  (void)b; return (int)tlfea_internal_force(m, x, NULL, NULL, f, s); }\n")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", inc, "-c", str(src),
                        "-o", str(tmp_path / "use.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def _t10_rule_tables():
    """The 5-point degree-3 rule and the App. A.1 gradient table at its
    points, written out here from the paper's table (rows of the 10-node
    tetrahedron's shape-function derivatives)."""
    a, b = 1.0 / 6.0, 0.5
    pts = [(0.25, 0.25, 0.25), (a, a, a), (b, a, a), (a, b, a), (a, a, b)]
    w = np.array([-4.0 / 5.0 / 6.0] + [9.0 / 20.0 / 6.0] * 4)
    G = np.zeros((5, 10, 3))
    for q, (x, y, z) in enumerate(pts):
        G[q] = [[4 * x + 4 * y + 4 * z - 3] * 3, [4 * x - 1, 0, 0], [0, 4 * y - 1, 0], [0, 0, 4 * z - 1],
                [-8 * x - 4 * y - 4 * z + 4, -4 * x, -4 * x], [4 * y, 4 * x, 0],
                [-4 * y, -4 * x - 8 * y - 4 * z + 4, -4 * y], [-4 * z, -4 * z, -4 * x - 4 * y - 8 * z + 4],
                [4 * z, 0, 4 * x], [0, 4 * z, 4 * y]]
    return w, G


def test_quadrature_table_of_the_builtin_rule_is_accepted(box):
    # the boundary takes the parent-element rule as data (Sec. 6); the
    # built-in one passes validation (on a machine without a GPU the call
    # then stops at the device step)
    X, conn = box
    w, G = _t10_rule_tables()
    st, h, msg = _create(X, [dict(conn=conn, qp_w=w, dsdxi=G)])
    assert st in (0, -4, -5), msg
    st, h, msg = _create(X, [dict(conn=conn, qp_w=w)])
    assert st in (0, -4, -5), msg
    # a table equal to the rule to rounding is the same rule
    st, h, msg = _create(X, [dict(conn=conn, dsdxi=G * (1 + 1e-16))])
    assert st in (0, -4, -5), msg


def test_other_quadrature_tables_are_refused(box):
    X, conn = box
    w, G = _t10_rule_tables()
    G2 = G.copy(); G2[3, 5, 1] += 1e-6
    st, _, msg = _create(X, [dict(conn=conn, dsdxi=G2)])
    assert st == -6 and "parent gradient [3][5][1]" in msg
    w2 = w.copy(); w2[0] *= -1
    st, _, msg = _create(X, [dict(conn=conn, qp_w=w2)])
    assert st == -6 and "weight of point 0" in msg
    # a 4-point rule (another degree)
    st, _, msg = _create(X, [dict(conn=conn, qp_w=np.full(4, 1 / 24), nq=4)])
    assert st == -6 and "4-point" in msg
    # an nq without a table, a nonzero reserved field, a negative density
    assert _create(X, [dict(conn=conn, nq=5)])[0] == -1
    assert _create(X, [dict(conn=conn, reserved=1)])[0] == -1
    assert _create(X, [dict(conn=conn, rho=-1.0)])[0] == -1
