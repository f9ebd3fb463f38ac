"""GPU parity: every output of the HIP path through the C ABI against the CPU
oracle on the same seeded inputs, element by element (norm-wise relative
error <= 1e-12), plus bitwise repeatability and the degenerate cases."""
import copy

import numpy as np
import pytest

import oracle as O
import synth
from _util import TOL, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

LAWS = {
    "SVK": (synth.SVK, np.array([5.769e6, 3.846e6, 0.0, 1.0e4, 3.0e3])),
    "NH": (synth.NH, np.array([1.7e6, 0.0, 1.72667e7, 1.0e4, 3.0e3])),
    "MR": (synth.MR, np.array([1.2e6, 0.45e6, 1.72667e7, 1.0e4, 3.0e3])),
}


def oc(p):
    """(X, blocks, x) for the oracle: the very inputs the GPU gets.  The
    oracle forms every element's positions relative to its first node, so
    its own FP64 error on these meshes stays below 1e-13 (measured against
    an extended-precision evaluation)."""
    return p.X, p.blocks, p.x


def say(*a):
    print(*a, flush=True)


def mesh_of(prob, flags=0, tile=None):
    from paper_2602_17002_amd import Mesh
    blocks = [copy.copy(b) for b in prob.blocks]
    if tile:
        for b in blocks:
            b.tile_elems = tile
    return Mesh(prob.X, blocks, flags=flags)


def make_problem(elem, law, damped, n=(7, 5, 3), seed=0, curved=False, per_elem=False, cell=0.02):
    rng = np.random.default_rng(seed)
    lid, th = LAWS[law]
    size = tuple(k * cell for k in n)
    X, conn = {synth.T10: synth.box_t10, synth.H8: synth.box_h8, synth.Q27: synth.box_q27}[elem](*n, size=size)
    if curved:
        if elem == synth.T10:
            X = synth.curve_midside_t10(X, conn, 0.08, rng)
        else:
            X = X + rng.uniform(-0.08 * cell, 0.08 * cell, X.shape)
    x = synth.sinusoidal_state(X, 0.05, rng)
    x = x + rng.normal(0, 0.02 * cell, X.shape)
    v = rng.normal(0, 0.5, X.shape) if damped else np.zeros_like(X)
    th = th.copy()
    if not damped:
        th[3:] = 0
    b = synth.Block(elem, lid, conn, th, damped=damped)
    if per_elem:
        b.theta_e = th[:, None] * rng.uniform(0.5, 2.0, (5, conn.shape[0]))
    p = synth.Problem(f"{synth.ELEM_NAMES[elem]}-{law}-{'KV' if damped else 'el'}", X, x, v, [b], cell=cell)
    p.w = rng.standard_normal(X.shape)
    p.dx = rng.standard_normal(X.shape) * cell
    p.dv = rng.standard_normal(X.shape)
    return p


CASES = [(e, l, d) for e in (synth.T10, synth.H8) for l in ("SVK", "NH", "MR") for d in (False, True)]


def _id(c):
    return f"{synth.ELEM_NAMES[c[0]]}-{c[1]}-{'KV' if c[2] else 'el'}"


@pytest.mark.parametrize("case", CASES, ids=_id)
@pytest.mark.parametrize("tile", [64, 256])
def test_forward_matches_oracle(case, tile):
    elem, law, damped = case
    p = make_problem(elem, law, damped, curved=(tile == 64))
    say("forward", p.name, "tile", tile, "elements", p.n_elem)
    m = mesh_of(p, tile=tile)
    f = to_host(m.internal_force(to_dev(p.x), to_dev(p.v) if damped else None))
    ref = O.internal_force(*oc(p), p.v)
    assert rel(f, ref) <= TOL, rel(f, ref)


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_vjp_matches_oracle(case):
    elem, law, damped = case
    p = make_problem(elem, law, damped, per_elem=True, curved=True, seed=1)
    say("vjp", p.name)
    m = mesh_of(p, tile=128)
    th = p.theta_all()
    gx, gv, gt = m.vjp(to_dev(p.x), to_dev(p.v) if damped else None, to_dev(p.w), to_dev(th))
    rx, rv, rt = O.vjp(*oc(p), p.v, p.w)
    assert rel(to_host(gx), rx) <= TOL
    if damped:
        assert rel(to_host(gv), rv) <= TOL
    else:
        assert np.all(to_host(gv) == 0)
    gt = to_host(gt)
    for r in range(5):
        if np.abs(rt[r]).max() == 0:
            assert np.all(gt[r] == 0), r
        else:
            assert rel(gt[r], rt[r]) <= TOL, (r, rel(gt[r], rt[r]))


# dv enters only through the viscous stress, so the dv directions are taken
# on damped bodies only
JVP_CASES = [(c, w) for w in ("dx+dv", "dx", "dv", "none") for c in CASES if c[2] or "dv" not in w]


@pytest.mark.parametrize("case,which", JVP_CASES, ids=lambda v: _id(v) if isinstance(v, tuple) else v)
def test_jvp_matches_oracle(case, which):
    elem, law, damped = case
    p = make_problem(elem, law, damped, per_elem=True, seed=2)
    say("jvp", p.name, which)
    m = mesh_of(p, tile=256)
    dx = p.dx if "dx" in which else None
    dv = p.dv if "dv" in which else None
    th = p.theta_all()
    df = to_host(m.jvp(to_dev(p.x), to_dev(p.v) if damped else None, None if dx is None else to_dev(dx),
                       None if dv is None else to_dev(dv), to_dev(th)))
    ref = O.jvp(*oc(p), p.v, dx, dv)
    if which == "none":
        assert np.all(df == 0)
    else:
        assert rel(df, ref) <= TOL, rel(df, ref)


@pytest.mark.parametrize("tile", [64, 128, 192, 256])
@pytest.mark.parametrize("elem", [synth.T10, synth.H8], ids=["T10", "H8"])
def test_every_operation_at_every_tile_size(elem, tile):
    # Each tile size gives every operation its own LDS budget, node cap and
    # number of components assembled per round; the damped Mooney-Rivlin
    # body has the longest records and the most registers.
    n = (9, 5, 4) if elem == synth.T10 else (12, 8, 5)
    p = make_problem(elem, "MR", True, n=n, per_elem=True, curved=True, seed=30 + tile)
    say("tile sizes", p.name, "tile", tile, "elements", p.n_elem)
    m = mesh_of(p, tile=tile)
    assert m.info()["tile_elems_t10" if elem == synth.T10 else "tile_elems_h8"] == tile
    th = p.theta_all()
    x, v = to_dev(p.x), to_dev(p.v)
    f = to_host(m.internal_force(x, v, to_dev(th)))
    assert rel(f, O.internal_force(*oc(p), p.v)) <= TOL
    gx, gv, gt = m.vjp(x, v, to_dev(p.w), to_dev(th))
    rx, rv, rt = O.vjp(*oc(p), p.v, p.w)
    assert rel(to_host(gx), rx) <= TOL and rel(to_host(gv), rv) <= TOL
    gt = to_host(gt)
    for r in range(5):
        assert rel(gt[r], rt[r]) <= TOL, r
    df = to_host(m.jvp(x, v, to_dev(p.dx), to_dev(p.dv), to_dev(th)))
    assert rel(df, O.jvp(*oc(p), p.v, p.dx, p.dv)) <= TOL


@pytest.mark.parametrize("law", ["SVK", "NH", "MR"])
@pytest.mark.parametrize("elem", [synth.T10, synth.H8], ids=["T10", "H8"])
def test_large_deformation(elem, law):
    # Strains up to 40 % (peak displacement gradient 0.4, with a volumetric
    # part) under a rigid rotation and fast velocities: every output against
    # the oracle, with every |det F| checked to stay clear of zero.
    rng = np.random.default_rng(60)
    lid, th = LAWS[law]
    n = (6, 4, 3)
    X, conn = (synth.box_t10 if elem == synth.T10 else synth.box_h8)(*n, size=tuple(0.02 * k for k in n))
    x = synth.sinusoidal_state(X, 0.4, rng)
    v = rng.normal(0, 5.0, X.shape)
    b = synth.Block(elem, lid, conn, th.copy(), damped=True)
    b.theta_e = th[:, None] * rng.uniform(0.5, 2.0, (5, conn.shape[0]))
    p = synth.Problem(f"large-{synth.ELEM_NAMES[elem]}-{law}", X, x, v, [b], cell=0.02)
    ninv, min_det = O.count_inverted(p.X, p.blocks, p.x)
    assert ninv == 0 and min_det > 0.2, (ninv, min_det)
    w, dx, dv = rng.standard_normal(X.shape), rng.standard_normal(X.shape) * 0.02, rng.standard_normal(X.shape)
    say("large deformation", p.name, "min det F", min_det)
    m = mesh_of(p)
    th_d = to_dev(p.theta_all())
    xd, vd = to_dev(x), to_dev(v)
    assert rel(to_host(m.internal_force(xd, vd, th_d)), O.internal_force(X, p.blocks, x, v)) <= TOL
    gx, gv, gt = m.vjp(xd, vd, to_dev(w), th_d)
    rx, rv, rt = O.vjp(X, p.blocks, x, v, w)
    assert rel(to_host(gx), rx) <= TOL and rel(to_host(gv), rv) <= TOL
    gt = to_host(gt)
    for r in range(5):
        if np.abs(rt[r]).max() > 0:
            assert rel(gt[r], rt[r]) <= TOL, r
    df = to_host(m.jvp(xd, vd, to_dev(dx), to_dev(dv), th_d))
    assert rel(df, O.jvp(X, p.blocks, x, v, dx, dv)) <= TOL


@pytest.mark.parametrize("damped", [False, True], ids=["undamped", "damped"])
@pytest.mark.parametrize("law", ["SVK", "NH", "MR"])
@pytest.mark.parametrize("elem", [synth.T10, synth.H8], ids=["T10", "H8"])
def test_reflected_state(elem, law, damped):
    # Every point inverted (a mirror image of a 10 % strain state, det F
    # near -1, every |det F| far from zero): the stress laws are evaluated
    # there as written (real cube roots of negative J), and every output,
    # the adjoint with and without the parameter gradients, matches the
    # oracle.
    rng = np.random.default_rng(61)
    lid, th = LAWS[law]
    n = (6, 4, 3)
    X, conn = (synth.box_t10 if elem == synth.T10 else synth.box_h8)(*n, size=tuple(0.02 * k for k in n))
    x = synth.sinusoidal_state(X, 0.1, rng) * np.array([[1.0], [-1.0], [1.0]])
    v = rng.normal(0, 1.0, X.shape) if damped else np.zeros_like(X)
    t = th.copy() if damped else np.concatenate([th[:3], [0.0, 0.0]])
    b = synth.Block(elem, lid, conn, t, damped=damped)
    b.theta_e = t[:, None] * rng.uniform(0.5, 2.0, (5, conn.shape[0]))
    p = synth.Problem(f"reflected-{synth.ELEM_NAMES[elem]}-{law}", X, x, v, [b], cell=0.02)
    ninv, min_det = O.count_inverted(p.X, p.blocks, p.x)
    assert ninv == p.n_qp and min_det > 0.2, (ninv, min_det)
    w, dx, dv = rng.standard_normal(X.shape), rng.standard_normal(X.shape) * 0.02, rng.standard_normal(X.shape)
    say("reflected", p.name, "damped", damped, "min |det F|", min_det)
    m = mesh_of(p)
    th_d = to_dev(p.theta_all())
    xd, vd = to_dev(x), to_dev(v)
    vo = v if damped else None
    assert rel(to_host(m.internal_force(xd, vd, th_d)), O.internal_force(X, p.blocks, x, vo)) <= TOL
    rx, rv, rt = O.vjp(X, p.blocks, x, v, w)
    gx, gv, gt = m.vjp(xd, vd, to_dev(w), th_d)
    assert rel(to_host(gx), rx) <= TOL
    if damped:
        assert rel(to_host(gv), rv) <= TOL
    gt = to_host(gt)
    for r in range(5):
        if np.abs(rt[r]).max() > 0:
            assert rel(gt[r], rt[r]) <= TOL, r
    gx2, _, _ = m.vjp(xd, vd, to_dev(w), th_d, want_theta=False)
    assert rel(to_host(gx2), rx) <= TOL
    df = to_host(m.jvp(xd, vd, to_dev(dx), to_dev(dv), th_d))
    assert rel(df, O.jvp(X, p.blocks, x, v, dx, dv if damped else np.zeros_like(dv))) <= TOL


@pytest.mark.parametrize("elem", [synth.T10, synth.H8], ids=["T10", "H8"])
def test_outputs_unchanged_by_exact_translation(elem):
    # Positions enter only through differences against each tile's
    # reference node; with coordinates on a 2^-40 m grid and an offset by
    # powers of two every translated coordinate and every difference is
    # exact, so the outputs must not change by a single bit.
    p = make_problem(elem, "NH", True, n=(8, 5, 4), per_elem=True, seed=50)
    q = 2.0 ** -40
    X, x = np.round(p.X / q) * q, np.round(p.x / q) * q
    T = np.array([[1024.0], [-2048.0], [512.0]])
    assert np.array_equal((X + T) - T, X) and np.array_equal((x + T) - T, x)
    say("translation", p.name)
    th = to_dev(p.theta_all())
    outs = []
    for XX, xx in ((X, x), (X + T, x + T)):
        pp = copy.copy(p)
        pp.X = np.ascontiguousarray(XX)
        m = mesh_of(pp)
        xd, vd = to_dev(xx), to_dev(p.v)
        f = to_host(m.internal_force(xd, vd, th))
        gx, gv, gt = (to_host(a) for a in m.vjp(xd, vd, to_dev(p.w), th))
        df = to_host(m.jvp(xd, vd, to_dev(p.dx), to_dev(p.dv), th))
        outs.append((f, gx, gv, gt, df))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    assert rel(outs[0][0], O.internal_force(X, p.blocks, x, p.v)) <= TOL


def test_c1_cantilever_all_outputs_and_repeatability():
    """The C1 cantilever: every output against the oracle, and every output
    of ten repeated calls bitwise equal (no atomics, fixed summation order)."""
    p = synth.config_c1()
    say("C1 cantilever", p.n_elem)
    m = mesh_of(p)
    rng = np.random.default_rng(3)
    w = rng.standard_normal(p.X.shape)
    dx, dv = rng.standard_normal(p.X.shape) * 0.05, rng.standard_normal(p.X.shape)
    xd, vd, wd, dxd, dvd = (to_dev(a) for a in (p.x, p.v, w, dx, dv))
    runs = []
    for rep in range(10):
        f = to_host(m.internal_force(xd, vd))
        gx, gv, gt = (to_host(a) for a in m.vjp(xd, vd, wd))
        df = to_host(m.jvp(xd, vd, dxd, dvd))
        runs.append((f, gx, gv, gt, df))
    for r in runs[1:]:
        for a, b in zip(r, runs[0]):
            assert np.array_equal(a, b)
    f, gx, gv, gt, df = runs[0]
    assert rel(f, O.internal_force(*oc(p), p.v)) <= TOL
    rx, rv, rt = O.vjp(*oc(p), p.v, w)
    assert rel(gx, rx) <= TOL and rel(gv, rv) <= TOL
    for r in (0, 1, 3):
        assert rel(gt[r], rt[r]) <= TOL
    assert np.all(gt[2] == 0) and rel(gt[4], rt[4]) <= TOL
    assert rel(df, O.jvp(*oc(p), p.v, dx, dv)) <= TOL


def test_keep_order_and_tile_sizes_agree():
    p = make_problem(synth.T10, "NH", True, n=(9, 4, 3), seed=4)
    say("orders", p.n_elem)
    ref = O.internal_force(*oc(p), p.v)
    from paper_2602_17002_amd import KEEP_ORDER
    for flags in (0, KEEP_ORDER):
        for tile in (64, 128, 256):
            m = mesh_of(p, flags=flags, tile=tile)
            f = to_host(m.internal_force(to_dev(p.x), to_dev(p.v)))
            assert rel(f, ref) <= TOL, (flags, tile)


def test_degenerate_meshes():
    from paper_2602_17002_amd import Mesh
    say("degenerate")
    # one element, and nodes that no element touches (output must be 0 there)
    X, conn = synth.box_t10(1, 1, 1, size=(0.1, 0.1, 0.1))
    extra = np.random.default_rng(5).uniform(0, 1, (3, 7))
    X2 = np.concatenate([X, extra], axis=1)
    b = synth.Block(synth.T10, synth.NH, conn[:1].copy(), LAWS["NH"][1], damped=True)
    rng = np.random.default_rng(6)
    x = X2 + rng.normal(0, 1e-3, X2.shape); v = rng.normal(0, 1, X2.shape)
    m = Mesh(X2, [b])
    f = to_host(m.internal_force(to_dev(x), to_dev(v)))
    Xc, xc = X2, x
    ref = O.internal_force(Xc, [b], xc, v)
    assert rel(f, ref) <= TOL
    untouched = np.setdiff1d(np.arange(X2.shape[1]), conn[0])
    assert np.all(f[:, untouched] == 0)
    # a block with no elements next to a real one
    e = synth.Block(synth.H8, synth.SVK, np.zeros((0, 8), np.int32), LAWS["SVK"][1], damped=False)
    m = Mesh(X2, [e, b])
    assert rel(to_host(m.internal_force(to_dev(x), to_dev(v))), ref) <= TOL
    # no elements at all: f == 0
    m = Mesh(X2, [e])
    assert np.all(to_host(m.internal_force(to_dev(x), to_dev(v))) == 0)


@pytest.mark.parametrize("tile", [64, 256])
def test_node_in_every_element(tile):
    """A fan of 700 T10 around one shared corner node: that node's slot group
    spans several threads' chunks in every tile (the reduction's long case)
    and it is shared by every tile.  Forward, adjoint and tangent against
    the oracle."""
    rng = np.random.default_rng(61)
    X, conn = synth.fan_t10(700, 0.02, rng)
    x = X + rng.normal(0, 2e-3, X.shape)
    v = rng.normal(0, 0.5, X.shape)
    b = synth.Block(synth.T10, synth.NH, conn, LAWS["NH"][1], damped=True)
    p = synth.Problem("fan", X, x, v, [b], cell=0.02)
    p.w = rng.standard_normal(X.shape)
    dx = rng.standard_normal(X.shape) * 0.02
    dv = rng.standard_normal(X.shape)
    say("fan", "tile", tile, "elements", p.n_elem)
    m = mesh_of(p, tile=tile)
    assert m.info()["n_tiles"] >= 700 // 66
    f = to_host(m.internal_force(to_dev(x), to_dev(v)))
    assert rel(f, O.internal_force(*oc(p), v)) <= TOL
    gx, gv, _ = m.vjp(to_dev(x), to_dev(v), to_dev(p.w), want_theta=False)
    rx, rv, _ = O.vjp(*oc(p), v, p.w)
    assert rel(to_host(gx), rx) <= TOL and rel(to_host(gv), rv) <= TOL
    df = to_host(m.jvp(to_dev(x), to_dev(v), to_dev(dx), to_dev(dv)))
    assert rel(df, O.jvp(*oc(p), v, dx, dv)) <= TOL


def test_node_order_renumbering():
    """tlfea_node_order is a permutation; a mesh built from the renumbered
    problem gives the renumbered outputs (to rounding) and matches the oracle."""
    p = make_problem(synth.T10, "NH", True, n=(9, 7, 4), seed=11)
    say("node order", p.name, p.n_elem)
    m = mesh_of(p)
    order = m.node_order()
    assert np.array_equal(np.sort(order), np.arange(p.n_nodes))
    q = p.renumbered(order)
    mq = mesh_of(q)
    f = to_host(m.internal_force(to_dev(p.x), to_dev(p.v)))
    fq = to_host(mq.internal_force(to_dev(q.x), to_dev(q.v)))
    gx, gv, _ = m.vjp(to_dev(p.x), to_dev(p.v), to_dev(p.w), want_theta=False)
    gxq, gvq, _ = mq.vjp(to_dev(q.x), to_dev(q.v), to_dev(q.w), want_theta=False)
    assert rel(fq, f[:, order]) <= 1e-13
    assert rel(to_host(gxq), to_host(gx)[:, order]) <= 1e-13
    assert rel(to_host(gvq), to_host(gv)[:, order]) <= 1e-13
    Xc, xc = q.X, q.x
    assert rel(fq, O.internal_force(Xc, q.blocks, xc, q.v)) <= TOL


@pytest.mark.parametrize("tile", [64, 256])
def test_count_inverted_matches_oracle(tile):
    """Integer count of points with det F <= 0, exact against the oracle on
    tangled T10 and H8 boxes (seeds whose smallest |det F| is far from the
    rounding of either side), plus the reference, reflected, collapsed and
    multi-block cases."""
    say("count_inverted tile", tile)
    cases = []
    for elem, n, size, seed in ((synth.T10, (4, 2, 2), (0.4, 0.2, 0.2), 1), (synth.H8, (4, 3, 2), (0.4, 0.3, 0.2), 0)):
        X, conn = (synth.box_t10 if elem == synth.T10 else synth.box_h8)(*n, size=size)
        b = synth.Block(elem, synth.SVK, conn, LAWS["SVK"][1], damped=False)
        b.tile_elems = tile
        x = X + np.random.default_rng(seed).normal(0, 0.04, X.shape)
        cases.append((X, [b], x))
    # the two bodies side by side in one mesh
    X0, b0, x0 = cases[0]
    X1, b1, x1 = cases[1]
    bb = copy.copy(b1[0]); bb.conn = b1[0].conn + X0.shape[1]
    cases.append((np.concatenate([X0, X1], 1), [b0[0], bb], np.concatenate([x0, x1], 1)))
    from paper_2602_17002_amd import Mesh
    for X, blocks, x in cases:
        n_qp = sum(bl.conn.shape[0] * len(O.quadrature(bl.elem)[1]) for bl in blocks)
        m = Mesh(X, blocks)
        ref, mn = O.count_inverted(X, blocks, x)
        assert 0 < ref < n_qp and mn > 1e-3
        assert int(m.count_inverted(to_dev(x)).item()) == ref
        assert int(m.count_inverted(to_dev(X)).item()) == 0
        assert int(m.count_inverted(to_dev(X * np.array([[1.0], [-1.0], [1.0]]))).item()) == n_qp
        assert int(m.count_inverted(to_dev(np.zeros_like(X))).item()) == n_qp


def test_multibody_batched_graph_equals_plain_and_oracle():
    from paper_2602_17002_amd import BATCHED, Mesh
    import torch
    p = synth.config_multibody(12, 150, 3000, seed=7, directions=True)
    say("multibody", len(p.blocks), p.n_elem)
    ref = O.internal_force(*oc(p), p.v)
    rx, rv, rt = O.vjp(*oc(p), p.v, p.w, want_gv=False)
    rj = O.jvp(*oc(p), p.v, p.dx)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x, w, dx = to_dev(p.x), to_dev(p.w), to_dev(p.dx)
        plain = mesh_of(p)
        batched = mesh_of(p, flags=BATCHED)
        fp = plain.internal_force(x)
        fb = torch.empty_like(x); gx = torch.empty_like(x); dfb = torch.empty_like(x)
        gt = torch.empty((5, p.n_elem), dtype=torch.float64, device="cuda")
        outs = []
        for rep in range(3):   # first call captures, later calls replay the graph
            for t in (fb, gx, dfb, gt):
                t.fill_(float("nan"))
            batched.internal_force(x, out=fb)
            batched.vjp(x, None, w, want_v=False, out=(gx, None, gt))
            batched.jvp(x, None, dx, out=dfb)
            torch.cuda.synchronize()
            outs.append((to_host(fb), to_host(gx), to_host(gt), to_host(dfb)))
        torch.cuda.synchronize()
    fp = to_host(fp)
    assert rel(fp, ref) <= TOL
    for fb, gx, gt, dfb in outs:
        assert np.array_equal(fb, fp)
        assert rel(gx, rx) <= TOL
        assert rel(dfb, rj) <= TOL
        for r in range(3):
            if np.abs(rt[r]).max() > 0:
                assert rel(gt[r], rt[r]) <= TOL
    # per-body plain meshes give bitwise the same forces as the batched mesh
    for bi in (0, 1, 5):
        b = p.blocks[bi]
        n0, n1 = p.body_nodes[bi]
        bb = copy.copy(b); bb.conn = b.conn - n0
        mb = Mesh(p.X[:, n0:n1], [bb])
        fb1 = to_host(mb.internal_force(to_dev(p.x[:, n0:n1])))
        assert np.array_equal(fb1, outs[0][0][:, n0:n1])


def test_batched_graph_cache_eviction():
    # A batched mesh keeps one graph per (operation, operand pointers,
    # stream), at most eight, evicting the least recently used one after its
    # last launch has finished.  Twelve output buffers, cycled twice on one
    # stream without synchronising, force in-place updates of cached graphs
    # while earlier launches may still run; every output must equal the plain
    # mesh's bitwise.
    import torch
    from paper_2602_17002_amd import BATCHED
    p = synth.config_multibody(6, 150, 1500, seed=9, directions=True)
    say("graph cache", len(p.blocks), p.n_elem)
    plain, batched = mesh_of(p), mesh_of(p, flags=BATCHED)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x, w = to_dev(p.x), to_dev(p.w)
        ref_f = to_host(plain.internal_force(x))
        ref_g = to_host(plain.vjp(x, None, w, want_v=False, want_theta=False)[0])
        fs = [torch.empty_like(x) for _ in range(12)]
        gs = [torch.empty_like(x) for _ in range(12)]
        for rep in range(2):
            for f, g in zip(fs, gs):
                f.fill_(float("nan"))
                g.fill_(float("nan"))
                batched.internal_force(x, out=f)
                batched.vjp(x, None, w, want_v=False, want_theta=False, out=(g, None, None))
        torch.cuda.synchronize()
    for f, g in zip(fs, gs):
        assert np.array_equal(to_host(f), ref_f)
        assert np.array_equal(to_host(g), ref_g)
    # with all eight graphs in use, new operand pointers update a cached
    # graph of the same operation in place
    info = batched.info()
    say("graphs built", info["graphs_built"], "updated", info["graphs_updated"])
    assert info["graphs_built"] >= 2 and info["graphs_updated"] > 0


def test_autograd_function():
    import torch
    from paper_2602_17002_amd import TLInternalForce
    p = make_problem(synth.T10, "NH", True, n=(3, 3, 2), seed=8, per_elem=True)
    say("autograd", p.n_elem)
    m = mesh_of(p)
    x = to_dev(p.x).requires_grad_(True)
    v = to_dev(p.v).requires_grad_(True)
    th = to_dev(p.theta_all()).requires_grad_(True)
    w = to_dev(p.w)
    f = TLInternalForce.apply(x, v, th, m)
    (f * w).sum().backward()
    rx, rv, rt = O.vjp(*oc(p), p.v, p.w)
    assert rel(to_host(x.grad), rx) <= TOL
    assert rel(to_host(v.grad), rv) <= TOL
    gth = to_host(th.grad)
    for r in range(5):   # Neo-Hookean + KV: rows 0, 2, 3, 4; the unused row 1 is exactly 0
        if np.abs(rt[r]).max() > 0:
            assert rel(gth[r], rt[r]) <= TOL, r
        else:
            assert np.all(gth[r] == 0), r
    # forward mode
    import torch.autograd.forward_ad as fwAD
    dx, dv = to_dev(p.dx), to_dev(p.dv)
    dth = to_dev(p.theta_all() * 0.1)
    with fwAD.dual_level():
        out = TLInternalForce.apply(fwAD.make_dual(x.detach(), dx), fwAD.make_dual(v.detach(), dv),
                                    fwAD.make_dual(th.detach(), dth), m)
        tangent = to_host(fwAD.unpack_dual(out).tangent)
    ref = O.jvp(*oc(p), p.v, p.dx, p.dv)
    b2 = copy.copy(p.blocks[0]); b2.theta_e = p.theta_all() * 0.1
    ref = ref + O.internal_force(oc(p)[0], [b2], oc(p)[2], p.v)
    assert rel(tangent, ref) <= TOL


def _h8_body():
    """A large H8 body (64x64x32 cells = 131,072 trilinear hexahedra, 2x2x2
    Gauss), Mooney-Rivlin with Kelvin-Voigt damping, under a rigid motion and
    a 3 % smooth deformation: the batched sets' other element type and the
    paper's general law, at a size that fills the GPU."""
    rng = np.random.default_rng(np.random.SeedSequence(1006))
    n = (64, 64, 32)
    X, conn = synth.box_h8(*n, size=tuple(0.01 * k for k in n))
    x = synth.sinusoidal_state(X, 0.03, rng)
    v = rng.normal(0.0, 0.01, X.shape)
    b = synth.Block(synth.H8, synth.MR, conn, np.array([1.2e6, 0.45e6, 1.72667e7, 1.0e4, 3.0e3]), damped=True)
    p = synth.Problem("H8-MR-KV-131k", X, x, v, [b], cell=0.01)
    p.w = rng.standard_normal(X.shape)
    p.dx = rng.standard_normal(X.shape) * 0.01
    return p


def _full_size(cfg):
    return {"C2": synth.config_c2, "C4": synth.config_c4, "H8": _h8_body}[cfg]()


def _check_whole(name, got, ref):
    """Norm-wise bound per output array; a parameter-gradient array is
    checked row by row (rows a law does not use must be exactly 0)."""
    if got.ndim == 2 and got.shape[0] == 5 and name.startswith("gtheta"):
        for r in range(5):
            if np.abs(ref[r]).max() == 0:
                assert np.all(got[r] == 0), (name, r)
            else:
                e = rel(got[r], ref[r])
                say(name, "row", r, "rel", e)
                assert e <= TOL, (name, r, e)
        return
    e = rel(got, ref)
    say(name, "rel", e)
    assert e <= TOL, (name, e)


@pytest.mark.parametrize("cfg", ["C2", "C4", "H8"])
def test_full_size_whole_outputs_against_oracle(cfg):
    """The benchmark's mesh sizes and launch configuration (library default
    tiling, nodes renumbered once with tlfea_node_order as the benchmark
    does): forward, adjoint (gx, gv, gtheta) and tangent over the whole
    mesh, every node and every element compared with the oracle on the same
    inputs (the oracle split over CPU worker processes by element ranges)."""
    import time

    import torch

    import _oracle_pool
    p = _full_size(cfg)
    damped = p.blocks[0].damped
    say(cfg, "elements", p.n_elem, "nodes", p.n_nodes)
    m0 = mesh_of(p)
    order = m0.node_order()
    m0.close()
    p = p.renumbered(order)
    if p.dx is None:
        p.dx = np.random.default_rng(12).standard_normal(p.X.shape) * p.cell
    if damped and p.dv is None:
        p.dv = np.random.default_rng(14).standard_normal(p.X.shape)
    m = mesh_of(p)
    x, v, w = to_dev(p.x), to_dev(p.v), to_dev(p.w)
    th = to_dev(p.theta_all())
    dx = to_dev(p.dx)
    dv = to_dev(p.dv) if damped else None
    vv = v if damped else None
    f = to_host(m.internal_force(x, vv, th))
    gx, gv, gt = (to_host(a) for a in m.vjp(x, vv, w, th))
    df = to_host(m.jvp(x, vv, dx, dv, th))
    # a smooth 2-5 % deformation inverts nothing; the whole mesh is counted
    assert int(m.count_inverted(x).item()) == 0
    torch.cuda.synchronize()
    t0 = time.time()
    ref = _oracle_pool.run(p.X, p.blocks, dict(x=p.x, v=p.v, w=p.w, dx=p.dx, dv=p.dv if damped else None),
                           ["f", "vjp", "gtheta", "jvp"])
    say(cfg, "oracle over the whole mesh in", round(time.time() - t0, 1), "s on", _oracle_pool.n_workers(), "workers")
    _check_whole(cfg + " f", f, ref["f"])
    _check_whole(cfg + " gx", gx, ref["gx"])
    if damped:
        _check_whole(cfg + " gv", gv, ref["gv"])
    else:
        assert np.all(gv == 0)
    _check_whole(cfg + " df", df, ref["df"])
    _check_whole("gtheta " + cfg, gt, ref["gtheta"])


def _sample_bodies(p, cap):
    """Bodies to check one by one: the smallest of each element type and
    law, and the largest under `cap` elements of each element type."""
    picks = set()
    sizes = [b.conn.shape[0] for b in p.blocks]
    for elem in (synth.T10, synth.H8):
        for law in (synth.SVK, synth.NH):
            cand = [i for i, b in enumerate(p.blocks) if b.elem == elem and b.law == law]
            if cand:
                picks.add(min(cand, key=lambda i: sizes[i]))
        cand = [i for i, b in enumerate(p.blocks) if b.elem == elem and sizes[i] <= cap]
        if cand:
            picks.add(max(cand, key=lambda i: sizes[i]))
    return sorted(picks)


def _body(p, bi):
    b = p.blocks[bi]
    n0, n1 = p.body_nodes[bi]
    bb = copy.copy(b)
    bb.conn = b.conn - n0
    return p.X[:, n0:n1], [bb], p.x[:, n0:n1], n0, n1


@pytest.mark.parametrize("cfg", ["C3", "C5"])
def test_full_size_multibody_whole_outputs_against_oracle(cfg):
    """The 512-body forward (batched mesh, graph replay) and the 256-body
    forward + adjoint + tangent (autotuned batched mesh captured in one
    graph), at full size as the benchmark runs them: every body's outputs
    against the oracle, body by body, and for C5 every body also bitwise
    against a plain mesh of that body alone with the tile size the
    autotuner chose."""
    import time

    import torch

    import _oracle_pool
    from paper_2602_17002_amd import AUTOTUNE, BATCHED, Mesh
    p = synth.config_c3() if cfg == "C3" else synth.config_c5()
    say("full-size multibody", cfg, len(p.blocks), "bodies", p.n_elem, "elements")
    m = mesh_of(p, flags=BATCHED | (AUTOTUNE if cfg == "C5" else 0))
    info = m.info()
    e0 = np.concatenate([[0], np.cumsum([b.conn.shape[0] for b in p.blocks])])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x = to_dev(p.x)
        f = torch.empty_like(x)
        if cfg == "C3":
            m.internal_force(x, out=f)
            m.internal_force(x, out=f)   # the graph replay
        else:
            w, dx = to_dev(p.w), to_dev(p.dx)
            gx, df = torch.empty_like(x), torch.empty_like(x)
            gt = torch.empty((5, p.n_elem), dtype=torch.float64, device="cuda")
            m.internal_force(x, out=f)
            m.vjp(x, None, w, want_v=False, out=(gx, None, gt))
            m.jvp(x, None, dx, out=df)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                m.internal_force(x, out=f)
                m.vjp(x, None, w, want_v=False, out=(gx, None, gt))
                m.jvp(x, None, dx, out=df)
            for t in (f, gx, gt, df):
                t.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
        torch.cuda.synchronize()
    f = to_host(f)
    ops = ["f"] if cfg == "C3" else ["f", "vjp", "gtheta", "jvp"]
    t0 = time.time()
    ref = _oracle_pool.run(p.X, p.blocks, dict(x=p.x, w=p.w, dx=p.dx), ops)
    say(cfg, "oracle over every body in", round(time.time() - t0, 1), "s")
    if cfg == "C5":
        gx, gt, df = to_host(gx), to_host(gt), to_host(df)
    worst = {}
    for bi in range(len(p.blocks)):
        n0, n1 = p.body_nodes[bi]
        pairs = [("f", f, ref["f"])]
        if cfg == "C5":
            pairs += [("gx", gx, ref["gx"]), ("df", df, ref["df"])]
        for k, a, b in pairs:
            e = rel(a[:, n0:n1], b[:, n0:n1])
            worst[k] = max(worst.get(k, 0.0), e)
            assert e <= TOL, (cfg, bi, k, e)
        if cfg == "C5":
            gtb, rtb = gt[:, e0[bi]:e0[bi + 1]], ref["gtheta"][:, e0[bi]:e0[bi + 1]]
            for r in range(3):
                if np.abs(rtb[r]).max() > 0:
                    e = rel(gtb[r], rtb[r])
                    worst["gtheta"] = max(worst.get("gtheta", 0.0), e)
                    assert e <= TOL, (cfg, bi, r, e)
                else:
                    assert np.all(gtb[r] == 0), (cfg, bi, r)
    say(cfg, "worst per-body rel", worst)
    if cfg == "C5":
        # a plain mesh of each of a few bodies alone, with the tile size the
        # autotuner chose for its element type, sums in the same order
        for bi in _sample_bodies(p, 12000):
            Xc, blk, xc, n0, n1 = _body(p, bi)
            bb = copy.copy(blk[0])
            bb.tile_elems = info["tile_elems_t10" if bb.elem == synth.T10 else "tile_elems_h8"]
            mb = Mesh(Xc, [bb])
            xb = to_dev(xc)
            gxb, _, gtb = mb.vjp(xb, None, to_dev(p.w[:, n0:n1]), want_v=False)
            assert np.array_equal(to_host(mb.internal_force(xb)), f[:, n0:n1]), bi
            assert np.array_equal(to_host(gxb), gx[:, n0:n1]), bi
            assert np.array_equal(to_host(gtb), gt[:, e0[bi]:e0[bi + 1]]), bi
            assert np.array_equal(to_host(mb.jvp(xb, None, to_dev(p.dx[:, n0:n1]))), df[:, n0:n1]), bi


def test_c4_finite_differences_and_adjoint_consistency():
    """The 204,000-element Neo-Hookean body with per-element (mu, lambda):
    the tangent against central differences of the GPU forward (h = 1e-6
    relative), the parameter gradient against exact differences (f is linear
    in the parameters), and w . (K dx) = gx . dx."""
    import torch
    p = synth.config_c4()
    say("C4 finite differences", p.n_elem)
    m = mesh_of(p)
    x, w, dx = to_dev(p.x), to_dev(p.w), to_dev(p.dx)
    th = to_dev(p.theta_all())
    gx, _, gt = m.vjp(x, None, w, th, want_v=False)
    kdx = m.jvp(x, None, dx, None, th)
    h = 1e-6
    fd = (m.internal_force(x + h * dx, None, th) - m.internal_force(x - h * dx, None, th)) / (2 * h)
    e_fd = float((fd - kdx).abs().max() / kdx.abs().max())
    say("C4 K.dx vs central differences", e_fd)
    assert e_fd <= 1e-7
    a, b = float((w * kdx).sum()), float((gx * dx).sum())
    say("C4 w.(K dx) vs gx.dx", abs(a - b) / abs(b))
    assert abs(a - b) <= 1e-12 * float((w.abs() * kdx.abs()).sum())
    d = torch.from_numpy(np.random.default_rng(21).standard_normal(th.shape) * 0.01).to("cuda") * th
    e1 = float((w * m.internal_force(x, None, th + d)).sum())
    e0 = float((w * m.internal_force(x, None, th - d)).sum())
    lin = float((gt * d).sum())
    say("C4 gtheta vs exact differences", abs((e1 - e0) / 2 - lin) / abs(lin))
    assert abs((e1 - e0) / 2 - lin) <= 1e-10 * abs(lin)
    torch.cuda.synchronize()


def test_one_graph_forward_adjoint_tangent_autotuned_batch():
    """Forward, adjoint and tangent of an autotuned multibody batch captured
    by the caller into one graph; every replay (with eager work between
    replays) equals the eager calls bitwise and the oracle within the bound."""
    import torch
    from paper_2602_17002_amd import AUTOTUNE, BATCHED
    p = synth.config_multibody(10, 300, 4000, seed=31, directions=True)
    say("one graph", len(p.blocks), p.n_elem)
    m = mesh_of(p, flags=BATCHED | AUTOTUNE)
    info = m.info()
    assert info["tile_elems_t10"] in (64, 128, 192, 256) and info["tile_elems_h8"] in (64, 128, 192, 256)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x, w, dx = to_dev(p.x), to_dev(p.w), to_dev(p.dx)
        f, gx, df = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
        gt = torch.empty((5, p.n_elem), dtype=torch.float64, device="cuda")
        m.internal_force(x, out=f)
        m.vjp(x, None, w, want_v=False, out=(gx, None, gt))
        m.jvp(x, None, dx, out=df)
        torch.cuda.synchronize()
        ref = [t.clone() for t in (f, gx, gt, df)]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            m.internal_force(x, out=f)
            m.vjp(x, None, w, want_v=False, out=(gx, None, gt))
            m.jvp(x, None, dx, out=df)
        for rep in range(3):
            for t in (f, gx, gt, df):
                t.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for a, b in zip((f, gx, gt, df), ref):
                assert torch.equal(a, b), rep
            # eager work between replays
            m.internal_force(x + 0.0, out=torch.empty_like(x))
            torch.cuda.synchronize()
    Xc, xc = p.X, p.x
    assert rel(to_host(f), O.internal_force(Xc, p.blocks, xc)) <= TOL
    rx, _, rt = O.vjp(Xc, p.blocks, xc, None, p.w, want_gv=False)
    assert rel(to_host(gx), rx) <= TOL
    gth = to_host(gt)
    for r in (0, 1, 2):
        if np.abs(rt[r]).max() > 0:
            assert rel(gth[r], rt[r]) <= TOL
    assert rel(to_host(df), O.jvp(Xc, p.blocks, xc, None, p.dx)) <= TOL
