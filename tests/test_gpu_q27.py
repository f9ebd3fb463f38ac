"""GPU parity of the 27-node hexahedron (App. A, Q27, 3x3x3 Gauss) through
the C ABI: every operation against the oracle on the same seeded inputs
(norm-wise relative error <= 1e-12 per output array), the exact count of
inverted points, a mesh mixing Q27 with T10 and H8 bodies (batched graph
bitwise equal to per-body plain meshes), and a 131,072-element body in the
launch configuration the benchmark times (whole outputs against the oracle
over the whole mesh)."""
import copy

import numpy as np
import pytest

import oracle as O
import synth
from _util import TOL, rel, to_dev, to_host
from test_gpu_parity import LAWS, make_problem, mesh_of, oc, say

pytestmark = pytest.mark.gpu

CASES = [(l, d) for l in ("SVK", "NH", "MR") for d in (False, True)]


def _id(c):
    return f"Q27-{c[0]}-{'KV' if c[1] else 'el'}"


def q27_problem(law, damped, n=(5, 4, 3), seed=0, curved=True, per_elem=False):
    return make_problem(synth.Q27, law, damped, n=n, seed=seed, curved=curved, per_elem=per_elem)


@pytest.mark.parametrize("case", CASES, ids=_id)
@pytest.mark.parametrize("tile", [64, 128])
def test_q27_forward_matches_oracle(case, tile):
    law, damped = case
    p = q27_problem(law, damped, seed=10 + tile)
    say("q27 forward", p.name, "tile", tile, "elements", p.n_elem)
    m = mesh_of(p, tile=tile)
    f = to_host(m.internal_force(to_dev(p.x), to_dev(p.v) if damped else None))
    ref = O.internal_force(*oc(p), p.v)
    assert rel(f, ref) <= TOL, rel(f, ref)


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_q27_vjp_matches_oracle(case):
    law, damped = case
    p = q27_problem(law, damped, n=(4, 3, 3), seed=20, per_elem=True)
    say("q27 vjp", p.name)
    m = mesh_of(p)
    th = p.theta_all()
    for want_theta in (False, True):
        gx, gv, gt = m.vjp(to_dev(p.x), to_dev(p.v) if damped else None, to_dev(p.w), to_dev(th),
                           want_theta=want_theta)
        rx, rv, rt = O.vjp(*oc(p), p.v, p.w)
        assert rel(to_host(gx), rx) <= TOL, rel(to_host(gx), rx)
        if damped:
            assert rel(to_host(gv), rv) <= TOL
        else:
            assert np.all(to_host(gv) == 0)
        if want_theta:
            gt = to_host(gt)
            for r in range(5):
                if np.abs(rt[r]).max() == 0:
                    assert np.all(gt[r] == 0), r
                else:
                    assert rel(gt[r], rt[r]) <= TOL, (r, rel(gt[r], rt[r]))


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_q27_jvp_matches_oracle(case):
    law, damped = case
    p = q27_problem(law, damped, n=(4, 3, 3), seed=30, per_elem=True)
    say("q27 jvp", p.name)
    m = mesh_of(p)
    th = p.theta_all()
    dv = p.dv if damped else None
    df = to_host(m.jvp(to_dev(p.x), to_dev(p.v) if damped else None, to_dev(p.dx),
                       None if dv is None else to_dev(dv), to_dev(th)))
    ref = O.jvp(*oc(p), p.v, p.dx, dv)
    assert rel(df, ref) <= TOL, rel(df, ref)
    # the parameter direction: the stress is linear in theta, so the tangent
    # in dtheta alone is the force at theta = dtheta
    dth = p.theta_all() * np.random.default_rng(31).uniform(-1, 1, th.shape)
    dfth = to_host(m.jvp(to_dev(p.x), to_dev(p.v) if damped else None, None, None, to_dev(th),
                         dtheta=to_dev(dth)))
    q = copy.copy(p)
    q.blocks = [copy.copy(b) for b in p.blocks]
    q.blocks[0].theta_e = dth
    assert rel(dfth, O.internal_force(q.X, q.blocks, q.x, q.v)) <= TOL


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_q27_reflected_state(case):
    """Every point inverted (the mirror image of the state, det F near -1):
    forward, adjoint with and without the parameter gradients, and tangent
    against the oracle."""
    law, damped = case
    p = q27_problem(law, damped, n=(3, 3, 2), seed=50, per_elem=True)
    p.x = p.x * np.array([[1.0], [-1.0], [1.0]])
    ninv, min_det = O.count_inverted(p.X, p.blocks, p.x)
    assert ninv == p.n_qp and min_det > 0.2, (ninv, min_det)
    say("q27 reflected", p.name, "min |det F|", min_det)
    m = mesh_of(p)
    th = to_dev(p.theta_all())
    xd, vd = to_dev(p.x), (to_dev(p.v) if damped else None)
    assert rel(to_host(m.internal_force(xd, vd, th)), O.internal_force(*oc(p), p.v)) <= TOL
    rx, rv, rt = O.vjp(*oc(p), p.v, p.w)
    for want_theta in (False, True):
        gx, gv, gt = m.vjp(xd, vd, to_dev(p.w), th, want_theta=want_theta)
        assert rel(to_host(gx), rx) <= TOL
        if damped:
            assert rel(to_host(gv), rv) <= TOL
        if want_theta:
            gt = to_host(gt)
            for r in range(5):
                if np.abs(rt[r]).max() > 0:
                    assert rel(gt[r], rt[r]) <= TOL, r
    dv = p.dv if damped else None
    df = to_host(m.jvp(xd, vd, to_dev(p.dx), None if dv is None else to_dev(dv), th))
    assert rel(df, O.jvp(*oc(p), p.v, p.dx, dv)) <= TOL


@pytest.mark.parametrize("damped", [False, True], ids=["el", "KV"])
def test_q27_mass_step_and_newton_operator_match_oracle(damped):
    p = q27_problem("NH", damped, n=(4, 4, 3), seed=40, per_elem=True)
    for b in p.blocks:
        b.rho = 1250.0
    say("q27 mass / step", p.name)
    m = mesh_of(p)
    rng = np.random.default_rng(41)
    u = rng.normal(0, 1, p.X.shape)
    assert rel(to_host(m.mass_action(to_dev(u))), O.mass_action(p.X, p.blocks, u)) <= TOL
    h = 1e-4
    q_n, v_n = p.x, rng.normal(0, 0.3, p.X.shape)
    v = v_n + rng.normal(0, 0.3, p.X.shape)
    f_ext = rng.normal(0, 10.0, p.X.shape)
    dv = rng.normal(0, 1.0, p.X.shape)
    th = to_dev(p.theta_all())
    g = to_host(m.step_residual(to_dev(q_n), to_dev(v_n), to_dev(v), h, th, to_dev(f_ext)))
    assert rel(g, O.step_residual(p.X, p.blocks, q_n, v_n, v, h, f_ext)) <= TOL
    y = to_host(m.newton_operator(to_dev(q_n), to_dev(v), h, th, to_dev(dv)))
    assert rel(y, O.newton_operator(p.X, p.blocks, q_n, v, h, dv)) <= TOL


def test_q27_count_inverted_matches_oracle():
    """Exact count of points with det F <= 0 on a tangled Q27 box (a seed
    whose smallest |det F| is far from rounding), and the reference,
    reflected and collapsed states."""
    X, conn = synth.box_q27(4, 3, 2, size=(0.4, 0.3, 0.2))
    b = synth.Block(synth.Q27, synth.SVK, conn, LAWS["SVK"][1], damped=False)
    x = X + np.random.default_rng(2).normal(0, 0.03, X.shape)
    from paper_2602_17002_amd import Mesh
    n_qp = conn.shape[0] * 27
    for tile in (64, 128):
        bb = copy.copy(b)
        bb.tile_elems = tile
        m = Mesh(X, [bb])
        ref, mn = O.count_inverted(X, [bb], x)
        say("q27 inverted", tile, ref, mn)
        assert 0 < ref < n_qp and mn > 1e-4
        assert int(m.count_inverted(to_dev(x)).item()) == ref
        assert int(m.count_inverted(to_dev(X)).item()) == 0
        assert int(m.count_inverted(to_dev(X * np.array([[1.0], [-1.0], [1.0]]))).item()) == n_qp
        assert int(m.count_inverted(to_dev(np.zeros_like(X))).item()) == n_qp


def _mixed_problem(seed):
    """Three bodies side by side: Q27 (Neo-Hookean, damped), T10 (SVK) and
    H8 (Mooney-Rivlin, damped)."""
    parts = [q27_problem("NH", True, n=(4, 3, 3), seed=seed),
             make_problem(synth.T10, "SVK", False, n=(5, 4, 3), seed=seed + 1, curved=True),
             make_problem(synth.H8, "MR", True, n=(6, 4, 3), seed=seed + 2, curved=True)]
    X, x, v, w, dx, blocks, off = [], [], [], [], [], [], 0
    for q in parts:
        X.append(q.X + np.array([[off * 0.3], [0.0], [0.0]]))
        x.append(q.x + np.array([[off * 0.3], [0.0], [0.0]]))
        v.append(q.v); w.append(q.w); dx.append(q.dx)
        b = copy.copy(q.blocks[0])
        b.conn = q.blocks[0].conn + sum(a.shape[1] for a in X[:-1])
        blocks.append(b)
        off += 1
    p = synth.Problem("mixed Q27/T10/H8", np.concatenate(X, 1), np.concatenate(x, 1), np.concatenate(v, 1),
                      blocks, cell=0.02)
    p.w, p.dx = np.concatenate(w, 1), np.concatenate(dx, 1)
    return p


def test_q27_in_a_batched_mixed_mesh():
    """Q27, T10 and H8 bodies in one batched mesh (one graph per call): forward,
    adjoint and tangent against the oracle, and bitwise equal to the plain
    mesh of the same bodies."""
    from paper_2602_17002_amd import BATCHED
    p = _mixed_problem(50)
    say("q27 mixed", p.n_elem)
    mb, mp = mesh_of(p, flags=BATCHED), mesh_of(p)
    x, v, w, dx = to_dev(p.x), to_dev(p.v), to_dev(p.w), to_dev(p.dx)
    outs = []
    for m in (mb, mp):
        f = to_host(m.internal_force(x, v))
        gx, gv, _ = m.vjp(x, v, w, want_theta=False)
        df = to_host(m.jvp(x, v, dx, None))
        outs.append((f, to_host(gx), to_host(gv), df))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    f, gx, gv, df = outs[0]
    assert rel(f, O.internal_force(*oc(p), p.v)) <= TOL
    rx, rv, _ = O.vjp(*oc(p), p.v, p.w, want_gtheta=False)
    assert rel(gx, rx) <= TOL and rel(gv, rv) <= TOL
    assert rel(df, O.jvp(*oc(p), p.v, p.dx)) <= TOL


def test_q27_full_size_body_whole_outputs_against_oracle():
    """The 131,072-element Q27 body (64 x 64 x 32 cells, 1,081,665 nodes,
    3,538,944 points) in the benchmark's launch configuration (nodes
    renumbered once with tlfea_node_order, default tiles): forward, adjoint
    (gx, gv) and tangent over the whole mesh against the oracle over the
    whole mesh (CPU worker processes by element ranges)."""
    import time
    import _oracle_pool
    p = synth.config_q27()
    m0 = mesh_of(p)
    order = m0.node_order()
    m0.close()
    p = p.renumbered(order)
    say("q27 full size", p.n_elem, "elements", p.n_nodes, "nodes")
    m = mesh_of(p)
    x, v, w, dx, dv = to_dev(p.x), to_dev(p.v), to_dev(p.w), to_dev(p.dx), to_dev(p.dv)
    f = to_host(m.internal_force(x, v))
    gx, gv, _ = m.vjp(x, v, w, want_theta=False)
    gx, gv = to_host(gx), to_host(gv)
    df = to_host(m.jvp(x, v, dx, dv))
    assert int(m.count_inverted(x).item()) == 0
    t0 = time.time()
    ref = _oracle_pool.run(p.X, p.blocks, dict(x=p.x, v=p.v, w=p.w, dx=p.dx, dv=p.dv), ["f", "vjp", "jvp"])
    say("q27 oracle over the whole mesh in", round(time.time() - t0, 1), "s on", _oracle_pool.n_workers(), "workers")
    for name, got, want in (("f", f, ref["f"]), ("gx", gx, ref["gx"]), ("gv", gv, ref["gv"]), ("df", df, ref["df"])):
        e = rel(got, want)
        say("q27", name, "rel", e)
        assert e <= TOL, (name, e)


def test_q27_single_element_and_rigid_motion():
    """One curved Q27 element: every operation against the oracle; under a
    rigid rotation and translation of the reference the force is zero to
    rounding."""
    p = q27_problem("MR", True, n=(1, 1, 1), seed=70, per_elem=True)
    m = mesh_of(p)
    x, v, w, dx = to_dev(p.x), to_dev(p.v), to_dev(p.w), to_dev(p.dx)
    th = p.theta_all()
    assert rel(to_host(m.internal_force(x, v, to_dev(th))), O.internal_force(*oc(p), p.v)) <= TOL
    gx, gv, gt = m.vjp(x, v, w, to_dev(th))
    rx, rv, rt = O.vjp(*oc(p), p.v, p.w)
    assert rel(to_host(gx), rx) <= TOL and rel(to_host(gv), rv) <= TOL
    assert rel(to_host(m.jvp(x, v, dx, None, to_dev(th))), O.jvp(*oc(p), p.v, p.dx)) <= TOL
    R = synth.random_rotation(np.random.default_rng(71))
    xr = R @ p.X + np.array([[0.3], [-0.2], [0.1]])
    f = to_host(m.internal_force(to_dev(xr), to_dev(np.zeros_like(p.X)), to_dev(th)))
    scale = np.abs(to_host(m.internal_force(x, v, to_dev(th)))).max()
    assert np.abs(f).max() <= 1e-12 * scale
