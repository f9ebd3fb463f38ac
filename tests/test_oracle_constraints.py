"""Pins of the oracle's revolute joint (Sec. 2.2 CD and DP1 rows, App. B.1
row weights): point evaluation at nodes, the Jacobian against central
differences of the constraint values, zero violation under rigid motion
and under rotation about the hinge axis (the joint's one free degree of
freedom), violation under any other relative rotation, the weights of
fibers of length delta, and zero net force of the transpose scatter."""
import numpy as np
import pytest

import oracle as O
import synth


def _rot(axis, angle):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * K @ K


def _locate(X, conn, elem, target):
    """A hosting element and parent coordinates of the reference point
    `target` (Newton on the element map; the element whose corner centroid
    is nearest)."""
    nen = conn.shape[1]
    ncorner = 4 if elem == synth.T10 else 8
    cent = X[:, conn[:, :ncorner]].mean(axis=2)
    e = int(np.argmin(((cent - target[:, None]) ** 2).sum(axis=0)))
    xi = np.array([0.25, 0.25, 0.25]) if elem == synth.T10 else np.zeros(3)
    for _ in range(30):
        r = X[:, conn[e]] @ O.shape(elem, xi) - target
        J = X[:, conn[e]] @ O.dshape(elem, xi)
        xi = xi - np.linalg.solve(J, r)
    assert np.abs(X[:, conn[e]] @ O.shape(elem, xi) - target).max() < 1e-13
    return (elem, conn[e].tolist(), xi.tolist())


def two_bodies(elem_b=synth.T10, elem_c=synth.H8, delta=0.004, seed=0):
    """Body b (a T10 box) and body c (an H8 box) side by side along x,
    touching at x = 0.06; a hinge at a point of the shared face with its
    axis along z; fibers of length delta."""
    rng = np.random.default_rng(seed)
    Xb, cb = (synth.box_t10 if elem_b == synth.T10 else synth.box_h8)(3, 2, 2, size=(0.06, 0.04, 0.04))
    Xc, cc = (synth.box_t10 if elem_c == synth.T10 else synth.box_h8)(3, 2, 2, size=(0.06, 0.04, 0.04),
                                                                      origin=(0.06, 0.0, 0.0))
    X = np.concatenate([Xb, Xc], axis=1)
    cc = cc + Xb.shape[1]
    hinge = np.array([0.06, 0.02, 0.02])
    P = _locate(X, cb, elem_b, hinge)
    Q = _locate(X, cb, elem_b, hinge + np.array([-1e-3, 0, delta]))
    R = _locate(X, cc, elem_c, hinge)
    S = _locate(X, cc, elem_c, hinge + np.array([delta, 0, 0]))
    T = _locate(X, cc, elem_c, hinge + np.array([0, delta, 0]))
    joint = dict(P=P, Q=Q, R=R, S=S, T=T)
    return X, (cb, cc), joint, rng


def test_point_evaluation_at_nodes_is_the_node():
    X, conn = synth.box_t10(1, 1, 1)
    nodes = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (.5, 0, 0), (.5, .5, 0), (0, .5, 0), (0, 0, .5),
             (.5, 0, .5), (0, .5, .5)]
    for a, xi in enumerate(nodes):
        r = O.point_position(X, (synth.T10, conn[0].tolist(), xi))
        assert np.abs(r - X[:, conn[0][a]]).max() <= 1e-15


def test_jacobian_matches_central_differences():
    X, _, joint, rng = two_bodies()
    q = X + rng.normal(0, 2e-4, X.shape)
    joints = [joint, dict(joint)]
    J = O.revolute_jacobian(X, q, joints)
    for trial in range(3):
        dq = rng.normal(0, 1, X.shape)
        eps = 1e-4
        fd = (O.revolute_values(X, q + eps * dq, joints) - O.revolute_values(X, q - eps * dq, joints)) / (2 * eps)
        lin = (J @ dq.ravel()).reshape(len(joints), 5)
        # CD rows are linear and DP1 rows quadratic in q: central
        # differences are exact up to rounding
        assert np.abs(fd - lin).max() <= 1e-9 * np.abs(lin).max()


def test_reference_configuration_and_rigid_motion_satisfy_the_joint():
    X, _, joint, rng = two_bodies()
    assert np.abs(O.revolute_values(X, X, [joint])).max() <= 1e-15
    for seed in range(3):
        r = np.random.default_rng(seed)
        Rm = _rot(r.normal(size=3), r.uniform(0, np.pi))
        q = Rm @ X + r.normal(0, 1, (3, 1))
        c = O.revolute_values(X, q, [joint])
        assert np.abs(c).max() <= 1e-13, c


def test_rotation_about_the_hinge_axis_is_free_others_are_not():
    X, (cb, cc), joint, rng = two_bodies()
    nb = int(cb.max()) + 1
    hinge = O.point_position(X, joint["P"])
    axis = O.point_position(X, joint["Q"]) - hinge
    for angle in (0.3, -1.1):
        q = X.copy()
        q[:, nb:] = _rot(axis, angle) @ (X[:, nb:] - hinge[:, None]) + hinge[:, None]
        assert np.abs(O.revolute_values(X, q, [joint])).max() <= 1e-12
        # about an axis perpendicular to the hinge: the DP1 rows are violated
        q2 = X.copy()
        q2[:, nb:] = _rot([1.0, 1.0, 0.0], angle) @ (X[:, nb:] - hinge[:, None]) + hinge[:, None]
        c = O.revolute_values(X, q2, [joint])[0]
        # the normalised DP1 rows are of order delta sin(angle)
        assert np.abs(c[:3]).max() <= 1e-12 and np.abs(c[3:]).min() > 1e-4


def test_row_weights_of_fibers_of_length_delta():
    for delta in (0.002, 0.005):
        X, _, joint, _ = two_bodies(delta=delta)
        f, w = O.reference_data(X, joint)
        a0 = O.point_position(X, joint["Q"]) - O.point_position(X, joint["P"])
        b10 = O.point_position(X, joint["S"]) - O.point_position(X, joint["R"])
        assert np.allclose(w[:3], 1.0)
        assert abs(w[3] - 1.0 / np.sqrt(a0 @ a0 + b10 @ b10)) <= 1e-15 * w[3]
        # |a0| ~ |b0| ~ delta: the DP1 weights are about 1 / (delta sqrt 2)
        assert 0.5 < w[3] * delta * np.sqrt(2) < 1.5


def test_transpose_scatter_has_no_net_force():
    """Every row depends on differences of point positions, and the shape
    functions sum to one, so the scattered forces of each joint sum to zero
    (a dropped sign or a wrong point fails this)."""
    X, _, joint, rng = two_bodies()
    q = X + rng.normal(0, 5e-4, X.shape)
    lam = rng.normal(0, 1, (1, 5))
    g = O.revolute_scatter(X, q, [joint], lam, rho=1e3, h=1e-3)
    assert np.abs(g.sum(axis=1)).max() <= 1e-15 * np.abs(g).max() * g.shape[1]
    # linear in (lambda, rho c)
    g2 = O.revolute_scatter(X, q, [joint], 2 * lam, rho=2e3, h=1e-3)
    assert np.abs(g2 - 2 * g).max() <= 1e-14 * np.abs(g).max()
