"""Shared helpers of the test suite."""
import copy

import numpy as np

TOL = 1e-12   # norm-wise relative error bound of GPU results against the oracle


def rel(a, b):
    """max |a - b| / max |b| (norm-wise; per-DOF relative error is meaningless
    at interior nodes where element contributions cancel)."""
    a = np.asarray(a); b = np.asarray(b)
    den = np.abs(b).max() if b.size else 0.0
    if den == 0.0:
        return float(np.abs(a).max()) if a.size else 0.0
    return float(np.abs(a - b).max() / den)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()


def sub_blocks(prob, nodes):
    """Blocks restricted to the elements incident to ``nodes`` (so the oracle
    can evaluate assembled values at exactly those nodes), plus the column
    indices of those elements in the concatenated element order."""
    out, cols, base = [], [], 0
    mask = np.zeros(prob.n_nodes, dtype=bool)
    mask[nodes] = True
    for b in prob.blocks:
        sel = np.nonzero(mask[b.conn].any(axis=1))[0]
        nb = copy.copy(b)
        nb.conn = np.ascontiguousarray(b.conn[sel])
        if b.theta_e is not None:
            nb.theta_e = np.ascontiguousarray(b.theta_e[:, sel])
        out.append(nb)
        cols.append(base + sel)
        base += b.n_elem
    return out, np.concatenate(cols)


def patch(prob, node, arrays=("x", "v", "w", "dx", "dv")):
    """The elements incident to ``node`` as a small stand-alone problem with
    local node numbering (the same coordinates, copied): everything the
    oracle needs to evaluate assembled values at that node.  Returns
    (X, blocks, {name: array}, local index of node, element columns)."""
    sub, cols = sub_blocks(prob, [node])
    used = np.unique(np.concatenate([b.conn.ravel() for b in sub if b.n_elem] + [np.array([node])]))
    loc = np.full(prob.n_nodes, -1, dtype=np.int64)
    loc[used] = np.arange(used.size)
    out = []
    for b in sub:
        nb = copy.copy(b)
        nb.conn = np.ascontiguousarray(loc[b.conn].astype(np.int32))
        out.append(nb)
    X = prob.X[:, used]
    vals = {}
    for name in arrays:
        a = getattr(prob, name, None)
        if a is not None:
            vals[name] = np.ascontiguousarray(a[:, used])
    return np.ascontiguousarray(X), out, vals, int(loc[node]), cols


def sample_nodes(prob, n_random, n_surface, seed):
    """Random nodes plus random nodes on the boundary of the bounding box
    (where the assembled forces are largest)."""
    rng = np.random.default_rng(seed)
    X = prob.X
    lo, hi = X.min(axis=1, keepdims=True), X.max(axis=1, keepdims=True)
    on_surface = np.nonzero(np.any(np.isclose(X, lo) | np.isclose(X, hi), axis=0))[0]
    a = rng.choice(prob.n_nodes, n_random, replace=False)
    b = rng.choice(on_surface, min(n_surface, on_surface.size), replace=False)
    return np.unique(np.concatenate([a, b]))
