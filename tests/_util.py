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
