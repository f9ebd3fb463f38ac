"""PyTorch-facing wrapper of a revolute-joint set (tlfea_create_joints).

A joint is a dict with keys P, Q, R, S, T, each a material point
(element type, node ids of the hosting element in its node order, parent
coordinates).  Torch supplies only device memory and the stream; the
values and the scatter run in the library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import Point, Revolute, check


def _point(pt):
    elem, nodes, xi = pt
    p = Point()
    p.elem = int(elem)
    for i, n in enumerate(nodes):
        p.nodes[i] = int(n)
    for k in range(3):
        p.xi[k] = float(xi[k])
    return p


_POINT_DTYPE = np.dtype([("elem", np.int32), ("nodes", np.int32, (27,)), ("xi", np.float64, (3,))], align=True)


class Joints:
    """Revolute joints on one GPU (Sec. 2.2); see include/tlfea.h."""

    def __init__(self, X, joints, device=None):
        arr = (Revolute * max(1, len(joints)))()
        for j, jt in enumerate(joints):
            for k in ("P", "Q", "R", "S", "T"):
                setattr(arr[j], k, _point(jt[k]))
        self._create(X, arr, len(joints), device)

    @classmethod
    def from_arrays(cls, X, elem, nodes, xi, device=None):
        """Joints from arrays: elem [n][5] element types, nodes [n][5][nen]
        hosting-element node ids, xi [n][5][3] parent coordinates (points in
        the order P, Q, R, S, T)."""
        n = int(np.asarray(elem).shape[0])
        rec = np.zeros((max(1, n), 5), dtype=_POINT_DTYPE)
        assert rec.dtype.itemsize == C.sizeof(Point)
        nodes = np.asarray(nodes)
        rec["elem"][:n] = elem
        rec["nodes"][:n, :, :nodes.shape[2]] = nodes
        rec["xi"][:n] = xi
        arr = (Revolute * max(1, n)).from_buffer(rec)
        obj = cls.__new__(cls)
        obj._keep = rec
        obj._create(X, arr, n, device)
        return obj

    def _create(self, X, arr, n_joints, device):
        L = _lib.lib()
        X = np.ascontiguousarray(X, dtype=np.float64)
        self.n_nodes = int(X.shape[1])
        self.n_joints = n_joints
        joints = arr
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            s = C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            st = L.tlfea_create_joints(self.n_nodes, X.ctypes.data_as(C.POINTER(C.c_double)), n_joints, joints, s,
                                       C.byref(h))
        check(st, "tlfea_create_joints")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().tlfea_destroy_joints(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _nodal(self, t, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if tuple(t.shape) != (3, self.n_nodes):
            raise ValueError(f"{name} must have shape (3, {self.n_nodes})")
        return t.contiguous()

    def values(self, q):
        """Row-normalised constraint values c_hat, [n_joints][5]."""
        q = self._nodal(q, "q")
        c = torch.empty((self.n_joints, 5), dtype=torch.float64, device=self.device)
        s = C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        check(_lib.lib().tlfea_joint_values(self._h, C.c_void_p(q.data_ptr()), C.c_void_p(c.data_ptr()), s),
              "tlfea_joint_values")
        return c

    def scatter(self, q, lam=None, rho=0.0, h=1.0, out=None, accumulate=False):
        """g (+)= h C_hat^T (lambda + rho c_hat) as a [3][n_nodes] tensor."""
        q = self._nodal(q, "q")
        if lam is not None:
            lam = lam.contiguous()
            if tuple(lam.shape) != (self.n_joints, 5) or lam.dtype != torch.float64:
                raise ValueError(f"lambda must be float64 of shape ({self.n_joints}, 5)")
        g = torch.empty((3, self.n_nodes), dtype=torch.float64, device=self.device) if out is None else out
        if accumulate and out is None:
            raise ValueError("accumulate needs out")
        s = C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        check(_lib.lib().tlfea_joint_scatter(self._h, C.c_void_p(q.data_ptr()),
                                             None if lam is None else C.c_void_p(lam.data_ptr()), C.c_double(rho),
                                             C.c_double(h), C.c_void_p(g.data_ptr()), int(bool(accumulate)), s),
              "tlfea_joint_scatter")
        return g
