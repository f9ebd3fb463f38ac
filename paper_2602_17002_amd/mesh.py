"""PyTorch-facing wrapper of a tlfea mesh.

Torch supplies only device memory (float64 CUDA/HIP tensors) and the current
stream; every step of the computation runs in the HIP kernels of libtlfea.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import Block, MeshInfo, check


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Mesh:
    """An immutable mesh on one GPU (tlfea_create_mesh).

    X: [3][n_nodes] reference nodes (host array).  blocks: objects with
    ``elem``, ``law``, ``conn`` ([n_elem][nen] int), ``theta`` ([5]),
    ``damped`` and optionally ``tile_elems``.  flags: tlfea create flags.
    """

    def __init__(self, X, blocks, flags=0, device=None):
        L = _lib.lib()
        X = np.ascontiguousarray(X, dtype=np.float64)
        if X.ndim != 2 or X.shape[0] != 3:
            raise ValueError("X must have shape (3, n_nodes)")
        self.n_nodes = int(X.shape[1])
        self._conns = []
        arr = (Block * max(1, len(blocks)))()
        self.n_elem = 0
        self.blocks = []
        for i, b in enumerate(blocks):
            conn = np.ascontiguousarray(b.conn, dtype=np.int32)
            self._conns.append(conn)
            arr[i].elem = int(b.elem)
            arr[i].law = int(b.law)
            arr[i].n_elem = int(conn.shape[0])
            arr[i].conn = conn.ctypes.data_as(C.POINTER(C.c_int32))
            th = np.asarray(b.theta, dtype=np.float64).reshape(-1)
            for p in range(5):
                arr[i].theta[p] = float(th[p]) if p < th.size else 0.0
            arr[i].damped = int(bool(b.damped))
            arr[i].tile_elems = int(getattr(b, "tile_elems", 0) or 0)
            self.n_elem += int(conn.shape[0])
            self.blocks.append((int(b.elem), int(b.law), int(conn.shape[0]), bool(b.damped)))
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device) \
            if torch.cuda.is_available() else torch.device("cpu")
        self.damped = any(b[3] for b in self.blocks)
        h = C.c_void_p()
        ctx = torch.cuda.device(self.device) if self.device.type == "cuda" else _null_ctx()
        with ctx:
            st = L.tlfea_create_mesh(self.n_nodes, X.ctypes.data_as(C.POINTER(C.c_double)), len(blocks), arr,
                                     int(flags), C.byref(h))
        check(st, "tlfea_create_mesh")
        self._h = h
        self._conns = None

    @classmethod
    def from_problem(cls, prob, flags=0, tile_elems=None):
        blocks = prob.blocks
        if tile_elems is not None:
            for b in blocks:
                b.tile_elems = tile_elems
        return cls(prob.X, blocks, flags=flags)

    # ------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().tlfea_destroy_mesh(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("mesh is closed")
        return self._h

    def info(self):
        inf = MeshInfo()
        check(_lib.lib().tlfea_get_mesh_info(self.handle, C.byref(inf)), "tlfea_get_mesh_info")
        return {k: getattr(inf, k) for k, _ in MeshInfo._fields_}

    def node_order(self):
        """tlfea_node_order: order[k] = the node that should become node k."""
        order = np.empty(self.n_nodes, dtype=np.int32)
        check(_lib.lib().tlfea_node_order(self.handle, order.ctypes.data_as(C.POINTER(C.c_int32))),
              "tlfea_node_order")
        return order

    # ------------------------------------------------------------ checks
    def _nodal(self, t, name, required=True):
        if t is None:
            if required:
                raise ValueError(f"{name} is required")
            return None
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if tuple(t.shape) != (3, self.n_nodes):
            raise ValueError(f"{name} must have shape (3, {self.n_nodes}), got {tuple(t.shape)}")
        return t.contiguous()

    def _theta(self, t, name="theta"):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if tuple(t.shape) != (5, self.n_elem):
            raise ValueError(f"{name} must have shape (5, {self.n_elem}), got {tuple(t.shape)}")
        return t.contiguous()

    def _out(self, t, name, shape, dtype=torch.float64):
        """An output buffer the library writes in place: right dtype, device,
        shape and contiguous (a copy would silently lose the result)."""
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != self.device:
            raise TypeError(f"{name} must be a {dtype} tensor on {self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _stream(self, stream):
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        return C.c_void_p(s.cuda_stream)

    def _empty_nodal(self):
        return torch.empty((3, self.n_nodes), dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------ compute
    def internal_force(self, x, v=None, theta=None, out=None, stream=None):
        """f_int(x, v) as a new (or the given) [3][n_nodes] tensor."""
        x = self._nodal(x, "x")
        v = self._nodal(v, "v", required=False)
        theta = self._theta(theta)
        f = self._empty_nodal() if out is None else self._out(out, "out", (3, self.n_nodes))
        check(_lib.lib().tlfea_internal_force(self.handle, _ptr(x), _ptr(v), _ptr(theta), _ptr(f),
                                              self._stream(stream)), "tlfea_internal_force")
        return f

    def vjp(self, x, v, w, theta=None, want_x=True, want_v=True, want_theta=True, out=None, stream=None):
        """(gx, gv, gtheta) = w^T df/dx, w^T df/dv, w^T df/dtheta (None where not wanted)."""
        x = self._nodal(x, "x")
        v = self._nodal(v, "v", required=False)
        w = self._nodal(w, "w")
        theta = self._theta(theta)
        gx = gv = gt = None
        if out is not None:
            gx, gv, gt = out
            gx = self._out(gx, "gx", (3, self.n_nodes))
            gv = self._out(gv, "gv", (3, self.n_nodes))
            gt = self._out(gt, "gtheta", (5, self.n_elem))
        if want_x and gx is None:
            gx = self._empty_nodal()
        if want_v and gv is None:
            gv = self._empty_nodal()
        if want_theta and gt is None:
            gt = torch.empty((5, self.n_elem), dtype=torch.float64, device=self.device)
        check(_lib.lib().tlfea_internal_force_vjp(self.handle, _ptr(x), _ptr(v), _ptr(theta), _ptr(w), _ptr(gx),
                                                  _ptr(gv), _ptr(gt), self._stream(stream)),
              "tlfea_internal_force_vjp")
        return gx, gv, gt

    def count_inverted(self, x, out=None, stream=None):
        """Device int64 tensor [1]: quadrature points with det F <= 0."""
        x = self._nodal(x, "x")
        if out is None:
            out = torch.empty(1, dtype=torch.int64, device=self.device)
        out = self._out(out, "out", (1,), torch.int64)
        check(_lib.lib().tlfea_count_inverted(self.handle, _ptr(x), _ptr(out), self._stream(stream)),
              "tlfea_count_inverted")
        return out

    def jvp(self, x, v=None, dx=None, dv=None, theta=None, out=None, stream=None):
        """df = (df/dx) dx + (df/dv) dv."""
        x = self._nodal(x, "x")
        v = self._nodal(v, "v", required=False)
        dx = self._nodal(dx, "dx", required=False)
        dv = self._nodal(dv, "dv", required=False)
        theta = self._theta(theta)
        df = self._empty_nodal() if out is None else self._out(out, "out", (3, self.n_nodes))
        check(_lib.lib().tlfea_tangent_jvp(self.handle, _ptr(x), _ptr(v), _ptr(theta), _ptr(dx), _ptr(dv),
                                           _ptr(df), self._stream(stream)), "tlfea_tangent_jvp")
        return df

    # ------------------------------------------------------------ timing
    def set_profiling(self, on=True):
        check(_lib.lib().tlfea_set_profiling(self.handle, int(bool(on))), "tlfea_set_profiling")

    def profile(self):
        """{kernel: (launches, total_ms)} accumulated since the last reset."""
        counts = (C.c_int32 * len(_lib.KERNEL_IDS))()
        ms = (C.c_double * len(_lib.KERNEL_IDS))()
        check(_lib.lib().tlfea_get_profile(self.handle, counts, ms), "tlfea_get_profile")
        return {k: (counts[i], ms[i]) for i, k in enumerate(_lib.KERNEL_IDS)}

    def reset_profile(self):
        check(_lib.lib().tlfea_reset_profile(self.handle), "tlfea_reset_profile")


class _null_ctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False
