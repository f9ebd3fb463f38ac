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
    ``damped`` and optionally ``tile_elems``, ``rho`` (reference density),
    ``qp_w`` ([nq]) and ``dsdxi`` ([nq][nen][3]) (the quadrature table; the
    library accepts only its built-in rule).  flags: tlfea create flags.

    Every compute call enqueues on ``stream`` (default: the current stream).
    When ``stream`` is another stream, it first waits for the current
    stream (inputs and freshly allocated outputs are made there), every
    tensor handed to the library is marked as used on ``stream``, and the
    outputs are ready on ``stream``: synchronise with it before reading them
    elsewhere.
    """

    def __init__(self, X, blocks, flags=0, device=None):
        L = _lib.lib()
        X = np.ascontiguousarray(X, dtype=np.float64)
        if X.ndim != 2 or X.shape[0] != 3:
            raise ValueError("X must have shape (3, n_nodes)")
        self.n_nodes = int(X.shape[1])
        keep = []
        arr = (Block * max(1, len(blocks)))()
        self.n_elem = 0
        self.blocks = []
        for i, b in enumerate(blocks):
            conn = np.ascontiguousarray(b.conn, dtype=np.int32)
            keep.append(conn)
            arr[i].elem = int(b.elem)
            arr[i].law = int(b.law)
            arr[i].n_elem = int(conn.shape[0])
            arr[i].conn = conn.ctypes.data_as(C.POINTER(C.c_int32))
            th = np.asarray(b.theta, dtype=np.float64).reshape(-1)
            for p in range(5):
                arr[i].theta[p] = float(th[p]) if p < th.size else 0.0
            arr[i].damped = int(bool(b.damped))
            arr[i].tile_elems = int(getattr(b, "tile_elems", 0) or 0)
            arr[i].rho = float(getattr(b, "rho", 0.0) or 0.0)
            qw, dg = getattr(b, "qp_w", None), getattr(b, "dsdxi", None)
            nq = 0
            if qw is not None:
                qw = np.ascontiguousarray(qw, dtype=np.float64).reshape(-1)
                keep.append(qw)
                arr[i].qp_w = qw.ctypes.data_as(C.POINTER(C.c_double))
                nq = qw.size
            if dg is not None:
                dg = np.ascontiguousarray(dg, dtype=np.float64)
                keep.append(dg)
                arr[i].dsdxi = dg.ctypes.data_as(C.POINTER(C.c_double))
                nq = dg.shape[0]
            arr[i].nq = nq
            self.n_elem += int(conn.shape[0])
            self.blocks.append((int(b.elem), int(b.law), int(conn.shape[0]), bool(b.damped)))
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device) \
            if torch.cuda.is_available() else torch.device("cpu")
        self.damped = any(b[3] for b in self.blocks)
        h = C.c_void_p()
        if self.device.type == "cuda":
            with torch.cuda.device(self.device):
                s = C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
                st = L.tlfea_create_mesh(self.n_nodes, X.ctypes.data_as(C.POINTER(C.c_double)), len(blocks), arr,
                                         int(flags), s, C.byref(h))
        else:
            st = L.tlfea_create_mesh(self.n_nodes, X.ctypes.data_as(C.POINTER(C.c_double)), len(blocks), arr,
                                     int(flags), None, C.byref(h))
        check(st, "tlfea_create_mesh")
        self._h = h
        del keep

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

    def _empty_nodal(self):
        return torch.empty((3, self.n_nodes), dtype=torch.float64, device=self.device)

    def _call(self, fn, what, args, tensors, stream):
        """Enqueue a library call on ``stream`` (default: the current
        stream).  On another stream: wait for the current one first, and mark
        every tensor handed over as used there, so the caching allocator does
        not recycle it before the kernels are done."""
        cur = torch.cuda.current_stream(self.device)
        s = cur if stream is None else stream
        other = s.cuda_stream != cur.cuda_stream
        if other:
            s.wait_stream(cur)
        check(fn(*args, C.c_void_p(s.cuda_stream)), what)
        if other:
            for t in tensors:
                if t is not None:
                    t.record_stream(s)

    # ------------------------------------------------------------ compute
    def internal_force(self, x, v=None, theta=None, out=None, stream=None):
        """f_int(x, v) as a new (or the given) [3][n_nodes] tensor."""
        x = self._nodal(x, "x")
        v = self._nodal(v, "v", required=False)
        theta = self._theta(theta)
        f = self._empty_nodal() if out is None else self._out(out, "out", (3, self.n_nodes))
        self._call(_lib.lib().tlfea_internal_force, "tlfea_internal_force",
                   (self.handle, _ptr(x), _ptr(v), _ptr(theta), _ptr(f)), (x, v, theta, f), stream)
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
        self._call(_lib.lib().tlfea_internal_force_vjp, "tlfea_internal_force_vjp",
                   (self.handle, _ptr(x), _ptr(v), _ptr(theta), _ptr(w), _ptr(gx), _ptr(gv), _ptr(gt)),
                   (x, v, theta, w, gx, gv, gt), stream)
        return gx, gv, gt

    def count_inverted(self, x, out=None, stream=None):
        """Device int64 tensor [1]: quadrature points with det F <= 0."""
        x = self._nodal(x, "x")
        if out is None:
            out = torch.empty(1, dtype=torch.int64, device=self.device)
        out = self._out(out, "out", (1,), torch.int64)
        self._call(_lib.lib().tlfea_count_inverted, "tlfea_count_inverted", (self.handle, _ptr(x), _ptr(out)),
                   (x, out), stream)
        return out

    def jvp(self, x, v=None, dx=None, dv=None, theta=None, dtheta=None, out=None, stream=None):
        """df = (df/dx) dx + (df/dv) dv + (df/dtheta) dtheta."""
        x = self._nodal(x, "x")
        v = self._nodal(v, "v", required=False)
        dx = self._nodal(dx, "dx", required=False)
        dv = self._nodal(dv, "dv", required=False)
        theta = self._theta(theta)
        dtheta = self._theta(dtheta, "dtheta")
        df = self._empty_nodal() if out is None else self._out(out, "out", (3, self.n_nodes))
        self._call(_lib.lib().tlfea_tangent_jvp, "tlfea_tangent_jvp",
                   (self.handle, _ptr(x), _ptr(v), _ptr(theta), _ptr(dx), _ptr(dv), _ptr(dtheta), _ptr(df)),
                   (x, v, theta, dx, dv, dtheta, df), stream)
        return df

    def mass_action(self, u, out=None, stream=None):
        """y = M u, the consistent mass of the blocks' densities (Sec. 4.1)."""
        u = self._nodal(u, "u")
        y = self._empty_nodal() if out is None else self._out(out, "out", (3, self.n_nodes))
        self._call(_lib.lib().tlfea_mass_action, "tlfea_mass_action", (self.handle, _ptr(u), _ptr(y)), (u, y), stream)
        return y

    def step_residual(self, q_n, v_n, v, h, theta=None, f_ext=None, out=None, stream=None):
        """g = M (v - v_n)/h + f_int(q_n + h v, v) - f_ext (Sec. 7, no constraints)."""
        q_n, v_n, v = self._nodal(q_n, "q_n"), self._nodal(v_n, "v_n"), self._nodal(v, "v")
        f_ext = self._nodal(f_ext, "f_ext", required=False)
        theta = self._theta(theta)
        g = self._empty_nodal() if out is None else self._out(out, "out", (3, self.n_nodes))
        self._call(_lib.lib().tlfea_step_residual, "tlfea_step_residual",
                   (self.handle, _ptr(q_n), _ptr(v_n), _ptr(v), C.c_double(h), _ptr(theta), _ptr(f_ext), _ptr(g)),
                   (q_n, v_n, v, theta, f_ext, g), stream)
        return g

    def newton_operator(self, q_n, v, h, theta, dv, out=None, stream=None):
        """y = (M/h + h K + C) dv at q = q_n + h v (the residual's v-derivative)."""
        q_n, v, dv = self._nodal(q_n, "q_n"), self._nodal(v, "v"), self._nodal(dv, "dv")
        theta = self._theta(theta)
        y = self._empty_nodal() if out is None else self._out(out, "out", (3, self.n_nodes))
        self._call(_lib.lib().tlfea_newton_operator, "tlfea_newton_operator",
                   (self.handle, _ptr(q_n), _ptr(v), C.c_double(h), _ptr(theta), _ptr(dv), _ptr(y)),
                   (q_n, v, theta, dv, y), stream)
        return y

    def newton_workspace(self, restart=30):
        """Doubles of device workspace newton_step needs."""
        n = C.c_int64()
        check(_lib.lib().tlfea_newton_workspace(self.handle, int(restart), C.byref(n)), "tlfea_newton_workspace")
        return n.value

    def newton_step(self, q_n, v_n, v, h, theta=None, f_ext=None, restart=30, max_iters=300, rtol=1e-10,
                    out=None, work=None, stream=None):
        """One Newton-Krylov step of the step residual: v_out = v + dv with
        (M/h + h K + C) dv = -g(v) solved by restarted GMRES.  Returns
        (v_out, info) with info = dict(iters, converged, g_norm, res_norm).
        Synchronises the stream."""
        q_n, v_n, v = self._nodal(q_n, "q_n"), self._nodal(v_n, "v_n"), self._nodal(v, "v")
        f_ext = self._nodal(f_ext, "f_ext", required=False)
        theta = self._theta(theta)
        L = _lib.lib()
        n = C.c_int64()
        check(L.tlfea_newton_workspace(self.handle, int(restart), C.byref(n)), "tlfea_newton_workspace")
        if work is None:
            work = torch.empty(n.value, dtype=torch.float64, device=self.device)
        vo = self._empty_nodal() if out is None else self._out(out, "out", (3, self.n_nodes))
        opts = _lib.KrylovOpts(int(restart), int(max_iters), float(rtol))
        info = _lib.KrylovInfo()
        self._call(L.tlfea_newton_step, "tlfea_newton_step",
                   (self.handle, _ptr(q_n), _ptr(v_n), _ptr(v), C.c_double(h), _ptr(theta), _ptr(f_ext),
                    C.byref(opts), _ptr(vo), _ptr(work), C.c_int64(work.numel()), C.byref(info)),
                   (q_n, v_n, v, theta, f_ext, vo, work), stream)
        return vo, {k: getattr(info, k) for k, _ in _lib.KrylovInfo._fields_}

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
