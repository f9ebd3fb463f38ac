"""torch.autograd.Function around the library's forward, adjoint and tangent calls.

Reverse mode: backward(w) = (gx, gv, gtheta) from tlfea_internal_force_vjp,
with F recomputed from x inside the adjoint kernel (nothing but the inputs is
saved).  Forward mode: jvp(dx, dv, dtheta) = K dx + C dv + (df/dtheta) dtheta
from tlfea_tangent_jvp, which forms all three terms in its kernels.
"""
from __future__ import annotations

import torch


class TLInternalForce(torch.autograd.Function):
    @staticmethod
    def forward(x, v, theta, mesh):
        return mesh.internal_force(x, v, theta)

    @staticmethod
    def setup_context(ctx, inputs, output):
        x, v, theta, mesh = inputs
        ctx.mesh = mesh
        ctx.save_for_backward(x, v, theta)
        ctx.save_for_forward(x, v, theta)

    @staticmethod
    def backward(ctx, gf):
        x, v, theta = ctx.saved_tensors
        nx, nv, nt, _ = ctx.needs_input_grad
        gx, gv, gt = ctx.mesh.vjp(x, v, gf.contiguous(), theta, want_x=nx, want_v=nv and v is not None,
                                  want_theta=nt and theta is not None)
        return gx, gv, gt, None

    @staticmethod
    def jvp(ctx, dx, dv, dtheta, _dmesh):
        x, v, theta = ctx.saved_tensors
        return ctx.mesh.jvp(x, v, dx, dv, theta, dtheta=dtheta)


def internal_force(x, v, theta, mesh):
    """Differentiable f_int(x, v; theta) (theta may be None: block defaults)."""
    return TLInternalForce.apply(x, v, theta, mesh)
