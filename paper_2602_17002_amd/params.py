"""Material parameters in the library's [5][n_elem] layout, as differentiable
torch ops (so that autograd chains the library's parameter gradients to the
engineering constants a caller optimises).

Neo-Hookean in the paper's form (Sec. 3.2.2, Mooney-Rivlin with mu01 = 0):
mu10 = mu / 2 and k = lambda + 2 mu / 3, the pair whose small-strain shear
and bulk moduli equal the Lame pair (mu, lambda).  Saint Venant-Kirchhoff
(Sec. 3.2.1) takes (lambda, mu) directly.
"""
from __future__ import annotations

import torch


def nh_theta_from_lame(mu, lam, mu_v=None, lam_v=None):
    """[5][n] parameter rows (mu10, 0, k, mu_v, lambda_v) from per-element
    Lame pairs (1-D tensors of one length); Kelvin-Voigt rows default to 0."""
    zero = torch.zeros_like(mu)
    return torch.stack([0.5 * mu, zero, lam + (2.0 / 3.0) * mu,
                        zero if mu_v is None else mu_v, zero if lam_v is None else lam_v])


def svk_theta_from_lame(mu, lam, mu_v=None, lam_v=None):
    """[5][n] parameter rows (lambda, mu, 0, mu_v, lambda_v)."""
    zero = torch.zeros_like(mu)
    return torch.stack([lam, mu, zero, zero if mu_v is None else mu_v, zero if lam_v is None else lam_v])
