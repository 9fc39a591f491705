"""torch.autograd.Function over the fine operator: y = H(U) psi with
H = Gamma5 D_dwf (Sec. 3), differentiable in psi and in the gauge links.

The backward pass runs two library kernels and nothing else:
  * grad_psi = H grad_y, since H is Hermitian (hdcr_apply_fine);
  * grad_U = dL/dRe U + i dL/dIm U of L = Re <grad_y, H psi>, the gauge-link
    gradient of the fermion force kernel (hdcr_fermion_force).
Both follow torch's convention for complex tensors: for a real loss, the
gradient of z is dLoss/dRe z + i dLoss/dIm z, so a first-order change of the
loss is Re sum conj(grad_z) dz.  For a real loss the su(3) force along
U -> exp(eps X) U is fermion_force(...)[1].
"""
from __future__ import annotations

import torch

from . import Lattice, apply_fine, fermion_force


class ApplyH(torch.autograd.Function):
    """y = H(U) psi on device tensors (gauge [V4, 4, 3, 3], fermion [12, V4, Ls])."""

    @staticmethod
    def forward(ctx, U, psi, lat: Lattice):
        U = U.contiguous()
        psi = psi.contiguous()
        ctx.lat = lat
        ctx.save_for_backward(U, psi)
        return apply_fine(lat, U, psi)

    @staticmethod
    def backward(ctx, grad_y):
        U, psi = ctx.saved_tensors
        g = grad_y.contiguous()
        grad_U = grad_psi = None
        if ctx.needs_input_grad[1]:
            grad_psi = apply_fine(ctx.lat, U, g)
        if ctx.needs_input_grad[0]:
            grad_U, _ = fermion_force(ctx.lat, U, g, psi, want_t=False)
        return grad_U, grad_psi, None


def apply_h(lat: Lattice, U, psi):
    """Differentiable y = H(U) psi."""
    return ApplyH.apply(U, psi, lat)
