"""torch.autograd wrapper of the sigma map y = (A - omega) x (the perturbed-amplitude
operator of Eqs. tx1, tx2).  Forward and backward both run in the library's HIP
kernels (lrcc_apply_sigma_dev and lrcc_sigma_vjp_dev); this module only hands over
device pointers and the current stream.

Inputs and outputs are complex128 CUDA tensors in the caller layouts of the C ABI:
x1 [R][nk][nocc][nvir], x2 [R][nk][nk][nk][nocc][nocc][nvir][nvir] with antisymmetric
doubles.  Gradients follow PyTorch's complex convention and are taken within the
space of antisymmetric doubles (the incoming doubles gradient is projected on it).
omega (real, [R]) is treated as a constant."""
from __future__ import annotations

import torch

from .lrcc import FP64


class _Sigma(torch.autograd.Function):
    @staticmethod
    def forward(fctx, lctx, x1, x2, omega, precision):
        x1 = x1.contiguous()
        x2 = x2.contiguous()
        y1 = torch.empty_like(x1)
        y2 = torch.empty_like(x2)
        lctx.apply_sigma_dev(x1, x2, y1, y2, omega, precision, torch.cuda.current_stream(x1.device).cuda_stream)
        fctx.lctx = lctx
        fctx.precision = precision
        fctx.save_for_backward(omega if omega is not None else torch.empty(0))
        fctx.has_omega = omega is not None
        return y1, y2

    @staticmethod
    def backward(fctx, g1, g2):
        (omega,) = fctx.saved_tensors
        g1 = g1.contiguous()
        g2 = g2.contiguous()
        gx1 = torch.empty_like(g1)
        gx2 = torch.empty_like(g2)
        fctx.lctx.sigma_vjp_dev(g1, g2, gx1, gx2, omega if fctx.has_omega else None, fctx.precision,
                                torch.cuda.current_stream(g1.device).cuda_stream)
        return None, gx1, gx2, None, None


def sigma(lctx, x1, x2, omega=None, precision=FP64):
    """Differentiable y1, y2 = (A - omega) (x1, x2) through the library context `lctx`."""
    if omega is not None:
        omega = omega.to(device=x1.device, dtype=torch.float64).contiguous()
    return _Sigma.apply(lctx, x1, x2, omega, precision)
