"""torch.autograd wrappers: the sigma map y = (A - omega) x (the perturbed-amplitude
operator of Eqs. tx1, tx2), and the polarizability alpha(f, L, mu) (Eq. lrf) as a
function of the Fock matrix, the Cholesky vectors and the dipole matrices.  Forward
and backward both run in the library's HIP kernels (lrcc_apply_sigma_dev and
lrcc_sigma_vjp_dev; lrcc_solve and the three gradient entry points); this module
only hands over pointers, host arrays and the current stream.

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


def _herm_project(g):
    """Orthogonal projection (real inner product) onto Hermitian [..., n, n] blocks."""
    return 0.5 * (g + g.conj().transpose(-1, -2))


def _pair_project(g):
    """Orthogonal projection onto Cholesky arrays with the Hermitian pairing
    L[k2][k1][Q] = conj(L[k1][k2][Q])^T."""
    return 0.5 * (g + g.conj().permute(1, 0, 2, 4, 3))


class _Alpha(torch.autograd.Function):
    """alpha[j][X][Y] per cell at the frequencies `omegas` for the Hamiltonian (f, L, mu) with
    the ground-state amplitudes held at (t1, t2) (the partial derivative of the response function
    as evaluated, lambda and the response amplitudes re-solved).  backward: for a real loss l with
    dl = Re sum conj(g_alpha) d alpha, the gradient of an input h is sum_{j,X,Y} g_alpha[j,X,Y]
    conj(d alpha[j,X,Y] / d h), projected on the admissible perturbations (Hermitian f and mu,
    paired L), from lrcc_alpha_fock_gradient, lrcc_alpha_chol_gradient and
    lrcc_alpha_dipole_gradient."""

    @staticmethod
    def forward(fctx, lctx, nocc, fock, chol, dip, t1, t2, omegas, opts):
        import numpy as np
        host = lambda t: np.ascontiguousarray(t.detach().cpu().numpy())
        lctx.set_hamiltonian(nocc, host(fock), host(chol), host(dip))
        lctx.set_amplitudes(host(t1), host(t2))
        alpha, _ = lctx.solve(list(omegas), **opts)
        fctx.lctx = lctx
        fctx.opts = opts
        fctx.omegas = list(omegas)
        fctx.dev = fock.device
        return torch.from_numpy(alpha).to(fock.device)

    @staticmethod
    def backward(fctx, galpha):
        import numpy as np
        lctx, opts = fctx.lctx, fctx.opts
        ga = galpha.detach().cpu().numpy()
        gf = gl = gd = 0
        for j in range(len(fctx.omegas)):
            for x in range(3):
                for y in range(3):
                    w = ga[j, x, y]
                    if w == 0:
                        continue
                    gf = gf + w * np.conj(lctx.alpha_fock_gradient(j, x, y, **opts))
                    gl = gl + w * np.conj(lctx.alpha_chol_gradient(j, x, y, **opts))
                    gd = gd + w * np.conj(lctx.alpha_dipole_gradient(j, x, y, **opts))
        dev = fctx.dev
        out = []
        for g, proj in ((gf, _herm_project), (gl, _pair_project), (gd, _herm_project)):
            out.append(None if np.isscalar(g) else proj(torch.from_numpy(g)).to(dev))
        return None, None, out[0], out[1], out[2], None, None, None, None


def alpha(lctx, nocc, fock, chol, dip, t1, t2, omegas, **opts):
    """Differentiable alpha[j][X][Y] (complex128) of the Hamiltonian (fock [nk][n][n], chol
    [nk][nk][naux][n][n], dip [3][nk][n][n], complex128 tensors) at fixed amplitudes (t1, t2,
    caller layouts, per-cell normalisation) through the library context `lctx`; opts are solver
    options (tol, precision, ...).  Gradients flow to fock, chol and dip."""
    return _Alpha.apply(lctx, nocc, fock, chol, dip, t1, t2, tuple(omegas), opts)
