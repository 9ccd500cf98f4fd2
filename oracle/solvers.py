"""Iterative solvers of the oracle.

* CCSD ground state: the Jacobi update of Sec. II.C (amplitude += residual /
  orbital-energy denominator, Eq. D) accelerated by DIIS on the amplitude
  change, with a Hermitian error matrix (the paper's complex-number remark in
  Sec. II.C).  Converged far below the paper's thresholds, to max|Omega| <= tol.
* Linear systems M x = b with a diagonal preconditioner: restarted GMRES with
  modified Gram-Schmidt, used for the response and lambda equations.
Vectors are flat complex numpy arrays.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ccsd


def _flat(a, b):
    return np.concatenate([np.asarray(a).ravel(), np.asarray(b).ravel()])


def solve_ccsd(h: ccsd.DenseHam, tol=1e-12, max_iter=400, ndiis=8, t_init=None, verbose=False):
    """Returns (t1, t2, E, n_iter) as torch tensors / complex."""
    no, nv = h.no, h.nv
    d1, d2 = ccsd.denominators(h)
    if t_init is None:
        t1 = torch.zeros((no, nv), dtype=torch.complex128)
        t2 = torch.zeros((no, no, nv, nv), dtype=torch.complex128)
    else:
        t1, t2 = (x.clone() for x in t_init)
    hist_t, hist_e = [], []
    n1 = no * nv
    for it in range(1, max_iter + 1):
        r1, r2 = ccsd.residual(t1, t2, h)
        rmax = max(float(r1.abs().max()) if r1.numel() else 0.0, float(r2.abs().max()))
        if verbose:
            print(f"ccsd it {it} max|Omega| {rmax:.3e}")
        if rmax <= tol:
            return t1, t2, complex(ccsd.energy(t1, t2, h)), it
        n1_ = t1 + r1 / d1
        n2_ = t2 + r2 / d2
        err = _flat((n1_ - t1).numpy(), (n2_ - t2).numpy())
        hist_t.append(_flat(n1_.numpy(), n2_.numpy()))
        hist_e.append(err)
        if len(hist_t) > ndiis:
            hist_t.pop(0)
            hist_e.pop(0)
        if len(hist_t) >= 2:
            m = len(hist_t)
            B = np.zeros((m + 1, m + 1), dtype=np.complex128)
            for a in range(m):
                for b in range(m):
                    B[a, b] = np.vdot(hist_e[a], hist_e[b])
            B[m, :m] = -1
            B[:m, m] = -1
            rhs = np.zeros(m + 1, dtype=np.complex128)
            rhs[m] = -1
            c = np.linalg.lstsq(B, rhs, rcond=None)[0][:m]
            vec = sum(ci * ti for ci, ti in zip(c, hist_t))
        else:
            vec = hist_t[-1]
        t1 = torch.from_numpy(vec[:n1].reshape(no, nv).copy())
        t2 = torch.from_numpy(vec[n1:].reshape(no, no, nv, nv).copy())
    raise RuntimeError(f"CCSD not converged in {max_iter} iterations (max|Omega| = {rmax:.3e})")


def gmres(apply, b, precond, tol=1e-12, restart=60, max_restarts=40, x0=None):
    """Solve apply(x) = b.  `precond(r)` approximates the inverse (right
    preconditioning).  Stops when ||b - apply(x)|| <= tol * ||b||.
    Returns (x, relative residual, number of operator applications)."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0.0, 0
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    napply = 0
    for _ in range(max_restarts):
        r = b - apply(x)
        napply += 1
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            return x, beta / bnorm, napply
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        k_used = 0
        for k in range(restart):
            z = precond(V[k])
            Z.append(z)
            w = apply(z)
            napply += 1
            for j in range(k + 1):
                H[j, k] = np.vdot(V[j], w)
                w = w - H[j, k] * V[j]
            H[k + 1, k] = np.linalg.norm(w)
            k_used = k + 1
            y, *_ = np.linalg.lstsq(H[:k + 2, :k + 1], g[:k + 2], rcond=None)
            res = np.linalg.norm(g[:k + 2] - H[:k + 2, :k + 1] @ y)
            if res <= 0.1 * tol * bnorm or H[k + 1, k] == 0:
                break
            V.append(w / H[k + 1, k])
        y, *_ = np.linalg.lstsq(H[:k_used + 1, :k_used], g[:k_used + 1], rcond=None)
        for j in range(k_used):
            x = x + y[j] * Z[j]
    r = b - apply(x)
    rel = np.linalg.norm(r) / bnorm
    if rel > tol:
        raise RuntimeError(f"GMRES not converged: relative residual {rel:.3e}")
    return x, rel, napply
