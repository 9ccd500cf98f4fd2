"""Linear-response CCSD quantities on dense collective indices (oracle).

Definitions (standard LR-CC theory that Sec. II.B follows; readings listed
in the design notes):
  A            = dOmega/dT, the CCSD Jacobian.  The paper's perturbed
                 amplitude equations (Eqs. tx1, tx2) are this operator with
                 its terms grouped into pre-built intermediates.
  sigma(X)     = A X, computed as the exact 5-point central difference of the
                 residual polynomial (degree 4 in T, so the stencil has no
                 truncation error for any step).
  xi^X         = <mu| exp(-T) X exp(T) |HF>: the residual with f -> X and no
                 two-electron part (Omega is linear in (f, v); Eq. rhs is the
                 paper's explicit form of this vector).
  t^X(w)       solves (A - w) t = -xi^X (the paper's perturbed amplitudes of
                 Eqs. tx1, tx2 solve the same system with its sign conventions).
  lambda       makes L = E + <lambda, Omega> stationary in T (Eqs. l1, l2).
  eta^X . t    = directional derivative of L(T; f -> X, v -> 0) along t.
  F(x, y)      = mixed second directional derivative of L along x and y.
  alpha_XY(w)  = -1/2 C^{+-w} [eta^X t^Y(w) + eta^Y t^X(-w) + F(t^X(-w), t^Y(w))],
                 C^{+-w} g(w) = g(w) + conj(g(-w)); divided by Nk per cell
                 (the symmetric response function of Eq. lrf).
Pairing <lambda, x> = sum lambda1 x1 + 1/4 sum lambda2 x2 (x2 antisymmetric).
Amplitude vectors are tuples (x1[i,a], x2[i,j,a,b]) of torch complex128 tensors.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ccsd
from .kmesh import mesh_of
from .solvers import gmres

_C = torch.complex128


def _scale(x):
    m = max(float(x[0].abs().max()) if x[0].numel() else 0.0, float(x[1].abs().max()))
    return m if m > 0 else 1.0


def _axpy(t, s, x):
    return (t[0] + s * x[0], t[1] + s * x[1])


def sigma(t, x, h: ccsd.DenseHam, step=0.05):
    """A x by the 5-point central difference (exact for the quartic residual)."""
    hs = step / _scale(x)
    r = {}
    for s in (-2, -1, 1, 2):
        r[s] = ccsd.residual(*_axpy(t, s * hs, x), h)
    return tuple((r[-2][k] - 8 * r[-1][k] + 8 * r[1][k] - r[2][k]) / (12 * hs) for k in range(2))


def zero_v(h: ccsd.DenseHam, f):
    return ccsd.DenseHam(f=torch.as_tensor(f, dtype=_C), v=torch.zeros_like(h.v), no=h.no)


def xi(t, op, h: ccsd.DenseHam):
    """xi^X for the dense one-body operator op (N x N)."""
    return ccsd.residual(t[0], t[1], zero_v(h, op))


def antisym2(x2):
    return 0.25 * (x2 - x2.transpose(0, 1) - x2.transpose(2, 3) + x2.transpose(0, 1).transpose(2, 3))


def pack(x):
    return np.concatenate([x[0].detach().resolve_conj().numpy().ravel(), x[1].detach().resolve_conj().numpy().ravel()])


def unpack(vec, no, nv):
    n1 = no * nv
    return (torch.from_numpy(np.ascontiguousarray(vec[:n1]).reshape(no, nv)),
            torch.from_numpy(np.ascontiguousarray(vec[n1:]).reshape(no, no, nv, nv)))


def _precond(h):
    d1, d2 = ccsd.denominators(h)
    return d1, d2


def solve_response(t, h: ccsd.DenseHam, rhs, omega, tol=1e-12, x0=None):
    """Solve (A - omega) x = rhs (rhs an amplitude tuple) with right-preconditioned GMRES."""
    no, nv = h.no, h.nv
    d1, d2 = _precond(h)
    m1 = (-d1 - omega).numpy()
    m2 = (-d2 - omega).numpy()

    def apply(vec):
        x = unpack(vec, no, nv)
        s = sigma(t, x, h)
        return pack((s[0] - omega * x[0], s[1] - omega * x[1]))

    def prec(vec):
        x = unpack(vec, no, nv)
        return pack((x[0] / torch.from_numpy(m1), antisym2(x[1] / torch.from_numpy(m2))))

    sol, rel, nap = gmres(apply, pack(rhs), prec, tol=tol,
                          x0=None if x0 is None else pack(x0))
    return unpack(sol, no, nv), rel, nap


def pairing(lam, x):
    return (lam[0] * x[0]).sum() + 0.25 * (lam[1] * x[1]).sum()


def lagrangian(t, lam, h: ccsd.DenseHam):
    return ccsd.energy(t[0], t[1], h) + pairing(lam, ccsd.residual(t[0], t[1], h))


def transpose_product(t, lam, h: ccsd.DenseHam):
    """d<lam, Omega(T)>/dT, doubles part antisymmetrised and scaled by 4 so that
    for a diagonal Jacobian it reads D*lam (same scale as A)."""
    t1 = t[0].detach().clone().requires_grad_(True)
    t2 = t[1].detach().clone().requires_grad_(True)
    val = pairing(lam, ccsd.residual(t1, t2, h))
    # holomorphic scalar: torch returns conj(dval/dT)
    g1, g2 = torch.autograd.grad(val, (t1, t2), grad_outputs=torch.ones_like(val))
    return torch.conj_physical(g1), 4.0 * antisym2(torch.conj_physical(g2))


def energy_gradient(t, h: ccsd.DenseHam):
    t1 = t[0].detach().clone().requires_grad_(True)
    t2 = t[1].detach().clone().requires_grad_(True)
    val = ccsd.energy(t1, t2, h)
    g1, g2 = torch.autograd.grad(val, (t1, t2), grad_outputs=torch.ones_like(val))
    return torch.conj_physical(g1), 4.0 * antisym2(torch.conj_physical(g2))


def solve_lambda(t, h: ccsd.DenseHam, tol=1e-12):
    """Stationarity of L = E + <lam, Omega>: A^T lam = -dE/dT (Eqs. l1, l2)."""
    no, nv = h.no, h.nv
    d1, d2 = _precond(h)
    m1, m2 = (-d1).numpy(), (-d2).numpy()
    b = energy_gradient(t, h)

    def apply(vec):
        return pack(transpose_product(t, unpack(vec, no, nv), h))

    def prec(vec):
        x = unpack(vec, no, nv)
        return pack((x[0] / torch.from_numpy(m1), antisym2(x[1] / torch.from_numpy(m2))))

    sol, rel, nap = gmres(apply, -pack(b), prec, tol=tol)
    return unpack(sol, no, nv), rel, nap


def eta_dot(t, lam, op, x, h: ccsd.DenseHam, step=0.05):
    """eta^X . x: derivative of L(T; f->X, v->0) along x (5-point, exact)."""
    hx = zero_v(h, op)
    hs = step / _scale(x)
    vals = {s: lagrangian(_axpy(t, s * hs, x), lam, hx) for s in (-2, -1, 1, 2)}
    return (vals[-2] - 8 * vals[-1] + 8 * vals[1] - vals[2]) / (12 * hs)


def _second(t, lam, z, h, step):
    hs = step / _scale(z)
    vals = {s: lagrangian(_axpy(t, s * hs, z), lam, h) for s in (-2, -1, 0, 1, 2)}
    return (-vals[-2] + 16 * vals[-1] - 30 * vals[0] + 16 * vals[1] - vals[2]) / (12 * hs * hs)


def f_form(t, lam, x, y, h: ccsd.DenseHam, step=0.05):
    """F(x, y) = d2 L(T + e x + d y)/de dd, by polarisation of exact 5-point second differences.
    x and y are first brought to a common scale to keep the stencils well conditioned."""
    sx, sy = _scale(x), _scale(y)
    xs = (x[0] / sx, x[1] / sx)
    ys = (y[0] / sy, y[1] / sy)
    qp = _second(t, lam, (xs[0] + ys[0], xs[1] + ys[1]), h, step)
    qm = _second(t, lam, (xs[0] - ys[0], xs[1] - ys[1]), h, step)
    return 0.25 * (qp - qm) * sx * sy


def polarizability(t, lam, ops, omegas, h: ccsd.DenseHam, nk=1, tol=1e-12, sols=None):
    """alpha[w][X][Y] per cell for the list of one-body operators `ops` (3 axes).
    Returns (alpha, sols) where sols[(X, w, sign)] are the response amplitudes."""
    nax = len(ops)
    xis = [xi(t, op, h) for op in ops]
    if sols is None:
        sols = {}
    for X in range(nax):
        for iw, w in enumerate(omegas):
            for sgn in (+1, -1):
                key = (X, iw, sgn)
                if key in sols:
                    continue
                rhs = (-xis[X][0], -xis[X][1])
                sols[key] = solve_response(t, h, rhs, sgn * w, tol=tol)[0]
    alpha = np.zeros((len(omegas), nax, nax), dtype=np.complex128)
    for iw, w in enumerate(omegas):
        def g(X, Y, s):
            # g(X,Y, s*w) = eta^X t^Y(s w) + eta^Y t^X(-s w) + F(t^X(-s w), t^Y(s w))
            tY = sols[(Y, iw, s)]
            tX = sols[(X, iw, -s)]
            return complex(eta_dot(t, lam, ops[X], tY, h) + eta_dot(t, lam, ops[Y], tX, h)
                           + f_form(t, lam, tX, tY, h))
        for X in range(nax):
            for Y in range(nax):
                alpha[iw, X, Y] = -0.5 * (g(X, Y, +1) + np.conj(g(X, Y, -1))) / mesh_of(nk).size
    return alpha, sols


def polarizability_velocity(t, lam, moms, omegas, h: ccsd.DenseHam, nk=1, tol=1e-12):
    """Velocity-gauge polarizability from momentum operators `moms` (3 axes, dense N x N).

    With the momentum operator as the perturbation the response function gives
    <<p_X; p_Y>>_w, and alpha^VG_XY(w) = -(<<p_X; p_Y>>_w - <<p_X; p_Y>>_0) / w^2:
    the static response is subtracted in place of the diamagnetic term, which equals
    it for an exact state in a complete basis (the modified velocity gauge of the
    reference cited with the velocity gauge in Sec. V).  `polarizability` with the
    momentum operators returns a(w) = -<<p;p>>_w per cell, so alpha^VG = (a(w) - a(0)) / w^2.
    Every frequency must be non-zero.  Returns alpha[w][X][Y]."""
    if any(w == 0 for w in omegas):
        raise ValueError("the velocity-gauge polarizability is defined for non-zero frequencies")
    a, _ = polarizability(t, lam, moms, [0.0] + list(omegas), h, nk=nk, tol=tol)
    return np.stack([(a[i + 1] - a[0]) / w ** 2 for i, w in enumerate(omegas)])


def antisym_basis(no, nv):
    """Index lists of the independent amplitudes (singles, doubles i<j, a<b)."""
    singles = [(i, a) for i in range(no) for a in range(nv)]
    doubles = [(i, j, a, b) for i in range(no) for j in range(i + 1, no)
               for a in range(nv) for b in range(a + 1, nv)]
    return singles, doubles


def unit_vector(k, no, nv, singles, doubles):
    x1 = torch.zeros((no, nv), dtype=_C)
    x2 = torch.zeros((no, no, nv, nv), dtype=_C)
    if k < len(singles):
        i, a = singles[k]
        x1[i, a] = 1.0
    else:
        i, j, a, b = doubles[k - len(singles)]
        x2[i, j, a, b] = 1.0
        x2[j, i, a, b] = -1.0
        x2[i, j, b, a] = -1.0
        x2[j, i, b, a] = 1.0
    return x1, x2


def to_independent(x, singles, doubles):
    return np.array([complex(x[0][i, a]) for i, a in singles]
                    + [complex(x[1][i, j, a, b]) for i, j, a, b in doubles])


def dense_jacobian(t, h: ccsd.DenseHam):
    """Explicit A on the independent amplitudes (tiny systems only)."""
    singles, doubles = antisym_basis(h.no, h.nv)
    n = len(singles) + len(doubles)
    A = np.zeros((n, n), dtype=np.complex128)
    for k in range(n):
        A[:, k] = to_independent(sigma(t, unit_vector(k, h.no, h.nv, singles, doubles), h),
                                 singles, doubles)
    return A


def excitation_energies(t, h: ccsd.DenseHam, nk=1):
    """EOM-CCSD excitation energies: the eigenvalues of the CCSD Jacobian, i.e. the
    poles of the linear response function (Sec. II.B), on the excitations that
    conserve crystal momentum (k_i = k_a, k_i + k_j = k_a + k_b on the k mesh;
    Eq. momentum), in ascending order of their real part.  Dense: tiny systems only."""
    m = mesh_of(nk)
    no, nv = h.no, h.nv
    o, v = no // m.size, nv // m.size
    singles, doubles = antisym_basis(no, nv)
    ks = [(i, a) for (i, a) in singles if i // o == a // v]
    kd = [(i, j, a, b) for (i, j, a, b) in doubles
          if m.signed([(1, i // o), (1, j // o), (-1, a // v), (-1, b // v)]) == 0]
    n = len(ks) + len(kd)
    A = np.zeros((n, n), dtype=np.complex128)
    for k in range(n):
        A[:, k] = to_independent(sigma(t, unit_vector(k, no, nv, ks, kd), h), ks, kd)
    w = np.linalg.eigvals(A)
    return w[np.argsort(w.real, kind="stable")]
