"""Spin-orbital CCSD residual and energy on dense collective indices (oracle).

The paper solves Eqs. ene, t1 and t2 (Sec. II.B) with Gauss-Stanton style
intermediates (their S1-S6, which are not reproduced in the main text).  The
residual itself is unique: Omega_mu(T) = <mu| exp(-T) H exp(T) |HF> with
H = sum f_pq {p+ q} + 1/4 sum <pq||rs> {p+ q+ s r}.  It is written out here
with the standard Stanton-Gauss intermediates (F_ae, F_mi, F_me, W_mnij,
W_abef, W_mbej) for a general, non-canonical Fock matrix: the diagonal of f
is kept inside F_ae and F_mi instead of being moved into the denominators of
Eq. D, so Omega(T) = 0 is the exact CCSD condition and
t <- t + Omega / D is the Jacobi step of Sec. II.C.

Integrals are written with creators first: f_pq and <pq||rs> with p,q
created and r,s annihilated.  The singles driver is therefore f_ai and the
doubles driver <ab||ij> (the paper writes the latter as <ij||ab>*, equal
under the Hermitian integral symmetry it assumes in Sec. II.C).

All arrays are torch complex128 CPU tensors so that the transpose products
needed by the Lagrangian (lambda equations) can be taken by reverse-mode
differentiation of this same polynomial.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import torch

_C = torch.complex128


@dataclasses.dataclass
class DenseHam:
    """Dense crystal-normalised Hamiltonian on collective indices."""
    f: torch.Tensor      # (N, N), occupied block first
    v: torch.Tensor      # (N, N, N, N) antisymmetrised <pq||rs>
    no: int              # N_O

    @property
    def nv(self):
        return self.f.shape[0] - self.no

    def with_fock(self, f):
        return DenseHam(f=f, v=self.v, no=self.no)

    @staticmethod
    def from_numpy(f, v, no):
        return DenseHam(f=torch.as_tensor(np.ascontiguousarray(f), dtype=_C),
                        v=torch.as_tensor(np.ascontiguousarray(v), dtype=_C), no=no)


def _e(spec, *ops):
    return torch.einsum(spec, *ops)


def _pij(x):
    """P_(ij) x_ij.. = x_ij.. - x_ji.. on the first two indices."""
    return x - x.transpose(0, 1)


def _pab(x):
    """P_(ab) on the last two indices."""
    return x - x.transpose(2, 3)


def tau(t1, t2):
    return t2 + _e('ia,jb->ijab', t1, t1) - _e('ib,ja->ijab', t1, t1)


def tau_tilde(t1, t2):
    return t2 + 0.5 * (_e('ia,jb->ijab', t1, t1) - _e('ib,ja->ijab', t1, t1))


def residual(t1, t2, h: DenseHam):
    """Omega = (Omega1[i,a], Omega2[i,j,a,b]) for amplitudes t1[i,a], t2[i,j,a,b]."""
    no = h.no
    o, v = slice(0, no), slice(no, None)
    f, g = h.f, h.v
    fov, foo, fvv, fvo = f[o, v], f[o, o], f[v, v], f[v, o]
    oovv = g[o, o, v, v]
    ovvv = g[o, v, v, v]
    ooov = g[o, o, o, v]
    ovvo = g[o, v, v, o]
    ovoo = g[o, v, o, o]
    oooo = g[o, o, o, o]
    vvvo = g[v, v, v, o]
    vvoo = g[v, v, o, o]
    vvvv = g[v, v, v, v]
    vovv = g[v, o, v, v]
    oovo = g[o, o, v, o]
    ovov = g[o, v, o, v]

    tt = tau_tilde(t1, t2)
    ta = tau(t1, t2)

    Fae = (fvv - 0.5 * _e('me,ma->ae', fov, t1) + _e('mf,mafe->ae', t1, ovvv)
           - 0.5 * _e('mnaf,mnef->ae', tt, oovv))
    Fmi = (foo + 0.5 * _e('ie,me->mi', t1, fov) + _e('ne,mnie->mi', t1, ooov)
           + 0.5 * _e('inef,mnef->mi', tt, oovv))
    Fme = fov + _e('nf,mnef->me', t1, oovv)

    x = _e('je,mnie->mnij', t1, ooov)
    Wmnij = oooo + (x - x.transpose(2, 3)) + 0.25 * _e('ijef,mnef->mnij', ta, oovv)
    y = _e('mb,amef->abef', t1, vovv)
    Wabef = vvvv - (y - y.transpose(0, 1)) + 0.25 * _e('mnab,mnef->abef', ta, oovv)
    Wmbej = (ovvo + _e('jf,mbef->mbej', t1, ovvv) - _e('nb,mnej->mbej', t1, oovo)
             - _e('jnfb,mnef->mbej', 0.5 * t2 + _e('jf,nb->jnfb', t1, t1), oovv))

    # singles
    r1 = (fvo.T.clone()
          + _e('ie,ae->ia', t1, Fae) - _e('ma,mi->ia', t1, Fmi)
          + _e('imae,me->ia', t2, Fme)
          - _e('nf,naif->ia', t1, g[o, v, o, v])
          - 0.5 * _e('imef,maef->ia', t2, ovvv)
          - 0.5 * _e('mnae,nmei->ia', t2, oovo))

    # doubles
    r2 = vvoo.permute(2, 3, 0, 1).clone()
    Fbe_bar = Fae - 0.5 * _e('mb,me->be', t1, Fme)
    r2 = r2 + _pab(_e('ijae,be->ijab', t2, Fbe_bar))
    Fmj_bar = Fmi + 0.5 * _e('je,me->mj', t1, Fme)
    r2 = r2 - _pij(_e('imab,mj->ijab', t2, Fmj_bar))
    r2 = r2 + 0.5 * _e('mnab,mnij->ijab', ta, Wmnij)
    r2 = r2 + 0.5 * _e('ijef,abef->ijab', ta, Wabef)
    ring = _e('imae,mbej->ijab', t2, Wmbej) - _e('ie,ma,mbej->ijab', t1, t1, ovvo)
    r2 = r2 + _pij(_pab(ring))
    r2 = r2 + _pij(_e('ie,abej->ijab', t1, vvvo))
    r2 = r2 - _pab(_e('ma,mbij->ijab', t1, ovoo))
    return r1, r2


def energy(t1, t2, h: DenseHam):
    """Correlation energy (Eq. ene, crystal normalisation, whole supercell):
    E = sum f_ia t_ia + 1/4 sum <ij||ab> tau_ijab."""
    no = h.no
    o, v = slice(0, no), slice(no, None)
    oovv = h.v[o, o, v, v]
    return (_e('ia,ia->', h.f[o, v], t1) + 0.25 * _e('ijab,ijab->', oovv, t2)
            + 0.5 * _e('ijab,ia,jb->', oovv, t1, t1))


def denominators(h: DenseHam):
    """Orbital-energy differences of Eq. D from the diagonal of f."""
    d = torch.diagonal(h.f).real
    eo, ev = d[:h.no], d[h.no:]
    d1 = eo[:, None] - ev[None, :]
    d2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return d1.to(_C), d2.to(_C)
