"""k-blocked CCSD residual and Jacobian products (oracle, second tier).

The same spin-orbital CCSD residual as `ccsd.residual`, written with explicit
sums over crystal momenta: every tensor is stored only on its momentum-allowed
blocks (Eq. momentum: one-electron blocks with k_p = k_q, two-electron blocks
with k_p + k_q = k_r + k_s), and every contraction of the dense formula runs
over exactly the block combinations that conserve momentum in all operands,
which is the "explicit summation over k points" the paper names as the
obvious improvement of its collective-index code (Sec. V).  Crystal
normalisation, as in `ccsd`.  Tensors are torch complex128 CPU tensors so the
lambda equations can use reverse-mode derivatives as in `response`.

Storage: a four-index tensor is [k0][k1][k2][d0][d1][d2][d3] with k3 implied by
its momentum rule s0 k0 + s1 k1 + s2 k2 + s3 k3 = 0 on the k mesh (`kmesh`:
componentwise modulo the mesh extents; for a 1D chain, modulo Nk); a
two-index tensor is [k][d0][d1].
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import torch

from .kmesh import mesh_of

_C = torch.complex128


class KT:
    """Block tensor: data[k-prefix][block], `sig` the momentum signs per index."""

    def __init__(self, data, sig, nk):
        self.data = data
        self.sig = tuple(sig)
        self.mesh = mesh_of(nk)
        self.nk = self.mesh.size

    @property
    def nidx(self):
        return len(self.sig)

    def implied(self, ks):
        """k of the last index from the first nidx-1."""
        return self.mesh.signed([(-self.sig[-1] * a, b) for a, b in zip(self.sig[:-1], ks)])

    def block(self, ks):
        return self.data[tuple(ks[:-1])]

    def allowed(self, ks):
        return self.mesh.signed(list(zip(self.sig, ks))) == 0

    @staticmethod
    def zeros(nk, shape, sig):
        pre = (mesh_of(nk).size,) * (len(sig) - 1)
        return KT(torch.zeros(pre + tuple(shape), dtype=_C), sig, nk)

    def new_like(self, data):
        return KT(data, self.sig, self.mesh)

    def __add__(self, other):
        return self.new_like(self.data + other.data)

    def __sub__(self, other):
        return self.new_like(self.data - other.data)

    def __mul__(self, s):
        return self.new_like(self.data * s)

    __rmul__ = __mul__


STD4 = (1, 1, -1, -1)
DIAG2 = (1, -1)


def kein(spec, *ops, out_shape, out_sig):
    """Block einsum: sum over all momentum assignments allowed by every operand.

    spec 'lab1,lab2,...->out' as for torch.einsum; each operand a KT whose
    labels follow its index order.  Returns a new KT with signs out_sig."""
    lhs, rhs = spec.split('->')
    labs = lhs.split(',')
    nk = ops[0].nk
    out = KT.zeros(ops[0].mesh, out_shape, out_sig)
    summed = sorted(set(''.join(labs)) - set(rhs))
    blocks_out = itertools.product(range(nk), repeat=len(rhs) - 1)
    for pre in blocks_out:
        kmap = dict(zip(rhs[:-1], pre))
        kmap[rhs[-1]] = out.implied(pre)
        acc = None
        for ks in itertools.product(range(nk), repeat=len(summed)):
            kmap.update(zip(summed, ks))
            blocks = []
            ok = True
            for lab, op in zip(labs, ops):
                kk = [kmap[c] for c in lab]
                if not op.allowed(kk):
                    ok = False
                    break
                blocks.append(op.block(kk))
            if not ok:
                continue
            val = torch.einsum(spec, *blocks)
            acc = val if acc is None else acc + val
        if acc is not None:
            out.data[pre] = acc
    return out


def permute(t: KT, perm, sig=None):
    """out[idx] = t[idx permuted]: out index d is t's index perm[d]."""
    nk = t.nk
    n = t.nidx
    sig_out = tuple(t.sig[p] for p in perm) if sig is None else sig
    shape = tuple(t.data.shape[n - 1 + p] for p in perm)
    out = KT.zeros(t.mesh, shape, sig_out)
    for pre in itertools.product(range(nk), repeat=n - 1):
        ks = list(pre) + [out.implied(pre)]
        src = [None] * n
        for d, p in enumerate(perm):
            src[p] = ks[d]
        out.data[pre] = t.block(src).permute(*perm)
    return out


def p_ij(t):
    """P_(ij) on indices 0,1 of a four-index tensor."""
    return t - permute(t, (1, 0, 2, 3))


def p_ab(t):
    return t - permute(t, (0, 1, 3, 2))


class KHam:
    """k-blocked Hamiltonian in crystal normalisation, built from the inputs of
    the library boundary: fock [nk][n][n], chol [nk][nk][naux][n][n] (per-cell),
    on the k mesh `mesh` (default: a 1D chain of fock.shape[0] points)."""

    def __init__(self, fock, chol, nocc, mesh=None):
        fock = np.asarray(fock)
        chol = np.asarray(chol)
        self.mesh = mesh_of(fock.shape[0] if mesh is None else mesh)
        if self.mesh.size != fock.shape[0]:
            raise ValueError(f"{self.mesh} does not have {fock.shape[0]} points")
        self.nk = nk = fock.shape[0]
        self.n = n = fock.shape[1]
        self.no = o = nocc
        self.nv = n - o
        self.f = torch.as_tensor(fock, dtype=_C)
        self.L = torch.as_tensor(chol, dtype=_C)
        self._eri = {}

    def slice(self, c):
        return slice(0, self.no) if c == 'o' else slice(self.no, self.n)

    def ext(self, c):
        return self.no if c == 'o' else self.nv

    def fblock(self, cls):
        """One-electron block f_{pq} of orbital classes cls (k-diagonal)."""
        a, b = self.slice(cls[0]), self.slice(cls[1])
        return KT(self.f[:, a, b].clone(), DIAG2, self.mesh)

    def eri(self, cls):
        """<pq||rs> blocks for orbital classes cls (e.g. 'oovv'), crystal normalised:
        (pr|qs) = (1/Nk) sum_Q L[kp][kr][Q][p][r] conj(L[ks][kq][Q][s][q])."""
        if cls in self._eri:
            return self._eri[cls]
        nk = self.nk
        sp, sq, sr, ss = (self.slice(c) for c in cls)
        out = KT.zeros(self.mesh, tuple(self.ext(c) for c in cls), STD4)
        for kp, kq, kr in itertools.product(range(nk), repeat=3):
            ks = self.mesh.comb(kp, kq, kr)
            Lpr = self.L[kp, kr][:, sp, sr]
            Lsq = self.L[ks, kq][:, ss, sq]
            Lps = self.L[kp, ks][:, sp, ss]
            Lrq = self.L[kr, kq][:, sr, sq]
            coul = torch.einsum('xpr,xsq->pqrs', Lpr, Lsq.conj())
            exch = torch.einsum('xps,xrq->pqrs', Lps, Lrq.conj())
            out.data[kp, kq, kr] = (coul - exch) / nk
        self._eri[cls] = out
        return out

    def with_fock(self, fock):
        h = KHam.__new__(KHam)
        h.__dict__.update(self.__dict__)
        h.f = torch.as_tensor(fock, dtype=_C)
        return h

    def zero_two_body(self, fock):
        """Same sizes, one-electron part `fock`, no two-electron part."""
        h = self.with_fock(fock)
        h.L = torch.zeros_like(self.L)
        h._eri = {}
        return h


def t1_kt(t1, nk):
    return KT(torch.as_tensor(np.asarray(t1), dtype=_C) if not torch.is_tensor(t1) else t1, DIAG2, nk)


def t2_kt(t2, nk):
    return KT(torch.as_tensor(np.asarray(t2), dtype=_C) if not torch.is_tensor(t2) else t2, STD4, nk)


def _tau(t1: KT, t2: KT, c):
    """t2_ijab + c (t_ia t_jb - t_ib t_ja), k-blocked."""
    nk, o, v = t2.nk, t2.data.shape[3], t2.data.shape[5]
    pair = kein('ia,jb->ijab', t1, t1, out_shape=(o, o, v, v), out_sig=STD4)
    return t2 + c * p_ab(pair)


def residual(h: KHam, t1: KT, t2: KT):
    """Omega1 [k][i][a], Omega2 [ki][kj][ka][i][j][a][b]: the CCSD residual
    (Eqs. t1, t2 with the Stanton-Gauss intermediates, full Fock matrix)."""
    nk, o, v = h.nk, h.no, h.nv
    E = kein
    fov, foo, fvv, fvo = h.fblock('ov'), h.fblock('oo'), h.fblock('vv'), h.fblock('vo')
    oovv, ovvv, ooov, ovvo = h.eri('oovv'), h.eri('ovvv'), h.eri('ooov'), h.eri('ovvo')
    ovoo, oooo, vvvo, vvoo = h.eri('ovoo'), h.eri('oooo'), h.eri('vvvo'), h.eri('vvoo')
    vvvv, vovv, oovo, ovov = h.eri('vvvv'), h.eri('vovv'), h.eri('oovo'), h.eri('ovov')
    tt = _tau(t1, t2, 0.5)
    ta = _tau(t1, t2, 1.0)
    S2 = (o, o, v, v)

    Fae = (fvv - 0.5 * E('me,ma->ae', fov, t1, out_shape=(v, v), out_sig=DIAG2)
           + E('mf,mafe->ae', t1, ovvv, out_shape=(v, v), out_sig=DIAG2)
           - 0.5 * E('mnaf,mnef->ae', tt, oovv, out_shape=(v, v), out_sig=DIAG2))
    Fmi = (foo + 0.5 * E('ie,me->mi', t1, fov, out_shape=(o, o), out_sig=DIAG2)
           + E('ne,mnie->mi', t1, ooov, out_shape=(o, o), out_sig=DIAG2)
           + 0.5 * E('inef,mnef->mi', tt, oovv, out_shape=(o, o), out_sig=DIAG2))
    Fme = fov + E('nf,mnef->me', t1, oovv, out_shape=(o, v), out_sig=DIAG2)

    x = E('je,mnie->mnij', t1, ooov, out_shape=(o, o, o, o), out_sig=STD4)
    Wmnij = oooo + (x - permute(x, (0, 1, 3, 2))) + 0.25 * E('ijef,mnef->mnij', ta, oovv, out_shape=(o, o, o, o), out_sig=STD4)
    y = E('mb,amef->abef', t1, vovv, out_shape=(v, v, v, v), out_sig=STD4)
    Wabef = vvvv - (y - permute(y, (1, 0, 2, 3))) + 0.25 * E('mnab,mnef->abef', ta, oovv, out_shape=(v, v, v, v), out_sig=STD4)
    t1t1 = E('jf,nb->jnfb', t1, t1, out_shape=S2, out_sig=STD4)
    Wmbej = (ovvo + E('jf,mbef->mbej', t1, ovvv, out_shape=(o, v, v, o), out_sig=STD4)
             - E('nb,mnej->mbej', t1, oovo, out_shape=(o, v, v, o), out_sig=STD4)
             - E('jnfb,mnef->mbej', 0.5 * t2 + t1t1, oovv, out_shape=(o, v, v, o), out_sig=STD4))

    r1 = (permute_2(fvo)
          + E('ie,ae->ia', t1, Fae, out_shape=(o, v), out_sig=DIAG2)
          - E('ma,mi->ia', t1, Fmi, out_shape=(o, v), out_sig=DIAG2)
          + E('imae,me->ia', t2, Fme, out_shape=(o, v), out_sig=DIAG2)
          - E('nf,naif->ia', t1, ovov, out_shape=(o, v), out_sig=DIAG2)
          - 0.5 * E('imef,maef->ia', t2, ovvv, out_shape=(o, v), out_sig=DIAG2)
          - 0.5 * E('mnae,nmei->ia', t2, oovo, out_shape=(o, v), out_sig=DIAG2))

    r2 = permute(vvoo, (2, 3, 0, 1), STD4)
    Fbe_bar = Fae - 0.5 * E('mb,me->be', t1, Fme, out_shape=(v, v), out_sig=DIAG2)
    r2 = r2 + p_ab(E('ijae,be->ijab', t2, Fbe_bar, out_shape=S2, out_sig=STD4))
    Fmj_bar = Fmi + 0.5 * E('je,me->mj', t1, Fme, out_shape=(o, o), out_sig=DIAG2)
    r2 = r2 - p_ij(E('imab,mj->ijab', t2, Fmj_bar, out_shape=S2, out_sig=STD4))
    r2 = r2 + 0.5 * E('mnab,mnij->ijab', ta, Wmnij, out_shape=S2, out_sig=STD4)
    r2 = r2 + 0.5 * E('ijef,abef->ijab', ta, Wabef, out_shape=S2, out_sig=STD4)
    ring = (E('imae,mbej->ijab', t2, Wmbej, out_shape=S2, out_sig=STD4)
            - E('ie,ma,mbej->ijab', t1, t1, ovvo, out_shape=S2, out_sig=STD4))
    r2 = r2 + p_ij(p_ab(ring))
    r2 = r2 + p_ij(E('ie,abej->ijab', t1, vvvo, out_shape=S2, out_sig=STD4))
    r2 = r2 - p_ab(E('ma,mbij->ijab', t1, ovoo, out_shape=S2, out_sig=STD4))
    return r1, r2


def permute_2(t: KT):
    """Transpose of a k-diagonal two-index tensor."""
    return KT(t.data.transpose(1, 2).clone(), DIAG2, t.mesh)


def energy(h: KHam, t1: KT, t2: KT):
    """Eq. ene in crystal normalisation: sum f_ia t_ia + 1/4 sum <ij||ab> tau_ijab (whole supercell)."""
    o, v = h.no, h.nv
    oovv = h.eri('oovv')
    e1 = (h.fblock('ov').data * t1.data).sum()
    ta = _tau(t1, t2, 1.0)
    e2 = (oovv.data * ta.data).sum()
    return e1 + 0.25 * e2


def sigma(h: KHam, t, x, step=0.05):
    """A x (Jacobian of the residual) by the exact 5-point central difference.
    t = (t1 [nk][o][v], t2 [nk^3 blocks]) and x likewise, crystal normalisation."""
    nk = h.mesh
    T1, T2 = t1_kt(t[0], nk), t2_kt(t[1], nk)
    X1, X2 = t1_kt(x[0], nk), t2_kt(x[1], nk)
    sc = max(float(X1.data.abs().max()), float(X2.data.abs().max()))
    hs = step / (sc if sc > 0 else 1.0)
    r = {}
    for s in (-2, -1, 1, 2):
        r[s] = residual(h, T1 + (s * hs) * X1, T2 + (s * hs) * X2)
    out1 = (r[-2][0] - 8 * r[-1][0] + 8 * r[1][0] - r[2][0]) * (1.0 / (12 * hs))
    out2 = (r[-2][1] - 8 * r[-1][1] + 8 * r[1][1] - r[2][1]) * (1.0 / (12 * hs))
    return out1.data, out2.data


def xi(h: KHam, t, op):
    """xi^X: the residual with f -> X (per-k one-body matrices [nk][n][n]) and no two-electron part."""
    hx = h.zero_two_body(op)
    r1, r2 = residual(hx, t1_kt(t[0], h.mesh), t2_kt(t[1], h.mesh))
    return r1.data, r2.data
