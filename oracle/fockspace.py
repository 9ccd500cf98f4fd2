"""Determinant-space brute force for tiny systems (oracle pins).

Spin-orbitals 0..N-1 (occupied reference orbitals 0..N_O-1, the same dense
ordering as `layout`), determinants of N_O electrons stored as bit strings,
|D> = a+_{p1} a+_{p2} ... |vac> with p1 < p2 < ...  Everything is applied
matrix-free through the one-body replacement operators E_pq = a+_p a_q:
  H   = sum h_pq E_pq + 1/4 sum <pq||rs> (E_pr E_qs - delta_qr E_ps)
  T   = sum t_ia E_ai + 1/4 sum t_ijab E_ai E_bj
with h = f - sum_i <pi||qi>, so that f is the Fock matrix of the reference.
From these the CC quantities follow from their definitions:
  Omega_mu = <mu| exp(-T) H exp(T) |HF>,  E_corr = <HF|exp(-T) H exp(T)|HF> - E_HF,
  |Phi_i^a> = E_ai|HF>,  |Phi_ij^ab> = E_ai E_bj |HF>.
"""
from __future__ import annotations

import itertools
import numpy as np


class FockSpace:
    def __init__(self, nso, nel):
        self.nso, self.nel = nso, nel
        dets = []
        for occ in itertools.combinations(range(nso), nel):
            b = 0
            for p in occ:
                b |= 1 << p
            dets.append(b)
        self.dets = np.array(dets, dtype=np.int64)
        self.index = {int(d): i for i, d in enumerate(dets)}
        self.dim = len(dets)
        self.hf = self.index[(1 << nel) - 1]
        # replacement tables: tgt[p,q,D] (-1 if zero), sgn[p,q,D]
        tgt = -np.ones((nso, nso, self.dim), dtype=np.int64)
        sgn = np.zeros((nso, nso, self.dim))
        for D, bits in enumerate(dets):
            for q in range(nso):
                if not (bits >> q) & 1:
                    continue
                s1 = (-1) ** bin(bits & ((1 << q) - 1)).count('1')
                b1 = bits & ~(1 << q)
                for p in range(nso):
                    if (b1 >> p) & 1:
                        continue
                    s2 = (-1) ** bin(b1 & ((1 << p) - 1)).count('1')
                    tgt[p, q, D] = self.index[b1 | (1 << p)]
                    sgn[p, q, D] = s1 * s2
        self.tgt, self.sgn = tgt, sgn
        self.valid = tgt >= 0

    # --- primitive: all E_pq applied to one vector -> (nso, nso, dim)
    def all_E(self, psi):
        out = np.zeros((self.nso, self.nso, self.dim), dtype=np.complex128)
        p, q, D = np.nonzero(self.valid)
        out[p, q, self.tgt[p, q, D]] = self.sgn[p, q, D] * psi[D]
        return out

    def gather_E(self, Y):
        """sum_pq E_pq Y[p,q,:] -> (dim,)."""
        out = np.zeros(self.dim, dtype=np.complex128)
        p, q, D = np.nonzero(self.valid)
        np.add.at(out, self.tgt[p, q, D], self.sgn[p, q, D] * Y[p, q, D])
        return out

    def apply_one(self, h, psi):
        """sum_pq h_pq E_pq psi."""
        return self.gather_E(h[:, :, None] * psi[None, None, :])

    def apply_H(self, h, g, psi):
        W = self.all_E(psi)                                  # E_qs psi
        Y = 0.25 * np.einsum('pqrs,qsD->prD', g, W)          # 1/4 sum g_pqrs E_qs psi
        two = self.gather_E(Y)                               # sum E_pr Y_pr
        corr = 0.25 * np.einsum('pqqs->ps', g)               # delta_qr term
        return self.apply_one(h, psi) + two - self.apply_one(corr, psi)

    def apply_T(self, t1, t2, psi):
        no = t1.shape[0]
        nso = self.nso
        full1 = np.zeros((nso, nso), dtype=np.complex128)
        full1[no:, :no] = t1.T                               # coefficient of E_ai
        out = self.apply_one(full1, psi)
        W = self.all_E(psi)[no:, :no]                        # E_bj psi  [b,j,D]
        Y = 0.25 * np.einsum('ijab,bjD->aiD', t2, W)
        Yf = np.zeros((nso, nso, self.dim), dtype=np.complex128)
        Yf[no:, :no] = Y
        return out + self.gather_E(Yf)

    def exp_T(self, t1, t2, psi, sign=+1):
        term = psi.copy()
        out = psi.copy()
        for k in range(1, self.nel + 2):
            term = sign * self.apply_T(t1, t2, term) / k
            if not np.any(term):
                break
            out = out + term
        return out

    def hf_vector(self):
        e = np.zeros(self.dim, dtype=np.complex128)
        e[self.hf] = 1.0
        return e

    def project(self, chi, no, nv):
        """(<Phi_i^a|chi>, <Phi_ij^ab|chi>) with |Phi> = E_ai|HF>, E_ai E_bj|HF>."""
        hfv = self.hf_vector()
        E1 = self.all_E(hfv)                                 # E_pq |HF>
        r1 = np.zeros((no, nv), dtype=np.complex128)
        r2 = np.zeros((no, no, nv, nv), dtype=np.complex128)
        for i in range(no):
            for a in range(nv):
                r1[i, a] = np.vdot(E1[no + a, i], chi)
        for j in range(no):
            for b in range(nv):
                Eb = self.all_E(E1[no + b, j])               # E_pq E_bj |HF>
                for i in range(no):
                    for a in range(nv):
                        r2[i, j, a, b] = np.vdot(Eb[no + a, i], chi)
        return r1, r2


def core_hamiltonian(f, g, no):
    """h = f - sum_i <pi||qi> (the reference is the Hartree-Fock-like determinant of f)."""
    return f - np.einsum('piqi->pq', g[:, :no, :, :no])


def hf_energy(f, g, no):
    return np.trace(f[:no, :no]) - 0.5 * np.einsum('ijij->', g[:no, :no, :no, :no])


def cc_transformed(fs, f, g, no, t1, t2, op=None):
    """exp(-T) O exp(T) |HF> for O = H (op None) or a one-body operator op."""
    psi = fs.exp_T(t1, t2, fs.hf_vector(), +1)
    if op is None:
        h = core_hamiltonian(f, g, no)
        phi = fs.apply_H(h, g, psi)
    else:
        phi = fs.apply_one(op, psi)
    return fs.exp_T(t1, t2, phi, -1)


def brute_residual(f, g, no, t1, t2):
    nso = f.shape[0]
    fs = FockSpace(nso, no)
    chi = cc_transformed(fs, f, g, no, t1, t2)
    r1, r2 = fs.project(chi, no, nso - no)
    ecorr = chi[fs.hf] - hf_energy(f, g, no)
    return r1, r2, ecorr


def brute_xi(f, g, no, t1, t2, x):
    """xi^X_mu = <mu| exp(-T) X exp(T) |HF> for a one-body operator X."""
    nso = f.shape[0]
    fs = FockSpace(nso, no)
    chi = cc_transformed(fs, f, g, no, t1, t2, op=x)
    return fs.project(chi, no, nso - no)


def fci_polarizability(f, g, no, mux, muy, omegas):
    """Exact sum-over-states alpha_XY(omega) in the N_O-electron space:
    sum_n [<0|X|n><n|Y|0>/(w_n - w) + <0|Y|n><n|X|0>/(w_n + w)]."""
    nso = f.shape[0]
    fs = FockSpace(nso, no)
    h = core_hamiltonian(f, g, no)
    H = np.zeros((fs.dim, fs.dim), dtype=np.complex128)
    for D in range(fs.dim):
        e = np.zeros(fs.dim, dtype=np.complex128)
        e[D] = 1.0
        H[:, D] = fs.apply_H(h, g, e)
    w, U = np.linalg.eigh(H)
    X = np.zeros_like(H)
    Y = np.zeros_like(H)
    for D in range(fs.dim):
        e = np.zeros(fs.dim, dtype=np.complex128)
        e[D] = 1.0
        X[:, D] = fs.apply_one(mux, e)
        Y[:, D] = fs.apply_one(muy, e)
    Xn = U.conj().T @ X @ U
    Yn = U.conj().T @ Y @ U
    out = []
    for om in omegas:
        s = 0.0
        for n in range(1, fs.dim):
            wn = w[n] - w[0]
            s += Xn[0, n] * Yn[n, 0] / (wn - om) + Yn[0, n] * Xn[n, 0] / (wn + om)
        out.append(s)
    return np.array(out), w[0] - hf_energy(f, g, no), w[1:] - w[0]
