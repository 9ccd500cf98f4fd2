"""k-block <-> dense collective-index conversions and dense integrals (oracle).

Collective index (Sec. II.A, Table index): occupied I = k*o + i for I < N_O,
virtual A = N_O + k*v + a.  One-electron arrays are k-diagonal and
two-electron arrays vanish unless k_p + k_q = k_r + k_s (Eq. momentum).

Two-electron integrals from Cholesky vectors (crystal normalisation):
  (PR|QS) = (1/Nk) sum_Q L^Q_{p kp, r kr} conj(L^Q_{s ks, q kq})  if kr-kp == kq-ks (mod Nk)
  <PQ|RS> = (PR|QS),  <PQ||RS> = <PQ|RS> - <PQ|SR>           (Sec. II.B notation)
"""
from __future__ import annotations

import numpy as np


def orbital_index(nk, o, v):
    """Dense index of every (k, p) spin orbital, occupied first."""
    n = o + v
    idx = np.empty((nk, n), dtype=np.int64)
    for k in range(nk):
        idx[k, :o] = k * o + np.arange(o)
        idx[k, o:] = nk * o + k * v + np.arange(v)
    return idx


def dense_one_body(mat, nk, o, v):
    """[nk][n][n] k-diagonal matrix -> dense (N, N)."""
    n = o + v
    N = nk * n
    idx = orbital_index(nk, o, v)
    out = np.zeros((N, N), dtype=np.complex128)
    for k in range(nk):
        out[np.ix_(idx[k], idx[k])] = mat[k]
    return out


def dense_cholesky(chol, nk, o, v):
    """Cholesky vectors as dense (Nk*naux, N, N): aux function (dk, Q) carries
    momentum transfer dk = k2 - k1."""
    naux = chol.shape[2]
    n = o + v
    N = nk * n
    idx = orbital_index(nk, o, v)
    out = np.zeros((nk * naux, N, N), dtype=np.complex128)
    for k1 in range(nk):
        for k2 in range(nk):
            dk = (k2 - k1) % nk
            out[np.ix_(np.arange(dk * naux, (dk + 1) * naux), idx[k1], idx[k2])] = chol[k1, k2]
    return out


def dense_eri(chol, nk, o, v):
    """Antisymmetrised crystal integrals <PQ||RS> as a dense (N,N,N,N) array."""
    L = dense_cholesky(chol, nk, o, v)
    # (PR|QS) = (1/Nk) sum_x L[x,P,R] conj(L[x,S,Q])
    chem = np.einsum('xpr,xsq->prqs', L, np.conj(L), optimize=True) / nk
    phys = chem.transpose(0, 2, 1, 3)          # <PQ|RS> = (PR|QS)
    return phys - phys.transpose(0, 1, 3, 2)


def dense_t1(t1, nk, o, v):
    """[nk][o][v] -> (N_O, N_V)."""
    out = np.zeros((nk * o, nk * v), dtype=np.complex128)
    for k in range(nk):
        out[k * o:(k + 1) * o, k * v:(k + 1) * v] = t1[k]
    return out


def dense_t2(t2, nk, o, v):
    """[nk][nk][nk][o][o][v][v] (kb implied) -> (N_O, N_O, N_V, N_V)."""
    out = np.zeros((nk * o, nk * o, nk * v, nk * v), dtype=np.complex128)
    for ki in range(nk):
        for kj in range(nk):
            for ka in range(nk):
                kb = (ki + kj - ka) % nk
                out[ki * o:(ki + 1) * o, kj * o:(kj + 1) * o, ka * v:(ka + 1) * v, kb * v:(kb + 1) * v] = t2[ki, kj, ka]
    return out


def block_t1(d, nk, o, v):
    return np.stack([d[k * o:(k + 1) * o, k * v:(k + 1) * v] for k in range(nk)])


def block_t2(d, nk, o, v):
    out = np.zeros((nk, nk, nk, o, o, v, v), dtype=np.complex128)
    for ki in range(nk):
        for kj in range(nk):
            for ka in range(nk):
                kb = (ki + kj - ka) % nk
                out[ki, kj, ka] = d[ki * o:(ki + 1) * o, kj * o:(kj + 1) * o, ka * v:(ka + 1) * v, kb * v:(kb + 1) * v]
    return out


def forbidden_mask_t2(nk, o, v):
    """True where a dense (N_O,N_O,N_V,N_V) element violates momentum conservation."""
    ko = np.repeat(np.arange(nk), o)
    kv = np.repeat(np.arange(nk), v)
    tot = ko[:, None, None, None] + ko[None, :, None, None] - kv[None, None, :, None] - kv[None, None, None, :]
    return (tot % nk) != 0


def to_crystal_t2(t2_paper, nk):
    """Paper normalisation (each 2E quantity carries a factor Nk) -> crystal."""
    return t2_paper / nk


def to_paper_t2(t2_crystal, nk):
    return t2_crystal * nk
