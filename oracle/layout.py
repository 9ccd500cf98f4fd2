"""k-block <-> dense collective-index conversions and dense integrals (oracle).

Collective index (Sec. II.A, Table index): occupied I = k*o + i for I < N_O,
virtual A = N_O + k*v + a.  One-electron arrays are k-diagonal and
two-electron arrays vanish unless k_p + k_q = k_r + k_s (Eq. momentum), the
sum taken on the k mesh (`kmesh`: a 1D chain of Nk points or a 3D mesh).

Two-electron integrals from Cholesky vectors (crystal normalisation):
  (PR|QS) = (1/Nk) sum_Q L^Q_{p kp, r kr} conj(L^Q_{s ks, q kq})  if kr-kp == kq-ks on the mesh
  <PQ|RS> = (PR|QS),  <PQ||RS> = <PQ|RS> - <PQ|SR>           (Sec. II.B notation)
"""
from __future__ import annotations

import numpy as np

from .kmesh import mesh_of


def orbital_index(nk, o, v):
    """Dense index of every (k, p) spin orbital, occupied first."""
    nk = mesh_of(nk).size
    n = o + v
    idx = np.empty((nk, n), dtype=np.int64)
    for k in range(nk):
        idx[k, :o] = k * o + np.arange(o)
        idx[k, o:] = nk * o + k * v + np.arange(v)
    return idx


def dense_one_body(mat, nk, o, v):
    """[nk][n][n] k-diagonal matrix -> dense (N, N)."""
    nk = mesh_of(nk).size
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
    m = mesh_of(nk)
    nk = m.size
    naux = chol.shape[2]
    n = o + v
    N = nk * n
    idx = orbital_index(nk, o, v)
    out = np.zeros((nk * naux, N, N), dtype=np.complex128)
    for k1 in range(nk):
        for k2 in range(nk):
            dk = m.sub(k2, k1)
            out[np.ix_(np.arange(dk * naux, (dk + 1) * naux), idx[k1], idx[k2])] = chol[k1, k2]
    return out


def dense_eri(chol, nk, o, v):
    """Antisymmetrised crystal integrals <PQ||RS> as a dense (N,N,N,N) array."""
    L = dense_cholesky(chol, nk, o, v)
    nk = mesh_of(nk).size
    # (PR|QS) = (1/Nk) sum_x L[x,P,R] conj(L[x,S,Q])
    chem = np.einsum('xpr,xsq->prqs', L, np.conj(L), optimize=True) / nk
    phys = chem.transpose(0, 2, 1, 3)          # <PQ|RS> = (PR|QS)
    return phys - phys.transpose(0, 1, 3, 2)


def dense_t1(t1, nk, o, v):
    """[nk][o][v] -> (N_O, N_V)."""
    nk = mesh_of(nk).size
    out = np.zeros((nk * o, nk * v), dtype=np.complex128)
    for k in range(nk):
        out[k * o:(k + 1) * o, k * v:(k + 1) * v] = t1[k]
    return out


def dense_t2(t2, nk, o, v):
    """[nk][nk][nk][o][o][v][v] (kb implied) -> (N_O, N_O, N_V, N_V)."""
    m = mesh_of(nk)
    nk = m.size
    out = np.zeros((nk * o, nk * o, nk * v, nk * v), dtype=np.complex128)
    for ki in range(nk):
        for kj in range(nk):
            for ka in range(nk):
                kb = m.comb(ki, kj, ka)
                out[ki * o:(ki + 1) * o, kj * o:(kj + 1) * o, ka * v:(ka + 1) * v, kb * v:(kb + 1) * v] = t2[ki, kj, ka]
    return out


def block_t1(d, nk, o, v):
    nk = mesh_of(nk).size
    return np.stack([d[k * o:(k + 1) * o, k * v:(k + 1) * v] for k in range(nk)])


def block_t2(d, nk, o, v):
    m = mesh_of(nk)
    nk = m.size
    out = np.zeros((nk, nk, nk, o, o, v, v), dtype=np.complex128)
    for ki in range(nk):
        for kj in range(nk):
            for ka in range(nk):
                kb = m.comb(ki, kj, ka)
                out[ki, kj, ka] = d[ki * o:(ki + 1) * o, kj * o:(kj + 1) * o, ka * v:(ka + 1) * v, kb * v:(kb + 1) * v]
    return out


def forbidden_mask_t2(nk, o, v):
    """True where a dense (N_O,N_O,N_V,N_V) element violates momentum conservation."""
    m = mesh_of(nk)
    bad = np.zeros((m.size * o, m.size * o, m.size * v, m.size * v), dtype=bool)
    for d in range(3):
        nd = m.dims[d]
        comp = np.array([m.vec(k)[d] for k in range(m.size)])
        ko = np.repeat(comp, o)
        kv = np.repeat(comp, v)
        tot = ko[:, None, None, None] + ko[None, :, None, None] - kv[None, None, :, None] - kv[None, None, None, :]
        bad |= (tot % nd) != 0
    return bad


def to_crystal_t2(t2_paper, nk):
    """Paper normalisation (each 2E quantity carries a factor Nk) -> crystal."""
    return t2_paper / mesh_of(nk).size


def to_paper_t2(t2_crystal, nk):
    return t2_crystal * mesh_of(nk).size
