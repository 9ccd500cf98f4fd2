"""Seeded synthetic inputs for the k-blocked LR-CCSD sigma path.

This module only draws random numbers and arranges them in the k-block
layouts that both the HIP library and the CPU oracle consume.  It holds
none of the method's arithmetic (no integrals, no amplitude equations).

Layouts (row-major, crystal momentum index k = 0..nk-1, k_j = 2*pi*j/nk on a 1D
chain; on a 3D mesh n0 x n1 x n2, nk = n0 n1 n2 and k is the flat index
(j0 n1 + j1) n2 + j2 of the point (j0/n0, j1/n1, j2/n2); momenta add
componentwise modulo the mesh extents):
  fock   [nk][n][n]              Hermitian per k, n = nocc + nvir, occupied first
  chol   [nk][nk][naux][n][n]    chol[k1][k2][Q][p][q] = L^Q_{p k1, q k2}, momentum
                                 transfer k2 - k1; Hermitian pairing
                                 chol[k2][k1][Q] = conj(chol[k1][k2][Q]).T
  dip    [3][nk][n][n]           Hermitian per axis per k
  t1     [nk][o][v]              t_{i k}^{a k}
  t2     [nk][nk][nk][o][o][v][v]  blocks (ki, kj, ka), kb = ki + kj - ka on the mesh,
                                 antisymmetric in (i,j) and in (a,b)

Distributions follow the workload description of the paper's test systems
re-stated for synthetic data (periodic 1D chain, Sec. II.A): orbital energies
drawn once per band, a cosine band shift, Gaussian Cholesky vectors and
Gaussian Hermitian dipole matrices.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = ["Workload", "WORKLOADS", "rng_for", "hamiltonian", "random_amplitudes", "uneven_batch",
           "random_vectors", "kb_of", "mesh_dims", "mesh_size", "omega_grid"]


@dataclasses.dataclass(frozen=True)
class Workload:
    cfg_id: int
    nk: int
    nocc: int
    nvir: int
    naux: int
    omegas: tuple          # frequencies in a.u.
    signs: tuple           # which signs of omega are solved
    band_shift: bool

    @property
    def n(self):
        return self.nocc + self.nvir

    @property
    def chol_sigma(self):
        """Standard deviation of the Cholesky entries.  0.05 for the molecular-limit
        and three-k workloads; for larger ones it is reduced so that the random
        two-electron coupling of one amplitude row, which grows like
        nvir * sqrt(naux / nk) * sigma^2, stays at the molecular-limit value
        (with 0.05 at nvir=40, naux=144 the response operator is nearly singular)."""
        if self.cfg_id <= 2:
            return 0.05
        ref = 12 * (48 / 1) ** 0.5
        return 0.05 * (ref / (self.nvir * (self.naux / self.nk) ** 0.5)) ** 0.5


WORKLOADS = {
    # molecular limit, 2 frequencies
    "c1": Workload(1, 1, 4, 12, 48, (0.0, 0.0656), (+1, -1), False),
    # 1D chain, three k points
    "c2": Workload(2, 3, 4, 20, 72, (0.0, 0.0656), (+1, -1), True),
    # batched mixed-precision workload: 3 axes x +-omega x 8 frequencies = 48 RHS
    "c3": Workload(3, 5, 8, 40, 144, tuple(0.1 * j / 7 for j in range(8)), (+1, -1), True),
    # adjoint workload and its three-k slice
    "c4": Workload(4, 7, 10, 60, 210, (0.0656,), (+1, -1), True),
    "c4s": Workload(4, 3, 10, 60, 210, (0.0656,), (+1, -1), True),
}


def rng_for(cfg_id, nk, nocc, nvir, extra=()):
    """Per-workload generator: seed = [1266, cfg_id, nk, nocc, nvir, *extra]."""
    return np.random.default_rng([1266, int(cfg_id), int(nk), int(nocc), int(nvir), *[int(e) for e in extra]])


def mesh_dims(nk):
    """(n0, n1, n2) of a k mesh given as an int (1D chain) or a tuple of extents."""
    d = (int(nk),) if np.isscalar(nk) else tuple(int(x) for x in nk)
    return d + (1,) * (3 - len(d))


def mesh_size(nk):
    n0, n1, n2 = mesh_dims(nk)
    return n0 * n1 * n2


def kb_of(ki, kj, ka, nk):
    """ki + kj - ka on the k mesh (flat indices)."""
    n0, n1, n2 = mesh_dims(nk)

    def vec(k):
        return (k // (n1 * n2), (k // n2) % n1, k % n2)
    a, b, c = vec(ki), vec(kj), vec(ka)
    j = [(a[d] + b[d] - c[d]) % n for d, n in enumerate((n0, n1, n2))]
    return (j[0] * n1 + j[1]) * n2 + j[2]


def _cnormal(rng, shape, sigma):
    return sigma * rng.standard_normal(shape) + 1j * sigma * rng.standard_normal(shape)


def hamiltonian(nk, nocc, nvir, naux, rng, band_shift=True, chol_sigma=0.05, dip_sigma=0.5):
    """Draw (fock, chol, dip, eps) for one synthetic chain (nk an int) or 3D mesh
    (nk a tuple of extents).

    fock is diagonal (canonical orbitals): occupied energies U[-1.5,-0.3],
    virtual energies U[0.2,3.0] (Hartree), drawn once per band, plus
    0.1*cos(2 pi k / nk) for every band when band_shift is set (on a mesh, the
    mean of cos(2 pi j_d / n_d) over the periodic directions d with n_d > 1).
    chol entries are complex Gaussians N(0, chol_sigma^2) per real and
    imaginary part; the k1 == k2 blocks are made Hermitian with (A + A^H)/sqrt2
    and the k1 > k2 blocks are the conjugate transposes of the k1 < k2 ones.
    dip entries are N(0, dip_sigma^2) complex Gaussians made Hermitian with
    (A + A^H)/2, independently per axis and per k.
    """
    dims = mesh_dims(nk)
    nk = mesh_size(nk)
    n = nocc + nvir
    e_occ = rng.uniform(-1.5, -0.3, size=nocc)
    e_vir = rng.uniform(0.2, 3.0, size=nvir)
    band = np.concatenate([np.sort(e_occ), np.sort(e_vir)])
    eps = np.empty((nk, n))
    per = [d for d in range(3) if dims[d] > 1]
    for k in range(nk):
        j = (k // (dims[1] * dims[2]), (k // dims[2]) % dims[1], k % dims[2])
        shift = np.mean([np.cos(2.0 * np.pi * j[d] / dims[d]) for d in per]) if per else 1.0
        eps[k] = band + (0.1 * shift if band_shift else 0.0)
    fock = np.zeros((nk, n, n), dtype=np.complex128)
    for k in range(nk):
        fock[k][np.arange(n), np.arange(n)] = eps[k]
    chol = np.zeros((nk, nk, naux, n, n), dtype=np.complex128)
    for k1 in range(nk):
        for k2 in range(k1, nk):
            a = _cnormal(rng, (naux, n, n), chol_sigma)
            if k1 == k2:
                chol[k1, k1] = (a + np.conj(np.swapaxes(a, 1, 2))) / np.sqrt(2.0)
            else:
                chol[k1, k2] = a
                chol[k2, k1] = np.conj(np.swapaxes(a, 1, 2))
    dip = np.zeros((3, nk, n, n), dtype=np.complex128)
    for x in range(3):
        for k in range(nk):
            a = _cnormal(rng, (n, n), dip_sigma)
            dip[x, k] = (a + np.conj(a.T)) / 2.0
    return dict(fock=fock, chol=chol, dip=dip, eps=eps)


def _antisym_blocks(raw, nk, mesh=None):
    """Antisymmetrize raw [nk][nk][nk][o][o][v][v] blocks over (i,j) and (a,b)
    across k-blocks: out[ki,kj,ka] = r[ki,kj,ka] - r[kj,ki,ka]^(ij) - r[ki,kj,kb]^(ab) + r[kj,ki,kb]^(ij)(ab)."""
    out = np.zeros_like(raw)
    for ki in range(nk):
        for kj in range(nk):
            for ka in range(nk):
                kb = kb_of(ki, kj, ka, nk if mesh is None else mesh)
                out[ki, kj, ka] = (raw[ki, kj, ka]
                                   - raw[kj, ki, ka].transpose(1, 0, 2, 3)
                                   - raw[ki, kj, kb].transpose(0, 1, 3, 2)
                                   + raw[kj, ki, kb].transpose(1, 0, 3, 2)) / 2.0
    return out


def random_amplitudes(nk, nocc, nvir, rng, s1=0.02, s2=0.02):
    """Random (t1, t2) with the structure of CCSD amplitudes: t2 antisymmetric
    in (i,j) and (a,b) and momentum conserving (kb implied).  nk: int or mesh."""
    mesh, nk = nk, mesh_size(nk)
    t1 = _cnormal(rng, (nk, nocc, nvir), s1)
    raw = _cnormal(rng, (nk, nk, nk, nocc, nocc, nvir, nvir), s2)
    return t1, _antisym_blocks(raw, nk, mesh)


def random_vectors(nrhs, nk, nocc, nvir, rng, s1=1.0, s2=1.0):
    """nrhs random amplitude-shaped vectors x1 [nrhs][nk][o][v], x2 [nrhs][nk][nk][nk][o][o][v][v]
    (nk: int or mesh)."""
    mesh, nk = nk, mesh_size(nk)
    x1 = np.stack([_cnormal(rng, (nk, nocc, nvir), s1) for _ in range(nrhs)])
    x2 = np.stack([_antisym_blocks(_cnormal(rng, (nk, nk, nk, nocc, nocc, nvir, nvir), s2), nk, mesh)
                   for _ in range(nrhs)])
    return x1, x2


def omega_grid(w: Workload):
    """List of (omega, sign) pairs solved for a workload."""
    return [(om, s) for om in w.omegas for s in w.signs]


def uneven_batch(max_elems_per_chain=3.0e8, nrhs=12, seed=1266, max_draws=200):
    """Twelve chains of an uneven batch: three each with Nk in {3, 5, 7, 9}, nocc drawn
    from {6..12}, nvir from {30..80}, Naux = 3 (nocc + nvir), nrhs right-hand sides
    (3 axes x 4 frequencies).  A chain whose doubles vector would exceed
    max_elems_per_chain complex elements (nrhs * Nk^3 * nocc^2 * nvir^2) is re-drawn,
    so the larger k meshes end up at the small end of the orbital ranges.  Returns a
    list of Workload records (cfg_id 5)."""
    rng = np.random.default_rng([seed, 5])
    out = []
    for nk in (3, 3, 3, 5, 5, 5, 7, 7, 7, 9, 9, 9):
        for _ in range(max_draws):
            o = int(rng.integers(6, 13))
            v = int(rng.integers(30, 81))
            if nrhs * nk ** 3 * o * o * v * v <= max_elems_per_chain:
                break
        else:
            o, v = 6, 30
        out.append(Workload(5, nk, o, v, 3 * (o + v), (0.02, 0.04, 0.0656, 0.1), (+1, -1), True))
    return out
