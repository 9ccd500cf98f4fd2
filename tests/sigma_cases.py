"""Seeded sigma parity cases: library inputs (k-blocked, paper normalisation)
and the oracle's expected outputs for them."""
import numpy as np
import torch

import synth
from oracle import ccsd, layout, response

# Bound on the max-norm relative error of a complex64 sigma (matrix-core products in fp32,
# inputs and outputs complex128) against the complex128 oracle.  The error is set by fp32
# rounding of the products and sums: about 1e-7 at the small sizes and 3e-7 at the batched
# Nk=5, o=8, v=40 workload; 1e-5 leaves a factor of about 30, far below what any defect
# confined to the complex64 path (a wrong term, a dropped block) would produce.
FP32_REL = 1e-5


def _rng(base, nk, o, v, mesh):
    """Per-case generator; a 3D mesh adds its extents to the seed."""
    if mesh is None:
        return synth.rng_for(base, nk, o, v)
    return synth.rng_for(base, nk, o, v, extra=synth.mesh_dims(mesh))


def _noncanonical(H, nk, o, v, seed, scale):
    """Add a Hermitian k-diagonal part with off-diagonal (occupied-virtual, occupied-occupied,
    virtual-virtual) elements to the Fock matrix: complex Gaussian N(0, scale^2) entries made
    Hermitian with (A + A^H)/2, drawn from a generator of their own so that the other inputs of
    a case do not change."""
    if not scale:
        return H
    rng = synth.rng_for(4000 + seed, nk, o, v)
    n = o + v
    H = dict(H)
    H['fock'] = H['fock'].copy()
    for k in range(nk):
        a = scale * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        H['fock'][k] += (a + a.conj().T) / 2
    return H


def make_case(nk, o, v, naux, nrhs, seed, tscale=0.02, band_shift=True, mesh=None, noncanonical=0.0):
    """mesh: None (1D chain of nk points) or k-mesh extents whose product is nk; noncanonical:
    scale of a Hermitian off-diagonal part added to the Fock matrix (0: diagonal f)."""
    km = nk if mesh is None else tuple(mesh)
    assert synth.mesh_size(km) == nk
    rng = _rng(500 + seed, nk, o, v, mesh)
    H = synth.hamiltonian(km, o, v, naux, rng, band_shift=band_shift)
    H = _noncanonical(H, nk, o, v, seed, noncanonical)
    t1k, t2k_cr = synth.random_amplitudes(km, o, v, rng, tscale, tscale)
    x1k, x2k_cr = synth.random_vectors(nrhs, km, o, v, rng, 0.1, 0.1)
    omega = np.linspace(-0.1, 0.1, nrhs) if nrhs > 1 else np.array([0.0656])
    # library inputs use the paper's per-cell normalisation: 2E quantities x Nk
    return dict(nk=nk, km=km, o=o, v=v, naux=naux, H=H, t1=t1k, t2=t2k_cr * nk, x1=x1k, x2=x2k_cr * nk,
                omega=omega)


def oracle_sigma(case):
    nk, o, v = case['nk'], case['o'], case['v']
    km = case.get('km', nk)
    H = case['H']
    f = layout.dense_one_body(H['fock'], km, o, v)
    g = layout.dense_eri(H['chol'], km, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    t = (torch.from_numpy(layout.dense_t1(case['t1'], km, o, v)),
         torch.from_numpy(layout.dense_t2(case['t2'] / nk, km, o, v)))
    y1 = np.empty_like(case['x1'])
    y2 = np.empty_like(case['x2'])
    for r in range(case['x1'].shape[0]):
        x = (torch.from_numpy(layout.dense_t1(case['x1'][r], km, o, v)),
             torch.from_numpy(layout.dense_t2(case['x2'][r] / nk, km, o, v)))
        s1, s2 = response.sigma(t, x, h)
        w = case['omega'][r]
        y1[r] = layout.block_t1(s1.numpy(), km, o, v) - w * case['x1'][r]
        y2[r] = nk * layout.block_t2(s2.numpy(), km, o, v) - w * case['x2'][r]
    return y1, y2


def oracle_sigma_adjoint(case, z1, z2):
    """y = (A_p - w)^T z in the library's (per-cell) normalisation: with S = diag(1, Nk)
    the per-cell operator is A_p = S A_c S^-1, so A_p^T = S^-1 A_c^T S, A_c^T being the
    oracle's transpose product (pairing sum u1 w1 + 1/4 sum u2 w2)."""
    nk, o, v = case['nk'], case['o'], case['v']
    km = case.get('km', nk)
    H = case['H']
    f = layout.dense_one_body(H['fock'], km, o, v)
    g = layout.dense_eri(H['chol'], km, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    t = (torch.from_numpy(layout.dense_t1(case['t1'], km, o, v)),
         torch.from_numpy(layout.dense_t2(case['t2'] / nk, km, o, v)))
    y1 = np.empty_like(z1)
    y2 = np.empty_like(z2)
    for r in range(z1.shape[0]):
        zc = (torch.from_numpy(layout.dense_t1(z1[r], km, o, v)),
              torch.from_numpy(layout.dense_t2(z2[r] * nk, km, o, v)))
        g1, g2 = response.transpose_product(t, zc, h)
        w = case['omega'][r]
        y1[r] = layout.block_t1(g1.numpy(), km, o, v) - w * z1[r]
        y2[r] = layout.block_t2(g2.numpy(), km, o, v) / nk - w * z2[r]
    return y1, y2


def oracle_solve(case, b1, b2, tol=1e-12):
    """Oracle solution of (A_p - w_r) x_r = b_r in the library normalisation:
    (A_c - w) S^-1 x = S^-1 b with S = diag(1, Nk)."""
    nk, o, v = case['nk'], case['o'], case['v']
    km = case.get('km', nk)
    H = case['H']
    f = layout.dense_one_body(H['fock'], km, o, v)
    g = layout.dense_eri(H['chol'], km, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    t = (torch.from_numpy(layout.dense_t1(case['t1'], km, o, v)),
         torch.from_numpy(layout.dense_t2(case['t2'] / nk, km, o, v)))
    x1 = np.empty_like(b1)
    x2 = np.empty_like(b2)
    for r in range(b1.shape[0]):
        rhs = (torch.from_numpy(layout.dense_t1(b1[r], km, o, v)),
               torch.from_numpy(layout.dense_t2(b2[r] / nk, km, o, v)))
        sol, rel, _ = response.solve_response(t, h, rhs, case['omega'][r], tol=tol)
        x1[r] = layout.block_t1(sol[0].numpy(), km, o, v)
        x2[r] = nk * layout.block_t2(sol[1].numpy(), km, o, v)
    return x1, x2


def make_ccsd_case(nk, o, v, naux, seed, band_shift=True, chol_sigma=0.05, mesh=None, noncanonical=0.0):
    """Synthetic chain (or 3D k mesh) with converged CCSD amplitudes (oracle) and its lambda;
    noncanonical as for make_case."""
    from oracle import solvers
    km = nk if mesh is None else tuple(mesh)
    assert synth.mesh_size(km) == nk
    rng = _rng(600 + seed, nk, o, v, mesh)
    H = synth.hamiltonian(km, o, v, naux, rng, band_shift=band_shift, chol_sigma=chol_sigma)
    H = _noncanonical(H, nk, o, v, 100 + seed, noncanonical)
    f = layout.dense_one_body(H['fock'], km, o, v)
    g = layout.dense_eri(H['chol'], km, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    t1, t2, E, _ = solvers.solve_ccsd(h, tol=1e-12)
    return dict(nk=nk, km=km, o=o, v=v, naux=naux, H=H, h=h, t=(t1, t2), E=E,
                t1=layout.block_t1(t1.numpy(), km, o, v), t2=nk * layout.block_t2(t2.numpy(), km, o, v))


def oracle_alpha(case, omegas, ops=None, velocity=False):
    """Oracle alpha[w][X][Y] per cell for the dipoles of the case, or for the one-body
    operators `ops` ([3][nk][n][n] k-blocked); velocity=True: the velocity-gauge form
    with `ops` the momentum matrices."""
    nk, o, v = case['nk'], case['o'], case['v']
    km = case.get('km', nk)
    lam, rel, _ = response.solve_lambda(case['t'], case['h'])
    src = case['H']['dip'] if ops is None else ops
    dense = [torch.from_numpy(layout.dense_one_body(src[x], km, o, v)) for x in range(3)]
    if velocity:
        return response.polarizability_velocity(case['t'], lam, dense, list(omegas), case['h'], nk=km), lam
    al, _ = response.polarizability(case['t'], lam, dense, list(omegas), case['h'], nk=km)
    return al, lam
