"""Seeded sigma parity cases: library inputs (k-blocked, paper normalisation)
and the oracle's expected outputs for them."""
import numpy as np
import torch

import synth
from oracle import ccsd, layout, response


def make_case(nk, o, v, naux, nrhs, seed, tscale=0.02, band_shift=True):
    rng = synth.rng_for(500 + seed, nk, o, v)
    H = synth.hamiltonian(nk, o, v, naux, rng, band_shift=band_shift)
    t1k, t2k_cr = synth.random_amplitudes(nk, o, v, rng, tscale, tscale)
    x1k, x2k_cr = synth.random_vectors(nrhs, nk, o, v, rng, 0.1, 0.1)
    omega = np.linspace(-0.1, 0.1, nrhs) if nrhs > 1 else np.array([0.0656])
    # library inputs use the paper's per-cell normalisation: 2E quantities x Nk
    return dict(nk=nk, o=o, v=v, naux=naux, H=H, t1=t1k, t2=t2k_cr * nk, x1=x1k, x2=x2k_cr * nk,
                omega=omega)


def oracle_sigma(case):
    nk, o, v = case['nk'], case['o'], case['v']
    H = case['H']
    f = layout.dense_one_body(H['fock'], nk, o, v)
    g = layout.dense_eri(H['chol'], nk, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    t = (torch.from_numpy(layout.dense_t1(case['t1'], nk, o, v)),
         torch.from_numpy(layout.dense_t2(case['t2'] / nk, nk, o, v)))
    y1 = np.empty_like(case['x1'])
    y2 = np.empty_like(case['x2'])
    for r in range(case['x1'].shape[0]):
        x = (torch.from_numpy(layout.dense_t1(case['x1'][r], nk, o, v)),
             torch.from_numpy(layout.dense_t2(case['x2'][r] / nk, nk, o, v)))
        s1, s2 = response.sigma(t, x, h)
        w = case['omega'][r]
        y1[r] = layout.block_t1(s1.numpy(), nk, o, v) - w * case['x1'][r]
        y2[r] = nk * layout.block_t2(s2.numpy(), nk, o, v) - w * case['x2'][r]
    return y1, y2


def oracle_sigma_adjoint(case, z1, z2):
    """y = (A_p - w)^T z in the library's (per-cell) normalisation: with S = diag(1, Nk)
    the per-cell operator is A_p = S A_c S^-1, so A_p^T = S^-1 A_c^T S, A_c^T being the
    oracle's transpose product (pairing sum u1 w1 + 1/4 sum u2 w2)."""
    nk, o, v = case['nk'], case['o'], case['v']
    H = case['H']
    f = layout.dense_one_body(H['fock'], nk, o, v)
    g = layout.dense_eri(H['chol'], nk, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    t = (torch.from_numpy(layout.dense_t1(case['t1'], nk, o, v)),
         torch.from_numpy(layout.dense_t2(case['t2'] / nk, nk, o, v)))
    y1 = np.empty_like(z1)
    y2 = np.empty_like(z2)
    for r in range(z1.shape[0]):
        zc = (torch.from_numpy(layout.dense_t1(z1[r], nk, o, v)),
              torch.from_numpy(layout.dense_t2(z2[r] * nk, nk, o, v)))
        g1, g2 = response.transpose_product(t, zc, h)
        w = case['omega'][r]
        y1[r] = layout.block_t1(g1.numpy(), nk, o, v) - w * z1[r]
        y2[r] = layout.block_t2(g2.numpy(), nk, o, v) / nk - w * z2[r]
    return y1, y2


def oracle_solve(case, b1, b2, tol=1e-12):
    """Oracle solution of (A_p - w_r) x_r = b_r in the library normalisation:
    (A_c - w) S^-1 x = S^-1 b with S = diag(1, Nk)."""
    nk, o, v = case['nk'], case['o'], case['v']
    H = case['H']
    f = layout.dense_one_body(H['fock'], nk, o, v)
    g = layout.dense_eri(H['chol'], nk, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    t = (torch.from_numpy(layout.dense_t1(case['t1'], nk, o, v)),
         torch.from_numpy(layout.dense_t2(case['t2'] / nk, nk, o, v)))
    x1 = np.empty_like(b1)
    x2 = np.empty_like(b2)
    for r in range(b1.shape[0]):
        rhs = (torch.from_numpy(layout.dense_t1(b1[r], nk, o, v)),
               torch.from_numpy(layout.dense_t2(b2[r] / nk, nk, o, v)))
        sol, rel, _ = response.solve_response(t, h, rhs, case['omega'][r], tol=tol)
        x1[r] = layout.block_t1(sol[0].numpy(), nk, o, v)
        x2[r] = nk * layout.block_t2(sol[1].numpy(), nk, o, v)
    return x1, x2


def make_ccsd_case(nk, o, v, naux, seed, band_shift=True, chol_sigma=0.05):
    """Synthetic chain with converged CCSD amplitudes (oracle) and its lambda."""
    from oracle import solvers
    rng = synth.rng_for(600 + seed, nk, o, v)
    H = synth.hamiltonian(nk, o, v, naux, rng, band_shift=band_shift, chol_sigma=chol_sigma)
    f = layout.dense_one_body(H['fock'], nk, o, v)
    g = layout.dense_eri(H['chol'], nk, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    t1, t2, E, _ = solvers.solve_ccsd(h, tol=1e-12)
    return dict(nk=nk, o=o, v=v, naux=naux, H=H, h=h, t=(t1, t2), E=E,
                t1=layout.block_t1(t1.numpy(), nk, o, v), t2=nk * layout.block_t2(t2.numpy(), nk, o, v))


def oracle_alpha(case, omegas):
    nk, o, v = case['nk'], case['o'], case['v']
    lam, rel, _ = response.solve_lambda(case['t'], case['h'])
    ops = [torch.from_numpy(layout.dense_one_body(case['H']['dip'][x], nk, o, v)) for x in range(3)]
    al, _ = response.polarizability(case['t'], lam, ops, list(omegas), case['h'], nk=nk)
    return al, lam
