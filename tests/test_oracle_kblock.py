"""Pins of the k-blocked oracle tier: it must reproduce the dense
collective-index tier (and through it the determinant-space definitions)
on systems where both run, for the residual, the energy, the Jacobian
product and the perturbation vector."""
import numpy as np
import pytest
import torch

from oracle import ccsd, fockspace, kblock, layout, response
from tests.oracle_cases import dipoles, random_direction, tiny_system


@pytest.mark.parametrize("nk,o,v", [(1, 2, 3), (2, 2, 3), (3, 2, 2), (4, 1, 2), (5, 1, 1)])
def test_kblock_residual_energy_match_dense(nk, o, v):
    s = tiny_system(nk, o, v, tscale=0.1)
    h = kblock.KHam(s['fock'], s['H']['chol'], o)
    t1k, t2k = s['tk']
    r1, r2 = kblock.residual(h, kblock.t1_kt(t1k, nk), kblock.t2_kt(t2k, nk))
    d1, d2 = ccsd.residual(*s['t'], s['h'])
    assert np.abs(layout.dense_t1(r1.data.numpy(), nk, o, v) - d1.numpy()).max() < 1e-14
    assert np.abs(layout.dense_t2(r2.data.numpy(), nk, o, v) - d2.numpy()).max() < 1e-14
    ek = complex(kblock.energy(h, kblock.t1_kt(t1k, nk), kblock.t2_kt(t2k, nk)))
    assert abs(ek - complex(ccsd.energy(*s['t'], s['h']))) < 1e-14


def test_kblock_residual_matches_determinants_directly():
    nk, o, v = 3, 1, 2
    s = tiny_system(nk, o, v, tscale=0.1, noncanonical=0.05)
    h = kblock.KHam(s['fock'], s['H']['chol'], o)
    t1k, t2k = s['tk']
    r1, r2 = kblock.residual(h, kblock.t1_kt(t1k, nk), kblock.t2_kt(t2k, nk))
    b1, b2, _ = fockspace.brute_residual(s['f'], s['g'], nk * o, s['t'][0].numpy(), s['t'][1].numpy())
    assert np.abs(layout.dense_t1(r1.data.numpy(), nk, o, v) - b1).max() < 1e-13
    assert np.abs(layout.dense_t2(r2.data.numpy(), nk, o, v) - b2).max() < 1e-13


@pytest.mark.parametrize("nk,o,v", [(2, 2, 2), (3, 2, 3)])
def test_kblock_sigma_and_xi_match_dense(nk, o, v):
    s = tiny_system(nk, o, v, tscale=0.05)
    h = kblock.KHam(s['fock'], s['H']['chol'], o)
    rng = s['rng']
    import synth
    x1, x2 = synth.random_vectors(1, nk, o, v, rng)
    xd = (torch.from_numpy(layout.dense_t1(x1[0], nk, o, v)), torch.from_numpy(layout.dense_t2(x2[0], nk, o, v)))
    k1, k2 = kblock.sigma(h, s['tk'], (x1[0], x2[0]))
    d1, d2 = response.sigma(s['t'], xd, s['h'])
    sc = float(d2.abs().max())
    assert np.abs(layout.dense_t1(k1.numpy(), nk, o, v) - d1.numpy()).max() < 1e-12 * sc
    assert np.abs(layout.dense_t2(k2.numpy(), nk, o, v) - d2.numpy()).max() < 1e-12 * sc
    op = s['H']['dip'][1]
    q1, q2 = kblock.xi(h, s['tk'], op)
    e1, e2 = response.xi(s['t'], dipoles(s)[1], s['h'])
    assert np.abs(layout.dense_t1(q1.numpy(), nk, o, v) - e1.numpy()).max() < 1e-14
    assert np.abs(layout.dense_t2(q2.numpy(), nk, o, v) - e2.numpy()).max() < 1e-14
