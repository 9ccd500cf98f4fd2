"""Gradient of the polarizability with respect to the dipole matrices.  At fixed
ground-state amplitudes and lambda, alpha_XY is bilinear in (mu_X, mu_Y), so the
central difference of the oracle's alpha along any dipole perturbation is exact up
to rounding and solver tolerance; the library's adjoint gradient must reproduce it."""
import numpy as np
import pytest
import torch

import synth
from tests.sigma_cases import make_ccsd_case

pytestmark = pytest.mark.gpu

OMEGAS = [0.0, 0.0656]


def _oracle_alpha_dip(case, lam, dip):
    from oracle import layout, response
    nk, o, v = case['nk'], case['o'], case['v']
    ops = [torch.from_numpy(layout.dense_one_body(dip[x], nk, o, v)) for x in range(3)]
    al, _ = response.polarizability(case['t'], lam, ops, OMEGAS, case['h'], nk=nk)
    return al


@pytest.mark.parametrize("x,y", [(2, 2), (0, 1)])
@pytest.mark.parametrize("nk,o,v,naux,seed", [(1, 2, 4, 6, 21), (2, 2, 3, 6, 22), (3, 1, 3, 5, 23)])
def test_alpha_dipole_gradient_matches_oracle(nk, o, v, naux, seed, x, y):
    import paper_2508_01266_amd as lr
    from oracle import response
    print(f"case nk={nk} o={o} v={v} naux={naux} alpha_{x}{y}", flush=True)
    case = make_ccsd_case(nk, o, v, naux, seed)
    H = case['H']
    # Hermitian dipole perturbations of all three axes (drawn like the dipoles)
    V = synth.hamiltonian(nk, o, v, naux, synth.rng_for(700 + seed, nk, o, v))['dip']
    lam, _, _ = response.solve_lambda(case['t'], case['h'])
    hstep = 0.5
    ap = _oracle_alpha_dip(case, lam, H['dip'] + hstep * V)
    am = _oracle_alpha_dip(case, lam, H['dip'] - hstep * V)
    ref = (ap - am)[:, x, y] / (2 * hstep)

    c = lr.Context(0)
    c.set_hamiltonian(o, H['fock'], H['chol'], H['dip'])
    c.set_amplitudes(case['t1'], case['t2'])
    c.solve(OMEGAS, tol=1e-12, precision=lr.FP64)
    for j in range(len(OMEGAS)):
        g = c.alpha_dipole_gradient(j, x, y, tol=1e-12, precision=lr.FP64)
        for z in range(3):
            if z not in (x, y):
                assert np.abs(g[z]).max() == 0.0
        got = np.sum(g * V)
        err = abs(got - ref[j])
        print(f"omega {OMEGAS[j]}: d alpha {got:.10f} oracle {ref[j]:.10f} err {err:.2e}", flush=True)
        assert err < 1e-8 * max(1.0, abs(ref[j]))
    c.close()


def _oracle_alpha_fock(case, fock):
    """Oracle alpha with the Fock matrix replaced, amplitudes fixed, lambda re-solved."""
    from oracle import ccsd, layout, response
    nk, o, v = case['nk'], case['o'], case['v']
    f = layout.dense_one_body(fock, nk, o, v)
    g = layout.dense_eri(case['H']['chol'], nk, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    lam, _, _ = response.solve_lambda(case['t'], h)
    ops = [torch.from_numpy(layout.dense_one_body(case['H']['dip'][x], nk, o, v)) for x in range(3)]
    al, _ = response.polarizability(case['t'], lam, ops, OMEGAS, h, nk=nk)
    return al


@pytest.mark.parametrize("x,y", [(2, 2), (0, 1)])
@pytest.mark.parametrize("nk,o,v,naux,seed", [(1, 2, 4, 6, 21), (2, 2, 3, 6, 22)])
def test_alpha_fock_gradient_matches_oracle(nk, o, v, naux, seed, x, y):
    """d alpha / d f at fixed amplitudes against a 5-point central difference of the oracle's
    alpha (lambda and the response amplitudes re-solved at every displaced Fock matrix)."""
    import paper_2508_01266_amd as lr
    print(f"case nk={nk} o={o} v={v} naux={naux} alpha_{x}{y}", flush=True)
    case = make_ccsd_case(nk, o, v, naux, seed)
    H = case['H']
    # a Hermitian, k-diagonal perturbation of the Fock matrix
    dF = 0.1 * synth.hamiltonian(nk, o, v, naux, synth.rng_for(800 + seed, nk, o, v))['dip'][0]
    h = 1e-3
    vals = [_oracle_alpha_fock(case, H['fock'] + s * h * dF)[:, x, y] for s in (-2, -1, 1, 2)]
    ref = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
    c = lr.Context(0)
    c.set_hamiltonian(o, H['fock'], H['chol'], H['dip'])
    c.set_amplitudes(case['t1'], case['t2'])
    c.solve(OMEGAS, tol=1e-12, precision=lr.FP64)
    for j in range(len(OMEGAS)):
        g = c.alpha_fock_gradient(j, x, y, tol=1e-12, precision=lr.FP64)
        got = np.sum(g * dF)
        err = abs(got - ref[j])
        print(f"omega {OMEGAS[j]}: d alpha {got:.10f} oracle {ref[j]:.10f} err {err:.2e}", flush=True)
        # 5-point difference error O(h^4) plus solver tolerance / h
        assert err < 1e-7 * max(1.0, abs(ref[j]))
    c.close()
