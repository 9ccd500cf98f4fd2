"""EOM-CCSD excitation energies (the poles of the response function) from the
device Davidson iteration against the oracle's dense Jacobian eigenvalues on the
momentum-conserving excitations, and the exact two-electron spectrum."""
import numpy as np
import pytest

from tests.sigma_cases import make_ccsd_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nk,o,v,naux,seed,nroots", [(1, 2, 4, 6, 21, 4), (2, 2, 3, 6, 22, 3),
                                                      (3, 1, 3, 5, 23, 3), (1, 4, 8, 24, 25, 5)])
def test_eom_roots_match_oracle(nk, o, v, naux, seed, nroots):
    import paper_2508_01266_amd as lr
    from oracle import response
    print(f"case nk={nk} o={o} v={v} naux={naux} nroots={nroots}", flush=True)
    case = make_ccsd_case(nk, o, v, naux, seed)
    ref = response.excitation_energies(case['t'], case['h'], nk=nk)[:nroots]
    c = lr.Context(0)
    c.set_hamiltonian(o, case['H']['fock'], case['H']['chol'], case['H']['dip'])
    c.set_amplitudes(case['t1'], case['t2'])
    w, rep = c.eom_roots(nroots, tol=1e-9)
    err = np.abs(w - ref).max()
    print(f"roots {np.round(w.real, 8)} max err {err:.2e} {rep}", flush=True)
    assert err < 1e-8
    c.close()


def test_eom_two_electron_roots_are_exact():
    import paper_2508_01266_amd as lr
    from oracle import fockspace, layout
    case = make_ccsd_case(1, 2, 5, 8, 31, chol_sigma=0.15)
    f = layout.dense_one_body(case['H']['fock'], 1, 2, 5)
    g = layout.dense_eri(case['H']['chol'], 1, 2, 5)
    op = layout.dense_one_body(case['H']['dip'][0], 1, 2, 5)
    _, _, exc = fockspace.fci_polarizability(f, g, 2, op, op, [0.0])
    c = lr.Context(0)
    c.set_hamiltonian(2, case['H']['fock'], case['H']['chol'], case['H']['dip'])
    c.set_amplitudes(case['t1'], case['t2'])
    w, _ = c.eom_roots(4, tol=1e-10)
    assert np.abs(w.real - np.sort(exc)[:4]).max() < 1e-9
    c.close()
