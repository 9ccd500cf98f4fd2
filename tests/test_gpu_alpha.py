"""GPU polarizability against the oracle (FP64 path: 1e-9 a.u.; mixed path:
1e-7 relative), plus the exact two-electron sum-over-states limit."""
import json
import os

import numpy as np
import pytest

from tests.sigma_cases import make_ccsd_case, oracle_alpha

pytestmark = pytest.mark.gpu

CASES = [(1, 2, 4, 6, 21), (2, 2, 3, 6, 22), (3, 1, 3, 5, 23), (1, 4, 12, 48, 24)]
OMEGAS = [0.0, 0.0656]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_alpha.json")


def _ctx(case, ladder_mode=0):
    import paper_2508_01266_amd as lr
    c = lr.Context(0)
    c.set_hamiltonian(case['o'], case['H']['fock'], case['H']['chol'], case['H']['dip'])
    c.set_ladder_mode(ladder_mode)
    c.set_amplitudes(case['t1'], case['t2'])
    return c


@pytest.mark.parametrize("nk,o,v,naux,seed", CASES)
def test_alpha_matches_oracle(nk, o, v, naux, seed):
    import paper_2508_01266_amd as lr
    case = make_ccsd_case(nk, o, v, naux, seed)
    print(f"case nk={nk} o={o} v={v} naux={naux}: E_ccsd {case['E']}", flush=True)
    ref, lam = oracle_alpha(case, OMEGAS)
    c = _ctx(case)
    a64, rep = c.solve(OMEGAS, tol=1e-11, precision=lr.FP64)
    err64 = np.abs(a64 - ref).max()
    print(f"fp64 alpha max abs err {err64:.2e} (|alpha| {np.abs(ref).max():.3f}); {rep}", flush=True)
    assert err64 < 1e-9
    a32, rep32 = c.solve(OMEGAS, tol=1e-11, precision=lr.FP32)
    rel32 = np.abs(a32 - ref).max() / np.abs(ref).max()
    print(f"mixed alpha max rel err {rel32:.2e}; {rep32}", flush=True)
    assert rel32 < 1e-7
    # lambda against the oracle (per-cell normalisation: l2_paper = l2_crystal / Nk)
    from oracle import layout
    l1, l2 = c.get_lambda()
    r1 = layout.block_t1(lam[0].numpy(), nk, o, v)
    r2 = layout.block_t2(lam[1].numpy(), nk, o, v) / nk
    assert np.abs(l1 - r1).max() < 1e-9 * max(1, np.abs(r1).max())
    assert np.abs(l2 - r2).max() < 1e-9 * max(1, np.abs(r2).max())
    c.close()
    # stored ladder integrals (2) and integrals built one momentum class at a time (3): the lambda
    # equations and the F term then read them through the transposed product
    for mode in (2, 3):
        c = _ctx(case, mode)
        s64, _ = c.solve(OMEGAS, tol=1e-11, precision=lr.FP64)
        errs = np.abs(s64 - ref).max()
        print(f"fp64 alpha, ladder mode {mode}: max abs err {errs:.2e}", flush=True)
        assert errs < 1e-9
        c.close()


def test_alpha_two_electron_sum_over_states():
    """Two electrons: LR-CCSD is exact; the device alpha equals the FCI sum over states."""
    import paper_2508_01266_amd as lr
    from oracle import fockspace, layout
    case = make_ccsd_case(1, 2, 5, 8, 31, chol_sigma=0.15)
    nk, o, v = 1, 2, 5
    c = _ctx(case)
    a64, _ = c.solve(OMEGAS, tol=1e-12, precision=lr.FP64)
    f = layout.dense_one_body(case['H']['fock'], nk, o, v)
    g = layout.dense_eri(case['H']['chol'], nk, o, v)
    ops = [layout.dense_one_body(case['H']['dip'][x], nk, o, v) for x in range(3)]
    ref = np.zeros_like(a64)
    for X in range(3):
        for Y in range(3):
            ref[:, X, Y] = fockspace.fci_polarizability(f, g, nk * o, ops[X], ops[Y], OMEGAS)[0] / nk
    err = np.abs(a64 - ref).max()
    print(f"device alpha vs FCI sum over states: {err:.2e}", flush=True)
    assert err < 1e-9


@pytest.mark.parametrize("nk,o,v,naux,seed", [(1, 2, 4, 6, 21), (2, 2, 3, 6, 22), (1, 4, 12, 48, 24)])
def test_ccsd_ground_state_matches_oracle(nk, o, v, naux, seed):
    """Device CCSD (exact residual from the Jacobian) against the oracle's CCSD."""
    import paper_2508_01266_amd as lr
    case = make_ccsd_case(nk, o, v, naux, seed)
    c = lr.Context(0)
    c.set_hamiltonian(o, case['H']['fock'], case['H']['chol'], case['H']['dip'])
    t1, t2, e, rep = c.solve_ccsd(tol=1e-11, max_iter=300)
    print(f"ccsd nk={nk} o={o} v={v}: E/cell {e:.12f} (oracle {case['E'].real / nk:.12f}) {rep}", flush=True)
    assert rep['converged'] == 1
    assert abs(e - case['E'].real / nk) < 1e-10
    assert np.abs(t1 - case['t1']).max() < 1e-9
    assert np.abs(t2 - case['t2']).max() < 1e-9
    # alpha from the device amplitudes equals alpha from the oracle's amplitudes
    ref, _ = oracle_alpha(case, OMEGAS)
    a64, _ = c.solve(OMEGAS, tol=1e-11, precision=lr.FP64)
    assert np.abs(a64 - ref).max() < 1e-9


@pytest.mark.parametrize("nk,o,v,naux,seed", [(1, 2, 4, 6, 21), (2, 2, 3, 6, 22), (3, 1, 3, 5, 23)])
def test_lambda_bar_form_equals_symmetric_alpha(nk, o, v, naux, seed):
    """The non-symmetric form with perturbed multipliers reproduces the symmetric alpha
    (and hence the oracle), including complex off-diagonal elements at finite frequency."""
    import paper_2508_01266_amd as lr
    case = make_ccsd_case(nk, o, v, naux, seed)
    ref, _ = oracle_alpha(case, OMEGAS)
    c = _ctx(case)
    a_sym, _ = c.solve(OMEGAS, tol=1e-12, precision=lr.FP64)
    a_lb, rep = c.alpha_lambda_bar(len(OMEGAS), tol=1e-12)
    d = np.abs(a_lb - a_sym).max()
    print(f"lambda-bar vs symmetric alpha: {d:.2e}; vs oracle {np.abs(a_lb - ref).max():.2e}; {rep}", flush=True)
    assert d < 1e-9
    assert np.abs(a_lb - ref).max() < 1e-9
    c.close()


@pytest.mark.parametrize("nk,o,v,naux,seed", [(1, 2, 4, 6, 25), (2, 2, 3, 6, 26)])
def test_alpha_noncanonical_fock_matches_oracle(nk, o, v, naux, seed):
    """A Fock matrix with off-diagonal elements (f_ov, f_oo, f_vv): the library keeps the full f in
    its one-body blocks and uses only its diagonal for the preconditioner."""
    import paper_2508_01266_amd as lr
    case = make_ccsd_case(nk, o, v, naux, seed, noncanonical=0.05)
    ref, _ = oracle_alpha(case, OMEGAS)
    c = _ctx(case)
    a64, rep = c.solve(OMEGAS, tol=1e-11, precision=lr.FP64)
    err = np.abs(a64 - ref).max()
    a32, _ = c.solve(OMEGAS, tol=1e-11, precision=lr.FP32)
    rel32 = np.abs(a32 - ref).max() / np.abs(ref).max()
    print(f"non-canonical f: fp64 alpha err {err:.2e}, mixed rel err {rel32:.2e}; {rep}", flush=True)
    assert err < 1e-9 and rel32 < 1e-7
    c.close()


def test_alpha_three_k_chain_workload_matches_oracle():
    """The three-k chain workload verbatim (Nk=3, nocc=4, nvir=20, Naux=72, band shift, 3 axes at
    omega in {0, 0.0656}): device CCSD, then alpha on the FP64 and the mixed path, against the
    oracle's alpha from its own CCSD (tests/golden/c2_alpha.json, written by
    tests/golden/make_c2_alpha.py from the oracle alone).  Both CCSD solutions are converged far
    below the alpha tolerance, so they agree to ~1e-11."""
    import synth
    import paper_2508_01266_amd as lr
    assert os.path.exists(GOLDEN), "run tests/golden/make_c2_alpha.py"
    gold = json.load(open(GOLDEN))
    w = synth.WORKLOADS["c2"]
    assert gold["workload"]["seed"] == [1266, w.cfg_id, w.nk, w.nocc, w.nvir]
    ref = np.array(gold["alpha_re"]) + 1j * np.array(gold["alpha_im"])
    rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir)
    H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift, chol_sigma=w.chol_sigma)
    c = lr.Context(0)
    c.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
    _, _, e, crep = c.solve_ccsd(tol=1e-11, max_iter=300)
    e_ref = gold["ccsd_energy_per_cell"][0]
    print(f"c2: device E/cell {e:.12f} oracle {e_ref:.12f}; {crep}", flush=True)
    assert abs(e - e_ref) < 1e-10
    a64, rep = c.solve(gold["omegas"], tol=1e-11, precision=lr.FP64)
    err = np.abs(a64 - ref)
    print(f"c2 fp64 alpha: max abs err {err.max():.2e} (|alpha| up to {np.abs(ref).max():.3f}); {rep}", flush=True)
    for j, wj in enumerate(gold["omegas"]):
        for x in range(3):
            print(f"  w={wj}: alpha_{x}{x} device {a64[j, x, x].real:.12f} oracle {ref[j, x, x].real:.12f}", flush=True)
    assert err.max() < 1e-9
    a32, rep32 = c.solve(gold["omegas"], tol=1e-11, precision=lr.FP32)
    rel = np.abs(a32 - ref).max() / np.abs(ref).max()
    print(f"c2 mixed alpha: max rel err {rel:.2e}; {rep32}", flush=True)
    assert rel < 1e-7
    c.close()
