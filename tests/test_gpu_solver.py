"""GPU response solver: (A - w) x = b solved on the device (FP64 GMRES and
FP32-inner / FP64-refined) against the oracle's GMRES solution."""
import numpy as np
import pytest

import synth
from tests.sigma_cases import make_case, oracle_sigma, oracle_solve

pytestmark = pytest.mark.gpu

CASES = [(1, 2, 4, 6, 3, 11), (3, 2, 3, 5, 2, 12), (1, 4, 12, 48, 4, 13)]


def _ctx(case):
    import paper_2508_01266_amd as lr
    c = lr.Context(0)
    c.set_hamiltonian(case['o'], case['H']['fock'], case['H']['chol'], case['H']['dip'])
    c.set_amplitudes(case['t1'], case['t2'])
    return c


@pytest.mark.parametrize("nk,o,v,naux,nrhs,seed", CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_solve_response_matches_oracle(nk, o, v, naux, nrhs, seed, prec):
    case = make_case(nk, o, v, naux, nrhs, seed)
    rng = synth.rng_for(8000 + seed, nk, o, v)
    b1, b2 = synth.random_vectors(nrhs, nk, o, v, rng, 0.1, 0.1)
    b2 = b2 * nk
    c = _ctx(case)
    x1, x2, rep = c.solve_response(b1, b2, case['omega'], tol=1e-11, precision=prec)
    print(f"case {nk},{o},{v} prec {prec}: {rep}", flush=True)
    assert rep['converged'] == 1
    r1, r2 = oracle_solve(case, b1, b2)
    err = max(np.abs(x1 - r1).max() / np.abs(r1).max(), np.abs(x2 - r2).max() / np.abs(r2).max())
    print(f"solution rel err vs oracle {err:.2e}", flush=True)
    assert err < 1e-9
    if prec == 1:
        assert rep['sigma_fp32'] > rep['sigma_fp64']


@pytest.mark.parametrize("prec", [0, 1])
def test_captured_arnoldi_steps_replay_like_eager(prec):
    """With graphs on, every Arnoldi step (preconditioner, sigma, Gram-Schmidt, rotation, status
    copy) is captured once and replayed; a restart length of 4 replays each step graph over many
    cycles (and, on the mixed path, over several refinement steps), with eager residual products
    and host synchronisations between the replays.  Every solve must equal the eager one."""
    import paper_2508_01266_amd as lr
    nk, o, v, naux, nrhs, seed = 1, 4, 12, 48, 4, 13
    case = make_case(nk, o, v, naux, nrhs, seed)
    rng = synth.rng_for(8000 + seed, nk, o, v)
    b1, b2 = synth.random_vectors(nrhs, nk, o, v, rng, 0.1, 0.1)
    b2 = b2 * nk
    c = _ctx(case)
    x1e, x2e, rep_e = c.solve_response(b1, b2, case['omega'], tol=1e-11, precision=prec, krylov=4)
    c.set_graphs(True)
    for rep in range(3):
        x1g, x2g, rep_g = c.solve_response(b1, b2, case['omega'], tol=1e-11, precision=prec, krylov=4)
        d = max(np.abs(x1g - x1e).max(), np.abs(x2g - x2e).max())
        print(f"precision {prec} replay {rep}: eager {rep_e['sigma_fp64']}+{rep_e['sigma_fp32']} products, "
              f"graphs {rep_g['sigma_fp64']}+{rep_g['sigma_fp32']}; max |x_graph - x_eager| {d:.1e}", flush=True)
        assert rep_g['converged'] == 1
        assert (rep_g['sigma_fp64'], rep_g['sigma_fp32']) == (rep_e['sigma_fp64'], rep_e['sigma_fp32'])
        assert d <= 1e-13 * max(np.abs(x2e).max(), 1.0)
    c.close()
