"""Chains of different sizes applied together (one persistent ladder launch for
all of them) give bitwise the per-chain sigmas, which match the oracle."""
import numpy as np
import pytest

from tests.sigma_cases import make_case, oracle_sigma

pytestmark = pytest.mark.gpu

# (nk, o, v, naux, nrhs, seed): >= 320 (rhs, i, j) rows each, so all join the shared launch,
# plus one small chain that runs its own ladder
CHAINS = [(2, 3, 5, 7, 40, 61), (3, 2, 4, 6, 96, 62), (1, 4, 12, 48, 24, 63), (2, 2, 3, 5, 2, 64)]


def test_group_matches_per_chain_and_oracle():
    import torch
    import paper_2508_01266_amd as lr
    dev = torch.device("cuda:0")
    cases = [make_case(*c) for c in CHAINS]
    ctxs = []
    for case in cases:
        c = lr.Context(0)
        c.set_hamiltonian(case['o'], case['H']['fock'], case['H']['chol'], case['H']['dip'])
        c.set_amplitudes(case['t1'], case['t2'])
        ctxs.append(c)
    X1 = [torch.from_numpy(c['x1']).to(dev) for c in cases]
    X2 = [torch.from_numpy(c['x2']).to(dev) for c in cases]
    OM = [torch.from_numpy(c['omega']).to(dev) for c in cases]
    st = torch.cuda.current_stream().cuda_stream
    g = lr.Group(ctxs)
    for prec in (lr.FP64, lr.FP32):
        ref = []
        for i, c in enumerate(ctxs):
            y1, y2 = torch.empty_like(X1[i]), torch.empty_like(X2[i])
            c.apply_sigma_dev(X1[i], X2[i], y1, y2, OM[i], prec, st)
            ref.append((y1, y2))
        for rep in range(2):
            Y1 = [torch.zeros_like(x) for x in X1]
            Y2 = [torch.zeros_like(x) for x in X2]
            g.apply_sigma_dev(X1, X2, Y1, Y2, OM, prec, st)
            torch.cuda.synchronize()
            for i in range(len(ctxs)):
                assert torch.equal(Y1[i], ref[i][0]) and torch.equal(Y2[i], ref[i][1]), (prec, rep, i)
        print(f"precision {prec}: group == per-chain (bitwise) for {len(ctxs)} chains", flush=True)
    # one chain against the oracle
    r1, r2 = oracle_sigma(cases[0])
    y1 = ref[0][0].cpu().numpy()
    assert np.abs(y1 - r1).max() / np.abs(r1).max() < 1e-5
    g.close()
    for c in ctxs:
        c.close()
