"""Chains of different sizes applied together (one persistent ladder launch for
all of them) give bitwise the per-chain sigmas, which match the oracle."""
import numpy as np
import pytest

from tests.sigma_cases import make_case, oracle_sigma

pytestmark = pytest.mark.gpu

# (nk, o, v, naux, nrhs, seed): >= 320 (rhs, i, j) rows each, so all join the shared launch (the
# ladder with its integrals rebuilt in LDS, mode 1), plus one small chain in the default mode (its
# blocks built by momentum class) that runs its own program
CHAINS = [(2, 3, 5, 7, 40, 61), (3, 2, 4, 6, 96, 62), (1, 4, 12, 48, 24, 63), (2, 2, 3, 5, 2, 64)]
MODES = [1, 1, 1, 0]
# complex64 sigma against the complex128 oracle: max-norm relative error bound (the measured
# error of these sizes is near 1e-7; rounding of the longest contractions, K <= 500, stays far below)
FP32_REL = 1e-5


def test_group_matches_per_chain_and_oracle():
    import torch
    import paper_2508_01266_amd as lr
    dev = torch.device("cuda:0")
    cases = [make_case(*c) for c in CHAINS]
    ctxs = []
    for case, mode in zip(cases, MODES):
        c = lr.Context(0)
        c.set_hamiltonian(case['o'], case['H']['fock'], case['H']['chol'], case['H']['dip'])
        c.set_ladder_mode(mode)
        c.set_amplitudes(case['t1'], case['t2'])
        ctxs.append(c)
    print("ladder paths:", [c.ladder_path(case['x1'].shape[0], lr.FP32) for c, case in zip(ctxs, cases)],
          flush=True)
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
    # every chain against the oracle (ref holds the complex64 results of the last loop)
    for i, case in enumerate(cases):
        r1, r2 = oracle_sigma(case)
        e1 = np.abs(ref[i][0].cpu().numpy() - r1).max() / np.abs(r1).max()
        e2 = np.abs(ref[i][1].cpu().numpy() - r2).max() / np.abs(r2).max()
        print(f"chain {i} (complex64) vs oracle: singles {e1:.1e} doubles {e2:.1e}", flush=True)
        assert e1 < FP32_REL and e2 < FP32_REL
    # a chain gets a new Hamiltonian of another shape: the group rebuilds its launch tables
    # (they hold the chain's buffer addresses and sizes) and still matches the chain alone
    new = make_case(2, 3, 4, 6, 40, 65)
    ctxs[0].set_hamiltonian(new['o'], new['H']['fock'], new['H']['chol'], new['H']['dip'])
    ctxs[0].set_amplitudes(new['t1'], new['t2'])
    X1[0] = torch.from_numpy(new['x1']).to(dev)
    X2[0] = torch.from_numpy(new['x2']).to(dev)
    OM[0] = torch.from_numpy(new['omega']).to(dev)
    for prec in (lr.FP64, lr.FP32):
        y1, y2 = torch.empty_like(X1[0]), torch.empty_like(X2[0])
        ctxs[0].apply_sigma_dev(X1[0], X2[0], y1, y2, OM[0], prec, st)
        Y1 = [torch.zeros_like(x) for x in X1]
        Y2 = [torch.zeros_like(x) for x in X2]
        g.apply_sigma_dev(X1, X2, Y1, Y2, OM, prec, st)
        torch.cuda.synchronize()
        assert torch.equal(Y1[0], y1) and torch.equal(Y2[0], y2), prec
    r1, r2 = oracle_sigma(new)
    assert np.abs(Y2[0].cpu().numpy() - r2).max() / np.abs(r2).max() < FP32_REL
    print("group after a new Hamiltonian on chain 0 == chain alone == oracle", flush=True)
    g.close()
    for c in ctxs:
        c.close()
