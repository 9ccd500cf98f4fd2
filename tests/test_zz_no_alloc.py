"""The sigma entry point that allocates no device memory (lrcc_apply_sigma_dev_noalloc,
work tensors and launch tables in the library's static device array) against the
allocating lrcc_apply_sigma_dev on the same inputs: two calls in a row, the second
with a smaller input, both precisions; then a batch too large for the array
(LRCC_E_OOM before any launch) and a call that works again."""
import numpy as np
import pytest
import torch

from tests.sigma_cases import make_case

pytestmark = pytest.mark.gpu


def _ctx(case):
    # ladder mode 1 (integrals rebuilt in LDS), the path the no-allocation call takes in the
    # automatic mode, so that both entry points run the same launches
    import paper_2508_01266_amd as lr
    c = lr.Context(0)
    c.set_hamiltonian(case['o'], case['H']['fock'], case['H']['chol'], case['H']['dip'])
    c.set_ladder_mode(1)
    c.set_amplitudes(case['t1'], case['t2'])
    return c


def _run(c, case, nrhs, prec, noalloc, st):
    dev = torch.device("cuda:0")
    x1 = torch.from_numpy(case['x1'][:nrhs].copy()).to(dev)
    x2 = torch.from_numpy(case['x2'][:nrhs].copy()).to(dev)
    om = torch.from_numpy(case['omega'][:nrhs].copy()).to(dev)
    y1 = torch.full_like(x1, float('nan'))
    y2 = torch.full_like(x2, float('nan'))
    f = c.apply_sigma_dev_noalloc if noalloc else c.apply_sigma_dev
    f(x1, x2, y1, y2, om, prec, st)
    torch.cuda.synchronize()
    return y1.cpu().numpy(), y2.cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_noalloc_sigma_matches_allocating_entry_point():
    import paper_2508_01266_amd as lr
    st = torch.cuda.Stream().cuda_stream
    big = make_case(2, 3, 5, 7, 40, 81)         # 360 (rhs, i, j) rows: the pipelined ladder
    small = make_case(1, 2, 4, 6, 3, 82)
    cb, cs = _ctx(big), _ctx(small)
    for prec, tol in ((lr.FP64, 1e-13), (lr.FP32, 1e-6)):
        # two calls in a row on the array, the second with a smaller input: fewer right-hand
        # sides on the same context, then a smaller problem on another context
        for c, case, nrhs in ((cb, big, 40), (cb, big, 7), (cs, small, 3), (cs, small, 1)):
            a1, a2 = _run(c, case, nrhs, prec, True, st)
            r1, r2 = _run(c, case, nrhs, prec, False, st)
            same = np.array_equal(a1, r1) and np.array_equal(a2, r2)
            e = max(_rel(a1, r1), _rel(a2, r2))
            print(f"precision {prec} nk={case['nk']} nrhs={nrhs}: no-alloc vs allocating rel {e:.1e} "
                  f"(bitwise {same})", flush=True)
            assert np.isfinite(a1).all() and np.isfinite(a2).all()
            assert e <= tol
    cb.close()
    # a batch whose work tensors exceed the static array: refused before any launch, then the
    # entry point works again
    c1 = make_case(1, 4, 12, 48, 1, 83)
    c = _ctx(c1)
    dev = torch.device("cuda:0")
    R = 2600
    x1 = torch.zeros((R, 1, 4, 12), dtype=torch.complex128, device=dev)
    x2 = torch.zeros((R, 1, 1, 1, 4, 4, 12, 12), dtype=torch.complex128, device=dev)
    y1, y2 = torch.empty_like(x1), torch.empty_like(x2)
    with pytest.raises(lr.LrccError) as err:
        c.apply_sigma_dev_noalloc(x1, x2, y1, y2, None, lr.FP64, st)
    print(f"oversized batch: {err.value}", flush=True)
    assert err.value.status == 4
    del x1, x2, y1, y2
    a1, a2 = _run(cs, small, 3, lr.FP64, True, st)
    r1, r2 = _run(cs, small, 3, lr.FP64, False, st)
    assert max(_rel(a1, r1), _rel(a2, r2)) <= 1e-13
    c.close()
    cs.close()
