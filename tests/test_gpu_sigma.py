"""GPU sigma parity: the HIP library (through the C ABI) against the oracle's
exact-stencil Jacobian-vector product, element by element."""
import numpy as np
import pytest

from tests.sigma_cases import FP32_REL, make_case, oracle_sigma

pytestmark = pytest.mark.gpu

CASES = [
    # (nk, o, v, naux, nrhs, seed): several tiles and ragged tails in every GEMM dimension
    (1, 2, 4, 6, 1, 1),
    (3, 2, 3, 5, 2, 2),
    (2, 3, 5, 7, 3, 3),
    (1, 4, 12, 48, 3, 4),      # molecular-limit workload sizes (c1)
    (3, 4, 20, 72, 2, 5),      # three-k chain workload sizes (c2)
    (2, 3, 5, 7, 24, 6),       # >= 192 (rhs, i, j) rows: 256-row packed ladder tiles, ragged
    (1, 4, 12, 48, 12, 7),     # c1 sizes with 12 right-hand sides (192 rows)
    (2, 3, 5, 7, 40, 8),       # >= 320 rows: one ragged 384-row pipelined ladder tile
    (1, 4, 12, 48, 30, 9),     # c1 sizes, 480 rows: two pipelined tiles, the second ragged
    (5, 8, 4, 10, 1, 10),      # one right-hand side, 156 unique rows per momentum class (ki <= kj pairs
                               # with one ki + kj share the pipelined tiles), as the one-vector products
]


def _ctx(case, ladder_mode=0):
    import paper_2508_01266_amd as lr
    c = lr.Context(0)
    H = case['H']
    c.set_hamiltonian(case['o'], H['fock'], H['chol'], H['dip'])
    c.set_ladder_mode(ladder_mode)
    c.set_amplitudes(case['t1'], case['t2'])
    return c


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# ladder integrals rebuilt in LDS (1), stored blocks (2), blocks built one momentum class at a time (3)
MODES = {1: "rebuild", 2: "stored", 3: "by class"}


@pytest.mark.parametrize("nk,o,v,naux,nrhs,seed", CASES)
def test_sigma_fp64_matches_oracle(nk, o, v, naux, nrhs, seed):
    import paper_2508_01266_amd as lr
    case = make_case(nk, o, v, naux, nrhs, seed)
    print(f"case nk={nk} o={o} v={v} naux={naux} nrhs={nrhs}", flush=True)
    ref1, ref2 = oracle_sigma(case)
    for mode, name in MODES.items():
        c = _ctx(case, mode)
        y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], lr.FP64)
        e1, e2 = _rel(y1, ref1), _rel(y2, ref2)
        print(f"fp64 ({name} ladder) rel err singles {e1:.2e} doubles {e2:.2e}", flush=True)
        # FP64 GEMM rounding: well below 1e-11 relative (max-norm)
        assert e1 < 1e-11 and e2 < 1e-11
        c.close()


@pytest.mark.parametrize("nk,o,v,naux,nrhs,seed", CASES)
def test_sigma_fp32_matches_oracle(nk, o, v, naux, nrhs, seed):
    import paper_2508_01266_amd as lr
    case = make_case(nk, o, v, naux, nrhs, seed)
    ref1, ref2 = oracle_sigma(case)
    tol = FP32_REL
    for mode, name in MODES.items():
        c = _ctx(case, mode)
        y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], lr.FP32)
        e1, e2 = _rel(y1, ref1), _rel(y2, ref2)
        print(f"fp32 ({name} ladder) rel err singles {e1:.2e} doubles {e2:.2e} (tol {tol:.1e})", flush=True)
        assert e1 < tol and e2 < tol
        c.close()


def test_ladder_mode_is_fixed_after_amplitudes():
    import paper_2508_01266_amd as lr
    case = make_case(1, 2, 4, 6, 1, 1)
    c = _ctx(case)
    with pytest.raises(lr.LrccError):
        c.set_ladder_mode(1)
    c.close()


@pytest.mark.parametrize("nk,o,v,naux,nrhs,seed", CASES)
def test_sigma_adjoint_fp64_matches_oracle_and_dot_identity(nk, o, v, naux, nrhs, seed):
    import synth
    import paper_2508_01266_amd as lr
    from tests.sigma_cases import oracle_sigma_adjoint
    case = make_case(nk, o, v, naux, nrhs, seed)
    rng = synth.rng_for(7000 + seed, nk, o, v)
    z1, z2 = synth.random_vectors(nrhs, nk, o, v, rng, 0.1, 0.1)
    z2 = z2 * nk
    ref1, ref2 = oracle_sigma_adjoint(case, z1, z2)
    print(f"case nk={nk} o={o} v={v} naux={naux} nrhs={nrhs}", flush=True)
    for mode, name in MODES.items():
        c = _ctx(case, mode)
        a1, a2 = c.apply_sigma_adjoint(z1, z2, case['omega'], lr.FP64)
        y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], lr.FP64)
        for r in range(nrhs):
            lhs = np.sum(z1[r] * y1[r]) + 0.25 * np.sum(z2[r] * y2[r])
            rhs = np.sum(a1[r] * case['x1'][r]) + 0.25 * np.sum(a2[r] * case['x2'][r])
            print(f"dot identity ({name} ladder) rhs {r}: rel {abs(lhs - rhs) / abs(lhs):.2e}", flush=True)
            assert abs(lhs - rhs) < 1e-12 * abs(lhs)
        e1, e2 = _rel(a1, ref1), _rel(a2, ref2)
        print(f"adjoint fp64 ({name} ladder) rel err singles {e1:.2e} doubles {e2:.2e}", flush=True)
        assert e1 < 1e-11 and e2 < 1e-11
        b1, b2 = c.apply_sigma_adjoint(z1, z2, case['omega'], lr.FP32)
        tol = FP32_REL
        assert _rel(b1, ref1) < tol and _rel(b2, ref2) < tol
        c.close()


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_every_launch_variant_matches_oracle(tmp_path, monkeypatch, prec_name):
    """Every launch variant the autotuner can pick (GEMM tile shapes including the complex64 tiles
    with three real products; the ladder kernels of the in-LDS
    path), forced for every op through the tuning cache, gives the oracle's forward and transpose
    products, in the default ladder path and with the integrals rebuilt in LDS."""
    import synth
    import paper_2508_01266_amd as lr
    from tests.sigma_cases import oracle_sigma_adjoint
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LRCC_TUNE_CACHE", str(cache))
    nk, o, v, naux, nrhs, seed = 1, 4, 12, 48, 30, 9   # 480 rows: 384-row ladder tiles, 128-row GEMM tiles
    case = make_case(nk, o, v, naux, nrhs, seed)
    ref1, ref2 = oracle_sigma(case)
    rng = synth.rng_for(7100 + seed, nk, o, v)
    z1, z2 = synth.random_vectors(nrhs, nk, o, v, rng, 0.1, 0.1)
    z2 = z2 * nk
    adj1, adj2 = oracle_sigma_adjoint(case, z1, z2)
    prec = lr.FP64 if prec_name == "fp64" else lr.FP32
    tol = 1e-11 if prec_name == "fp64" else FP32_REL
    for mode in (0, 1):
        cache.write_text("")
        c = _ctx(case, mode)
        c.set_autotune(True)
        c.apply_sigma(case['x1'], case['x2'], case['omega'], prec)
        c.apply_sigma_adjoint(z1, z2, case['omega'], prec)
        c.close()
        lines = [ln.split() for ln in cache.read_text().splitlines() if ln.strip()]
        assert any("forward" in ln[0] for ln in lines) and any("adjoint" in ln[0] for ln in lines)
        for cand in range(4):
            # candidate index `cand` for every tunable launch (clamped to each op's number of variants)
            cache.write_text("".join(" ".join([ln[0]] + [str(cand)] * (len(ln) - 1)) + "\n" for ln in lines))
            c = _ctx(case, mode)
            c.set_autotune(True)
            y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], prec)
            a1, a2 = c.apply_sigma_adjoint(z1, z2, case['omega'], prec)
            c.close()
            e = (_rel(y1, ref1), _rel(y2, ref2), _rel(a1, adj1), _rel(a2, adj2))
            print(f"{prec_name} ladder mode {mode}, variant {cand} for every op: rel err forward {e[0]:.1e} "
                  f"{e[1]:.1e} transpose {e[2]:.1e} {e[3]:.1e}", flush=True)
            assert max(e) < tol


def test_graph_replay_matches_eager():
    """Sigma through captured HIP graphs equals the eager launches on every replay
    (replays interleaved with eager work and with a second input set)."""
    import torch
    import paper_2508_01266_amd as lr
    case = make_case(1, 4, 12, 48, 3, 41)
    c = _ctx(case)
    dev = torch.device("cuda:0")
    xa1, xa2 = (torch.from_numpy(a).to(dev) for a in (case['x1'], case['x2']))
    xb1, xb2 = xa1.flip(0).contiguous(), xa2.flip(0).contiguous()
    om = torch.from_numpy(case['omega']).to(dev)
    st = torch.cuda.Stream()
    y1, y2 = torch.empty_like(xa1), torch.empty_like(xa2)
    ref = {}
    for name, (x1, x2) in (("a", (xa1, xa2)), ("b", (xb1, xb2))):
        c.apply_sigma_dev(x1, x2, y1, y2, om, lr.FP64, st.cuda_stream)
        st.synchronize()
        ref[name] = (y1.clone(), y2.clone())
    c.set_graphs(True)
    for rep, name in enumerate(("a", "b", "a", "a", "b")):
        x1, x2 = (xa1, xa2) if name == "a" else (xb1, xb2)
        y1.zero_()
        y2.zero_()
        c.apply_sigma_dev(x1, x2, y1, y2, om, lr.FP64, st.cuda_stream)
        st.synchronize()
        # eager work between replays
        z1, z2 = torch.empty_like(xa1), torch.empty_like(xa2)
        c.set_graphs(False) if rep == 2 else None
        c.apply_sigma_dev(xb1, xb2, z1, z2, om, lr.FP64, st.cuda_stream)
        st.synchronize()
        c.set_graphs(True)
        assert torch.equal(y1, ref[name][0]) and torch.equal(y2, ref[name][1]), (rep, name)
        assert torch.equal(z1, ref["b"][0]) and torch.equal(z2, ref["b"][1])


def test_autotuned_variants_match_and_cache(tmp_path, monkeypatch):
    """Autotuning picks launch variants without changing results; the choices are
    cached per program and reused by a new context."""
    import paper_2508_01266_amd as lr
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LRCC_TUNE_CACHE", str(cache))
    case = make_case(2, 3, 5, 7, 24, 6)   # >= 192 rows: packed ladder and large tiles are candidates
    ref1, ref2 = oracle_sigma(case)
    c = _ctx(case)
    c.set_autotune(True)
    for _ in range(2):
        y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], lr.FP64)
        assert _rel(y1, ref1) < 1e-11 and _rel(y2, ref2) < 1e-11
    text = cache.read_text()
    assert "forward" in text and len(text.splitlines()) >= 1
    c2 = _ctx(case)
    c2.set_autotune(True)
    z1, z2 = c2.apply_sigma(case['x1'], case['x2'], case['omega'], lr.FP64)
    assert _rel(z1, ref1) < 1e-11 and _rel(z2, ref2) < 1e-11
    assert cache.read_text() == text       # second context read the cache, tuned nothing new


# non-canonical Fock matrices: off-diagonal f_ov, f_oo and f_vv enter F_ae, F_mi, F_me and the
# singles driver; the oracle's residual keeps the full f
NONCANONICAL = [(1, 2, 4, 6, 2, 41), (2, 3, 5, 7, 3, 42), (3, 2, 3, 5, 40, 43)]


@pytest.mark.parametrize("nk,o,v,naux,nrhs,seed", NONCANONICAL)
def test_sigma_noncanonical_fock_matches_oracle(nk, o, v, naux, nrhs, seed):
    import paper_2508_01266_amd as lr
    from tests.sigma_cases import oracle_sigma_adjoint
    case = make_case(nk, o, v, naux, nrhs, seed, noncanonical=0.05)
    f = case['H']['fock']
    off = max(np.abs(f[k] - np.diag(np.diag(f[k]))).max() for k in range(nk))
    print(f"case nk={nk} o={o} v={v} nrhs={nrhs}: largest off-diagonal |f| {off:.3f}", flush=True)
    assert off > 0.01
    ref1, ref2 = oracle_sigma(case)
    z1, z2 = case['x1'][::-1].copy(), case['x2'][::-1].copy()
    adj1, adj2 = oracle_sigma_adjoint(case, z1, z2)
    for mode, name in MODES.items():
        c = _ctx(case, mode)
        for prec, tol in ((lr.FP64, 1e-11), (lr.FP32, FP32_REL)):
            y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], prec)
            g1, g2 = c.apply_sigma_adjoint(z1, z2, case['omega'], prec)
            e = (_rel(y1, ref1), _rel(y2, ref2), _rel(g1, adj1), _rel(g2, adj2))
            print(f"{name} ladder, precision {prec}: sigma {e[0]:.1e} {e[1]:.1e} transpose {e[2]:.1e} {e[3]:.1e}",
                  flush=True)
            assert max(e) < tol
        c.close()
