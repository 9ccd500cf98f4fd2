"""GPU parity on 3D k meshes (k = flat index of an n0 x n1 x n2 mesh, momenta added
componentwise modulo the extents) and of the velocity-gauge polarizability,
through the C ABI, against the oracle."""
import numpy as np
import pytest

import synth
from tests.sigma_cases import FP32_REL, make_case, make_ccsd_case, oracle_alpha, oracle_sigma, oracle_sigma_adjoint

pytestmark = pytest.mark.gpu

MESH_CASES = [
    # (mesh, o, v, naux, nrhs, seed)
    ((2, 2, 1), 2, 3, 5, 3, 1),      # Z2 x Z2: not cyclic
    ((2, 2, 2), 1, 3, 4, 2, 2),      # a 3D mesh, nk = 8
    ((3, 2, 1), 2, 4, 6, 2, 3),      # Z3 x Z2
    ((2, 2, 1), 3, 5, 7, 24, 4),     # >= 192 (rhs, i, j) rows: 256-row packed ladder tiles, ragged
    ((2, 2, 1), 3, 5, 7, 40, 5),     # >= 320 rows: a ragged 384-row pipelined ladder tile
]
MODES = {1: "rebuild", 2: "stored", 3: "by class"}


def _ctx(case, mode=0, amplitudes=True):
    import paper_2508_01266_amd as lr
    c = lr.Context(0)
    km = case['km']
    if not np.isscalar(km):
        c.set_kmesh(*synth.mesh_dims(km))
    H = case['H']
    c.set_hamiltonian(case['o'], H['fock'], H['chol'], H['dip'])
    c.set_ladder_mode(mode)
    if amplitudes:
        c.set_amplitudes(case['t1'], case['t2'])
    return c


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("mesh,o,v,naux,nrhs,seed", MESH_CASES)
def test_sigma_on_mesh_matches_oracle(mesh, o, v, naux, nrhs, seed):
    import paper_2508_01266_amd as lr
    nk = int(np.prod(mesh))
    case = make_case(nk, o, v, naux, nrhs, 300 + seed, mesh=mesh)
    print(f"mesh {mesh} o={o} v={v} naux={naux} nrhs={nrhs}", flush=True)
    ref1, ref2 = oracle_sigma(case)
    tol32 = FP32_REL
    for mode, name in MODES.items():
        c = _ctx(case, mode)
        y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], lr.FP64)
        e1, e2 = _rel(y1, ref1), _rel(y2, ref2)
        print(f"fp64 ({name}) rel err singles {e1:.2e} doubles {e2:.2e}", flush=True)
        assert e1 < 1e-11 and e2 < 1e-11
        y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], lr.FP32)
        e1, e2 = _rel(y1, ref1), _rel(y2, ref2)
        print(f"fp32 ({name}) rel err singles {e1:.2e} doubles {e2:.2e}", flush=True)
        assert e1 < tol32 and e2 < tol32
        c.close()
    # transpose product: the oracle's and the dot-product identity
    rng = synth.rng_for(7300 + seed, nk, o, v, extra=mesh)
    z1, z2 = synth.random_vectors(nrhs, mesh, o, v, rng, 0.1, 0.1)
    z2 = z2 * nk
    b1, b2 = oracle_sigma_adjoint(case, z1, z2)
    for mode, name in MODES.items():
        c = _ctx(case, mode)
        a1, a2 = c.apply_sigma_adjoint(z1, z2, case['omega'], lr.FP64)
        y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], lr.FP64)
        for r in range(nrhs):
            lhs = np.sum(z1[r] * y1[r]) + 0.25 * np.sum(z2[r] * y2[r])
            rhs = np.sum(a1[r] * case['x1'][r]) + 0.25 * np.sum(a2[r] * case['x2'][r])
            assert abs(lhs - rhs) < 1e-12 * abs(lhs)
        e1, e2 = _rel(a1, b1), _rel(a2, b2)
        print(f"transpose fp64 ({name}) rel err singles {e1:.2e} doubles {e2:.2e}", flush=True)
        assert e1 < 1e-11 and e2 < 1e-11
        c.close()


def _crt(j):
    return (j % 2) * 3 + (j % 3)


def test_sigma_on_mesh_equals_relabelled_chain():
    """Z6 = Z2 x Z3: a 6-point chain and the same inputs relabelled onto the 2 x 3 mesh
    give the same sigma, block for block, at sizes with several 256-row ladder tiles."""
    import paper_2508_01266_amd as lr
    nk, o, v, naux, R = 6, 4, 16, 48, 16
    case = make_case(nk, o, v, naux, R, 310)
    perm = np.array([_crt(j) for j in range(nk)])
    inv = np.argsort(perm)
    H = case['H']
    mcase = dict(case, km=(2, 3, 1))
    mcase['H'] = dict(H, fock=H['fock'][inv], chol=H['chol'][inv][:, inv], dip=H['dip'][:, inv])
    mcase['t1'] = case['t1'][inv]
    mcase['t2'] = case['t2'][inv][:, inv][:, :, inv]
    x1m = case['x1'][:, inv]
    x2m = case['x2'][:, inv][:, :, inv][:, :, :, inv]
    for prec, tol in ((lr.FP64, 1e-12), (lr.FP32, 1e-5)):
        c = _ctx(case)
        y1, y2 = c.apply_sigma(case['x1'], case['x2'], case['omega'], prec)
        c.close()
        cm = _ctx(mcase)
        m1, m2 = cm.apply_sigma(x1m, x2m, case['omega'], prec)
        cm.close()
        e1 = _rel(m1, y1[:, inv])
        e2 = _rel(m2, y2[:, inv][:, :, inv][:, :, :, inv])
        print(f"precision {prec}: mesh vs relabelled chain rel diff {e1:.2e} {e2:.2e}", flush=True)
        assert e1 < tol and e2 < tol


ALPHA_MESHES = [((2, 2, 1), 1, 3, 5, 21), ((2, 2, 2), 1, 2, 4, 22)]
OMEGAS = [0.0, 0.0656]


@pytest.mark.parametrize("mesh,o,v,naux,seed", ALPHA_MESHES)
def test_alpha_on_mesh_matches_oracle(mesh, o, v, naux, seed):
    import paper_2508_01266_amd as lr
    nk = int(np.prod(mesh))
    case = make_ccsd_case(nk, o, v, naux, 300 + seed, mesh=mesh)
    ref, _ = oracle_alpha(case, OMEGAS)
    c = _ctx(case)
    a64, rep = c.solve(OMEGAS, tol=1e-11, precision=lr.FP64)
    err64 = np.abs(a64 - ref).max()
    print(f"mesh {mesh}: fp64 alpha err {err64:.2e} (|alpha| {np.abs(ref).max():.3f}) {rep}", flush=True)
    assert err64 < 1e-9
    a32, _ = c.solve(OMEGAS, tol=1e-11, precision=lr.FP32)
    assert np.abs(a32 - ref).max() / np.abs(ref).max() < 1e-7
    # device CCSD on the mesh reproduces the oracle's ground state
    t1, t2, e, crep = c.solve_ccsd(tol=1e-11, max_iter=300)
    print(f"mesh {mesh}: ccsd E/cell {e:.12f} (oracle {case['E'].real / nk:.12f})", flush=True)
    assert abs(e - case['E'].real / nk) < 1e-10
    c.close()


VG_CASES = [(2, None, 2, 3, 6, 31), (4, (2, 2, 1), 1, 3, 5, 32)]
VG_OMEGAS = [0.1, 0.2]


def _momentum(case, seed):
    """Momentum-like matrices: i times a real antisymmetric matrix per axis and k (the form
    of momentum integrals in a real basis; Hermitian)."""
    km, o, v, naux = case['km'], case['o'], case['v'], case['naux']
    nk = case['nk']
    extra = () if np.isscalar(km) else synth.mesh_dims(km)
    d = synth.hamiltonian(km, o, v, naux, synth.rng_for(seed, nk, o, v, extra=extra))['dip'].imag
    return 1j * (d - np.swapaxes(d, -1, -2))


@pytest.mark.parametrize("nk,mesh,o,v,naux,seed", VG_CASES)
def test_velocity_gauge_matches_oracle(nk, mesh, o, v, naux, seed):
    import paper_2508_01266_amd as lr
    case = make_ccsd_case(nk, o, v, naux, 300 + seed, mesh=mesh)
    mom = _momentum(case, 990 + seed)
    ref, _ = oracle_alpha(case, VG_OMEGAS, ops=mom, velocity=True)
    assert np.abs(ref).max() > 0.1
    c = _ctx(case)
    for prec, tol in ((lr.FP64, 1e-8), (lr.FP32, 1e-6)):
        a, rep = c.alpha_velocity_gauge(VG_OMEGAS, mom, tol=1e-12, precision=prec)
        err = np.abs(a - ref).max() / np.abs(ref).max()
        print(f"velocity gauge nk={nk} mesh={mesh} precision {prec}: rel err {err:.2e} "
              f"(|alpha| {np.abs(ref).max():.3f}) {rep}", flush=True)
        assert err < tol
    # the dipoles of the Hamiltonian are back in place for length-gauge solves
    lg, _ = oracle_alpha(case, OMEGAS)
    a64, _ = c.solve(OMEGAS, tol=1e-11, precision=lr.FP64)
    assert np.abs(a64 - lg).max() < 1e-9
    with pytest.raises(lr.LrccError):
        c.alpha_velocity_gauge([0.0, 0.1], mom)
    c.close()


def test_mesh_size_must_match_hamiltonian():
    import paper_2508_01266_amd as lr
    case = make_case(4, 1, 2, 3, 1, 320, mesh=(2, 2, 1))
    c = lr.Context(0)
    c.set_kmesh(3, 1, 1)
    with pytest.raises(lr.LrccError):
        c.set_hamiltonian(1, case['H']['fock'], case['H']['chol'], case['H']['dip'])
    with pytest.raises(lr.LrccError):
        c.set_kmesh(0, 1, 1)
    c.close()


def test_eom_roots_on_mesh_match_oracle():
    """Excitation energies on the non-cyclic 2 x 2 mesh: the device Davidson roots equal the
    oracle's dense Jacobian eigenvalues on the excitations that conserve momentum on the mesh."""
    import paper_2508_01266_amd as lr
    from oracle import response
    from oracle.kmesh import Mesh
    mesh = (2, 2, 1)
    case = make_ccsd_case(4, 1, 2, 4, 340, mesh=mesh)
    ref = response.excitation_energies(case['t'], case['h'], nk=Mesh(mesh))[:3]
    c = _ctx(case)
    w, rep = c.eom_roots(3, tol=1e-9)
    err = np.abs(w - ref).max()
    print(f"mesh {mesh}: roots {np.round(w.real, 8)} max err {err:.2e} {rep}", flush=True)
    assert err < 1e-8
    c.close()


def test_group_of_mesh_and_chain_contexts():
    """A 2 x 2 x 2 mesh and a chain applied together in one persistent ladder launch (integrals
    rebuilt in LDS, ladder mode 1) give bitwise the per-context sigmas."""
    import torch
    import paper_2508_01266_amd as lr
    dev = torch.device("cuda:0")
    cases = [make_case(8, 2, 3, 5, 96, 350, mesh=(2, 2, 2)), make_case(3, 2, 4, 6, 96, 351)]
    ctxs = [_ctx(cs, 1) for cs in cases]
    X1 = [torch.from_numpy(cs['x1']).to(dev) for cs in cases]
    X2 = [torch.from_numpy(cs['x2']).to(dev) for cs in cases]
    OM = [torch.from_numpy(cs['omega']).to(dev) for cs in cases]
    st = torch.cuda.current_stream().cuda_stream
    g = lr.Group(ctxs)
    for prec in (lr.FP64, lr.FP32):
        ref = []
        for i, c in enumerate(ctxs):
            y1, y2 = torch.empty_like(X1[i]), torch.empty_like(X2[i])
            c.apply_sigma_dev(X1[i], X2[i], y1, y2, OM[i], prec, st)
            ref.append((y1, y2))
        Y1 = [torch.zeros_like(x) for x in X1]
        Y2 = [torch.zeros_like(x) for x in X2]
        g.apply_sigma_dev(X1, X2, Y1, Y2, OM, prec, st)
        torch.cuda.synchronize()
        for i in range(len(ctxs)):
            assert torch.equal(Y1[i], ref[i][0]) and torch.equal(Y2[i], ref[i][1]), (prec, i)
    g.close()
    for c in ctxs:
        c.close()
