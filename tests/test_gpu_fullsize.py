"""Parity at full workload sizes, in the launch configuration the benchmark times:
the batched sigma (all right-hand sides in one launch) against the k-blocked
oracle on sampled right-hand sides, and the large-orbital slice (Nk=3, o=10,
v=60, Naux=210) forward and transpose."""
import numpy as np
import pytest

from tests.sigma_cases import FP32_REL

import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _inputs(name, nrhs):
    w = synth.WORKLOADS[name]
    rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir)
    H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift, chol_sigma=w.chol_sigma)
    t1, t2 = synth.random_amplitudes(w.nk, w.nocc, w.nvir, rng, 0.02, 0.02)
    x1, x2 = synth.random_vectors(nrhs, w.nk, w.nocc, w.nvir, rng, 0.1, 0.1)
    omega = np.linspace(-0.1, 0.1, nrhs)
    return w, H, t1, t2 * w.nk, x1, x2 * w.nk, omega


def _oracle_one(w, H, t1, t2, x1, x2, om, adjoint=False):
    import torch
    from oracle import kblock
    nk = w.nk
    ham = kblock.KHam(H['fock'], H['chol'], w.nocc)
    t = (t1, t2 / nk)
    if not adjoint:
        s1, s2 = kblock.sigma(ham, t, (x1, x2 / nk))
        return s1.numpy() - om * x1, nk * s2.numpy() - om * x2
    raise NotImplementedError


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_batched_workload_sampled_rhs():
    """All 48 right-hand sides in one launch, both precisions, the three ladder modes (integrals
    stored / built one momentum class at a time / rebuilt in LDS), with the autotuned launch
    variants the benchmark times; sampled right-hand sides against the k-blocked oracle."""
    import paper_2508_01266_amd as lr
    w, H, t1, t2, x1, x2, om = _inputs("c3", 48)
    out = {}
    for mode in (2, 3, 1):
        c = lr.Context(0)
        c.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
        c.set_ladder_mode(mode)
        c.set_amplitudes(t1, t2)
        c.set_autotune(True)
        for prec in (lr.FP64, lr.FP32):
            y1, y2 = c.apply_sigma(x1, x2, om, prec)
            out[(mode, prec)] = (y1[[0, 29]], y2[[0, 29]])
        c.close()
        print(f"ladder mode {mode}: device sigmas done", flush=True)
    for i, r in enumerate((0, 29)):
        r1, r2 = _oracle_one(w, H, t1, t2, x1[r], x2[r], om[r])
        for (mode, prec), (y1, y2) in out.items():
            e1, e2 = _rel(y1[i], r1), _rel(y2[i], r2)
            tol = 1e-11 if prec == lr.FP64 else FP32_REL
            print(f"c3 48-rhs launch, rhs {r}, ladder mode {mode}, prec {prec}: rel err singles {e1:.2e} "
                  f"doubles {e2:.2e} (tol {tol:.1e})", flush=True)
            assert e1 < tol and e2 < tol


def test_large_orbital_slice_forward_and_transpose():
    import paper_2508_01266_amd as lr
    w, H, t1, t2, x1, x2, om = _inputs("c4s", 2)
    c = lr.Context(0)
    c.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
    c.set_amplitudes(t1, t2)
    y1, y2 = c.apply_sigma(x1, x2, om, lr.FP64)
    r1, r2 = _oracle_one(w, H, t1, t2, x1[0], x2[0], om[0])
    e1, e2 = _rel(y1[0], r1), _rel(y2[0], r2)
    print(f"Nk=3 o=10 v=60 slice: rel err singles {e1:.2e} doubles {e2:.2e}", flush=True)
    assert e1 < 1e-11 and e2 < 1e-11
    # transpose: dot-product identity against the verified forward product
    rng = synth.rng_for(99, 3, 10, 60)
    z1, z2 = synth.random_vectors(2, 3, 10, 60, rng, 0.1, 0.1)
    z2 = z2 * 3
    a1, a2 = c.apply_sigma_adjoint(z1, z2, om, lr.FP64)
    for r in range(2):
        lhs = np.sum(z1[r] * y1[r]) + 0.25 * np.sum(z2[r] * y2[r])
        rhs = np.sum(a1[r] * x1[r]) + 0.25 * np.sum(a2[r] * x2[r])
        print(f"slice dot identity rhs {r}: {abs(lhs - rhs) / abs(lhs):.2e}", flush=True)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_c4_forward_modes_and_transpose():
    """Nk=7, o=10, v=60, Naux=210 (2 RHS): the independent ladder paths (integrals rebuilt in
    LDS, stored integral blocks, blocks built one momentum class at a time) agree, and the
    transpose product satisfies the dot identity with the forward product in the rebuilt and
    by-class modes (properties that hold at any size; the oracle is too slow here)."""
    import paper_2508_01266_amd as lr
    w, H, t1, t2, x1, x2, om = _inputs("c4", 2)
    ys, adj = {}, {}
    rng = synth.rng_for(98, 7, 10, 60)
    z1, z2 = synth.random_vectors(2, 7, 10, 60, rng, 0.1, 0.1)
    z2 = z2 * 7
    for mode in (1, 2, 3):
        c = lr.Context(0)
        c.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
        c.set_ladder_mode(mode)
        c.set_amplitudes(t1, t2)
        ys[mode] = c.apply_sigma(x1, x2, om, lr.FP64)
        if mode != 2:
            adj[mode] = c.apply_sigma_adjoint(z1, z2, om, lr.FP64)
        c.close()
        print(f"c4 ladder mode {mode}: forward done", flush=True)
    for m in (2, 3):
        e1, e2 = _rel(ys[1][0], ys[m][0]), _rel(ys[1][1], ys[m][1])
        print(f"c4 rebuilt vs ladder mode {m}: rel diff singles {e1:.2e} doubles {e2:.2e}", flush=True)
        assert e1 < 1e-11 and e2 < 1e-11
    for m, (a1, a2) in adj.items():
        y1, y2 = ys[m]
        for r in range(2):
            lhs = np.sum(z1[r] * y1[r]) + 0.25 * np.sum(z2[r] * y2[r])
            rhs = np.sum(a1[r] * x1[r]) + 0.25 * np.sum(a2[r] * x2[r])
            print(f"c4 dot identity, ladder mode {m}, rhs {r}: {abs(lhs - rhs) / abs(lhs):.2e}", flush=True)
            assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_c4s_dipole_gradient_against_finite_difference():
    """Adjoint workload slice (Nk=3, o=10, v=60, Naux=210): device CCSD ground state,
    alpha_zz(0.0656) and its dipole gradient; alpha is bilinear in mu_z at fixed amplitudes, so
    the central difference along a Hermitian perturbation is exact up to the solver tolerance."""
    import paper_2508_01266_amd as lr
    w = synth.WORKLOADS["c4s"]
    rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir)
    H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift, chol_sigma=w.chol_sigma)
    V = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, synth.rng_for(97, w.nk, w.nocc, w.nvir))['dip']
    c = lr.Context(0)
    c.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
    t1, t2, e, rep = c.solve_ccsd(tol=1e-9, max_iter=300)
    print(f"c4s CCSD: E/cell {e:.10f} {rep}", flush=True)
    om = [0.0656]
    a0, r0 = c.solve(om, axis_mask=4, tol=1e-11, precision=lr.FP64)
    print(f"c4s alpha_zz {a0[0, 2, 2]} {r0}", flush=True)
    g = c.alpha_dipole_gradient(0, 2, 2, tol=1e-11)
    got = np.sum(g[2] * V[2])
    hstep = 0.5
    vals = []
    for sgn in (1, -1):
        dip = H['dip'].copy()
        dip[2] = dip[2] + sgn * hstep * V[2]
        c2 = lr.Context(0)
        c2.set_hamiltonian(w.nocc, H['fock'], H['chol'], dip)
        c2.set_amplitudes(t1, t2)
        a, _ = c2.solve(om, axis_mask=4, tol=1e-11, precision=lr.FP64)
        vals.append(a[0, 2, 2])
        c2.close()
    ref = (vals[0] - vals[1]) / (2 * hstep)
    print(f"c4s d alpha_zz: gradient {got:.10f} central difference {ref:.10f}", flush=True)
    assert abs(got - ref) < 1e-7 * max(1.0, abs(ref))
    c.close()


def test_c4s_fock_gradient_against_central_difference():
    """Adjoint workload slice (Nk=3, o=10, v=60, Naux=210): d alpha_zz(0.0656) / d f at the device
    CCSD amplitudes against the central difference of alpha_zz at f +- h df with h = 1e-5 (the
    amplitudes held at their input values and lambda re-solved, as the gradient is defined),
    along a Hermitian k-diagonal df with off-diagonal elements.  The oracle's own gradient at
    this size would take hours of host time (each oracle alpha needs tens of its ~10 s k-blocked
    residual evaluations per solve); the small sizes compare it with the oracle directly."""
    import paper_2508_01266_amd as lr
    w = synth.WORKLOADS["c4s"]
    rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir)
    H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift, chol_sigma=w.chol_sigma)
    dF = 0.1 * synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, synth.rng_for(96, w.nk, w.nocc, w.nvir))['dip'][0]
    c = lr.Context(0)
    c.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
    t1, t2, e, rep = c.solve_ccsd(tol=1e-10, max_iter=300)
    print(f"c4s CCSD: E/cell {e:.10f} {rep}", flush=True)
    om = [0.0656]
    a0, r0 = c.solve(om, axis_mask=4, tol=1e-12, precision=lr.FP64)
    g = c.alpha_fock_gradient(0, 2, 2, tol=1e-12)
    got = np.sum(g * dF)
    h = 1e-5
    vals = []
    for sgn in (1, -1):
        c2 = lr.Context(0)
        c2.set_hamiltonian(w.nocc, H['fock'] + sgn * h * dF, H['chol'], H['dip'])
        c2.set_amplitudes(t1, t2)
        a, _ = c2.solve(om, axis_mask=4, tol=1e-12, precision=lr.FP64)
        vals.append(a[0, 2, 2])
        c2.close()
    ref = (vals[0] - vals[1]) / (2 * h)
    err = abs(got - ref)
    print(f"c4s d alpha_zz / df . dF: gradient {got:.10f} central difference (h=1e-5) {ref:.10f} "
          f"err {err:.2e}", flush=True)
    # O(h^2) truncation (~1e-10 relative) plus the solver tolerance divided by h (1e-12 |alpha| / 1e-5)
    assert err < 1e-5 * max(1.0, abs(ref))
    c.close()


def test_cholesky_scale_reading_on_batched_workload():
    """The Cholesky scale of the batched workload (Nk=5, o=8, v=40, Naux=144): with the small
    workloads' N(0, 0.05^2) entries the random two-electron coupling outweighs the orbital-energy
    gaps and the device CCSD iteration does not converge, so there are no ground-state amplitudes
    to pose the response equations at; with the reduced scale the ground state converges and so
    does the response solve (the reading the synthetic inputs take for the larger workloads)."""
    import paper_2508_01266_amd as lr
    w = synth.WORKLOADS["c3"]
    out = {}
    for sig in (0.05, w.chol_sigma):
        rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir)
        H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift, chol_sigma=sig)
        c = lr.Context(0)
        c.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
        try:
            _, _, e, rep = c.solve_ccsd(tol=1e-9, max_iter=80)
            a, arep = c.solve([0.0656], axis_mask=4, tol=1e-10, precision=lr.FP64)
            out[sig] = (e, rep, a[0, 2, 2], arep)
            print(f"sigma {sig:.4f}: CCSD E/cell {e:.8f} in {rep['outer']} iterations, alpha_zz {a[0, 2, 2]:.6f} "
                  f"after {arep['sigma_fp64']} operator applications", flush=True)
        except lr.LrccError as err:
            out[sig] = err
            print(f"sigma {sig:.4f}: {err}", flush=True)
        c.close()
    assert isinstance(out[0.05], lr.LrccError) and out[0.05].status == 6
    e, rep, a, arep = out[w.chol_sigma]
    assert rep['converged'] and arep['converged'] and np.isfinite(a)
