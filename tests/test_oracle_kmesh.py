"""Pins of the oracle on 3D k meshes and of the velocity-gauge polarizability.

The mesh arithmetic is pinned by group structure (the Chinese-remainder
isomorphism Z6 = Z2 x Z3, the exponent of Z2 x Z2) and by the momentum rule
written on explicit integer 3-vectors; the k-blocked residual on a mesh is
pinned by invariance under that isomorphism (a relabelled 1D chain) and by the
dense collective-index tier on a non-cyclic mesh.  The velocity gauge is pinned
by the independent-particle sum rule and by the exact two-electron limit.
"""
import itertools

import numpy as np
import torch

import synth
from oracle import ccsd, fockspace, kblock, layout, response
from oracle.kmesh import Mesh


def _crt(j):
    """Z6 -> Z2 x Z3 (flat index on the mesh (2, 3, 1))."""
    return (j % 2) * 3 + (j % 3)


def test_mesh_group_structure():
    m = Mesh((2, 3, 1))
    assert sorted(_crt(j) for j in range(6)) == list(range(6))
    for a, b, c in itertools.product(range(6), repeat=3):
        assert m.comb(_crt(a), _crt(b), _crt(c)) == _crt((a + b - c) % 6)
    q = Mesh((2, 2, 1))
    assert all(q.add(a, a) == 0 for a in range(4))          # exponent 2: not the cyclic Z4
    assert Mesh((4,)).add(1, 1) == 2
    c = Mesh((3, 2, 2))
    for a, b in itertools.product(range(12), repeat=2):
        assert c.add(c.sub(a, b), b) == a


def _vec(m, k):
    n0, n1, n2 = m.dims
    return np.array([k // (n1 * n2), (k // n2) % n1, k % n2])


def test_momentum_rule_on_integer_vectors():
    """Non-zero ERI blocks and t2 blocks sit exactly where k_p + k_q - k_r - k_s is a
    reciprocal-lattice vector, computed on explicit integer coordinates."""
    m = Mesh((2, 2, 2))
    nk, o, v = m.size, 1, 1
    rng = synth.rng_for(951, nk, o, v, extra=(2, 2, 2))
    H = synth.hamiltonian((2, 2, 2), o, v, 2, rng, chol_sigma=0.3)
    g = layout.dense_eri(H['chol'], m, o, v)
    idx = layout.orbital_index(m, o, v)
    korb = np.empty(nk * (o + v), dtype=int)
    for k in range(nk):
        korb[idx[k]] = k
    dims = np.array(m.dims)
    N = nk * (o + v)
    for p, q, r, s in itertools.product(range(N), repeat=4):
        tot = _vec(m, korb[p]) + _vec(m, korb[q]) - _vec(m, korb[r]) - _vec(m, korb[s])
        allowed = np.all(tot % dims == 0)
        if not allowed:
            assert g[p, q, r, s] == 0
    assert np.abs(g).max() > 0.01
    mask = layout.forbidden_mask_t2(m, 1, 1)
    for i, j, a, b in itertools.product(range(nk), repeat=4):
        tot = _vec(m, i) + _vec(m, j) - _vec(m, a) - _vec(m, b)
        assert mask[i, j, a, b] == (not np.all(tot % dims == 0))


def _relabel_inputs(H, t1, t2, perm):
    """Move every k block to the label perm[k] (perm a group isomorphism)."""
    nk = len(perm)
    inv = np.argsort(perm)
    fock = H['fock'][inv]
    chol = H['chol'][inv][:, inv]
    t1r = t1[inv]
    t2r = t2[inv][:, inv][:, :, inv]
    return fock, chol, t1r, t2r


def test_residual_on_mesh_equals_relabelled_chain():
    """Z6 and Z2 x Z3 are isomorphic: the k-blocked residual of a 6-point chain and of
    the same Hamiltonian relabelled onto the 2 x 3 mesh agree block by block."""
    nk, o, v = 6, 1, 2
    rng = synth.rng_for(952, nk, o, v)
    H = synth.hamiltonian(nk, o, v, 2, rng, chol_sigma=0.2)
    t1, t2 = synth.random_amplitudes(nk, o, v, rng, 0.05, 0.05)
    h = kblock.KHam(H['fock'], H['chol'], o)
    r1, r2 = kblock.residual(h, kblock.t1_kt(t1, nk), kblock.t2_kt(t2, nk))
    perm = np.array([_crt(j) for j in range(6)])
    fock, chol, t1m, t2m = _relabel_inputs(H, t1, t2, perm)
    m = Mesh((2, 3, 1))
    hm = kblock.KHam(fock, chol, o, mesh=m)
    q1, q2 = kblock.residual(hm, kblock.t1_kt(t1m, m), kblock.t2_kt(t2m, m))
    inv = np.argsort(perm)
    e1 = r1.data.numpy()[inv]
    e2 = r2.data.numpy()[inv][:, inv][:, :, inv]
    sc = np.abs(e2).max()
    assert np.abs(q1.data.numpy() - e1).max() < 1e-13 * max(1, np.abs(e1).max())
    assert np.abs(q2.data.numpy() - e2).max() < 1e-13 * sc
    # a 1D relabelling by a map that is not a homomorphism changes the result
    bad = np.array([0, 1, 2, 3, 5, 4])
    fock_b, chol_b, t1b, t2b = _relabel_inputs(H, t1, t2, bad)
    hb = kblock.KHam(fock_b, chol_b, o, mesh=m)
    b1, b2 = kblock.residual(hb, kblock.t1_kt(t1b, m), kblock.t2_kt(t2b, m))
    assert np.abs(b2.data.numpy() - e2).max() > 1e-6 * sc


def test_kblock_matches_dense_on_noncyclic_mesh():
    """On the 2 x 2 mesh (not cyclic) the k-blocked residual and energy equal the dense
    collective-index CCSD built from the same Cholesky vectors."""
    m = Mesh((2, 2, 1))
    nk, o, v = 4, 1, 2
    rng = synth.rng_for(953, nk, o, v, extra=(2, 2, 1))
    H = synth.hamiltonian((2, 2), o, v, 3, rng, chol_sigma=0.2)
    t1, t2 = synth.random_amplitudes((2, 2), o, v, rng, 0.05, 0.05)
    h = kblock.KHam(H['fock'], H['chol'], o, mesh=m)
    T1, T2 = kblock.t1_kt(t1, m), kblock.t2_kt(t2, m)
    r1, r2 = kblock.residual(h, T1, T2)
    f = layout.dense_one_body(H['fock'], m, o, v)
    g = layout.dense_eri(H['chol'], m, o, v)
    hd = ccsd.DenseHam.from_numpy(f, g, nk * o)
    td = (torch.from_numpy(layout.dense_t1(t1, m, o, v)), torch.from_numpy(layout.dense_t2(t2, m, o, v)))
    d1, d2 = ccsd.residual(td[0], td[1], hd)
    assert np.abs(layout.dense_t1(r1.data.numpy(), m, o, v) - d1.numpy()).max() < 1e-14
    assert np.abs(layout.dense_t2(r2.data.numpy(), m, o, v) - d2.numpy()).max() < 1e-13
    # the dense residual has no weight on momentum-violating doubles
    assert np.abs(d2.numpy()[layout.forbidden_mask_t2(m, o, v)]).max() < 1e-15
    e_k = complex(kblock.energy(h, T1, T2))
    e_d = complex(ccsd.energy(td[0], td[1], hd))
    assert abs(e_k - e_d) < 1e-14


def _momentum_from_commutator(fock, dip):
    """p = i [f, r] per k and axis: the momentum matrix of an independent-particle
    Hamiltonian f (Heisenberg equation of motion of the position operator)."""
    return np.stack([np.stack([1j * (fock[k] @ dip[x][k] - dip[x][k] @ fock[k]) for k in range(fock.shape[0])])
                     for x in range(3)])


def test_velocity_gauge_sum_rule_independent_particles():
    """Without two-electron terms the CCSD state is the determinant.  With momentum
    matrices p = i[f, r] (p_ia = -i D r_ia, D = e_a - e_i) the velocity-gauge form
    (a_p(w) - a_p(0)) / w^2 is, in closed form, sum_ia (D / w) [A / (D - w) - B / (D + w)]
    with A = r^X_ia r^Y_ai, B = r^Y_ia r^X_ai; it differs from the length-gauge sum
    sum_ia [A / (D - w) + B / (D + w)] by sum_ia (A - B) / w, which vanishes when the
    position matrices commute (real symmetric r): then the two gauges agree."""
    m = Mesh((2, 1, 1))
    nk, o, v = 2, 2, 3
    rng = synth.rng_for(954, nk, o, v)
    H = synth.hamiltonian(nk, o, v, 2, rng)
    f = layout.dense_one_body(H['fock'], m, o, v)
    hd = ccsd.DenseHam.from_numpy(f, np.zeros((nk * (o + v),) * 4, dtype=np.complex128), nk * o)
    t = (torch.zeros(nk * o, nk * v, dtype=torch.complex128), torch.zeros((nk * o,) * 2 + (nk * v,) * 2,
                                                                           dtype=torch.complex128))
    lam, _, _ = response.solve_lambda(t, hd)
    eps = np.real(np.diag(f))
    N_O, N = nk * o, nk * (o + v)
    omegas = [0.05, 0.2]
    for real in (False, True):
        dip = H['dip'].real.astype(np.complex128) if real else H['dip']
        mom = _momentum_from_commutator(H['fock'], dip)
        rs = [torch.from_numpy(layout.dense_one_body(dip[x], m, o, v)) for x in range(3)]
        ps = [torch.from_numpy(layout.dense_one_body(mom[x], m, o, v)) for x in range(3)]
        a_lg, _ = response.polarizability(t, lam, rs, omegas, hd, nk=m)
        a_vg = response.polarizability_velocity(t, lam, ps, omegas, hd, nk=m)
        R = [r.numpy() for r in rs]
        lg = np.zeros_like(a_lg)
        vg = np.zeros_like(a_lg)
        for iw, w in enumerate(omegas):
            for X in range(3):
                for Y in range(3):
                    for i in range(N_O):
                        for a in range(N_O, N):
                            D = eps[a] - eps[i]
                            A, B = R[X][i, a] * R[Y][a, i], R[Y][i, a] * R[X][a, i]
                            lg[iw, X, Y] += (A / (D - w) + B / (D + w)) / nk
                            vg[iw, X, Y] += (D / w) * (A / (D - w) - B / (D + w)) / nk
        sc = np.abs(lg).max()
        assert np.abs(a_lg - lg).max() < 1e-10 * sc
        assert np.abs(a_vg - vg).max() < 1e-9 * sc
        if real:
            assert np.abs(a_vg - a_lg).max() < 1e-9 * sc
        else:
            assert np.abs(a_vg - a_lg).max() > 1e-3 * sc


def test_velocity_gauge_two_electron_exact():
    """Two electrons: LR-CCSD is exact, so the velocity-gauge polarizability equals
    (S(w) - S(0)) / w^2 with S the full-CI sum over states of the momentum operator."""
    nk, o, v = 1, 2, 4
    rng = synth.rng_for(955, nk, o, v)
    H = synth.hamiltonian(nk, o, v, 6, rng, chol_sigma=0.15)
    f = layout.dense_one_body(H['fock'], nk, o, v)
    g = layout.dense_eri(H['chol'], nk, o, v)
    hd = ccsd.DenseHam.from_numpy(f, g, nk * o)
    from oracle import solvers
    t1, t2, _, _ = solvers.solve_ccsd(hd, tol=1e-13)
    lam, _, _ = response.solve_lambda((t1, t2), hd)
    # momentum matrices of a real basis: i times a real antisymmetric matrix (Hermitian)
    d = synth.hamiltonian(nk, o, v, 6, synth.rng_for(956, nk, o, v))['dip'].imag
    mom = 1j * (d - np.swapaxes(d, -1, -2))
    ps = [torch.from_numpy(layout.dense_one_body(mom[x], nk, o, v)) for x in range(3)]
    omegas = [0.1, 0.3]
    a_vg = response.polarizability_velocity((t1, t2), lam, ps, omegas, hd, nk=nk)
    P = [p.numpy() for p in ps]
    for X in range(3):
        for Y in range(3):
            s = fockspace.fci_polarizability(f, g, nk * o, P[X], P[Y], [0.0] + omegas)[0]
            ref = [(s[i + 1] - s[0]) / w ** 2 for i, w in enumerate(omegas)]
            assert np.abs(a_vg[:, X, Y] - np.array(ref)).max() < 1e-8 * max(1.0, np.abs(ref).max())
    assert np.abs(a_vg).max() > 0.1
