"""Pins of the CPU oracle against facts that do not come from the oracle itself:
the determinant-space definition of every CC quantity, the exact two-electron
(CCSD = FCI) sum-over-states polarizability, finite-field derivatives, integral
symmetries and the momentum-conservation zero pattern (Sec. II.A, Eq. momentum)."""
import numpy as np
import pytest
import torch

import synth
from oracle import ccsd, fockspace, layout, response, solvers
from tests.oracle_cases import dipoles, random_direction, tiny_system


@pytest.mark.parametrize("nk,o,v", [(1, 2, 3), (1, 3, 3), (2, 2, 2), (3, 1, 2)])
def test_eri_symmetries(nk, o, v):
    s = tiny_system(nk, o, v)
    g = s['g']
    # Hermiticity <pq||rs>* = <rs||pq> (the assumption of Sec. II.C, exact here)
    assert np.abs(np.conj(g) - g.transpose(2, 3, 0, 1)).max() < 1e-15
    # antisymmetry
    assert np.abs(g + g.transpose(1, 0, 2, 3)).max() < 1e-15
    assert np.abs(g + g.transpose(0, 1, 3, 2)).max() < 1e-15
    # momentum conservation: k_p + k_q = k_r + k_s (Eq. momentum)
    idx = layout.orbital_index(nk, o, v)
    kof = np.empty(nk * (o + v), dtype=int)
    for k in range(nk):
        kof[idx[k]] = k
    tot = (kof[:, None, None, None] + kof[None, :, None, None]
           - kof[None, None, :, None] - kof[None, None, None, :]) % nk
    assert np.abs(g[tot != 0]).max(initial=0.0) == 0.0
    assert np.abs(g[tot == 0]).max() > 1e-3


@pytest.mark.parametrize("nk,o,v,nc", [(1, 2, 3, 0.0), (1, 3, 4, 0.08), (2, 2, 2, 0.08), (3, 1, 2, 0.0), (3, 2, 2, 0.05)])
def test_residual_and_energy_vs_determinants(nk, o, v, nc):
    """Omega_mu = <mu|e^-T H e^T|HF> and E_corr, complex integrals, non-canonical f."""
    s = tiny_system(nk, o, v, noncanonical=nc, tscale=0.1)
    t1, t2 = s['t']
    r1, r2 = ccsd.residual(t1, t2, s['h'])
    e = complex(ccsd.energy(t1, t2, s['h']))
    b1, b2, be = fockspace.brute_residual(s['f'], s['g'], nk * o, t1.numpy(), t2.numpy())
    assert np.abs(r1.numpy() - b1).max() < 1e-13 * max(1, np.abs(b1).max())
    assert np.abs(r2.numpy() - b2).max() < 1e-13 * max(1, np.abs(b2).max())
    assert abs(e - be) < 1e-13


@pytest.mark.parametrize("nk,o,v", [(1, 2, 4), (2, 2, 2)])
def test_xi_vs_determinants(nk, o, v):
    s = tiny_system(nk, o, v, tscale=0.1)
    op = dipoles(s)[1]
    x1, x2 = response.xi(s['t'], op, s['h'])
    b1, b2 = fockspace.brute_xi(s['f'], s['g'], nk * o, s['t'][0].numpy(), s['t'][1].numpy(), op.numpy())
    assert np.abs(x1.numpy() - b1).max() < 1e-13
    assert np.abs(x2.numpy() - b2).max() < 1e-13


def _brute_jvp(s, x):
    """<mu| e^-T [H, X] e^T |HF> in determinant space."""
    fs = fockspace.FockSpace(s['f'].shape[0], s['h'].no)
    t1, t2 = (a.numpy() for a in s['t'])
    h1 = fockspace.core_hamiltonian(s['f'], s['g'], s['h'].no)
    psi = fs.exp_T(t1, t2, fs.hf_vector(), +1)
    a = fs.apply_H(h1, s['g'], fs.apply_T(x[0].numpy(), x[1].numpy(), psi))
    b = fs.apply_T(x[0].numpy(), x[1].numpy(), fs.apply_H(h1, s['g'], psi))
    chi = fs.exp_T(t1, t2, a - b, -1)
    return fs.project(chi, s['h'].no, s['h'].nv)


@pytest.mark.parametrize("nk,o,v,nc", [(1, 2, 4, 0.05), (3, 1, 2, 0.0), (2, 2, 2, 0.05)])
def test_sigma_vs_commutator(nk, o, v, nc):
    """Stencil JVP equals the commutator definition A x = <mu|e^-T [H, X] e^T|HF>."""
    s = tiny_system(nk, o, v, noncanonical=nc, tscale=0.1)
    x = random_direction(s)
    s1, s2 = response.sigma(s['t'], x, s['h'])
    b1, b2 = _brute_jvp(s, x)
    sc = max(np.abs(b1).max(), np.abs(b2).max())
    assert np.abs(s1.numpy() - b1).max() < 1e-12 * sc
    assert np.abs(s2.numpy() - b2).max() < 1e-12 * sc


def test_sigma_zero_pattern_and_linearity():
    """sigma of a momentum-conserving X vanishes on forbidden blocks; sigma is linear."""
    nk, o, v = 3, 2, 3
    s = tiny_system(nk, o, v, tscale=0.05)
    x = random_direction(s)
    y = random_direction(s)
    sx = response.sigma(s['t'], x, s['h'])
    sy = response.sigma(s['t'], y, s['h'])
    sxy = response.sigma(s['t'], (x[0] + 2j * y[0], x[1] + 2j * y[1]), s['h'])
    mask = layout.forbidden_mask_t2(nk, o, v)
    assert float(sx[1].abs().max()) > 1e-2
    assert np.abs(sx[1].numpy()[mask]).max() <= 1e-14 * float(sx[1].abs().max())
    for k in range(2):
        assert float((sxy[k] - sx[k] - 2j * sy[k]).abs().max()) < 1e-12 * float(sxy[k].abs().max())


def test_dense_jacobian_solve_matches_gmres():
    """(A - w) t = -xi solved densely on the explicit Jacobian and by GMRES."""
    s = tiny_system(1, 2, 4, tscale=0.05)
    A = response.dense_jacobian(s['t'], s['h'])
    op = dipoles(s)[0]
    xi = response.xi(s['t'], op, s['h'])
    singles, doubles = response.antisym_basis(s['h'].no, s['h'].nv)
    w = 0.0656
    dense = np.linalg.solve(A - w * np.eye(A.shape[0]), -response.to_independent(xi, singles, doubles))
    it, rel, _ = response.solve_response(s['t'], s['h'], (-xi[0], -xi[1]), w)
    assert rel < 1e-12
    assert np.abs(response.to_independent(it, singles, doubles) - dense).max() < 1e-11


def test_transpose_product_dot_identity():
    """<z, A x> = <A^T z, x> (bilinear, no conjugation), A x from the stencil."""
    s = tiny_system(2, 2, 2, tscale=0.08)
    x = random_direction(s)
    z = random_direction(s)
    ax = response.sigma(s['t'], x, s['h'])
    atz = response.transpose_product(s['t'], z, s['h'])
    lhs = complex(response.pairing(z, ax))
    # atz doubles carry a factor 4 (same scale as A), so the pairing weight is 1/4
    rhs = complex((atz[0] * x[0]).sum() + 0.25 * (atz[1] * x[1]).sum())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("nk,o,v", [(1, 2, 4), (2, 1, 3)])
def test_alpha_equals_two_electron_sum_over_states(nk, o, v):
    """Two electrons: CCSD is exact, so the LR-CCSD alpha equals the exact
    sum-over-states polarizability (per cell), including the complex Hermitian
    off-diagonal elements at finite frequency."""
    s = tiny_system(nk, o, v, naux=8, seed=11)
    t1, t2, E, _ = solvers.solve_ccsd(s['h'])
    t = (t1, t2)
    lam, rel, _ = response.solve_lambda(t, s['h'])
    assert rel < 1e-12
    ops = dipoles(s)
    oms = [0.0, 0.0656]
    al, _ = response.polarizability(t, lam, ops, oms, s['h'], nk=nk)
    ref = np.zeros_like(al)
    for X in range(3):
        for Y in range(3):
            a, e0, exc = fockspace.fci_polarizability(s['f'], s['g'], nk * o, ops[X].numpy(), ops[Y].numpy(), oms)
            ref[:, X, Y] = a / nk
    assert abs(E - e0) < 1e-12
    assert np.abs(al - ref).max() < 1e-11
    # physical sanity (cf. every polarizability table): alpha_ii > 0 and grows with omega
    for X in range(3):
        assert al[0, X, X].real > 0 and al[1, X, X].real > al[0, X, X].real


def test_static_alpha_equals_finite_field():
    """alpha_XY(0) = -d2 E_corr / dF_X dF_Y with f -> f - F mu and CCSD re-solved
    (four electrons: not exact, so this pins lambda, eta and F independently)."""
    nk, o, v = 1, 4, 5
    s = tiny_system(nk, o, v, naux=8, seed=3, chol_sigma=0.12)
    h = s['h']
    ops = dipoles(s)
    t1, t2, E0, _ = solvers.solve_ccsd(h)
    lam, _, _ = response.solve_lambda((t1, t2), h)
    al, _ = response.polarizability((t1, t2), lam, ops, [0.0], h, nk=nk)

    def e_of(fx, fy, X, Y, guess):
        hf = h.with_fock(h.f - fx * ops[X] - fy * ops[Y])
        a, b, E, _ = solvers.solve_ccsd(hf, tol=1e-13, t_init=guess)
        return E

    hstep = 2e-3
    g = (t1, t2)
    # diagonal element: 5-point second derivative
    X = 2
    vals = {k: e_of(k * hstep, 0.0, X, X, g) for k in (-2, -1, 0, 1, 2)}
    d2 = (-vals[-2] + 16 * vals[-1] - 30 * vals[0] + 16 * vals[1] - vals[2]) / (12 * hstep ** 2)
    assert abs(-d2.real - al[0, X, X].real) < 2e-7 * max(1.0, abs(al[0, X, X]))
    # mixed element by 4-corner differences (real part; the static alpha is Hermitian)
    X, Y = 0, 1
    c = {(a, b): e_of(a * hstep, b * hstep, X, Y, g) for a in (-1, 1) for b in (-1, 1)}
    dxy = (c[(1, 1)] - c[(1, -1)] - c[(-1, 1)] + c[(-1, -1)]) / (4 * hstep ** 2)
    assert abs(-dxy.real - al[0, X, Y].real) < 2e-6 * max(1.0, abs(al[0, X, Y]))


def test_paper_rhs_equals_xi_of_transposed_operator():
    """Eq. rhs (crystal normalisation) is xi^X with X replaced by its transpose
    (= X* for a Hermitian X): the paper's X_IA / X*_KC / X_CA / X_IK slots are the
    transposed matrix elements of the standard <mu|e^-T X e^T|HF>."""
    s = tiny_system(2, 2, 3, tscale=0.1)
    t1, t2 = s['t']
    X = dipoles(s)[2]
    no = s['h'].no
    o, v = slice(0, no), slice(no, None)
    Xs = X.conj()
    e = torch.einsum
    r1 = (X[o, v] + e('ikac,kc->ia', t2, Xs[o, v]) - e('ic,ka,kc->ia', t1, t1, Xs[o, v])
          + e('ic,ca->ia', t1, X[v, v]) - e('ka,ik->ia', t1, X[o, o]))
    inner_ij = X[o, o] + e('ic,kc->ik', t1, Xs[o, v])
    a = e('ik,kjab->ijab', inner_ij, t2)
    inner_ab = X[v, v] - e('kb,kc->cb', t1, Xs[o, v])
    b = e('cb,ijac->ijab', inner_ab, t2)
    r2 = -(a - a.transpose(0, 1)) + (b - b.transpose(2, 3))
    x1, x2 = response.xi((t1, t2), X.T.contiguous(), s['h'])
    assert float((r1 - x1).abs().max()) < 1e-14
    assert float((r2 - x2).abs().max()) < 1e-14
    # for a real symmetric operator the two readings coincide
    Xr = X.real.to(torch.complex128)
    y1, y2 = response.xi((t1, t2), Xr, s['h'])
    z1, z2 = response.xi((t1, t2), Xr.T.contiguous(), s['h'])
    assert float((y1 - z1).abs().max()) < 1e-15 and float((y2 - z2).abs().max()) < 1e-15


@pytest.mark.parametrize("nk,o,v", [(1, 2, 4), (2, 1, 3)])
def test_excitation_energies_equal_two_electron_spectrum(nk, o, v):
    """Two electrons: EOM-CCSD is exact, so the eigenvalues of the CCSD Jacobian on the
    momentum-conserving excitations are excitation energies of the exact spectrum (all of
    them at Nk = 1, where singles and doubles span every excited determinant)."""
    s = tiny_system(nk, o, v, naux=8, seed=12)
    t1, t2, E, _ = solvers.solve_ccsd(s['h'])
    w = response.excitation_energies((t1, t2), s['h'], nk=nk)
    ops = dipoles(s)
    _, e0, exc = fockspace.fci_polarizability(s['f'], s['g'], nk * o, ops[0].numpy(), ops[0].numpy(), [0.0])
    assert np.abs(w.imag).max() < 1e-9
    for x in w.real:
        assert np.abs(exc - x).min() < 1e-10
    if nk == 1:
        assert len(w) == len(exc)
        assert np.abs(np.sort(w.real) - np.sort(exc)).max() < 1e-10


@pytest.mark.parametrize("nk,o,v", [(1, 2, 3), (2, 1, 2)])
def test_residual_degree_in_singles_and_doubles(nk, o, v):
    """The CCSD residual (Eqs. t1, t2), evaluated in determinant space, is a polynomial of degree 4 in
    the amplitudes but of degree 2 along the doubles alone: along T + e y the 5th differences vanish,
    and along a pure-doubles y the 3rd do.  So A(T) = dOmega/dT is cubic in T (the F stencil with the
    unshifted product and three shifted points is exact) and linear in t2 at fixed t1 (the blocks that
    depend on t2 alone change by e B(y) along y)."""
    s = tiny_system(nk, o, v, tscale=0.1, noncanonical=0.05)
    t1, t2 = (a.numpy() for a in s['t'])
    y1, y2 = (a.numpy() for a in random_direction(s, 0.5))

    def differences(d1, d2, h=0.5, n=6):
        vals = []
        for k in range(n):
            b1, b2, _ = fockspace.brute_residual(s['f'], s['g'], nk * o, t1 + k * h * d1, t2 + k * h * d2)
            vals.append(np.concatenate([b1.ravel(), b2.ravel()]))
        out = []
        for _ in range(n):
            out.append(np.abs(vals[0]).max())
            vals = [vals[i + 1] - vals[i] for i in range(len(vals) - 1)]
        return out

    gen, dbl, sgl = differences(y1, y2), differences(0 * y1, y2), differences(y1, 0 * y2)
    print(f"nk={nk}: general {gen}\n  doubles {dbl}\n  singles {sgl}", flush=True)
    assert gen[4] > 1e-4 and gen[5] < 1e-10 * gen[4]
    assert sgl[4] > 1e-4 and sgl[5] < 1e-10 * sgl[4]
    assert dbl[2] > 1e-4 and dbl[3] < 1e-10 * dbl[2] and dbl[4] < 1e-10 * dbl[2]
