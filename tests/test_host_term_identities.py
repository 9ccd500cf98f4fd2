"""The exact regroupings of Eq. tx2 terms that the library's sigma program uses, checked on random
tensors with the symmetries they rely on (one k point; the k-blocked sums are the same sums split
by momentum).  Each identity is stated where the sigma program applies it."""
import numpy as np
import pytest

O, V = 3, 4


def _rng(seed):
    return np.random.default_rng(seed)


def _c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _oovv_antisym(rng):
    """<mn||ef>: antisymmetric in (m, n) and in (e, f)."""
    g = _c(rng, O, O, V, V)
    g = g - g.transpose(1, 0, 2, 3)
    return g - g.transpose(0, 1, 3, 2)


def _pab(z):
    return z - z.transpose(0, 1, 3, 2)


def _pij(z):
    return z - z.transpose(1, 0, 2, 3)


def _d1(x, t):
    """x1 t1 part of d tau: x_ia t_jb + t_ia x_jb - x_ib t_ja - t_ib x_ja."""
    a = np.einsum('ia,jb->ijab', x, t) + np.einsum('ia,jb->ijab', t, x)
    return a - a.transpose(0, 1, 3, 2)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dfae_doubles_part_regrouped(seed):
    """-(x2 + dtau) <mn||ef> / 4 = -dtau <mn||ef> / 2 + (x_ma Fg_me + t_ma dFme_me) / 2."""
    rng = _rng(seed)
    g = _oovv_antisym(rng)
    x1, t1 = _c(rng, O, V), _c(rng, O, V)
    x2 = _pij(_pab(_c(rng, O, O, V, V)))
    dtau = x2 + _d1(x1, t1)
    lhs = -0.25 * np.einsum('mnaf,mnef->ae', x2 + dtau, g)
    fg = np.einsum('nf,mnef->me', t1, g)
    dfme = np.einsum('nf,mnef->me', x1, g)
    rhs = (-0.5 * np.einsum('mnaf,mnef->ae', dtau, g) + 0.5 * np.einsum('ma,me->ae', x1, fg)
           + 0.5 * np.einsum('ma,me->ae', t1, dfme))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_dfmi_doubles_part_regrouped(seed):
    """(x2 + dtau) <mn||ef> / 4 = dtau <mn||ef> / 2 - (x_ie Fg_me + t_ie dFme_me) / 2."""
    rng = _rng(seed)
    g = _oovv_antisym(rng)
    x1, t1 = _c(rng, O, V), _c(rng, O, V)
    x2 = _pij(_pab(_c(rng, O, O, V, V)))
    dtau = x2 + _d1(x1, t1)
    lhs = 0.25 * np.einsum('inef,mnef->mi', x2 + dtau, g)
    fg = np.einsum('nf,mnef->me', t1, g)
    dfme = np.einsum('nf,mnef->me', x1, g)
    rhs = (0.5 * np.einsum('inef,mnef->mi', dtau, g) - 0.5 * np.einsum('ie,me->mi', x1, fg)
           - 0.5 * np.einsum('ie,me->mi', t1, dfme))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()


@pytest.mark.parametrize("seed", [7, 8])
def test_hole_hole_tau_term_regrouped(seed):
    """Under P(ij)P(ab): Zmn t2 / 16 + Vx tau / 8 = (Zmn + 2 Vx) t2 / 16 - (-Vx t1 / 4)_ijan t_nb,
    tau = t2 + t_ma t_nb - t_mb t_na."""
    rng = _rng(seed)
    zmn, vx = _c(rng, O, O, O, O), _c(rng, O, O, O, O)
    t1 = _c(rng, O, V)
    t2 = _pij(_pab(_c(rng, O, O, V, V)))
    tau = t2 + np.einsum('ma,nb->mnab', t1, t1) - np.einsum('mb,na->mnab', t1, t1)
    z_old = np.einsum('ijmn,mnab->ijab', zmn, t2) / 16 + np.einsum('ijmn,mnab->ijab', vx, tau) / 8
    yx = -0.25 * np.einsum('ijmn,ma->ijan', vx, t1)
    z_new = np.einsum('ijmn,mnab->ijab', zmn + 2 * vx, t2) / 16 - np.einsum('ijan,nb->ijab', yx, t1)
    a, b = _pij(_pab(z_old)), _pij(_pab(z_new))
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()
    assert np.abs(z_old - z_new).max() > 1e-3 * np.abs(z_old).max()   # equal only after P(ij)P(ab)


@pytest.mark.parametrize("seed", [9, 10])
def test_x1_terms_summed_once(seed):
    """Under P(ij)P(ab): -S x_nb - Yp x_nb - Q/4 x_mb = -(S + Yp + Q/4) x_nb; x_ie H_abej + R_iabf x_jf =
    x_ie (H_abej - R_jabe); -G2_ijbm x_ma - 1/2 <mb||ij> x_ma = -(G2 + 1/2 <mb||ij>)_ijbm x_ma."""
    rng = _rng(seed)
    x1 = _c(rng, O, V)
    s_, yp, q = _c(rng, O, O, V, O), _c(rng, O, O, V, O), _c(rng, O, O, V, O)
    old = (-np.einsum('ijan,nb->ijab', s_, x1) - np.einsum('ijan,nb->ijab', yp, x1)
           - 0.25 * np.einsum('ijam,mb->ijab', q, x1))
    new = -np.einsum('ijan,nb->ijab', s_ + yp + 0.25 * q, x1)
    assert np.abs(old - new).max() < 1e-12 * np.abs(old).max()
    h, r = _c(rng, V, V, V, O), _c(rng, O, V, V, V)
    old = np.einsum('ie,abej->ijab', x1, h) + np.einsum('iabf,jf->ijab', r, x1)
    new = np.einsum('ie,abej->ijab', x1, h - r.transpose(1, 2, 3, 0))
    a, b = _pij(_pab(old)), _pij(_pab(new))
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()
    g2, ovoo = _c(rng, O, O, V, O), _c(rng, O, V, O, O)
    old = -np.einsum('ijbm,ma->ijab', g2, x1) - 0.5 * np.einsum('mbij,ma->ijab', ovoo, x1)
    new = -np.einsum('ijbm,ma->ijab', g2 + 0.5 * ovoo.transpose(2, 3, 1, 0), x1)
    assert np.abs(old - new).max() < 1e-12 * np.abs(old).max()
