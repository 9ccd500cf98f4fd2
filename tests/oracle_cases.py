"""Small seeded systems shared by the oracle pin tests (inputs only)."""
import numpy as np
import torch

import synth
from oracle import layout, ccsd


def tiny_system(nk, o, v, naux=6, seed=7, chol_sigma=0.15, noncanonical=0.0, tscale=0.0):
    rng = synth.rng_for(900 + seed, nk, o, v)
    H = synth.hamiltonian(nk, o, v, naux, rng, band_shift=True, chol_sigma=chol_sigma)
    fock = H['fock'].copy()
    if noncanonical:
        for k in range(nk):
            a = noncanonical * (rng.standard_normal((o + v, o + v)) + 1j * rng.standard_normal((o + v, o + v)))
            fock[k] += (a + a.conj().T) / 2
    f = layout.dense_one_body(fock, nk, o, v)
    g = layout.dense_eri(H['chol'], nk, o, v)
    h = ccsd.DenseHam.from_numpy(f, g, nk * o)
    out = dict(H=H, fock=fock, f=f, g=g, h=h, nk=nk, o=o, v=v, rng=rng)
    if tscale:
        t1k, t2k = synth.random_amplitudes(nk, o, v, rng, tscale, tscale)
        out['t'] = (torch.from_numpy(layout.dense_t1(t1k, nk, o, v)),
                    torch.from_numpy(layout.dense_t2(t2k, nk, o, v)))
        out['tk'] = (t1k, t2k)
    return out


def random_direction(s, scale=1.0):
    x1k, x2k = synth.random_vectors(1, s['nk'], s['o'], s['v'], s['rng'], scale, scale)
    return (torch.from_numpy(layout.dense_t1(x1k[0], s['nk'], s['o'], s['v'])),
            torch.from_numpy(layout.dense_t2(x2k[0], s['nk'], s['o'], s['v'])))


def dipoles(s):
    return [torch.from_numpy(layout.dense_one_body(s['H']['dip'][x], s['nk'], s['o'], s['v']))
            for x in range(3)]
