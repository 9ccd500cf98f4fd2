"""Writes tests/golden/c2_alpha.json: the oracle's polarizability of the three-k
chain workload (Nk=3, nocc=4, nvir=20, Naux=72, band shift, Cholesky sigma 0.05),
alpha_XY(w) per cell for all axes at w in {0, 0.0656} a.u. (Eq. lrf, symmetric
form), with the CCSD ground state (Eqs. ene, t1, t2) converged by the oracle to
1e-12 and lambda (Eqs. l1, l2) and every response solve to 1e-12.

Only the oracle and the seeded input generators are used: the inputs are the
same draws the benchmark and the GPU test make for this workload
(synth.WORKLOADS['c2'], seed [1266, 2, 3, 4, 20]).  Dense collective-index tier;
about an hour on 8 host cores.

    python tests/golden/make_c2_alpha.py
"""
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ccsd, layout, response, solvers  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_alpha.json")


def main():
    w = synth.WORKLOADS["c2"]
    t0 = time.time()
    rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir)
    H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift, chol_sigma=w.chol_sigma)
    f = layout.dense_one_body(H["fock"], w.nk, w.nocc, w.nvir)
    g = layout.dense_eri(H["chol"], w.nk, w.nocc, w.nvir)
    h = ccsd.DenseHam.from_numpy(f, g, w.nk * w.nocc)
    t1, t2, E, nit = solvers.solve_ccsd(h, tol=1e-12)
    print(f"ccsd: E {E} in {nit} iterations ({time.time() - t0:.0f} s)", flush=True)
    lam, rel, nap = response.solve_lambda((t1, t2), h)
    print(f"lambda: rel {rel:.1e} after {nap} products ({time.time() - t0:.0f} s)", flush=True)
    ops = [torch.from_numpy(layout.dense_one_body(H["dip"][x], w.nk, w.nocc, w.nvir)) for x in range(3)]
    omegas = list(w.omegas)
    alpha, _ = response.polarizability((t1, t2), lam, ops, omegas, h, nk=w.nk)
    print(f"alpha done ({time.time() - t0:.0f} s)", flush=True)
    out = {
        "what": "oracle alpha_XY(omega) per cell (Eq. lrf, symmetric form), dense collective-index tier",
        "workload": {"nk": w.nk, "nocc": w.nocc, "nvir": w.nvir, "naux": w.naux, "band_shift": w.band_shift,
                     "chol_sigma": w.chol_sigma, "seed": [1266, w.cfg_id, w.nk, w.nocc, w.nvir]},
        "omegas": omegas,
        "ccsd_energy_per_cell": [float(np.real(E)) / w.nk, float(np.imag(E)) / w.nk],
        "alpha_re": alpha.real.tolist(),
        "alpha_im": alpha.imag.tolist(),
        "tolerances": {"ccsd": 1e-12, "lambda": 1e-12, "response": 1e-12},
        "seconds": time.time() - t0,
        "threads": torch.get_num_threads(),
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
