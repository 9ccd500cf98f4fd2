"""Benchmark of the k-blocked LR-CCSD sigma path on one MI355X.

A step is one application of the CCSD Jacobian (the sigma vector of the
perturbed-amplitude equations) to the whole batch of right-hand sides of the
workload, with inputs resident in HBM.  The default workload is the batched
one: Nk=5, nocc=8, nvir=40, Naux=144, 3 axes x +-omega x 8 frequencies = 48
right-hand sides in one launch, computed on the matrix cores in complex64
(split into real fp32 MFMA products).  The FP64 form of the same batch is
timed beside it.  Then the device CCSD ground state of the same Hamiltonian and
the time to converged alpha(omega) for all 48 right-hand sides, mixed and FP64
(--no-alpha skips it; --alpha-modes 2,3 repeats both solves in other ladder
modes).  The sigma is also timed with the ladder integral blocks stored (ladder
mode 2) and built one momentum class at a time (mode 3).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sigma-vector TFLOP/s + s to converged α(ω), mixed-batched vs FP64, 1 GPU"

# HBM traffic of the complex64 ladder launches of one application on the batched workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE), each scaled by the counter's reading for a plain
# 2 GiB copy (fetch x2.0, write x1.0).  Valid only for the ladder path and kernel sources it was
# measured on.
LADDER_TRAFFIC = {  # ladder path -> measured HBM bytes per application of the complex64 sigma
    3: {"workload": "c3", "sources_sha256": "27b805843d1d6dd5d287c163d32cdadf2b8a817b279502c7d141fb47a5640af4",
        "bytes": 40.6e9},
    1: {"workload": "c3", "sources_sha256": "984e5f970a1f2d74bea898efacb6b789c5a66e58c32d231fc99c73581dd474cb",
        "bytes": 188.6e9},
}


LADDER_PATH_TEXT = {1: "ladder integrals rebuilt in LDS from the Cholesky vectors",
                    2: "ladder integral blocks stored for the unique momentum pairs",
                    3: "ladder integral blocks built from the Cholesky vectors one momentum class at a time "
                       "in every application"}
LADDER_KERNEL = {1: "ladder_kernel_pipe (one launch, integrals rebuilt in LDS)",
                 2: "gemm_kernel<..., 1, ...> over the stored blocks (one launch)",
                 3: "gemm_kernel<..., 1, ...> over the class-built blocks (one launch per momentum class)"}


def ladder_sources_sha(path):
    """sha256 of the kernel sources of a ladder path: the ladder kernels (path 1) or the GEMM
    kernel (paths 2 and 3), with the shared header."""
    import hashlib
    h = hashlib.sha256()
    for f in ("ladder.hip" if path == 1 else "gemm.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2508_01266_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


PEAK = {"f32": 157.3, "f64": 78.6}          # MI355X dense matrix-core TFLOP/s


def sigma_alg_flops(nk, o, v):
    """Algorithmic real flops of one sigma for one right-hand side: 8 per complex
    multiply-add over full index ranges of the ladder (Nk^4 o^2 v^4), ring and
    t1/tau dressing (2 Nk^4 o^3 v^3), hole-hole terms (3 Nk^4 o^4 v^2) and the
    remaining one- and two-index terms (4 Nk^3 (o^2 v^3 + o^3 v^2))."""
    return 8.0 * nk ** 4 * (o ** 2 * v ** 4 + 2 * o ** 3 * v ** 3 + 3 * o ** 4 * v ** 2) \
        + 32.0 * nk ** 3 * (o ** 2 * v ** 3 + o ** 3 * v ** 2)


def ladder_alg_flops(nk, o, v):
    return 8.0 * nk ** 4 * o ** 2 * v ** 4


def ladder_unique_flops(nk, o, v, nrhs):
    """The ladder's own work on a 1D chain: 8 real flops per complex multiply-add over the
    unique index pairs only.  The ladder input (dtau) and output are antisymmetric in
    (ki,i) <-> (kj,j), in (ka,a) <-> (kb,b) and in (ke,e) <-> (kf,f), so its independent
    products are unique rows (ki,i) < (kj,j) x unique outputs (ka,a) < (kb,b) x unique inputs
    (ke,e) < (kf,f), over momentum-conserving blocks (kb = ki+kj-ka, kf = ki+kj-ke).  The
    in-LDS rebuild of the integrals and tile padding are excluded (they are overhead)."""
    pairs_o = o * (o - 1) // 2
    total = 0
    for ki in range(nk):
        for kj in range(ki, nk):
            rows = nrhs * (o * o if ki < kj else pairs_o)
            K = (ki + kj) % nk
            uniq = 0
            for ka in range(nk):
                kb = (K - ka) % nk
                uniq += v * v if ka < kb else (v * (v - 1) // 2 if ka == kb else 0)
            total += rows * uniq * uniq
    return 8.0 * total


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload_inputs(name):
    import numpy as np
    import synth
    w = synth.WORKLOADS[name]
    rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir)
    H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift, chol_sigma=w.chol_sigma)
    # synthetic amplitudes with the structure (antisymmetry, momentum) of CCSD ones
    t1, t2 = synth.random_amplitudes(w.nk, w.nocc, w.nvir, rng, 0.02, 0.02)
    pairs = synth.omega_grid(w)
    nrhs = 3 * len(pairs)
    x1, x2 = synth.random_vectors(nrhs, w.nk, w.nocc, w.nvir, rng, 0.1, 0.1)
    omega = np.array([s * om for _ in range(3) for (om, s) in pairs])
    return w, H, t1, t2 * w.nk, x1, x2 * w.nk, omega


def time_sigma(ctx, x1, x2, y1, y2, om, prec, steps, warmup, torch):
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(warmup):
        ctx.apply_sigma_dev(x1, x2, y1, y2, om, prec, stream)
    torch.cuda.synchronize()
    ctx.read_profile()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.apply_sigma_dev(x1, x2, y1, y2, om, prec, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_profiling(False)
    prof = ctx.read_profile()
    # per application: seconds of the ladder products (one launch with the integrals rebuilt in
    # LDS or stored, one per momentum class when the blocks are built by class), launches, and
    # seconds of the class builds of the blocks
    return ((t1 - t0) / steps, prof["ladder"][0] / 1e3 / steps, prof["ladder"][1] / steps,
            prof["ladder_build"][0] / 1e3 / steps)


def mesh_sigma(lr, torch, steps, mesh=(2, 2, 2), nocc=8, nvir=40, naux=144, nfreq=2):
    """Sigma on a 3D k mesh (n0 x n1 x n2 Monkhorst-Pack points, momenta added componentwise):
    the batched workload's orbital sizes on the 2 x 2 x 2 mesh, 3 axes x +-omega x nfreq
    right-hand sides, complex64 and complex128, integrals rebuilt in LDS."""
    import numpy as np
    import synth
    nk = int(np.prod(mesh))
    rng = synth.rng_for(6, nk, nocc, nvir, extra=mesh)
    sig = 0.05 * ((12 * 48 ** 0.5) / (nvir * (naux / nk) ** 0.5)) ** 0.5
    H = synth.hamiltonian(mesh, nocc, nvir, naux, rng, chol_sigma=sig)
    t1, t2 = synth.random_amplitudes(mesh, nocc, nvir, rng, 0.02, 0.02)
    R = 6 * nfreq
    x1, x2 = synth.random_vectors(R, mesh, nocc, nvir, rng, 0.1, 0.1)
    om = np.array([s * 0.05 * (j + 1) for _ in range(3) for j in range(nfreq) for s in (1, -1)])
    ctx = lr.Context(0)
    ctx.set_kmesh(*mesh)
    ctx.set_hamiltonian(nocc, H['fock'], H['chol'], H['dip'])
    ctx.set_amplitudes(t1, t2 * nk)
    dev = torch.device("cuda:0")
    X1, X2 = torch.from_numpy(x1).to(dev), torch.from_numpy(x2 * nk).to(dev)
    del x1, x2
    Y1, Y2 = torch.empty_like(X1), torch.empty_like(X2)
    OM = torch.from_numpy(om).to(dev)
    alg = R * sigma_alg_flops(nk, nocc, nvir)
    out = {"mesh": list(mesh), "nk": nk, "nocc": nocc, "nvir": nvir, "naux": naux, "nrhs": R,
           "algorithmic_flops_per_step": alg}
    for prec, name in ((lr.FP32, "f32"), (lr.FP64, "f64")):
        dt, lad, _, bld = time_sigma(ctx, X1, X2, Y1, Y2, OM, prec, steps, 1, torch)
        out[name] = {"ms_per_step": dt * 1e3, "value": alg / dt / 1e12, "ladder_ms_per_step": lad * 1e3,
                     "ladder_build_ms_per_step": bld * 1e3, "ladder_path": ctx.ladder_path(R, prec),
                     "ladder_executed_frac": ctx.ladder_flops(R, prec) / lad / 1e12 / PEAK[name]}
        log(f"mesh {mesh} sigma ({name}): {dt * 1e3:.1f} ms")
    ctx.close()
    return out


def velocity_gauge_alpha(lr, torch, tol):
    """Time to the velocity-gauge polarizability on the three-k chain workload (Nk=3, nocc=4,
    nvir=20, Naux=72): device CCSD, then one batched solve of the momentum response at
    0 and the two frequencies, mixed and FP64; the length-gauge alpha of the same system
    beside it."""
    import numpy as np
    import synth
    w = synth.WORKLOADS["c2"]
    rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir)
    H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift)
    d = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, synth.rng_for(7, w.nk, w.nocc, w.nvir))['dip'].imag
    mom = 1j * (d - np.swapaxes(d, -1, -2))
    ctx = lr.Context(0)
    ctx.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
    _, _, e, crep = ctx.solve_ccsd(tol=1e-10, max_iter=300)
    om = [x for x in w.omegas if x != 0.0]
    out = {"workload": "c2", "omegas": om, "ccsd_energy_per_cell": e}
    for name, prec in (("mixed", lr.FP32), ("fp64", lr.FP64)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a, rep = ctx.alpha_velocity_gauge(om, mom, tol=tol, precision=prec)
        out[name] = {"seconds": time.perf_counter() - t0, "alpha_vg_diag": [float(a[0, x, x].real) for x in range(3)],
                     "report": rep}
        log(f"velocity-gauge alpha ({name}) in {out[name]['seconds']:.2f} s")
    ctx.close()
    return out


def latency_small(lr, torch, reps=50):
    """Microseconds per sigma on the molecular-limit workload (Nk=1, nocc=4, nvir=12,
    Naux=48; 3 axes x (0, +w, -w) = 9 right-hand sides), eager launches vs one HIP
    graph replay per application."""
    import numpy as np
    import synth
    w = synth.WORKLOADS["c1"]
    rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir)
    H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift)
    t1, t2 = synth.random_amplitudes(w.nk, w.nocc, w.nvir, rng, 0.02, 0.02)
    x1, x2 = synth.random_vectors(9, w.nk, w.nocc, w.nvir, rng, 0.1, 0.1)
    om = np.array([0.0, 0.0656, -0.0656] * 3)
    ctx = lr.Context(0)
    ctx.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
    ctx.set_amplitudes(t1, t2)
    ctx.set_autotune(True)       # the first (untimed) applications pick the launch variants
    dev = torch.device("cuda:0")
    X1, X2 = torch.from_numpy(x1).to(dev), torch.from_numpy(x2).to(dev)
    Y1, Y2 = torch.empty_like(X1), torch.empty_like(X2)
    OM = torch.from_numpy(om).to(dev)
    st = torch.cuda.Stream()
    out = {}
    for mode in ("eager", "graph"):
        ctx.set_graphs(mode == "graph")
        for prec, pname in ((lr.FP64, "f64"), (lr.FP32, "f32")):
            for _ in range(3):
                ctx.apply_sigma_dev(X1, X2, Y1, Y2, OM, prec, st.cuda_stream)
            st.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.apply_sigma_dev(X1, X2, Y1, Y2, OM, prec, st.cuda_stream)
            st.synchronize()
            out[f"{mode}_{pname}_us"] = (time.perf_counter() - t0) / reps * 1e6
    ctx.close()
    return out


def uneven_batch(lr, torch, steps):
    """Uneven batch of twelve chains (Nk in {3,5,7,9}, 12 right-hand sides each): complex64
    sigma of every chain with the integrals rebuilt in LDS (ladder mode 1), one after another vs
    all together with one persistent ladder launch; then one after another in the default mode
    (each chain's context alone on the device: the class-built blocks of twelve resident chains
    would not fit beside their work tensors)."""
    import numpy as np
    import synth
    chains = synth.uneven_batch()
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    out = {}

    def make(i, w, mode):
        rng = synth.rng_for(w.cfg_id, w.nk, w.nocc, w.nvir, (i,))
        H = synth.hamiltonian(w.nk, w.nocc, w.nvir, w.naux, rng, band_shift=w.band_shift, chol_sigma=0.02)
        t1, t2 = synth.random_amplitudes(w.nk, w.nocc, w.nvir, rng, 0.02, 0.02)
        x1, x2 = synth.random_vectors(12, w.nk, w.nocc, w.nvir, rng, 0.1, 0.1)
        c = lr.Context(0)
        c.set_hamiltonian(w.nocc, H['fock'], H['chol'], H['dip'])
        c.set_ladder_mode(mode)
        c.set_amplitudes(t1, t2 * w.nk)
        X1, X2 = torch.from_numpy(x1).to(dev), torch.from_numpy(x2 * w.nk).to(dev)
        om = np.array([f for _ in range(3) for f in w.omegas])
        return c, X1, X2, torch.empty_like(X1), torch.empty_like(X2), torch.from_numpy(om).to(dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    alg = sum(12 * sigma_alg_flops(w.nk, w.nocc, w.nvir) for w in chains)
    ctxs, X1, X2, Y1, Y2, OM = [], [], [], [], [], []
    for i, w in enumerate(chains):
        c, x1, x2, y1, y2, om = make(i, w, 1)
        ctxs.append(c); X1.append(x1); X2.append(x2); Y1.append(y1); Y2.append(y2); OM.append(om)
        log(f"chain {i}: Nk={w.nk} nocc={w.nocc} nvir={w.nvir} Naux={w.naux}")
    g = lr.Group(ctxs)

    def seq():
        for i, c in enumerate(ctxs):
            c.apply_sigma_dev(X1[i], X2[i], Y1[i], Y2[i], OM[i], lr.FP32, st)

    def grp():
        g.apply_sigma_dev(X1, X2, Y1, Y2, OM, lr.FP32, st)

    for name, fn in (("one_after_another", seq), ("one_persistent_ladder", grp)):
        dt = timed(fn)
        out[name] = {"ms_per_step": dt * 1e3, "tflops_algorithmic": alg / dt / 1e12}
        log(f"uneven batch, {name}: {dt * 1e3:.1f} ms")
    g.close()
    for c in ctxs:
        c.close()
    del X1, X2, Y1, Y2, OM
    torch.cuda.empty_cache()
    total, paths = 0.0, []
    for i, w in enumerate(chains):
        c, x1, x2, y1, y2, om = make(i, w, 0)
        total += timed(lambda: c.apply_sigma_dev(x1, x2, y1, y2, om, lr.FP32, st))
        paths.append(c.ladder_path(12, lr.FP32))
        c.close()
        del x1, x2, y1, y2, om
        torch.cuda.empty_cache()
    out["one_after_another_default_mode"] = {"ms_per_step": total * 1e3, "tflops_algorithmic": alg / total / 1e12,
                                             "ladder_paths": paths}
    log(f"uneven batch, one after another in the default mode: {total * 1e3:.1f} ms")
    out["chains"] = [[w.nk, w.nocc, w.nvir, w.naux] for w in chains]
    out["nrhs_per_chain"] = 12
    out["speedup"] = out["one_after_another"]["ms_per_step"] / out["one_persistent_ladder"]["ms_per_step"]
    return out


def cpu_baseline(w, H, t1, t2, x1, x2, nrhs):
    """The oracle's sigma on a bounded sample: the oracle computes A x as the exact
    5-point stencil of the CCSD residual, i.e. four residual evaluations per
    right-hand side.  One of those four evaluations (for one right-hand side) is
    timed after the integral blocks are built (their build, like the library's
    set-up, is outside the timed region) and the rate is scaled by 4."""
    import torch
    from oracle import kblock
    nk = w.nk
    ham = kblock.KHam(H['fock'], H['chol'], w.nocc)
    for cls in ('oovv', 'ovvv', 'ooov', 'ovvo', 'ovoo', 'oooo', 'vvvo', 'vvoo', 'vvvv', 'vovv', 'oovo', 'ovov'):
        ham.eri(cls)
    T1 = kblock.t1_kt(t1 + 1e-3 * x1, nk)
    T2 = kblock.t2_kt((t2 + 1e-3 * x2) / nk, nk)
    t0 = time.perf_counter()
    kblock.residual(ham, T1, T2)
    dt = 4 * (time.perf_counter() - t0)
    flops = sigma_alg_flops(nk, w.nocc, w.nvir)
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"1 of {nrhs} right-hand sides of the same workload, fp64: one of the four residual "
                      f"evaluations of the oracle's 5-point stencil sigma (k-blocked oracle tier) timed "
                      f"({dt / 4:.1f} s) and scaled by 4"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-alpha", action="store_true",
                    help="skip the time to converged alpha (device CCSD, then the mixed and FP64 solves)")
    ap.add_argument("--alpha-modes", type=lambda t: [int(x) for x in t.split(",") if x], default=[],
                    help="comma-separated ladder modes (2 stored, 3 built by momentum class) in which both "
                         "alpha solves are timed again after the headline mode")
    ap.add_argument("--no-legs", action="store_true",
                    help="time the headline ladder path only (no other ladder paths, latency probe or peaks)")
    ap.add_argument("--ladder-mode", type=int, default=0,
                    help="ladder mode of the headline context (0 automatic, 1 rebuilt in LDS, 2 stored, "
                         "3 built by momentum class)")
    ap.add_argument("--alpha-tol", type=float, default=1e-10)
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="relative tolerance of the complex64 correction solves (default: the library's)")
    ap.add_argument("--ccsd-iter", type=int, default=300)
    ap.add_argument("--no-tune", action="store_true", help="heuristic launch variants instead of autotuning")
    ap.add_argument("--uneven", action="store_true", help="also time the twelve-chain uneven batch")
    ap.add_argument("--mesh", action="store_true", help="also time the sigma on a 2x2x2 k mesh")
    ap.add_argument("--velocity", action="store_true", help="also time the velocity-gauge alpha (c2)")
    ap.add_argument("--counters", action="store_true",
                    help="only one complex64 sigma (the tuned launch variants: from the cache that "
                         "LRCC_TUNE_CACHE names, else timed first) and then a plain 2 GiB device copy that "
                         "calibrates hardware byte counters; prints no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is "
              "not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2508_01266_amd as lr

    log(f"generating inputs for {args.workload}")
    w, H, t1, t2, x1, x2, omega = workload_inputs(args.workload)
    nk, o, v = w.nk, w.nocc, w.nvir
    log("inputs ready; building library context")
    nrhs = len(omega)
    dev = torch.device("cuda:0")
    ctx = lr.Context(0)
    ctx.set_hamiltonian(o, H['fock'], H['chol'], H['dip'])
    ctx.set_ladder_mode(args.ladder_mode)
    ctx.set_amplitudes(t1, t2)
    # the warm-up application picks the launch variants (with LRCC_TUNE_CACHE naming the cache of a
    # timed run, --counters applies that run's choices without timing candidates)
    ctx.set_autotune(not args.no_tune)
    X1 = torch.from_numpy(x1).to(dev)
    X2 = torch.from_numpy(x2).to(dev)
    sample = (x1[0].copy(), x2[0].copy())
    Y1 = torch.empty_like(X1)
    Y2 = torch.empty_like(X2)
    OM = torch.from_numpy(omega).to(dev)
    del x1, x2
    if args.counters:
        ctx.apply_sigma_dev(X1, X2, Y1, Y2, OM, lr.FP32, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        log("counters: one complex64 sigma done")
        a = torch.ones(1 << 28, dtype=torch.float64, device=dev)     # 2 GiB read, 2 GiB written
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("counters: 2 GiB device copy done")
        ctx.close()
        return

    alg = nrhs * sigma_alg_flops(nk, o, v)
    lad = nrhs * ladder_alg_flops(nk, o, v)
    log("context ready; timing complex64 sigma")
    dt32, lad_s, lad_n, bld_s = time_sigma(ctx, X1, X2, Y1, Y2, OM, lr.FP32, args.steps, args.warmup, torch)
    log(f"complex64 sigma {dt32*1e3:.1f} ms; timing complex128 sigma")
    dt64, lad64_s, lad64_n, bld64_s = time_sigma(ctx, X1, X2, Y1, Y2, OM, lr.FP64, args.fp64_steps, 1, torch)
    path, path64 = ctx.ladder_path(nrhs, lr.FP32), ctx.ladder_path(nrhs, lr.FP64)
    # roofline of the ladder products: the method's own work (unique antisymmetric index pairs)
    # per second of the ladder launches against the matrix-core peak.  Integral rebuilds are
    # overhead: inside the kernel with the integrals rebuilt in LDS, separate launches (reported
    # beside, and in frac_with_builds) when the blocks are built by momentum class.  The products
    # the launches execute (rebuild and padding included) and their matrix-core instructions are
    # reported beside it
    lad_unique = ladder_unique_flops(nk, o, v, nrhs)
    lad_exec = ctx.ladder_flops(nrhs, lr.FP32)
    lad_exec64 = ctx.ladder_flops(nrhs, lr.FP64)
    lad_mfma = ctx.ladder_mfma_flops(nrhs, lr.FP32)
    achieved = lad_unique / lad_s / 1e12
    traffic = None
    tr = LADDER_TRAFFIC.get(path)
    if tr and args.workload == tr["workload"] and tr["sources_sha256"] == ladder_sources_sha(path):
        traffic = tr["bytes"]
    out = {
        "metric": METRIC,
        "value": alg / dt32 / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: 1D chain Nk={nk}, nocc={o}, nvir={v}, Naux={w.naux}, "
                               f"{nrhs} right-hand sides (3 axes x +-omega x {len(w.omegas)} frequencies) "
                               f"in one sigma launch, complex64 on the matrix cores, {LADDER_PATH_TEXT[path]}",
                   "nk": nk, "nocc": o, "nvir": v, "naux": w.naux, "nrhs": nrhs,
                   "ladder_mode": args.ladder_mode, "ladder_path": path},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK["f32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["f32"], "traffic": traffic, "kernel": LADDER_KERNEL[path],
                     "work": "unique antisymmetric pairs (rows, outputs, inputs); integral rebuilds are overhead",
                     "unique_flops_per_step": lad_unique, "launches_per_step": lad_n,
                     "ladder_ms_avg": lad_s / lad_n * 1e3, "ladder_ms_per_step": lad_s * 1e3,
                     "build_ms_per_step": bld_s * 1e3,
                     "frac_with_builds": lad_unique / (lad_s + bld_s) / 1e12 / PEAK["f32"],
                     "executed_flops_per_step": lad_exec, "executed_frac": lad_exec / lad_s / 1e12 / PEAK["f32"],
                     "mfma_flops_per_step": lad_mfma, "mfma_frac": lad_mfma / lad_s / 1e12 / PEAK["f32"],
                     "full_range_flops_per_step": lad, "full_range_tflops": lad / lad_s / 1e12},
        "fp64": {"value": alg / dt64 / 1e12, "ms_per_step": dt64 * 1e3, "steps": args.fp64_steps,
                 "ladder_path": path64, "ladder_ms_per_step": lad64_s * 1e3, "build_ms_per_step": bld64_s * 1e3,
                 "ladder_achieved": lad_unique / lad64_s / 1e12,
                 "ladder_frac": lad_unique / lad64_s / 1e12 / PEAK["f64"],
                 "ladder_frac_with_builds": lad_unique / (lad64_s + bld64_s) / 1e12 / PEAK["f64"],
                 "ladder_executed_frac": lad_exec64 / lad64_s / 1e12 / PEAK["f64"], "peak": PEAK["f64"]},
        "executed_flops_per_step": {"f32": ctx.sigma_flops(nrhs, lr.FP32), "f64": ctx.sigma_flops(nrhs, lr.FP64)},
        "algorithmic_flops_per_step": alg,
        "speedup_mixed_vs_fp64_sigma": dt64 / dt32,
    }
    log(f"complex128 sigma {dt64*1e3:.1f} ms")
    # the same sigma along the other ladder paths: integrals rebuilt in LDS (1), stored for the
    # unique momentum pairs once per amplitudes (2), built one momentum class at a time in every
    # application (3)
    notes = {1: "integrals rebuilt in LDS from the t1-dressed Cholesky vectors inside the ladder kernel; "
                "nothing of vvvv size in memory",
             2: "antisymmetrised integral blocks stored for unique momentum pairs, built once per "
                "amplitudes (0.9 GB complex64 + 1.8 GB complex128 here)",
             3: "the same blocks built in every application, one momentum class ka + kb at a time, into "
                "a scratch array of one class (184 MB complex64, 368 MB complex128 here) that the class's "
                "GEMM consumes"}
    for mode, key in ((1, "rebuilt_in_lds"), (2, "stored_integrals"), (3, "class_integrals")):
        if mode == path or args.no_legs:
            continue
        ctx2 = lr.Context(0)
        ctx2.set_hamiltonian(o, H['fock'], H['chol'], H['dip'])
        ctx2.set_ladder_mode(mode)
        ctx2.set_amplitudes(t1, t2)
        ctx2.set_autotune(not args.no_tune)
        s32, sl32, _, sb32 = time_sigma(ctx2, X1, X2, Y1, Y2, OM, lr.FP32, args.steps, args.warmup, torch)
        s64, sl64, _, sb64 = time_sigma(ctx2, X1, X2, Y1, Y2, OM, lr.FP64, args.fp64_steps, 1, torch)
        out[key] = {
            "ladder_mode": mode,
            "ms_per_step": s32 * 1e3, "value": alg / s32 / 1e12, "ladder_ms_per_step": sl32 * 1e3,
            "build_ms_per_step": sb32 * 1e3,
            "ladder_achieved": lad_unique / sl32 / 1e12, "ladder_frac": lad_unique / sl32 / 1e12 / PEAK["f32"],
            "ladder_frac_with_builds": lad_unique / (sl32 + sb32) / 1e12 / PEAK["f32"],
            "ladder_executed_frac": ctx2.ladder_flops(nrhs, lr.FP32) / sl32 / 1e12 / PEAK["f32"],
            "fp64_ms_per_step": s64 * 1e3, "fp64_value": alg / s64 / 1e12, "fp64_ladder_ms_per_step": sl64 * 1e3,
            "fp64_build_ms_per_step": sb64 * 1e3,
            "fp64_ladder_frac": lad_unique / sl64 / 1e12 / PEAK["f64"],
            "fp64_ladder_frac_with_builds": lad_unique / (sl64 + sb64) / 1e12 / PEAK["f64"],
            "fp64_ladder_executed_frac": ctx2.ladder_flops(nrhs, lr.FP64) / sl64 / 1e12 / PEAK["f64"],
            "note": f"ladder mode {mode}: {notes[mode]}"}
        log(f"ladder mode {mode}: complex64 sigma {s32*1e3:.1f} ms, complex128 {s64*1e3:.1f} ms")
        ctx2.close()
    if not args.no_legs:
        out["latency_c1_9rhs"] = latency_small(lr, torch)
        # attainable ceilings on this device (project microbenchmarks), beside the published peaks
        out["peaks_measured"] = lr.measure_peaks(0)
        out["peaks_measured"]["published"] = {"mfma_f32_tflops": PEAK["f32"], "mfma_f64_tflops": PEAK["f64"],
                                              "hbm_gbs": 8000.0}
        log(f"measured peaks {out['peaks_measured']}")
        log(f"c1 latency {out['latency_c1_9rhs']}")
    del X1, X2, Y1, Y2, OM
    torch.cuda.empty_cache()
    if not args.no_alpha:
        # the response and lambda equations are posed at converged ground-state amplitudes:
        # solve CCSD on the device first (the random amplitudes above only serve the timing)
        log("solving ground-state CCSD on the device")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t1c, t2c, ecorr, crep = ctx.solve_ccsd(tol=1e-9, max_iter=args.ccsd_iter)
        out["ccsd"] = {"seconds": time.perf_counter() - t0, "energy_per_cell": ecorr, "report": crep}
        log(f"CCSD: {out['ccsd']}")
        res = {}
        for name, prec in (("mixed", lr.FP32), ("fp64", lr.FP64)):
            log(f"solving for alpha ({name})")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            extra = {"inner_tol": args.inner_tol} if args.inner_tol else {}
            al, rep = ctx.solve(list(w.omegas), axis_mask=7, tol=args.alpha_tol, precision=prec,
                                reuse_lambda=0, **extra)
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t0, al, rep)
            log(f"alpha ({name}) in {res[name][0]:.1f} s: {rep}")
        am, af = res["mixed"][1], res["fp64"][1]
        dif = np.abs(am - af)
        out["s_to_alpha_mixed"] = res["mixed"][0]
        out["s_to_alpha_fp64"] = res["fp64"][0]
        out["alpha"] = {
            "s_to_alpha_mixed": res["mixed"][0], "s_to_alpha_fp64": res["fp64"][0],
            "speedup_mixed_vs_fp64": res["fp64"][0] / res["mixed"][0],
            "tol": args.alpha_tol,
            "inner_tol": args.inner_tol if args.inner_tol else ctx.solve_options().inner_tol,
            "mixed_vs_fp64_max_abs": float(dif.max()),
            "mixed_vs_fp64_max_rel": float(dif.max() / np.abs(af).max()),
            # per tensor element alpha_XY: the largest |mixed - fp64| over the frequencies, and
            # relative to the largest |alpha_XY| over the frequencies
            "mixed_vs_fp64_per_element_abs": [[float(dif[:, x, y].max()) for y in range(3)] for x in range(3)],
            "mixed_vs_fp64_per_element_rel": [[float(dif[:, x, y].max() / max(np.abs(af[:, x, y]).max(), 1e-300))
                                               for y in range(3)] for x in range(3)],
            "alpha_xx_over_freqs_fp64": [float(x) for x in af[:, 0, 0].real],
            "effective_sigma_tflops": {k: res[k][2]["rhs_sigmas"] * sigma_alg_flops(nk, o, v) / res[k][0] / 1e12
                                       for k in res},
            "reports": {k: res[k][2] for k in res},
        }
    for mode in ([] if args.no_alpha else args.alpha_modes):
        # the same solves in another ladder mode: the one-vector transpose products of the lambda
        # equations and of the F term are bound by the integral rebuild at one right-hand side,
        # which stored blocks (2) remove and class-built blocks (3) share over every row pair
        if mode == args.ladder_mode:
            continue
        am, af = res["mixed"][1], res["fp64"][1]
        if ctx is not None:
            ctx.close()
            ctx = None
        torch.cuda.empty_cache()
        cs = lr.Context(0)
        cs.set_hamiltonian(o, H['fock'], H['chol'], H['dip'])
        cs.set_ladder_mode(mode)
        cs.set_amplitudes(t1c, t2c)
        cs.set_autotune(not args.no_tune)
        # build and tune the 48-RHS programs outside the timed solves, as for the default context
        Z1 = torch.zeros((nrhs, nk, o, v), dtype=torch.complex128, device=dev)
        Z2 = torch.zeros((nrhs, nk, nk, nk, o, o, v, v), dtype=torch.complex128, device=dev)
        OMz = torch.zeros(nrhs, dtype=torch.float64, device=dev)
        for prec in (lr.FP32, lr.FP64):
            cs.apply_sigma_dev(Z1, Z2, Z1.clone(), torch.empty_like(Z2), OMz, prec,
                               torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        del Z1, Z2, OMz
        torch.cuda.empty_cache()
        rs = {}
        for name, prec in (("mixed", lr.FP32), ("fp64", lr.FP64)):
            log(f"solving for alpha ({name}, ladder mode {mode})")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            al, rep = cs.solve(list(w.omegas), axis_mask=7, tol=args.alpha_tol, precision=prec, reuse_lambda=0)
            torch.cuda.synchronize()
            rs[name] = (time.perf_counter() - t0, al, rep)
            log(f"alpha ({name}, ladder mode {mode}) in {rs[name][0]:.1f} s: {rep}")
        cs.close()
        out["alpha"][f"ladder_mode_{mode}"] = {
            "s_to_alpha_mixed": rs["mixed"][0], "s_to_alpha_fp64": rs["fp64"][0],
            "max_abs_vs_default_fp64": float(np.abs(rs["fp64"][1] - af).max()),
            "max_abs_vs_default_mixed": float(np.abs(rs["mixed"][1] - am).max()),
            "reports": {k: rs[k][2] for k in rs},
        }
    if (args.mesh or args.velocity or args.uneven) and ctx is not None:
        ctx.close()               # the extra workloads need the memory
        torch.cuda.empty_cache()
    if args.mesh:
        out["mesh_2x2x2"] = mesh_sigma(lr, torch, max(1, args.steps // 2))
    if args.velocity:
        out["velocity_gauge_c2"] = velocity_gauge_alpha(lr, torch, args.alpha_tol)
    if args.uneven:
        if ctx is not None:
            ctx.close()           # the twelve chains need the memory
        torch.cuda.empty_cache()
        out["uneven_batch"] = uneven_batch(lr, torch, max(1, args.steps))
    if not args.no_cpu:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(w, H, t1, t2, sample[0], sample[1], nrhs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
