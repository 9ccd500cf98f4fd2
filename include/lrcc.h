/*
 * lrcc.h - C ABI of the MI355X (gfx950) k-blocked LR-CCSD sigma library.
 *
 * The library applies the CCSD Jacobian (the linear-response "sigma vector",
 * the left-hand operator of the perturbed-amplitude equations, Sec. II.B,
 * Eqs. tx1 and tx2) to batches of perturbed amplitudes X1(w), X2(w) of a 1D
 * periodic system under crystal-momentum conservation (Sec. II.A,
 * Eq. momentum), and solves the response equations for the frequency-
 * dependent polarizability (Eq. lrf).
 *
 * Conventions shared by every entry point
 *   - complex numbers are interleaved (re, im) IEEE doubles ("c128"): a
 *     pointer to `double` addresses 2*count doubles;
 *   - k = 0..nk-1 labels k_j = 2*pi*j/nk; n = nocc + nvir, occupied first;
 *   - normalisation follows the paper: every two-electron quantity (the
 *     integrals built from `chol`, T2, X2, sigma2) is the per-cell quantity
 *     of Eqs. ene-lrf, i.e. Nk times the supercell-normalised one; one-
 *     electron quantities (f, mu, T1, X1, sigma1) are unscaled;
 *   - layouts (row-major):
 *       fock  [nk][n][n]                       f_{p k, q k}
 *       chol  [nk][nk][naux][n][n]             L^Q_{p k1, q k2}; integrals
 *             (p k1 r k2 | q k3 s k4) = sum_Q L^Q_{p k1, r k2} conj(L^Q_{s k4, q k3})
 *             for k2 - k1 = k3 - k4 (mod nk)
 *       dip   [3][nk][n][n]                    <p k|mu_x|q k>
 *       t1    [nk][nocc][nvir]                 t_{i k}^{a k}
 *       t2    [nk][nk][nk][nocc][nocc][nvir][nvir]   blocks (ki,kj,ka),
 *             kb = ki+kj-ka mod nk; antisymmetric in (i,j) and in (a,b)
 *       x1/y1 [nrhs][nk][nocc][nvir], x2/y2 [nrhs][nk][nk][nk][o][o][v][v]
 *   - ownership: the caller owns every buffer it passes; the library copies
 *     inputs during the call and writes outputs only on success.  A context
 *     owns its device memory; lrcc_destroy frees it.  A context is not
 *     thread-safe; distinct contexts are independent.
 *   - errors: every call returns an lrcc_status; nothing unwinds across the
 *     ABI; lrcc_last_error() describes the last failure of that context.
 */
#ifndef LRCC_H
#define LRCC_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrcc_ctx lrcc_ctx;

typedef enum {
    LRCC_OK = 0,
    LRCC_E_ARG = 1,      /* invalid argument (null pointer, bad size, broken symmetry) */
    LRCC_E_SHAPE = 2,    /* sizes inconsistent with the context                        */
    LRCC_E_STATE = 3,    /* call made before the inputs it needs were set               */
    LRCC_E_OOM = 4,      /* device allocation failed or exceeds the memory cap          */
    LRCC_E_HIP = 5,      /* HIP runtime error                                           */
    LRCC_E_NOCONV = 6,   /* iterative solve did not reach the tolerance, or a residual
                            norm is not finite (NaN/Inf in the inputs or iterates)     */
    LRCC_E_SINGULAR = 7  /* response operator numerically singular at this frequency:
                            the complex128 Krylov iteration met a Hessenberg pivot
                            below 1e-12 on a right-hand side that had not converged
                            (the preconditioned operator is O(1) by construction)   */
} lrcc_status;

enum { LRCC_FP64 = 0, LRCC_FP32 = 1 };

/* Options of the iterative response solver (lrcc_solve_opts_default fills them). */
typedef struct {
    double tol;            /* stop when ||b - (A - w) x|| <= tol ||b|| for every RHS (default 1e-10);
                              norm: sum |u1|^2 + 1/4 sum |u2|^2 over full arrays                      */
    int max_iter;          /* FP64 GMRES: maximum operator applications (default 400)                */
    int krylov;            /* GMRES restart length (at most 60); 0 (default) sizes it from free device
                              memory (85% of it, 4..60 vectors)                                       */
    int precision;         /* LRCC_FP64: GMRES in complex128; LRCC_FP32: complex64 matrix-core inner
                              GMRES corrections inside complex128 iterative refinement                */
    double inner_tol;      /* relative tolerance of each complex64 correction solve (default 1e-5;
                              at most 4 restart cycles per refinement step)                          */
    int max_outer;         /* maximum refinement steps (default 30)                                  */
    long long mem_cap_bytes; /* > 0: refuse (LRCC_E_OOM) if solver vectors would exceed this         */
    int reuse_lambda;      /* lrcc_solve: 1 (default) reuses lambda of the same amplitudes, 0 re-solves */
} lrcc_solve_opts;

typedef struct {
    int converged;           /* 1 if every RHS met tol (0 if any residual norm is NaN or Inf)       */
    int outer;               /* refinement steps (1 for LRCC_FP64)                                    */
    int sigma_fp64;          /* complex128 sigma applications (batched launches)                     */
    int sigma_fp32;          /* complex64 sigma applications (batched launches)                      */
    double max_rel_residual; /* largest final relative residual over the RHS (NaN if any is NaN)     */
    double seconds;          /* wall time of the solve                                               */
    long long rhs_sigmas;    /* full-Jacobian products counted per right-hand side (forward, adjoint,
                                both precisions): work in units of one single-RHS sigma               */
    double phase_seconds[3]; /* lrcc_solve: wall time of the lambda solve, of the batched response
                                solve (with eta), and of the F term and the contraction; 0 elsewhere */
} lrcc_solve_report;

/* Create a context on HIP device `hip_device`. *out is NULL on failure. */
lrcc_status lrcc_create(int hip_device, lrcc_ctx **out);

/* Destroy a context and free its device memory. NULL-safe. */
void lrcc_destroy(lrcc_ctx *ctx);

/* Text of the last error of this context (empty string if none).  Valid until
 * the next call on the same context.  ctx may be NULL (then: the last
 * lrcc_create failure). */
const char *lrcc_last_error(const lrcc_ctx *ctx);

/* Set the periodic Hamiltonian (Sec. II.A): Fock matrix per k, Cholesky
 * vectors of the two-electron integrals per k pair (momentum transfer
 * k2 - k1), and the three dipole matrices per k.  Checks Hermiticity of fock
 * and dip and the Hermitian pairing chol[k2][k1][Q] = conj(chol[k1][k2][Q])^T
 * (relative tolerance 1e-10) -> LRCC_E_ARG.  Discards any amplitudes set
 * before. */
lrcc_status lrcc_set_hamiltonian(lrcc_ctx *ctx, int nk, int nocc, int nvir, int naux,
                                 const double *fock, const double *chol, const double *dip);

/* Crystal-momentum mesh of the k points: n0 x n1 x n2 Monkhorst-Pack points
 * k = (j0/n0, j1/n1, j2/n2) (reciprocal-lattice units), for three-dimensional
 * periodicity (the extension of the 1D chains of Sec. II.A that Sec. V plans).
 * Momentum is conserved modulo a reciprocal-lattice vector (Eq. momentum), so k
 * points add componentwise modulo (n0, n1, n2).  Every k index of the other
 * calls is then the flat index k = (j0 n1 + j1) n2 + j2, nk = n0 n1 n2, and
 * every layout keeps its shape: t2 blocks (ki, kj, ka) with kb = ki + kj - ka on
 * the mesh, chol[k1][k2] with momentum transfer k2 - k1 on the mesh.  Without
 * this call (or with (nk, 1, 1)) the k points form a 1D chain.  Takes effect for
 * the next lrcc_set_hamiltonian, whose nk must equal n0 n1 n2 (else LRCC_E_SHAPE),
 * and discards the Hamiltonian, amplitudes and solutions set before.
 * LRCC_E_ARG unless every extent is >= 1. */
lrcc_status lrcc_set_kmesh(lrcc_ctx *ctx, int n0, int n1, int n2);

/* Set the converged ground-state amplitudes T1, T2 (Eqs. t1, t2; T2 in the
 * paper's per-cell normalisation) and build every amplitude-dependent
 * intermediate of the Jacobian once (the fixed "tilde" blocks of Sec. II.B).
 * Checks the (i,j)/(a,b) antisymmetry of t2 (tolerance 1e-10) -> LRCC_E_ARG;
 * before lrcc_set_hamiltonian -> LRCC_E_STATE. */
lrcc_status lrcc_set_amplitudes(lrcc_ctx *ctx, const double *t1, const double *t2);

/* Sigma vector for nrhs right-hand sides (Eqs. tx1, tx2 without -R and the
 * denominators): y_r = (A - omega_r) x_r with A the CCSD Jacobian dOmega/dT.
 * omega may be NULL (all zero).  x/y are HOST buffers in the layouts above.
 * precision LRCC_FP64 computes in complex128; LRCC_FP32 in complex64 on the
 * matrix cores (inputs and outputs stay complex128). */
lrcc_status lrcc_apply_sigma(lrcc_ctx *ctx, int nrhs, const double *omega,
                             const double *x1, const double *x2, double *y1, double *y2,
                             int precision);

/* Same as lrcc_apply_sigma on DEVICE buffers of the same layouts, enqueued on
 * `stream` (a hipStream_t; NULL = the null stream).  Returns after enqueueing. */
lrcc_status lrcc_apply_sigma_dev(lrcc_ctx *ctx, int nrhs, const double *omega,
                                 const void *x1, const void *x2, void *y1, void *y2,
                                 int precision, void *stream);

/* lrcc_apply_sigma_dev for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sigma, with the program's work tensors and launch tables placed in a
 * static device array of the library (256 MiB; each device the library runs on
 * holds one until the process ends) instead of context-owned allocations.  The
 * call allocates nothing: it synchronizes `stream` (the previous call on it may
 * still read the array), records the program into the array (launch tables by
 * synchronous host-to-device copies), and enqueues it on `stream`; no autotuning,
 * graph replay or profiling events.  Every call on a device shares that device's
 * array and overwrites it: calls that overlap on one device (other streams, other
 * threads, other contexts) race.  The context's amplitude-dependent blocks come
 * from lrcc_set_amplitudes as for the other calls.  LRCC_E_OOM, before any launch,
 * when the work tensors of nrhs right-hand sides exceed the array (about
 * 3 nrhs nk^3 o^2 v^2 complex elements of the precision, plus tables); other
 * errors as for lrcc_apply_sigma_dev.  In the automatic ladder mode the call
 * takes the integrals-rebuilt-in-LDS path (mode 1; mode 3 would put a momentum
 * class of integral blocks in the array too).  Results equal
 * lrcc_apply_sigma_dev's with the same ladder path and launch variants. */
lrcc_status lrcc_apply_sigma_dev_noalloc(lrcc_ctx *ctx, int nrhs, const double *omega, const void *x1,
                                         const void *x2, void *y1, void *y2, int precision, void *stream);

/* Kernel timing with HIP events recorded on the launch stream.  While enabled,
 * every sigma application records an event pair around each ladder launch and
 * around the whole application.  lrcc_read_profile waits for the recorded
 * events and returns, per category, the summed milliseconds and the number of
 * timed launches: index 0 unused, 1 = ladder products (one launch per
 * application with the integrals rebuilt in LDS or stored, one per momentum
 * class in ladder mode 3), 2 = whole sigma application, 3 = the integral-block
 * builds of ladder mode 3 (two per momentum class) (arrays of 4); it then
 * clears the record. */
lrcc_status lrcc_set_profiling(lrcc_ctx *ctx, int enable);
lrcc_status lrcc_read_profile(lrcc_ctx *ctx, double *ms, long long *count);

/* How the ladder term (the vvvv contraction of Eq. tx2) obtains its integrals.
 * 0 (default): automatic, per sigma program: mode 3 when one momentum class of
 * blocks in the program's precision takes at most an eighth of the free device
 * memory, else mode 1 (and mode 1 inside lrcc_apply_sigma_dev_noalloc).  1:
 * rebuilt in LDS from the t1-dressed Cholesky vectors inside the ladder kernel,
 * so nothing of vvvv size is ever stored.  2: stored blocks,
 * the antisymmetrised integrals for the unique momentum pairs (about Nk^3/4
 * blocks of nvir^4 complex values per precision, rebuilt with the other
 * amplitude-dependent blocks), after which the ladder is one dense matrix-core
 * GEMM; LRCC_E_OOM at lrcc_set_amplitudes if they would take more than half of
 * the free device memory.  The transpose product reads the same blocks in mode
 * 2 (a transposed GEMM over the unique momentum pairs into a scratch array of
 * the doubles' size, then an (e, f)-antisymmetric completion).  3: the same
 * blocks built in every sigma application, one momentum class K = ka + kb at a
 * time, into a scratch array of the largest class (about 1/Nk of the mode-2
 * blocks) that the class's GEMM consumes before the next class is built; each
 * block is rebuilt once per application for all row pairs ki + kj = K and all
 * right-hand sides.  The per-sigma profile (lrcc_read_profile) counts the
 * class builds and GEMMs as ladder launches.  Must precede the first
 * lrcc_set_amplitudes or lrcc_solve_ccsd (LRCC_E_STATE afterwards); LRCC_E_ARG
 * for other modes. */
lrcc_status lrcc_set_ladder_mode(lrcc_ctx *ctx, int mode);

/* Autotuning of launch variants: when enabled, the first application of each
 * sigma program (per problem size, nrhs, precision and direction) is run once
 * per candidate configuration (matrix-core GEMM tiles 64x64 or large; ladder
 * antisymmetry-packed or full-range), every tunable launch is timed with HIP
 * events and the fastest candidate is kept per launch.  If the environment
 * variable LRCC_TUNE_CACHE names a file, choices are read from and appended to
 * it (one line per program).  Results do not depend on the choice. */
lrcc_status lrcc_set_autotune(lrcc_ctx *ctx, int enable);

/* HIP-graph replay of the sigma (and transpose) applications: when enabled,
 * each application on a non-null stream is captured once per set of buffer
 * addresses and replayed as one graph launch (the solver uses a stream of its
 * own).  Profiling events are not recorded inside graphs.  Disabling frees the
 * captured graphs. */
lrcc_status lrcc_set_graphs(lrcc_ctx *ctx, int enable);

/* Real floating-point operations executed by one sigma application for nrhs
 * right-hand sides (matrix-core GEMMs and ladder, including the in-LDS
 * integral rebuild; streaming kernels excluded). */
lrcc_status lrcc_sigma_flops(lrcc_ctx *ctx, int nrhs, int precision, double *executed);

/* Real floating-point operations executed by the ladder products of one sigma
 * application (the profiling category 1 of lrcc_read_profile): the matrix-core
 * products over the unique momentum/index pairs when the integral blocks are
 * stored or built one momentum class at a time (the class builds, category 3,
 * are not included), or the ladder kernel's products including its in-LDS
 * rebuild for the kernel variant in use (after autotuning); 8 real flops per
 * complex multiply-add formed. */
lrcc_status lrcc_ladder_flops(lrcc_ctx *ctx, int nrhs, int precision, double *executed);
/* The same launches counted in real matrix-core flops (the work of their MFMA
 * instructions): the complex64 pipelined kernel forms the complex products of
 * its integral rebuild, and the complex64 GEMM tiles with three real products
 * (when the autotuner picks them) all their complex products, from three real
 * matrix-core products (Gauss' method), which count 6 instead of 8. */
lrcc_status lrcc_ladder_mfma_flops(lrcc_ctx *ctx, int nrhs, int precision, double *mfma);
/* Ladder path of the sigma program for nrhs right-hand sides and this precision
 * (recording it if needed): 1 integrals rebuilt in LDS, 2 stored blocks, 3 blocks
 * built one momentum class at a time (lrcc_set_ladder_mode; mode 0 resolves to
 * 3 or 1).  LRCC_E_STATE before amplitudes. */
lrcc_status lrcc_ladder_path(lrcc_ctx *ctx, int nrhs, int precision, int *path);

/* Measurement helper, not an operation of the method: the attainable dense
 * matrix-core rates of the device (streams of real 16x16x4 fp32 and fp64 MFMA
 * products on all compute units, best over 1, 2 and 4 waves per SIMD and 8 or
 * 16 independent accumulators per wave) in TFLOP/s and the bandwidth of a
 * 2 GiB device copy (bytes read + written per second, GB/s, best of four runs
 * at two grid sizes) -- the ceilings the sigma kernels' roofline is read
 * against, beside the published peaks.  Allocates and frees its own device
 * buffers (about 4 GiB).  LRCC_E_ARG for null outputs, LRCC_E_HIP / LRCC_E_OOM
 * on device errors. */
lrcc_status lrcc_measure_peaks(int hip_device, double *mfma_f32_tflops, double *mfma_f64_tflops,
                               double *hbm_copy_gbs);

/* Host-only validation of the launch plans for a problem size: records every
 * kernel of lrcc_set_hamiltonian, lrcc_set_amplitudes and lrcc_apply_sigma (FP64
 * and FP32, nrhs right-hand sides) without a device, checking that every
 * address each matrix-core GEMM can form lies inside its operands.  Needs no
 * GPU and allocates no device memory.  On failure writes a message into msg
 * (msglen bytes, may be NULL) and returns LRCC_E_ARG (or LRCC_E_OOM). */
lrcc_status lrcc_plan_check(int nk, int nocc, int nvir, int naux, int nrhs, char *msg, int msglen);
/* The same on an n0 x n1 x n2 k mesh (lrcc_set_kmesh); lrcc_plan_check is the
 * 1D chain (nk, 1, 1). */
lrcc_status lrcc_plan_check_mesh(int n0, int n1, int n2, int nocc, int nvir, int naux, int nrhs, char *msg,
                                 int msglen);

/* Transpose product (the operator of the lambda equations l1, l2, Sec. II.B):
 * y_r = (A - omega_r)^T x_r, the transpose taken with respect to the bilinear
 * pairing <u, w> = sum_singles u1 w1 + 1/4 sum_doubles u2 w2 over full arrays
 * in the layouts and normalisation above, so that <z, (A - w) x> =
 * <(A - w)^T z, x> for antisymmetric x, z.  The adjoint reuses the ladder
 * kernel with pair-transposed Cholesky slices; nothing of vvvv size is stored.
 * Host-buffer and device-buffer variants as for the sigma. */
lrcc_status lrcc_apply_sigma_adjoint(lrcc_ctx *ctx, int nrhs, const double *omega,
                                     const double *x1, const double *x2, double *y1, double *y2,
                                     int precision);
lrcc_status lrcc_apply_sigma_adjoint_dev(lrcc_ctx *ctx, int nrhs, const double *omega,
                                         const void *x1, const void *x2, void *y1, void *y2,
                                         int precision, void *stream);

/* Vector-Jacobian product of the sigma map y = (A - omega) x for reverse-mode
 * differentiation (the transpose operator of the lambda equations l1, l2,
 * Sec. II.B, in the complex-gradient convention of PyTorch):
 *   gx = conj((A - omega)^T conj(g)) restricted to antisymmetric doubles,
 * i.e. Re sum conj(gx) . dx = Re sum conj(g) . (A - omega) dx over full caller
 * arrays for every dx with antisymmetric doubles.  The doubles part of g is
 * projected onto the antisymmetric subspace on entry and gx2 is antisymmetric.
 * g1, gx1: [nrhs][nk][nocc][nvir]; g2, gx2: [nrhs][nk][nk][nk][nocc][nocc][nvir][nvir]
 * (complex128 device buffers, caller layout of the sigma).  omega: nrhs real
 * device values or NULL.  Grows a context-owned scratch of 2 x (input size)
 * on first use with a larger nrhs.  Errors as for the sigma. */
lrcc_status lrcc_sigma_vjp_dev(lrcc_ctx *ctx, int nrhs, const double *omega, const void *g1, const void *g2,
                               void *gx1, void *gx2, int precision, void *stream);

void lrcc_solve_opts_default(lrcc_solve_opts *opts);

/* Solve the perturbed-amplitude equations (Eqs. tx1, tx2 in operator form,
 * the Jacobi/DIIS iteration of Sec. II.C replaced by preconditioned GMRES with
 * the same orbital-energy denominators of Eq. D): (A - omega_r) x_r = b_r for
 * nrhs right-hand sides at once, each with its own frequency.  The doubles of
 * b and x are antisymmetric under (ki,i)<->(kj,j) and (ka,a)<->(kb,b), as every
 * doubles amplitude vector (the Krylov basis keeps one k block per orbit of
 * those swaps; a part of b2 outside that subspace is not in the operator's
 * range and is not solved for).  x holds the
 * initial guess on entry (zeros for none) and the solution on exit.  opts may
 * be NULL (defaults).  Returns LRCC_E_NOCONV (x and report still written) if
 * the tolerance is not reached or a residual norm is not finite (NaN/Inf in b
 * or x), LRCC_E_SINGULAR (x and report written) if (A - omega_r) is singular
 * (see the status codes), LRCC_E_OOM if opts->mem_cap_bytes is below the
 * Krylov vectors' size.  Host-buffer variant (omega host) and device
 * variant (omega, b, x device; enqueued on stream, returns after completion). */
lrcc_status lrcc_solve_response(lrcc_ctx *ctx, int nrhs, const double *omega,
                                const double *b1, const double *b2, double *x1, double *x2,
                                const lrcc_solve_opts *opts, lrcc_solve_report *report);
lrcc_status lrcc_solve_response_dev(lrcc_ctx *ctx, int nrhs, const double *omega,
                                    const void *b1, const void *b2, void *x1, void *x2,
                                    const lrcc_solve_opts *opts, lrcc_solve_report *report, void *stream);

/* Frequency-dependent polarizability (Eq. lrf, symmetric form) for the dipole
 * axes in axis_mask (bit x = axis x; axes whose dipole matrices vanish are
 * skipped, as in Sec. II.B) at nfreq frequencies omega (host array, a.u.).
 * Solves, on the device: the lambda equations (Eqs. l1, l2) once per set of
 * amplitudes, the perturbed amplitudes t^X(+-omega_j) for all axes and
 * frequencies as ONE batch of 2*nfreq*naxes right-hand sides (Eqs. tx1, tx2),
 * and contracts them in complex128 into
 *   alpha_XY(w) = -1/(2 Nk) [g_XY(w) + conj(g_XY(-w))],
 *   g_XY(w) = eta^X t^Y(w) + eta^Y t^X(-w) + F(t^X(-w), t^Y(w)),
 * the polarizability per cell (reading of the paper's sign and symmetrisation
 * conventions as documented with the library).  opts->precision selects the
 * plain complex128 solver or complex64 matrix-core corrections inside complex128
 * refinement (the one-vector lambda solve is always complex128); the residual
 * tolerance, subspace size and memory cap come from
 * opts (NULL: defaults).  Results stay in the context: lrcc_get_alpha,
 * lrcc_get_solution, lrcc_get_lambda.  Initial guesses stored with
 * lrcc_set_guess start the batched solve.  On LRCC_E_NOCONV / LRCC_E_SINGULAR
 * the report (if given) describes the failing solve and no polarizability is
 * stored.  LRCC_E_ARG for non-finite frequencies or bad options. */
lrcc_status lrcc_solve(lrcc_ctx *ctx, unsigned axis_mask, int nfreq, const double *omega,
                       const lrcc_solve_opts *opts, lrcc_solve_report *report);

/* Ground-state CCSD on the device (Eqs. t1, t2): Jacobi steps with the
 * denominators of Eq. D and DIIS on the amplitude change (Sec. II.C), from
 * T = 0, until the residual norm sqrt(sum |O1|^2 + 1/4 sum |O2|^2) (per-cell
 * normalisation) is <= tol.  The residual is evaluated exactly from the
 * Jacobian: Omega(T) = Omega(0) + int_0^1 A(sT) T ds with 2-point Gauss-Legendre
 * (the integrand is cubic in s).  On success the converged amplitudes become the
 * context's amplitudes (as after lrcc_set_amplitudes).  t1/t2/energy may be NULL;
 * energy is the correlation energy per cell (Eq. ene).  LRCC_E_NOCONV if
 * max_iter is reached. */
lrcc_status lrcc_solve_ccsd(lrcc_ctx *ctx, double tol, int max_iter, double *t1, double *t2, double *energy,
                            lrcc_solve_report *report);

/* Several chains (contexts with their own Hamiltonians and sizes, on one device)
 * whose sigma applications run together: every chain's steps up to the ladder,
 * then the ladders of all chains as ONE persistent launch that takes
 * (chain, k block, tile) work items from an atomic queue, most expensive
 * chains first (uneven batches keep the device busy through the tail), then the
 * remaining steps.  Chains whose ladder is not the rebuild-in-LDS pipelined
 * kernel (stored integrals, or fewer than 128 unique (rhs, i, j) rows in every
 * momentum class ki + kj) run their whole program on their own.  Results are bitwise those of
 * lrcc_apply_sigma_dev per chain.  The group does not own the contexts; destroy
 * it before them.  A chain may get a new Hamiltonian, k mesh or amplitudes
 * between calls: the group's launch tables record each context's state and are
 * rebuilt when it changed.  Arrays are indexed by chain; omega may be NULL.  Errors:
 * LRCC_E_ARG for null arrays, contexts on different devices or a bad precision,
 * LRCC_E_STATE if a chain has no amplitudes; the message is read with
 * lrcc_group_last_error. */
typedef struct lrcc_group lrcc_group;
lrcc_status lrcc_group_create(lrcc_ctx *const *ctxs, int n, lrcc_group **out);
void lrcc_group_destroy(lrcc_group *group);
const char *lrcc_group_last_error(const lrcc_group *group);
lrcc_status lrcc_group_apply_sigma_dev(lrcc_group *group, const int *nrhs, const double *const *omega,
                                       const void *const *x1, const void *const *x2, void *const *y1,
                                       void *const *y2, int precision, void *stream);

/* EOM-CCSD excitation energies: the nroots eigenvalues of the CCSD Jacobian with
 * the lowest real parts on the momentum-conserving excitations, i.e. the poles
 * of the linear response function (Sec. II.B) that alpha(omega) diverges at.
 * Davidson iteration on the device sigma (complex128) with the dressed diagonal
 * preconditioner; Rayleigh-Ritz on the small projected matrix on the host.
 * omega: host [nroots] complex (Hartree), ascending real part.  tol: residual
 * norm ||(A - theta) x|| for unit x (<= 0: 1e-8); max_iter (<= 0: 200).
 * LRCC_E_ARG unless 1 <= nroots <= nk*nocc*nvir; LRCC_E_STATE before amplitudes;
 * LRCC_E_NOCONV when not converged (omega then holds the current estimates). */
lrcc_status lrcc_eom_roots(lrcc_ctx *ctx, int nroots, double tol, int max_iter, double *omega,
                           lrcc_solve_report *report);

/* alpha [nfreq][3][3] (as lrcc_get_alpha) from the non-symmetric form of the
 * response function with perturbed multipliers (the formulation of Eq. lrf with
 * lambda-bar, Sec. II.B): lambda-bar^Y(s w) = (A + s w)^-T (eta^Y + F(., t^Y(s w)))
 * for every solved axis, frequency and sign in one batched transpose solve
 * (opts as for lrcc_solve, NULL: defaults), then
 *   g_XY(s w) = eta^X t^Y(s w) - <lambda-bar^Y(s w), xi^X>,
 *   alpha_XY(w) = -1/(2 Nk) [g_XY(w) + conj(g_XY(-w))].
 * Uses the response amplitudes and lambda of the last lrcc_solve (LRCC_E_STATE
 * without one; LRCC_E_ARG if nfreq differs); equals its symmetric alpha up to
 * the solver tolerances. */
lrcc_status lrcc_alpha_lambda_bar(lrcc_ctx *ctx, int nfreq, const lrcc_solve_opts *opts, double *alpha,
                                  lrcc_solve_report *report);

/* Polarizability in the velocity gauge (Sec. V): the perturbation operator is
 * the momentum operator instead of the dipole.  mom: host [3][nk][n][n] complex,
 * Hermitian per axis per k (matrix elements of the momentum operator p_x, p_y,
 * p_z; LRCC_E_ARG otherwise).  One batched solve (as lrcc_solve, with opts) of
 * the response to p at the frequencies 0, omega_0, ..., omega_{nfreq-1}, then
 *   alpha^VG_XY(w) = (a_XY(w) - a_XY(0)) / w^2,   a_XY(w) = -<<p_X; p_Y>>_w / Nk,
 * the symmetric response function of p in the form of lrcc_solve; subtracting
 * the static response removes the diamagnetic term (which it equals for an exact
 * state in a complete basis).  alpha: host [nfreq][3][3] complex (zeros for axes
 * outside axis_mask or with vanishing p).  Every omega must be non-zero
 * (LRCC_E_ARG).  The dipoles of lrcc_set_hamiltonian are kept for later solves;
 * the stored solutions of the last lrcc_solve are discarded (lambda is kept:
 * it does not depend on the perturbation). */
lrcc_status lrcc_alpha_velocity_gauge(lrcc_ctx *ctx, unsigned axis_mask, int nfreq, const double *omega,
                                      const double *mom, const lrcc_solve_opts *opts, double *alpha,
                                      lrcc_solve_report *report);

/* alpha [nfreq][3][3] complex (zeros for skipped axes) of the last lrcc_solve;
 * nfreq must match it. */
lrcc_status lrcc_get_alpha(const lrcc_ctx *ctx, int nfreq, double *alpha);

/* Gradient of one polarizability element of the last lrcc_solve with respect to
 * the dipole matrices (the perturbation operators of Eq. rhs, Sec. II.B), at
 * fixed ground-state amplitudes and lambda (neither depends on the dipoles):
 *   d alpha_xy(omega_ifreq) = sum_{Z,k,p,q} grad[Z][k][p][q] dmu_Z[k][p][q]
 * for every Hermitian perturbation dmu_Z of the dipole of axis Z.
 * grad: host [3][nk][n][n] complex (zeros for axes other than x, y).  alpha is
 * bilinear in (mu_x, mu_y); the gradient costs one batched transpose solve of
 * 4 right-hand sides (2 when x == y) with opts (NULL: defaults), 4 F-vector
 * stencils and a few one-body density evaluations on the device.
 * LRCC_E_STATE before lrcc_solve; LRCC_E_ARG for an axis the last solve did not
 * include or an out-of-range ifreq; LRCC_E_NOCONV if the transpose solve fails. */
lrcc_status lrcc_alpha_dipole_gradient(lrcc_ctx *ctx, int ifreq, int x, int y, const lrcc_solve_opts *opts,
                                       double *grad);

/* Gradient of one polarizability element of the last lrcc_solve with respect to
 * the Fock matrix (the one-electron part of the Hamiltonian of Sec. II.A) at
 * fixed ground-state amplitudes, with lambda re-solved (it depends on f):
 *   d alpha_xy(omega_ifreq) = sum_{k,p,q} grad[k][p][q] df[k][p][q]
 * for every Hermitian perturbation df.  grad: host [nk][n][n] complex.  The
 * residual is linear in f, so every f-dependence enters through one-body
 * densities of the perturbation residual; the cost is the transpose solves of
 * the dipole gradient (4 right-hand sides), one forward solve of 2 right-hand
 * sides, 6 stencils of the sigma and a few density evaluations.  Errors as for
 * lrcc_alpha_dipole_gradient. */
lrcc_status lrcc_alpha_fock_gradient(lrcc_ctx *ctx, int ifreq, int x, int y, const lrcc_solve_opts *opts,
                                     double *grad);

/* Gradient of one polarizability element of the last lrcc_solve with respect to
 * the Cholesky vectors of the two-electron integrals (Sec. II.A; they enter the
 * Jacobian of Eqs. tx1, tx2, the multiplier equations l1, l2 and the response
 * function of Eq. lrf), at fixed ground-state amplitudes with lambda and the
 * response amplitudes re-solved:
 *   d alpha_xy(omega_ifreq) = sum_{k1,k2,Q,p,q} grad[k1][k2][Q][p][q] dL[k1][k2][Q][p][q]
 * for every perturbation dL that keeps the Hermitian pairing of lrcc_set_hamiltonian
 * (dL[k2][k1][Q] = conj(dL[k1][k2][Q])^T).  grad: host [nk][nk][naux][n][n] complex.
 * The parameter derivative of the Jacobian is taken by reverse traversal of the
 * sigma's term list and of the amplitude-dependent blocks at fixed amplitudes; the
 * ladder's contribution is formed from the density D_ab,ef = sum u_ijab x_ijef one
 * momentum block at a time (never stored whole) and contracted with the Cholesky
 * vectors.  Costs the solves of the Fock gradient plus 14 parameter-derivative
 * passes of about one sigma each.  Errors as for lrcc_alpha_dipole_gradient. */
lrcc_status lrcc_alpha_chol_gradient(lrcc_ctx *ctx, int ifreq, int x, int y, const lrcc_solve_opts *opts,
                                     double *grad);

/* Perturbed amplitudes t^X(sign*omega_ifreq) of the last lrcc_solve (caller
 * layouts with nrhs = 1, per-cell normalisation). */
lrcc_status lrcc_get_solution(const lrcc_ctx *ctx, int axis, int ifreq, int sign, double *x1, double *x2);

/* Initial guess for one right-hand side of the NEXT lrcc_solve: the perturbed
 * amplitudes t^axis(sign*omega_ifreq) start from (x1, x2) instead of zero (the
 * restart of the iterative solution of Sec. II.C; e.g. the converged amplitudes
 * of a neighbouring frequency from lrcc_get_solution seed a shifted frequency
 * grid).  ifreq indexes the frequency list of that next call; x1
 * [nk][nocc][nvir], x2 [nk][nk][nk][nocc][nocc][nvir][nvir] (HOST buffers, caller
 * layouts, per-cell normalisation), copied into context-owned device memory
 * (one amplitude vector per guess; setting the same (axis, ifreq, sign) again
 * replaces it).  The next lrcc_solve consumes every stored guess (guesses for
 * axes or frequencies it does not solve are dropped); lrcc_set_hamiltonian and
 * lrcc_set_kmesh discard them.  The solution does not depend on the guess (up to
 * the solver tolerance), only the work does.  LRCC_E_ARG for an axis outside
 * 0..2, ifreq < 0, sign not +-1, null pointers or non-finite values;
 * LRCC_E_STATE before lrcc_set_hamiltonian. */
lrcc_status lrcc_set_guess(lrcc_ctx *ctx, int axis, int ifreq, int sign, const double *x1, const double *x2);

/* lambda amplitudes of the last lrcc_solve (layouts of t1/t2; pairing
 * sum l1 x1 + 1/4 sum l2 x2 with amplitudes in the per-cell normalisation). */
lrcc_status lrcc_get_lambda(lrcc_ctx *ctx, double *l1, double *l2);

/* Number of amplitude elements per right-hand side: singles and doubles. */
lrcc_status lrcc_sizes(const lrcc_ctx *ctx, long long *n1, long long *n2);

#ifdef __cplusplus
}
#endif
#endif /* LRCC_H */
