"""ctypes binding of liblrcc.so.  Argument marshalling only: every step of the
sigma path runs in the library's HIP kernels.  Raises if the library is not
built; there is no fallback."""
from __future__ import annotations

import ctypes
import os

import numpy as np

FP64, FP32 = 0, 1
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrcc.so")
_lib = None

_STATUS = {0: "LRCC_OK", 1: "LRCC_E_ARG", 2: "LRCC_E_SHAPE", 3: "LRCC_E_STATE", 4: "LRCC_E_OOM",
           5: "LRCC_E_HIP", 6: "LRCC_E_NOCONV", 7: "LRCC_E_SINGULAR"}


class LrccError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        L.lrcc_create.argtypes = [i, ctypes.POINTER(vp)]
        L.lrcc_destroy.argtypes = [vp]
        L.lrcc_destroy.restype = None
        L.lrcc_last_error.argtypes = [vp]
        L.lrcc_last_error.restype = ctypes.c_char_p
        L.lrcc_set_hamiltonian.argtypes = [vp, i, i, i, i, vp, vp, vp]
        L.lrcc_set_amplitudes.argtypes = [vp, vp, vp]
        L.lrcc_apply_sigma.argtypes = [vp, i, vp, vp, vp, vp, vp, i]
        L.lrcc_apply_sigma_dev.argtypes = [vp, i, vp, vp, vp, vp, vp, i, vp]
        L.lrcc_apply_sigma_dev_noalloc.argtypes = [vp, i, vp, vp, vp, vp, vp, i, vp]
        L.lrcc_apply_sigma_dev_noalloc.restype = ctypes.c_int
        L.lrcc_apply_sigma_adjoint.argtypes = [vp, i, vp, vp, vp, vp, vp, i]
        L.lrcc_apply_sigma_adjoint_dev.argtypes = [vp, i, vp, vp, vp, vp, vp, i, vp]
        L.lrcc_sigma_vjp_dev.argtypes = [vp, i, vp, vp, vp, vp, vp, i, vp]
        L.lrcc_set_profiling.argtypes = [vp, i]
        L.lrcc_set_graphs.argtypes = [vp, i]
        L.lrcc_group_create.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(vp)]
        L.lrcc_group_create.restype = ctypes.c_int
        L.lrcc_group_destroy.argtypes = [vp]
        L.lrcc_group_destroy.restype = None
        L.lrcc_group_last_error.argtypes = [vp]
        L.lrcc_group_last_error.restype = ctypes.c_char_p
        L.lrcc_group_apply_sigma_dev.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                                 ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i, vp]
        L.lrcc_group_apply_sigma_dev.restype = ctypes.c_int
        L.lrcc_alpha_lambda_bar.argtypes = [vp, i, ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveReport)]
        L.lrcc_alpha_lambda_bar.restype = ctypes.c_int
        L.lrcc_eom_roots.argtypes = [vp, i, ctypes.c_double, i, vp, ctypes.POINTER(SolveReport)]
        L.lrcc_eom_roots.restype = ctypes.c_int
        L.lrcc_set_kmesh.argtypes = [vp, i, i, i]
        L.lrcc_set_kmesh.restype = ctypes.c_int
        L.lrcc_alpha_velocity_gauge.argtypes = [vp, ctypes.c_uint, i, vp, vp, ctypes.POINTER(SolveOpts), vp,
                                                ctypes.POINTER(SolveReport)]
        L.lrcc_alpha_velocity_gauge.restype = ctypes.c_int
        L.lrcc_set_ladder_mode.argtypes = [vp, i]
        L.lrcc_set_ladder_mode.restype = ctypes.c_int
        L.lrcc_set_autotune.argtypes = [vp, i]
        L.lrcc_set_autotune.restype = ctypes.c_int
        L.lrcc_set_graphs.restype = ctypes.c_int
        L.lrcc_read_profile.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong)]
        L.lrcc_sigma_flops.argtypes = [vp, i, i, dp]
        L.lrcc_ladder_flops.argtypes = [vp, i, i, dp]
        L.lrcc_ladder_flops.restype = ctypes.c_int
        L.lrcc_ladder_mfma_flops.argtypes = [vp, i, i, dp]
        L.lrcc_ladder_mfma_flops.restype = ctypes.c_int
        L.lrcc_ladder_path.argtypes = [vp, i, i, ctypes.POINTER(i)]
        L.lrcc_ladder_path.restype = ctypes.c_int
        for f in ("lrcc_set_profiling", "lrcc_read_profile", "lrcc_sigma_flops"):
            getattr(L, f).restype = ctypes.c_int
        L.lrcc_solve_opts_default.argtypes = [ctypes.POINTER(SolveOpts)]
        L.lrcc_solve_opts_default.restype = None
        L.lrcc_solve_response.argtypes = [vp, i, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                          ctypes.POINTER(SolveReport)]
        L.lrcc_solve_response.restype = ctypes.c_int
        L.lrcc_solve_response_dev.argtypes = [vp, i, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                              ctypes.POINTER(SolveReport), vp]
        L.lrcc_solve_response_dev.restype = ctypes.c_int
        L.lrcc_solve.argtypes = [vp, ctypes.c_uint, i, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveReport)]
        L.lrcc_get_alpha.argtypes = [vp, i, vp]
        L.lrcc_alpha_dipole_gradient.argtypes = [vp, i, i, i, ctypes.POINTER(SolveOpts), vp]
        L.lrcc_alpha_dipole_gradient.restype = ctypes.c_int
        L.lrcc_alpha_fock_gradient.argtypes = [vp, i, i, i, ctypes.POINTER(SolveOpts), vp]
        L.lrcc_alpha_fock_gradient.restype = ctypes.c_int
        L.lrcc_alpha_chol_gradient.argtypes = [vp, i, i, i, ctypes.POINTER(SolveOpts), vp]
        L.lrcc_alpha_chol_gradient.restype = ctypes.c_int
        L.lrcc_solve_ccsd.argtypes = [vp, ctypes.c_double, i, vp, vp, dp, ctypes.POINTER(SolveReport)]
        L.lrcc_solve_ccsd.restype = ctypes.c_int
        L.lrcc_get_solution.argtypes = [vp, i, i, i, vp, vp]
        L.lrcc_get_lambda.argtypes = [vp, vp, vp]
        L.lrcc_set_guess.argtypes = [vp, i, i, i, vp, vp]
        L.lrcc_set_guess.restype = ctypes.c_int
        for f in ("lrcc_solve", "lrcc_get_alpha", "lrcc_get_solution", "lrcc_get_lambda"):
            getattr(L, f).restype = ctypes.c_int
        L.lrcc_plan_check.argtypes = [i, i, i, i, i, ctypes.c_char_p, i]
        L.lrcc_plan_check.restype = ctypes.c_int
        L.lrcc_measure_peaks.argtypes = [i, dp, dp, dp]
        L.lrcc_measure_peaks.restype = ctypes.c_int
        L.lrcc_plan_check_mesh.argtypes = [i, i, i, i, i, i, i, ctypes.c_char_p, i]
        L.lrcc_plan_check_mesh.restype = ctypes.c_int
        L.lrcc_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
        for f in ("lrcc_create", "lrcc_set_hamiltonian", "lrcc_set_amplitudes", "lrcc_apply_sigma",
                  "lrcc_apply_sigma_dev", "lrcc_apply_sigma_adjoint", "lrcc_apply_sigma_adjoint_dev", "lrcc_sizes"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("krylov", ctypes.c_int),
                ("precision", ctypes.c_int), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("mem_cap_bytes", ctypes.c_longlong), ("reuse_lambda", ctypes.c_int)]


class SolveReport(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int), ("outer", ctypes.c_int), ("sigma_fp64", ctypes.c_int),
                ("sigma_fp32", ctypes.c_int), ("max_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("rhs_sigmas", ctypes.c_longlong), ("phase_seconds", ctypes.c_double * 3)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["phase_seconds"] = list(d["phase_seconds"])
        return d


def _c128(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def measure_peaks(device=0):
    """Attainable matrix-core rates (fp32, fp64 TFLOP/s) and device-copy bandwidth (GB/s)
    measured by the library's microbenchmarks."""
    f32, f64, bw = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = lib().lrcc_measure_peaks(int(device), ctypes.byref(f32), ctypes.byref(f64), ctypes.byref(bw))
    if st != 0:
        raise LrccError(st, "microbenchmark failed")
    return {"mfma_f32_tflops": f32.value, "mfma_f64_tflops": f64.value, "hbm_copy_gbs": bw.value}


def plan_check(nk, nocc, nvir, naux, nrhs):
    """Host-only validation of all launch plans for a problem size (no GPU needed).
    nk: number of k points of a 1D chain, or a tuple (n0, n1, n2) of mesh extents."""
    buf = ctypes.create_string_buffer(512)
    if np.isscalar(nk):
        st = lib().lrcc_plan_check(int(nk), nocc, nvir, naux, nrhs, buf, 512)
    else:
        d = tuple(int(x) for x in nk) + (1,) * (3 - len(nk))
        st = lib().lrcc_plan_check_mesh(d[0], d[1], d[2], nocc, nvir, naux, nrhs, buf, 512)
    if st != 0:
        raise LrccError(st, buf.value.decode())


class Context:
    """One library context on HIP device `device` (owns its device memory)."""

    def __init__(self, device=0):
        self._L = lib()
        h = ctypes.c_void_p()
        st = self._L.lrcc_create(int(device), ctypes.byref(h))
        if st != 0:
            raise LrccError(st, self._L.lrcc_last_error(None).decode())
        self._h = h
        self.shape = None

    def _check(self, st):
        if st != 0:
            raise LrccError(st, self._L.lrcc_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.lrcc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_kmesh(self, n0, n1=1, n2=1):
        """k points on an n0 x n1 x n2 mesh (flat index (j0 n1 + j1) n2 + j2); call before
        set_hamiltonian.  Without it the k points form a 1D chain."""
        self._check(self._L.lrcc_set_kmesh(self._h, int(n0), int(n1), int(n2)))

    def set_hamiltonian(self, nocc, fock, chol, dip):
        """fock [nk][n][n], chol [nk][nk][naux][n][n], dip [3][nk][n][n] (complex128)."""
        nk, n = fock.shape[0], fock.shape[1]
        naux = chol.shape[2]
        f, c, d = (_c128(fock, (nk, n, n)), _c128(chol, (nk, nk, naux, n, n)), _c128(dip, (3, nk, n, n)))
        self.nk, self.n, self.naux = nk, n, naux
        self.no, self.nv = nocc, n - nocc
        self._check(self._L.lrcc_set_hamiltonian(self._h, self.nk, self.no, self.nv, self.naux,
                                                  _ptr(f), _ptr(c), _ptr(d)))

    def set_amplitudes(self, t1, t2):
        nk, o, v = self.nk, self.no, self.nv
        a = _c128(t1, (nk, o, v))
        b = _c128(t2, (nk, nk, nk, o, o, v, v))
        self._check(self._L.lrcc_set_amplitudes(self._h, _ptr(a), _ptr(b)))

    def apply_sigma_adjoint(self, x1, x2, omega=None, precision=FP64):
        """y = (A - omega)^T x for the pairing sum u1 w1 + 1/4 sum u2 w2."""
        return self.apply_sigma(x1, x2, omega, precision, adjoint=True)

    def apply_sigma(self, x1, x2, omega=None, precision=FP64, adjoint=False):
        nk, o, v = self.nk, self.no, self.nv
        R = x1.shape[0]
        a = _c128(x1, (R, nk, o, v))
        b = _c128(x2, (R, nk, nk, nk, o, o, v, v))
        y1 = np.empty_like(a)
        y2 = np.empty_like(b)
        om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64)
        f = self._L.lrcc_apply_sigma_adjoint if adjoint else self._L.lrcc_apply_sigma
        self._check(f(self._h, R, None if om is None else _ptr(om), _ptr(a), _ptr(b), _ptr(y1), _ptr(y2),
                      int(precision)))
        return y1, y2

    def solve_options(self, **kw):
        o = SolveOpts()
        self._L.lrcc_solve_opts_default(ctypes.byref(o))
        for k, val in kw.items():
            setattr(o, k, val)
        return o

    def solve_response(self, b1, b2, omega, x1=None, x2=None, **opts):
        """Solve (A - omega_r) x_r = b_r (host arrays, caller layouts). Returns (x1, x2, report dict)."""
        nk, o, v = self.nk, self.no, self.nv
        R = b1.shape[0]
        a = _c128(b1, (R, nk, o, v))
        b = _c128(b2, (R, nk, nk, nk, o, o, v, v))
        y1 = np.zeros_like(a) if x1 is None else _c128(x1, a.shape).copy()
        y2 = np.zeros_like(b) if x2 is None else _c128(x2, b.shape).copy()
        om = np.ascontiguousarray(omega, dtype=np.float64)
        oo = self.solve_options(**opts)
        rep = SolveReport()
        self._check(self._L.lrcc_solve_response(self._h, R, _ptr(om), _ptr(a), _ptr(b), _ptr(y1), _ptr(y2),
                                                ctypes.byref(oo), ctypes.byref(rep)))
        return y1, y2, rep.as_dict()

    def solve(self, omegas, axis_mask=7, **opts):
        """Polarizability alpha[nfreq][3][3] per cell (complex) at the frequencies `omegas`.
        Returns (alpha, report dict)."""
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        oo = self.solve_options(**opts)
        rep = SolveReport()
        self._check(self._L.lrcc_solve(self._h, int(axis_mask), len(om), _ptr(om), ctypes.byref(oo),
                                       ctypes.byref(rep)))
        alpha = np.zeros((len(om), 3, 3), dtype=np.complex128)
        self._check(self._L.lrcc_get_alpha(self._h, len(om), _ptr(alpha)))
        return alpha, rep.as_dict()

    def alpha_velocity_gauge(self, omegas, mom, axis_mask=7, **opts):
        """Velocity-gauge polarizability alpha^VG[nfreq][3][3] per cell from the momentum
        matrices mom [3][nk][n][n] at non-zero frequencies: (a(w) - a(0)) / w^2 with a the
        response of the momentum operator.  Returns (alpha, report dict)."""
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        m = _c128(mom, (3, self.nk, self.n, self.n))
        oo = self.solve_options(**opts)
        rep = SolveReport()
        a = np.zeros((len(om), 3, 3), dtype=np.complex128)
        self._check(self._L.lrcc_alpha_velocity_gauge(self._h, int(axis_mask), len(om), _ptr(om), _ptr(m),
                                                      ctypes.byref(oo), _ptr(a), ctypes.byref(rep)))
        return a, rep.as_dict()

    def alpha_dipole_gradient(self, ifreq, x, y, **opts):
        """d alpha_xy(omega_ifreq) / d mu: complex [3][nk][n][n] such that the change of
        alpha_xy under Hermitian dipole perturbations dmu is sum(grad * dmu).  Needs a
        preceding solve() that included axes x and y."""
        oo = self.solve_options(**opts)
        g = np.zeros((3, self.nk, self.n, self.n), dtype=np.complex128)
        self._check(self._L.lrcc_alpha_dipole_gradient(self._h, int(ifreq), int(x), int(y), ctypes.byref(oo),
                                                       _ptr(g)))
        return g

    def alpha_fock_gradient(self, ifreq, x, y, **opts):
        """d alpha_xy(omega_ifreq) / d f at fixed amplitudes (lambda re-solved): complex
        [nk][n][n] with d alpha = sum(grad * df) for Hermitian df.  Needs a preceding solve()."""
        oo = self.solve_options(**opts)
        g = np.zeros((self.nk, self.n, self.n), dtype=np.complex128)
        self._check(self._L.lrcc_alpha_fock_gradient(self._h, int(ifreq), int(x), int(y), ctypes.byref(oo), _ptr(g)))
        return g

    def alpha_chol_gradient(self, ifreq, x, y, **opts):
        """d alpha_xy(omega_ifreq) / d L at fixed amplitudes (lambda and the response re-solved):
        complex [nk][nk][naux][n][n] with d alpha = sum(grad * dL) for perturbations dL that keep the
        Hermitian pairing of the Cholesky vectors.  Needs a preceding solve()."""
        oo = self.solve_options(**opts)
        g = np.zeros((self.nk, self.nk, self.naux, self.n, self.n), dtype=np.complex128)
        self._check(self._L.lrcc_alpha_chol_gradient(self._h, int(ifreq), int(x), int(y), ctypes.byref(oo), _ptr(g)))
        return g

    def alpha_lambda_bar(self, nfreq, **opts):
        """alpha [nfreq][3][3] of the last solve() from the non-symmetric (perturbed-lambda) form."""
        oo = self.solve_options(**opts)
        a = np.zeros((nfreq, 3, 3), dtype=np.complex128)
        rep = SolveReport()
        self._check(self._L.lrcc_alpha_lambda_bar(self._h, int(nfreq), ctypes.byref(oo), _ptr(a), ctypes.byref(rep)))
        return a, rep.as_dict()

    def eom_roots(self, nroots, tol=1e-8, max_iter=200):
        """Lowest nroots EOM-CCSD excitation energies (complex, Hartree) and the report."""
        w = np.zeros(nroots, dtype=np.complex128)
        rep = SolveReport()
        self._check(self._L.lrcc_eom_roots(self._h, int(nroots), float(tol), int(max_iter), _ptr(w),
                                           ctypes.byref(rep)))
        return w, rep.as_dict()

    def solve_ccsd(self, tol=1e-9, max_iter=200):
        """Ground-state CCSD on the device; the result becomes the context's amplitudes.
        Returns (t1, t2, energy per cell, report)."""
        nk, o, v = self.nk, self.no, self.nv
        t1 = np.zeros((nk, o, v), dtype=np.complex128)
        t2 = np.zeros((nk, nk, nk, o, o, v, v), dtype=np.complex128)
        e = ctypes.c_double()
        rep = SolveReport()
        self._check(self._L.lrcc_solve_ccsd(self._h, float(tol), int(max_iter), _ptr(t1), _ptr(t2),
                                            ctypes.byref(e), ctypes.byref(rep)))
        return t1, t2, e.value, rep.as_dict()

    def get_solution(self, axis, ifreq, sign):
        nk, o, v = self.nk, self.no, self.nv
        x1 = np.zeros((nk, o, v), dtype=np.complex128)
        x2 = np.zeros((nk, nk, nk, o, o, v, v), dtype=np.complex128)
        self._check(self._L.lrcc_get_solution(self._h, int(axis), int(ifreq), int(sign), _ptr(x1), _ptr(x2)))
        return x1, x2

    def set_guess(self, axis, ifreq, sign, x1, x2):
        """Initial guess for t^axis(sign * omega_ifreq) of the next solve() (caller layouts, nrhs = 1)."""
        nk, o, v = self.nk, self.no, self.nv
        a = _c128(x1, (nk, o, v))
        b = _c128(x2, (nk, nk, nk, o, o, v, v))
        self._check(self._L.lrcc_set_guess(self._h, int(axis), int(ifreq), int(sign), _ptr(a), _ptr(b)))

    def get_lambda(self):
        nk, o, v = self.nk, self.no, self.nv
        l1 = np.zeros((nk, o, v), dtype=np.complex128)
        l2 = np.zeros((nk, nk, nk, o, o, v, v), dtype=np.complex128)
        self._check(self._L.lrcc_get_lambda(self._h, _ptr(l1), _ptr(l2)))
        return l1, l2

    def set_ladder_mode(self, mode):
        """0 automatic, 1 integrals rebuilt in LDS, 2 stored integral blocks, 3 integral blocks built
        one momentum class at a time in every application (before set_amplitudes)."""
        self._check(self._L.lrcc_set_ladder_mode(self._h, int(mode)))

    def set_autotune(self, on=True):
        self._check(self._L.lrcc_set_autotune(self._h, int(bool(on))))

    def set_graphs(self, on=True):
        self._check(self._L.lrcc_set_graphs(self._h, int(bool(on))))

    def set_profiling(self, on=True):
        self._check(self._L.lrcc_set_profiling(self._h, int(bool(on))))

    def read_profile(self):
        """{'ladder': (ms_total, launches), 'sigma': (ms_total, applications), 'ladder_build': (ms_total,
        launches)} since the last read."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_longlong * 4)()
        self._check(self._L.lrcc_read_profile(self._h, ms, cnt))
        return {"ladder": (ms[1], cnt[1]), "sigma": (ms[2], cnt[2]), "ladder_build": (ms[3], cnt[3])}

    def sigma_flops(self, nrhs, precision=FP64):
        out = ctypes.c_double()
        self._check(self._L.lrcc_sigma_flops(self._h, int(nrhs), int(precision), ctypes.byref(out)))
        return out.value

    def ladder_flops(self, nrhs, precision=FP64):
        out = ctypes.c_double()
        self._check(self._L.lrcc_ladder_flops(self._h, int(nrhs), int(precision), ctypes.byref(out)))
        return out.value

    def ladder_mfma_flops(self, nrhs, precision=FP64):
        out = ctypes.c_double()
        self._check(self._L.lrcc_ladder_mfma_flops(self._h, int(nrhs), int(precision), ctypes.byref(out)))
        return out.value

    def ladder_path(self, nrhs, precision=FP64):
        """1 integrals rebuilt in LDS, 2 stored blocks, 3 blocks built one momentum class at a time."""
        out = ctypes.c_int()
        self._check(self._L.lrcc_ladder_path(self._h, int(nrhs), int(precision), ctypes.byref(out)))
        return out.value

    def apply_sigma_dev(self, x1, x2, y1, y2, omega=None, precision=FP64, stream=None, adjoint=False):
        """Device-pointer variant for torch tensors (complex128, caller layouts)."""
        R = x1.shape[0]
        f = self._L.lrcc_apply_sigma_adjoint_dev if adjoint else self._L.lrcc_apply_sigma_dev
        st = f(
            self._h, R, None if omega is None else ctypes.c_void_p(omega.data_ptr()),
            ctypes.c_void_p(x1.data_ptr()), ctypes.c_void_p(x2.data_ptr()),
            ctypes.c_void_p(y1.data_ptr()), ctypes.c_void_p(y2.data_ptr()), int(precision),
            None if stream is None else ctypes.c_void_p(stream))
        self._check(st)

    def apply_sigma_dev_noalloc(self, x1, x2, y1, y2, omega=None, precision=FP64, stream=None):
        """lrcc_apply_sigma_dev without device allocation (work tensors in the library's static
        device array); torch tensors as for apply_sigma_dev."""
        st = self._L.lrcc_apply_sigma_dev_noalloc(
            self._h, x1.shape[0], None if omega is None else ctypes.c_void_p(omega.data_ptr()),
            ctypes.c_void_p(x1.data_ptr()), ctypes.c_void_p(x2.data_ptr()),
            ctypes.c_void_p(y1.data_ptr()), ctypes.c_void_p(y2.data_ptr()), int(precision),
            None if stream is None else ctypes.c_void_p(stream))
        self._check(st)

    def sigma_vjp_dev(self, g1, g2, gx1, gx2, omega=None, precision=FP64, stream=None):
        """Device-pointer vector-Jacobian product of the sigma (complex128 torch tensors,
        caller layouts): gx = conj((A - omega)^T conj(g)) on antisymmetric doubles."""
        R = g1.shape[0]
        st = self._L.lrcc_sigma_vjp_dev(
            self._h, R, None if omega is None else ctypes.c_void_p(omega.data_ptr()),
            ctypes.c_void_p(g1.data_ptr()), ctypes.c_void_p(g2.data_ptr()),
            ctypes.c_void_p(gx1.data_ptr()), ctypes.c_void_p(gx2.data_ptr()), int(precision),
            None if stream is None else ctypes.c_void_p(stream))
        self._check(st)


class Group:
    """Several chains whose sigma applications share one persistent ladder launch
    (lrcc_group_*).  Holds references to the contexts; close() before them."""

    def __init__(self, contexts):
        self._L = lib()
        self.contexts = list(contexts)
        arr = (ctypes.c_void_p * len(self.contexts))(*[c._h for c in self.contexts])
        h = ctypes.c_void_p()
        st = self._L.lrcc_group_create(arr, len(self.contexts), ctypes.byref(h))
        if st != 0:
            raise LrccError(st, "lrcc_group_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.lrcc_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_sigma_dev(self, xs1, xs2, ys1, ys2, omegas=None, precision=FP64, stream=None):
        """Per-chain torch tensors (complex128, caller layouts); omegas: per-chain float64 tensors or None."""
        n = len(self.contexts)
        vp = ctypes.c_void_p
        P = lambda ts: (vp * n)(*[t.data_ptr() for t in ts])
        nr = (ctypes.c_int * n)(*[int(t.shape[0]) for t in xs1])
        om = None if omegas is None else P(omegas)
        st = self._L.lrcc_group_apply_sigma_dev(self._h, nr, om, P(xs1), P(xs2), P(ys1), P(ys2), int(precision),
                                                None if stream is None else vp(stream))
        if st != 0:
            raise LrccError(st, self._L.lrcc_group_last_error(self._h).decode())
