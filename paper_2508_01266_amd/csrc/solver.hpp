// Launchers of the solver's streaming kernels (solver.hip).
#pragma once
#include "common.hpp"

namespace lrcc {
int dot_blocks(i64 n);
// out[r] = scale * sum_i conj(u[r][i]) v[r][i] (conj_u = 1) or sum_i u[r][i] v[r][i] (conj_u = 0);
// part needs R*dot_blocks(n) complex doubles
hipError_t batched_dot(const void *u, const void *v, int R, i64 n, double scale, void *part, void *out, hipStream_t s,
                       int conj_u = 1);
hipError_t batched_axpby(void *y, const void *x, const void *alpha, double beta, int R, i64 n, hipStream_t s);
// singles divided by (ev - eo - w), doubles by (ev2 + ev2 - eo2 - eo2 - w)
hipError_t precond(void *o1, void *o2, const void *i1, const void *i2, const double *eo, const double *ev,
                   const double *eo2, const double *ev2, const double *omega, KMesh km, int R, int no, int nv,
                   hipStream_t s);
hipError_t diag_real(const void *F, double *d, int nk, int n, hipStream_t s);
// Y[r] = beta Y[r] + sum_i C[r][i] V[i]  (complex128; V: [m][n], Y: [R][n], C: device [R][m])
hipError_t combine(void *Y, const void *V, const void *C, int R, int m, i64 n, double beta, hipStream_t s);
}  // namespace lrcc
