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
// Krylov vectors (and the vectors orthogonalised against them) are stored in complex128, or in
// complex64 with f32 = 1 (the complex64 inner solves); arithmetic is complex128 in both.
// y = beta y + alpha_r x on that storage
hipError_t basis_axpby(void *y, const void *x, const void *alpha, double beta, int R, i64 n, int f32, hipStream_t s);
// singles divided by (ev - eo - w), doubles by (ev2 + ev2 - eo2 - eo2 - w)
hipError_t precond(void *o1, void *o2, const void *i1, const void *i2, const double *eo, const double *ev,
                   const double *eo2, const double *ev2, const double *omega, KMesh km, int R, int no, int nv,
                   hipStream_t s);
hipError_t diag_real(const void *F, double *d, int nk, int n, hipStream_t s);

// Krylov vectors with packed doubles: one k block (o*o*v*v) per orbit of the antisymmetry swaps
// (ki,i) <-> (kj,j), (ka,a) <-> (kb,b), the block with ki <= kj and ka <= kb, scaled by
// sqrt(orbit size / 4): plain inner products of packed vectors equal the 1/4-weighted ones of the
// full (antisymmetric) vectors.  Device tables:
struct PackMap {
    int np = 0, nfull = 0;          // packed blocks, full blocks (nk^3)
    const int *canon = nullptr;     // [np] full block (ki*nk + kj)*nk + ka of packed block p
    const int *map = nullptr;       // [nfull] 4 p + 2 (ki > kj) + (ka > kb): the orbit's block, swaps
    const double *scale = nullptr;  // [np] sqrt(orbit size / 4)
};
// host tables of the k mesh; returns the number of packed blocks
int pack_tables(const KMesh &km, std::vector<int> &canon, std::vector<int> &map, std::vector<double> &scale);
// packed = a - b (b1, b2 may be null): singles [R][n1] copied, doubles [R][nfull][blk] gathered
// into [R][np][blk] and scaled
hipError_t pack_vec(void *o1, void *o2p, const void *a1, const void *a2, const void *b1, const void *b2,
                    const PackMap &pm, int R, i64 n1, i64 blk, int f32, hipStream_t s);
// full = the preconditioner (as precond) applied to the unpacked vector (antisymmetry signs filled in)
hipError_t unpack_precond(void *o1, void *o2, const void *i1, const void *i2p, const PackMap &pm, const double *eo,
                          const double *ev, const double *eo2, const double *ev2, const double *omega, KMesh km,
                          int R, int no, int nv, int f32, hipStream_t s);
// Y[r] = beta Y[r] + sum_i C[r][i] V[i]  (complex128; V: [m][n], Y: [R][n], C: device [R][m])
hipError_t combine(void *Y, const void *V, const void *C, int R, int m, i64 n, double beta, hipStream_t s);

// Device-resident GMRES state of R right-hand sides with restart length m (device arrays).
struct GmresState {
    int R, m;
    double2 *H;      // [R][(m+1)*m] Hessenberg matrices (rotated: upper triangular)
    double2 *cs, *sn;// [R][m] Givens rotations
    double2 *g;      // [R][m+1] rotated right-hand side of the least-squares problem
    double2 *scal;   // [R] scale of the next basis vector (0 for inactive right-hand sides)
    double *bn;      // [R] ||b||
    double *rel;     // [R] relative residual estimate (NaN for a non-finite one)
    int *act;        // [R] 1 while the right-hand side iterates
    int *kr;         // [R] Arnoldi steps that count for the right-hand side in this cycle
    int *sing;       // [R] 1 after a zero pivot (singular operator)
};
// Krylov vectors: vector i of right-hand side r at (Vs + (i*R + r)*n1, Vd + (i*R + r)*n2).
// out[r*ostride + i] = <V_i[r], w[r]> (conjugate-linear in V, doubles weighted by dw: 1/4 for full
// antisymmetric doubles, 1 for packed ones), i < k
int multidot_blocks(i64 n);
hipError_t multidot(const void *Vs, const void *Vd, const void *ws, const void *wd, int R, i64 n1, i64 n2, int k,
                    void *part, void *out, int ostride, double dw, int f32, hipStream_t s);
hipError_t selfdot(const void *ws, const void *wd, int R, i64 n1, i64 n2, void *part, void *out, double dw, int f32,
                   hipStream_t s);
// w[r] = beta w[r] + sign * sum_{i<k} C[r*cstride + i] V_i[r] (masked rows: w[r] = beta w[r]); k <= 64
hipError_t multiaxpy(void *ws, void *wd, const void *Vs, const void *Vd, const void *C, int cstride, double sign,
                     const int *mask, double beta, int R, i64 n1, i64 n2, int k, int f32, hipStream_t s);
hipError_t gmres_init(const GmresState &g, const void *beta2, double tol, hipStream_t s);
// h2: the second Gram-Schmidt pass's coefficients, or null after a single pass
hipError_t gmres_step(const GmresState &g, int j, const void *h1, const void *h2, const void *hn2, double tol,
                      double sing_pivot, hipStream_t s);
hipError_t gmres_solve(const GmresState &g, void *y, hipStream_t s);
hipError_t gmres_status(const GmresState &g, double *out, hipStream_t s);
}  // namespace lrcc
