// Launchers of the streaming kernels (definitions in elem.hip).
#pragma once
#include "common.hpp"

namespace lrcc {
template <typename Tin, typename Tout>
hipError_t rhs_to_block(const void *in, void *out, int R, i64 B, i64 E, double scale, hipStream_t s);
template <typename T>
hipError_t tau_like(const void *x1, const void *x2, const void *t1, void *out, KMesh km, int R, int o, int v,
                    double c, int x1_has_rhs, hipStream_t s);
template <typename T>
hipError_t pp_out(const void *Z, const void *x2, void *y2, const double *omega, KMesh km, int R, int o, int v,
                  double scale, hipStream_t s);
template <typename T>
hipError_t s1_out(const void *s1, const void *x1, void *y1, const double *omega, int nk, int R, int o, int v,
                  hipStream_t s);
template <typename Tout>
hipError_t chol_slice(const void *L, void *out, int nk, int naux, int n, int p0, int np, int q0, int nq,
                      double scale, int conj_pair, hipStream_t s);
template <typename Tout>
hipError_t one_body_slice(const void *in, void *out, int nk, int n, int p0, int np, int q0, int nq, hipStream_t s);
hipError_t convert_f64_f32(const void *in, void *out, i64 n, hipStream_t s);
template <typename Tout>
hipError_t axis_slice(const void *in, void *out, int nax, int nk, int n, int p0, int np, int q0, int nq, int transpose,
                      hipStream_t s);
hipError_t scale_copy(void *y, const void *x, double ar, double ai, i64 n, hipStream_t s);
// inverse of axis_slice (complex128 in and out): out[x][k][p0+p][q0+q] = in[k][x][p][q]
hipError_t axis_scatter(const void *in, void *out, int nax, int nk, int n, int p0, int np, int q0, int nq,
                        int transpose, hipStream_t s);
hipError_t conj_scale(void *y, const void *x, double s, i64 n, hipStream_t st);
// caller-layout doubles: out = scale * c(P(ij) P(ab) y), c = conjugation when conj != 0 (out of place)
hipError_t antisym(const void *y, void *out, int R, KMesh km, int o, int v, double scale, int conj, hipStream_t s);
// four-index complex128 permutation: output dim d = input dim perm[d]; output momentum signs sg_out
hipError_t permute4(const void *in, void *out, KMesh km, const int *ext_in, const int *perm, const int *sg_out,
                    hipStream_t s);
template <typename T>
hipError_t pp_in(const void *y, void *Z, KMesh km, int R, int o, int v, double scale, hipStream_t s);
// out += scale * (in - in with (a,b) and ka/kb swapped): completes a doubles array that holds one
// block of each (ka, kb) pair
template <typename T>
hipError_t expand_ab(const void *in, void *out, KMesh km, int R, int o, int v, double scale, hipStream_t s);
template <typename T>
hipError_t add_inplace(void *y, const void *x, i64 n, hipStream_t s);
template <typename T>
hipError_t zero_fill(void *y, i64 n, hipStream_t s);
template <typename T>
hipError_t pair_transpose(const void *in, void *out, int nk, int naux, int m, hipStream_t s);
// out[k1][k2][Q][p0+p][q0+q] += in[k1][k2][Q][p][q] (complex128; the reverse of chol_slice)
hipError_t slice_add(const void *in, void *out, int nk, int naux, int n, int p0, int np, int q0, int nq,
                     hipStream_t s);
// g[ki][kj][ki][i][j][a][b] += c x[ki][i][a] y[kj][j][b] (complex128, oovv-class blocks)
hipError_t outer_oovv(void *g, const void *x, const void *y, double c, int nk, int o, int v, hipStream_t s);
}  // namespace lrcc
