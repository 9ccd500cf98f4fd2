// Streaming (HBM-bound) kernels of the sigma path: layout transposes between
// the caller's rhs-major layout and the internal k-block-major layout, the
// amplitude products entering tau (Eq. t2 and the perturbed analogue), the
// final P_IJ P_AB antisymmetrisation with the -omega shift, Cholesky slices,
// and precision conversion.  Grid-stride loops (over elements, or over rows of
// the doubles arrays for the per-sigma kernels); consecutive threads touch
// consecutive elements of the innermost (unit-stride) index.
#include "common.hpp"
#include "elem.hpp"

#include <algorithm>

namespace lrcc {

namespace {
inline unsigned grid_for(i64 n, int bs = 256) {
    i64 g = (n + bs - 1) / bs;
    if (g > 65536 * 4) g = 65536 * 4;
    if (g < 1) g = 1;
    return (unsigned)g;
}
template <typename T> __device__ inline typename Cx<T>::type mk(T x, T y) {
    typename Cx<T>::type r; r.x = x; r.y = y; return r;
}
// Row-wise launches: a workgroup takes whole rows of `len` consecutive elements, so the
// row index (the same for every lane) is split with 64-bit arithmetic once per row and
// the position inside the row with 32-bit arithmetic; splitting a flat 64-bit element
// index with 64-bit divisions costs more than the memory traffic of these kernels.
inline unsigned rows_grid(i64 rows) {
    return (unsigned)std::max<i64>(1, std::min<i64>(rows, 65536 * 4));
}
}

// out[b][r][e] = scale * in[r][b][e]
template <typename Tin, typename Tout>
__global__ void k_rhs_to_block(const typename Cx<Tin>::type *in, typename Cx<Tout>::type *out,
                               int R, i64 B, i64 E, double scale) {
    // rows (b, r) of the output, E elements each (E < 2^31, checked by the launcher)
    const i64 rows = (i64)R * B;
    for (i64 row = blockIdx.x; row < rows; row += gridDim.x) {
        const int r = (int)(row % R);
        const i64 b = row / R;
        const typename Cx<Tin>::type *src = in + ((i64)r * B + b) * E;
        typename Cx<Tout>::type *dst = out + row * E;
        for (int e = threadIdx.x; e < (int)E; e += blockDim.x) {
            auto v = src[e];
            dst[e] = mk<Tout>((Tout)(scale * v.x), (Tout)(scale * v.y));
        }
    }
}

template <typename Tin, typename Tout>
hipError_t rhs_to_block(const void *in, void *out, int R, i64 B, i64 E, double scale, hipStream_t s) {
    if (E >= ((i64)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_rhs_to_block<Tin, Tout>), dim3(rows_grid((i64)R * B)), dim3(256), 0, s,
                       (const typename Cx<Tin>::type *)in, (typename Cx<Tout>::type *)out, R, B, E, scale);
    return hipGetLastError();
}

// out = x2 + c * (x_ia t_jb + t_ia x_jb - x_ib t_ja - t_ib x_ja), k-blocked, rhs inside the block.
// x1 [nk][R][o][v], t1 [nk][o][v], x2/out [nk^3][R][o][o][v][v]
template <typename T>
__global__ void k_tau_like(const typename Cx<T>::type *x1, const typename Cx<T>::type *x2,
                           const typename Cx<T>::type *t1, typename Cx<T>::type *out,
                           KMesh km, int R, int o, int v, T c, int x1_has_rhs) {
    const int nk = km.size(), vv = v * v;
    const i64 rows = (i64)nk * nk * nk * R * o * o;
    for (i64 row = blockIdx.x; row < rows; row += gridDim.x) {
        // row = (((ki nk + kj) nk + ka) R + r) o + i) o + j, elements (a, b)
        i64 q = row;
        const int j = (int)(q % o); q /= o;
        const int i = (int)(q % o); q /= o;
        const int r = (int)(q % R); q /= R;
        const int ka = (int)(q % nk); q /= nk;
        const int kj = (int)(q % nk); q /= nk;
        const int ki = (int)q;
        const int kb = km.comb(ki, kj, ka);
        const int rx = x1_has_rhs ? r : 0;
        const int Rx = x1_has_rhs ? R : 1;
        auto X = [&](int k, int ii, int aa) { return x1[(((i64)k * Rx + rx) * o + ii) * v + aa]; };
        auto Tt = [&](int k, int ii, int aa) { return t1[((i64)k * o + ii) * v + aa]; };
        const typename Cx<T>::type *src = x2 + row * vv;
        typename Cx<T>::type *dst = out + row * vv;
        for (int e = threadIdx.x; e < vv; e += blockDim.x) {
            const int a = e / v, b = e - a * v;
            auto acc = src[e];
            T sr = 0, si = 0;
            if (ka == ki) {     // x_ia t_jb + t_ia x_jb  (kb == kj)
                auto p = X(ki, i, a), q2 = Tt(kj, j, b), u = Tt(ki, i, a), w = X(kj, j, b);
                sr += p.x * q2.x - p.y * q2.y + u.x * w.x - u.y * w.y;
                si += p.x * q2.y + p.y * q2.x + u.x * w.y + u.y * w.x;
            }
            if (kb == ki) {     // - x_ib t_ja - t_ib x_ja  (ka == kj)
                auto p = X(ki, i, b), q2 = Tt(kj, j, a), u = Tt(ki, i, b), w = X(kj, j, a);
                sr -= p.x * q2.x - p.y * q2.y + u.x * w.x - u.y * w.y;
                si -= p.x * q2.y + p.y * q2.x + u.x * w.y + u.y * w.x;
            }
            dst[e] = mk<T>(acc.x + c * sr, acc.y + c * si);
        }
    }
}

template <typename T>
hipError_t tau_like(const void *x1, const void *x2, const void *t1, void *out, KMesh km, int R, int o, int v,
                    double c, int x1_has_rhs, hipStream_t s) {
    const int nk = km.size();
    const i64 rows = (i64)nk * nk * nk * R * o * o;
    hipLaunchKernelGGL(k_tau_like<T>, dim3(rows_grid(rows)), dim3(256), 0, s,
                       (const typename Cx<T>::type *)x1, (const typename Cx<T>::type *)x2,
                       (const typename Cx<T>::type *)t1, (typename Cx<T>::type *)out, km, R, o, v, (T)c,
                       x1_has_rhs);
    return hipGetLastError();
}

// y2[r][ki,kj,ka][i][j][a][b] = scale * (P_ij P_ab Z)[ki,kj,ka][r][i][j][a][b] - omega_r * x2[r][...]
// The four rows (ki,kj,ka,i,j), (kj,ki,ka,j,i), (ki,kj,kb,i,j), (kj,ki,kb,j,i) of one orbit of the
// antisymmetriser read the same four rows of Z: with P, Q, R, S those rows and A = P - Q - R^T + S^T
// (transposes in (a, b)) they are A, -A, -A^T and A^T.  The workgroup of the orbit's first row
// ((ki, i) <= (kj, j), ka <= kb) writes all of its distinct rows, so Z is read about once per output
// (the transposed reads of a row hit the cache lines its direct reads brought in); the other
// workgroups return at once.
template <typename T>
__global__ void k_pp_out(const typename Cx<T>::type *Z, const double2 *x2, double2 *y2, const double *omega,
                         KMesh km, int R, int o, int v, double scale) {
    const int nk = km.size(), vv = v * v;
    const i64 B = (i64)nk * nk * nk;
    const i64 rows = B * R * o * o;
    for (i64 row = blockIdx.x; row < rows; row += gridDim.x) {
        // row indexes the caller layout [r][blk][i][j], elements (a, b)
        i64 q = row;
        const int j = (int)(q % o); q /= o;
        const int i = (int)(q % o); q /= o;
        const i64 blk = q % B;
        const int r = (int)(q / B);
        const int ka = (int)(blk % nk), kj = (int)((blk / nk) % nk), ki = (int)(blk / (nk * nk));
        const int kb = km.comb(ki, kj, ka);
        const int pi = ki * o + i, pj = kj * o + j;
        if (pi > pj || ka > kb) continue;
        const bool two_pairs = pi != pj, two_blocks = ka != kb;
        auto zrow = [&](int k0, int k1, int k2, int p, int q3) {
            return Z + ((((i64)(k0 * nk + k1) * nk + k2) * R + r) * o + p) * o * vv + (i64)q3 * vv;
        };
        auto yrow = [&](int k0, int k1, int k2, int p, int q3) {
            return (((i64)r * B + ((i64)k0 * nk + k1) * nk + k2) * o + p) * o * vv + (i64)q3 * vv;
        };
        const typename Cx<T>::type *P = zrow(ki, kj, ka, i, j), *Q = zrow(kj, ki, ka, j, i);
        const typename Cx<T>::type *Rz = zrow(ki, kj, kb, i, j), *S = zrow(kj, ki, kb, j, i);
        const i64 o0 = row * vv, o1 = yrow(kj, ki, ka, j, i), o2 = yrow(ki, kj, kb, i, j), o3 = yrow(kj, ki, kb, j, i);
        const double w = omega ? omega[r] : 0.0;
        auto put = [&](i64 off, int e, double zr, double zi) {
            double2 out;
            out.x = scale * zr;
            out.y = scale * zi;
            if (omega) {
                const double2 xv = x2[off + e];
                out.x -= w * xv.x;
                out.y -= w * xv.y;
            }
            y2[off + e] = out;
        };
        for (int e = threadIdx.x; e < vv; e += blockDim.x) {
            const int a = e / v, b = e - a * v, et = b * v + a;
            const auto p = P[e], qd = Q[e], rt = Rz[et], st = S[et];
            const double ar = (double)p.x - (double)qd.x - (double)rt.x + (double)st.x;
            const double ai = (double)p.y - (double)qd.y - (double)rt.y + (double)st.y;
            put(o0, e, ar, ai);
            if (two_pairs) put(o1, e, -ar, -ai);
            if (two_blocks) {
                const auto pt = P[et], qt = Q[et], rd = Rz[e], sd = S[e];
                const double tr = (double)pt.x - (double)qt.x - (double)rd.x + (double)sd.x;
                const double ti = (double)pt.y - (double)qt.y - (double)rd.y + (double)sd.y;
                put(o2, e, -tr, -ti);
                if (two_pairs) put(o3, e, tr, ti);
            }
        }
    }
}

template <typename T>
hipError_t pp_out(const void *Z, const void *x2, void *y2, const double *omega, KMesh km, int R, int o, int v,
                  double scale, hipStream_t s) {
    const int nk = km.size();
    const i64 rows = (i64)nk * nk * nk * R * o * o;
    hipLaunchKernelGGL(k_pp_out<T>, dim3(rows_grid(rows)), dim3(256), 0, s, (const typename Cx<T>::type *)Z,
                       (const double2 *)x2, (double2 *)y2, omega, km, R, o, v, scale);
    return hipGetLastError();
}

// y1[r][k][i][a] = s1[k][r][i][a] - omega_r x1[r][k][i][a]
template <typename T>
__global__ void k_s1_out(const typename Cx<T>::type *s1, const double2 *x1, double2 *y1, const double *omega,
                         int nk, int R, int o, int v) {
    const i64 E = (i64)o * v;
    const i64 n = (i64)R * nk * E;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        const i64 e = t % E;
        const int k = (int)((t / E) % nk);
        const int r = (int)(t / (E * nk));
        auto sv = s1[((i64)k * R + r) * E + e];
        double2 out;
        out.x = (double)sv.x;
        out.y = (double)sv.y;
        if (omega) {
            const double w = omega[r];
            const double2 xv = x1[t];
            out.x -= w * xv.x;
            out.y -= w * xv.y;
        }
        y1[t] = out;
    }
}

template <typename T>
hipError_t s1_out(const void *s1, const void *x1, void *y1, const double *omega, int nk, int R, int o, int v,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_s1_out<T>, dim3(grid_for((i64)R * nk * o * v)), dim3(256), 0, s,
                       (const typename Cx<T>::type *)s1, (const double2 *)x1, (double2 *)y1, omega, nk, R, o, v);
    return hipGetLastError();
}

// Slice of Cholesky vectors: out[k1][k2][Q][p][q] = scale * L[k1][k2][Q][p0+p][q0+q]   (conj_pair = 0)
//                            out[k1][k2][Q][p][q] = scale * conj(L[k2][k1][Q][q0+q][p0+p])  (conj_pair = 1)
template <typename Tout>
__global__ void k_chol_slice(const double2 *L, typename Cx<Tout>::type *out, int nk, int naux, int n, int p0,
                             int np, int q0, int nq, double scale, int conj_pair) {
    const i64 n_out = (i64)nk * nk * naux * np * nq;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n_out; t += (i64)gridDim.x * blockDim.x) {
        i64 q = t;
        const int qq = (int)(q % nq); q /= nq;
        const int pp = (int)(q % np); q /= np;
        const int Q = (int)(q % naux); q /= naux;
        const int k2 = (int)(q % nk);
        const int k1 = (int)(q / nk);
        double2 v;
        if (!conj_pair) {
            v = L[(((i64)(k1 * nk + k2) * naux + Q) * n + (p0 + pp)) * n + (q0 + qq)];
        } else {
            v = L[(((i64)(k2 * nk + k1) * naux + Q) * n + (q0 + qq)) * n + (p0 + pp)];
            v.y = -v.y;
        }
        out[t] = mk<Tout>((Tout)(scale * v.x), (Tout)(scale * v.y));
    }
}

template <typename Tout>
hipError_t chol_slice(const void *L, void *out, int nk, int naux, int n, int p0, int np, int q0, int nq,
                      double scale, int conj_pair, hipStream_t s) {
    hipLaunchKernelGGL(k_chol_slice<Tout>, dim3(grid_for((i64)nk * nk * naux * np * nq)), dim3(256), 0, s,
                       (const double2 *)L, (typename Cx<Tout>::type *)out, nk, naux, n, p0, np, q0, nq, scale,
                       conj_pair);
    return hipGetLastError();
}

// Strided block copy of the 1E matrices: out[k][p][q] = in[k][p0+p][q0+q] (in: [nk][n][n])
template <typename Tout>
__global__ void k_one_body_slice(const double2 *in, typename Cx<Tout>::type *out, int nk, int n, int p0, int np,
                                 int q0, int nq) {
    const i64 N = (i64)nk * np * nq;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        const int qq = (int)(t % nq), pp = (int)((t / nq) % np), k = (int)(t / ((i64)nq * np));
        double2 v = in[((i64)k * n + p0 + pp) * n + q0 + qq];
        out[t] = mk<Tout>((Tout)v.x, (Tout)v.y);
    }
}

template <typename Tout>
hipError_t one_body_slice(const void *in, void *out, int nk, int n, int p0, int np, int q0, int nq, hipStream_t s) {
    hipLaunchKernelGGL(k_one_body_slice<Tout>, dim3(grid_for((i64)nk * np * nq)), dim3(256), 0, s,
                       (const double2 *)in, (typename Cx<Tout>::type *)out, nk, n, p0, np, q0, nq);
    return hipGetLastError();
}

template <typename Tout>
__global__ void k_axis_slice(const double2 *in, typename Cx<Tout>::type *out, int nax, int nk, int n, int p0, int np,
                             int q0, int nq, int transpose) {
    const i64 N = (i64)nk * nax * np * nq;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        i64 q = t;
        const int qq = (int)(q % nq); q /= nq;
        const int pp = (int)(q % np); q /= np;
        const int x = (int)(q % nax);
        const int k = (int)(q / nax);
        const double2 v = transpose ? in[(((i64)x * nk + k) * n + q0 + qq) * n + p0 + pp]
                                    : in[(((i64)x * nk + k) * n + p0 + pp) * n + q0 + qq];
        out[t] = mk<Tout>((Tout)v.x, (Tout)v.y);
    }
}

template <typename Tout>
hipError_t axis_slice(const void *in, void *out, int nax, int nk, int n, int p0, int np, int q0, int nq, int transpose,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_axis_slice<Tout>, dim3(grid_for((i64)nk * nax * np * nq)), dim3(256), 0, s,
                       (const double2 *)in, (typename Cx<Tout>::type *)out, nax, nk, n, p0, np, q0, nq, transpose);
    return hipGetLastError();
}

// Inverse of axis_slice: out[x][k][p0+p][q0+q] = in[k][x][p][q]
// (transpose: out[x][k][q0+q][p0+p] = in[k][x][p][q]); complex128.
__global__ void k_axis_scatter(const double2 *in, double2 *out, int nax, int nk, int n, int p0, int np, int q0,
                               int nq, int transpose) {
    const i64 N = (i64)nk * nax * np * nq;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        i64 q = t;
        const int qq = (int)(q % nq); q /= nq;
        const int pp = (int)(q % np); q /= np;
        const int x = (int)(q % nax);
        const int k = (int)(q / nax);
        const i64 dst = transpose ? (((i64)x * nk + k) * n + q0 + qq) * n + p0 + pp
                                  : (((i64)x * nk + k) * n + p0 + pp) * n + q0 + qq;
        out[dst] = in[t];
    }
}

hipError_t axis_scatter(const void *in, void *out, int nax, int nk, int n, int p0, int np, int q0, int nq,
                        int transpose, hipStream_t s) {
    hipLaunchKernelGGL(k_axis_scatter, dim3(grid_for((i64)nk * nax * np * nq)), dim3(256), 0, s,
                       (const double2 *)in, (double2 *)out, nax, nk, n, p0, np, q0, nq, transpose);
    return hipGetLastError();
}

// y = alpha * x (complex alpha, n elements, double2)
__global__ void k_scale_copy(double2 *y, const double2 *x, double ar, double ai, i64 n) {
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        const double2 v = x[t];
        y[t] = make_double2(ar * v.x - ai * v.y, ar * v.y + ai * v.x);
    }
}
hipError_t scale_copy(void *y, const void *x, double ar, double ai, i64 n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, s, (double2 *)y, (const double2 *)x, ar, ai, n);
    return hipGetLastError();
}

// out = in with permuted indices: output dim d is input dim perm[d]; output blocks
// [k0][k1][k2] with k3 from the output momentum signs sg (both tensors conserve momentum).
__global__ void k_permute4(const double2 *in, double2 *out, KMesh km, int e0, int e1, int e2, int e3, int p0, int p1,
                           int p2, int p3, int s0, int s1, int s2, int s3) {
    const int ein[4] = {e0, e1, e2, e3}, perm[4] = {p0, p1, p2, p3}, sg[4] = {s0, s1, s2, s3};
    int eo[4];
    for (int d = 0; d < 4; ++d) eo[d] = ein[perm[d]];
    const int nk = km.size();
    const i64 inner = (i64)e0 * e1 * e2 * e3;
    const i64 n = (i64)nk * nk * nk * inner;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        i64 q = t;
        int io[4], ko[4];
        for (int d = 3; d >= 0; --d) { io[d] = (int)(q % eo[d]); q /= eo[d]; }
        ko[2] = (int)(q % nk); q /= nk;
        ko[1] = (int)(q % nk); q /= nk;
        ko[0] = (int)q;
        ko[3] = km.sum3(-sg[3] * sg[0], ko[0], -sg[3] * sg[1], ko[1], -sg[3] * sg[2], ko[2]);
        int ii[4], ki[4];
        for (int d = 0; d < 4; ++d) { ii[perm[d]] = io[d]; ki[perm[d]] = ko[d]; }
        const i64 src = (((i64)(ki[0] * nk + ki[1]) * nk + ki[2]) * inner) +
                        (((i64)ii[0] * e1 + ii[1]) * e2 + ii[2]) * e3 + ii[3];
        out[t] = in[src];
    }
}

hipError_t permute4(const void *in, void *out, KMesh km, const int *ext_in, const int *perm, const int *sg_out,
                    hipStream_t s) {
    const int nk = km.size();
    const i64 n = (i64)nk * nk * nk * ext_in[0] * ext_in[1] * ext_in[2] * ext_in[3];
    hipLaunchKernelGGL(k_permute4, dim3(grid_for(n)), dim3(256), 0, s, (const double2 *)in, (double2 *)out, km,
                       ext_in[0], ext_in[1], ext_in[2], ext_in[3], perm[0], perm[1], perm[2], perm[3], sg_out[0],
                       sg_out[1], sg_out[2], sg_out[3]);
    return hipGetLastError();
}

// y = s * conj(x)
__global__ void k_conj_scale(double2 *y, const double2 *x, double s, i64 n) {
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        const double2 v = x[t];
        y[t] = make_double2(s * v.x, -s * v.y);
    }
}
hipError_t conj_scale(void *y, const void *x, double s, i64 n, hipStream_t st) {
    hipLaunchKernelGGL(k_conj_scale, dim3(grid_for(n)), dim3(256), 0, st, (double2 *)y, (const double2 *)x, s, n);
    return hipGetLastError();
}

// out = scale * c(y - y(ij swapped) - y(ab swapped) + y(both swapped)) on caller-layout doubles
// [R][ki][kj][ka][i][j][a][b] (kb implied), c = complex conjugation when conj != 0.  Out of place.
__global__ void k_antisym(const double2 *y, double2 *out, int R, KMesh km, int o, int v, double scale, int conj) {
    const int nk = km.size(), vv = v * v;
    const i64 B = (i64)nk * nk * nk;
    const i64 rows = (i64)R * B * o * o;
    for (i64 row = blockIdx.x; row < rows; row += gridDim.x) {
        // row = [r][ki][kj][ka][i][j], elements (a, b)
        i64 q = row;
        const int j = (int)(q % o); q /= o;
        const int i = (int)(q % o); q /= o;
        const int ka = (int)(q % nk); q /= nk;
        const int kj = (int)(q % nk); q /= nk;
        const int ki = (int)(q % nk);
        const i64 r = q / nk;
        const int kb = km.comb(ki, kj, ka);
        auto rowp = [&](int k0, int k1, int k2, int p, int q3) {
            return y + ((r * B + ((i64)k0 * nk + k1) * nk + k2) * o + p) * o * vv + (i64)q3 * vv;
        };
        const double2 *Y1 = rowp(ki, kj, ka, i, j), *Y2 = rowp(kj, ki, ka, j, i);
        const double2 *Y3 = rowp(ki, kj, kb, i, j), *Y4 = rowp(kj, ki, kb, j, i);
        double2 *dst = out + row * vv;
        for (int e = threadIdx.x; e < vv; e += blockDim.x) {
            const int a = e / v, b = e - a * v, et = b * v + a;
            const double2 z1 = Y1[e], z2 = Y2[e], z3 = Y3[et], z4 = Y4[et];
            const double re = scale * (z1.x - z2.x - z3.x + z4.x), im = scale * (z1.y - z2.y - z3.y + z4.y);
            dst[e] = make_double2(re, conj ? -im : im);
        }
    }
}

hipError_t antisym(const void *y, void *out, int R, KMesh km, int o, int v, double scale, int conj, hipStream_t s) {
    const int nk = km.size();
    const i64 rows = (i64)R * nk * nk * nk * o * o;
    hipLaunchKernelGGL(k_antisym, dim3(rows_grid(rows)), dim3(256), 0, s, (const double2 *)y, (double2 *)out, R, km, o,
                       v, scale, conj);
    return hipGetLastError();
}

__global__ void k_convert(const double2 *in, float2 *out, i64 n) {
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        double2 v = in[t];
        out[t] = make_float2((float)v.x, (float)v.y);
    }
}

hipError_t convert_f64_f32(const void *in, void *out, i64 n, hipStream_t s) {
    hipLaunchKernelGGL(k_convert, dim3(grid_for(n)), dim3(256), 0, s, (const double2 *)in, (float2 *)out, n);
    return hipGetLastError();
}

// Z[ki,kj,ka][r][i][j][a][b] = scale * (P_ij P_ab y)[r][ki,kj,ka][i][j][a][b]  (caller layout in, block layout out)
template <typename T>
__global__ void k_pp_in(const double2 *y, typename Cx<T>::type *Z, KMesh km, int R, int o, int v, double scale) {
    const int nk = km.size(), vv = v * v;
    const i64 B = (i64)nk * nk * nk;
    const i64 rows = B * R * o * o;
    for (i64 row = blockIdx.x; row < rows; row += gridDim.x) {
        // row indexes the block layout [blk][r][i][j], elements (a, b)
        i64 q = row;
        const int j = (int)(q % o); q /= o;
        const int i = (int)(q % o); q /= o;
        const int r = (int)(q % R);
        const i64 blk = q / R;
        const int ka = (int)(blk % nk), kj = (int)((blk / nk) % nk), ki = (int)(blk / (nk * nk));
        const int kb = km.comb(ki, kj, ka);
        auto rowp = [&](int k0, int k1, int k2, int p, int q3) {
            return y + (((i64)r * B + ((i64)k0 * nk + k1) * nk + k2) * o + p) * o * vv + (i64)q3 * vv;
        };
        const double2 *Y1 = rowp(ki, kj, ka, i, j), *Y2 = rowp(kj, ki, ka, j, i);
        const double2 *Y3 = rowp(ki, kj, kb, i, j), *Y4 = rowp(kj, ki, kb, j, i);
        typename Cx<T>::type *dst = Z + row * vv;
        for (int e = threadIdx.x; e < vv; e += blockDim.x) {
            const int a = e / v, b = e - a * v, et = b * v + a;
            const double2 z1 = Y1[e], z2 = Y2[e], z3 = Y3[et], z4 = Y4[et];
            dst[e] = mk<T>((T)(scale * (z1.x - z2.x - z3.x + z4.x)), (T)(scale * (z1.y - z2.y - z3.y + z4.y)));
        }
    }
}

template <typename T>
hipError_t pp_in(const void *y, void *Z, KMesh km, int R, int o, int v, double scale, hipStream_t s) {
    const int nk = km.size();
    const i64 rows = (i64)nk * nk * nk * R * o * o;
    hipLaunchKernelGGL(k_pp_in<T>, dim3(rows_grid(rows)), dim3(256), 0, s, (const double2 *)y,
                       (typename Cx<T>::type *)Z, km, R, o, v, scale);
    return hipGetLastError();
}

// out[blk][r][i][j][a][b] += scale * (in[blk][r][i][j][a][b] - in[blk'][r][i][j][b][a]), blk = (ki,kj,ka),
// blk' = (ki,kj,kb): the (a,b)-antisymmetric completion of a block-layout doubles array that holds
// only one block of each (ka, kb) pair
template <typename T>
__global__ void k_expand_ab(const typename Cx<T>::type *in, typename Cx<T>::type *out, KMesh km, int R, int o,
                            int v, T scale) {
    const int nk = km.size(), vv = v * v;
    const i64 inblk = (i64)R * o * o;
    const i64 rows = (i64)nk * nk * nk * inblk;
    for (i64 row = blockIdx.x; row < rows; row += gridDim.x) {
        // row = [blk][r][i][j], elements (a, b)
        const i64 blk = row / inblk, rest = row - blk * inblk;
        const int ka = (int)(blk % nk), kj = (int)((blk / nk) % nk), ki = (int)(blk / (nk * nk));
        const int kb = km.comb(ki, kj, ka);
        const typename Cx<T>::type *X1 = in + row * vv;
        const typename Cx<T>::type *X2 = in + ((((i64)ki * nk + kj) * nk + kb) * inblk + rest) * vv;
        typename Cx<T>::type *dst = out + row * vv;
        for (int e = threadIdx.x; e < vv; e += blockDim.x) {
            const int a = e / v, b = e - a * v;
            const auto x1 = X1[e], x2 = X2[b * v + a], y = dst[e];
            dst[e] = mk<T>(y.x + scale * (x1.x - x2.x), y.y + scale * (x1.y - x2.y));
        }
    }
}

template <typename T>
hipError_t expand_ab(const void *in, void *out, KMesh km, int R, int o, int v, double scale, hipStream_t s) {
    const int nk = km.size();
    const i64 rows = (i64)nk * nk * nk * R * o * o;
    hipLaunchKernelGGL(k_expand_ab<T>, dim3(rows_grid(rows)), dim3(256), 0, s, (const typename Cx<T>::type *)in,
                       (typename Cx<T>::type *)out, km, R, o, v, (T)scale);
    return hipGetLastError();
}

// y += x (complex, n elements)
template <typename T>
__global__ void k_add(typename Cx<T>::type *y, const typename Cx<T>::type *x, i64 n) {
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        auto a = y[t], b = x[t];
        y[t] = mk<T>(a.x + b.x, a.y + b.y);
    }
}
template <typename T>
hipError_t add_inplace(void *y, const void *x, i64 n, hipStream_t s) {
    hipLaunchKernelGGL(k_add<T>, dim3(grid_for(n)), dim3(256), 0, s, (typename Cx<T>::type *)y,
                       (const typename Cx<T>::type *)x, n);
    return hipGetLastError();
}

// zero fill (a kernel rather than a memset so that programs stay capturable)
template <typename T>
__global__ void k_zero(typename Cx<T>::type *y, i64 n) {
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) y[t] = mk<T>(0, 0);
}
template <typename T>
hipError_t zero_fill(void *y, i64 n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero<T>, dim3(grid_for(n)), dim3(256), 0, s, (typename Cx<T>::type *)y, n);
    return hipGetLastError();
}

// out[k2][k1][Q][q][p] = in[k1][k2][Q][p][q]   ([nk][nk][naux][m][m] blocks)
template <typename T>
__global__ void k_pair_transpose(const typename Cx<T>::type *in, typename Cx<T>::type *out, int nk, int naux, int m) {
    const i64 n = (i64)nk * nk * naux * m * m;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        i64 q = t;
        const int p = (int)(q % m); q /= m;
        const int qq = (int)(q % m); q /= m;
        const int Q = (int)(q % naux); q /= naux;
        const int k1 = (int)(q % nk);
        const int k2 = (int)(q / nk);
        // t = [k2][k1][Q][qq][p]
        out[t] = in[(((i64)(k1 * nk + k2) * naux + Q) * m + p) * m + qq];
    }
}
template <typename T>
hipError_t pair_transpose(const void *in, void *out, int nk, int naux, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_transpose<T>, dim3(grid_for((i64)nk * nk * naux * m * m)), dim3(256), 0, s,
                       (const typename Cx<T>::type *)in, (typename Cx<T>::type *)out, nk, naux, m);
    return hipGetLastError();
}

// Reverse of chol_slice (no conjugation, scale 1): out[k1][k2][Q][p0+p][q0+q] += in[k1][k2][Q][p][q]
// (complex128; out is a full [nk][nk][naux][n][n] array)
__global__ void k_slice_add(const double2 *in, double2 *out, int nk, int naux, int n, int p0, int np, int q0,
                            int nq) {
    const i64 N = (i64)nk * nk * naux * np * nq;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        i64 q = t;
        const int qq = (int)(q % nq); q /= nq;
        const int pp = (int)(q % np); q /= np;
        const i64 dst = (q * n + p0 + pp) * n + q0 + qq;   // q = (k1 * nk + k2) * naux + Q
        const double2 a = out[dst], b = in[t];
        out[dst] = make_double2(a.x + b.x, a.y + b.y);
    }
}

hipError_t slice_add(const void *in, void *out, int nk, int naux, int n, int p0, int np, int q0, int nq,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_slice_add, dim3(grid_for((i64)nk * nk * naux * np * nq)), dim3(256), 0, s,
                       (const double2 *)in, (double2 *)out, nk, naux, n, p0, np, q0, nq);
    return hipGetLastError();
}

// g[ki][kj][ki][i][j][a][b] += c x[ki][i][a] y[kj][j][b]: the k-diagonal singles x, y put into the
// blocks (ki, kj, ka = ki, kb = kj) of an oovv-class array (complex128)
__global__ void k_outer_oovv(double2 *g, const double2 *x, const double2 *y, double c, int nk, int o, int v) {
    const i64 N = (i64)nk * nk * o * o * v * v;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        i64 q = t;
        const int b = (int)(q % v); q /= v;
        const int a = (int)(q % v); q /= v;
        const int j = (int)(q % o); q /= o;
        const int i = (int)(q % o); q /= o;
        const int kj = (int)(q % nk);
        const int ki = (int)(q / nk);
        const double2 xv = x[((i64)ki * o + i) * v + a], yv = y[((i64)kj * o + j) * v + b];
        const i64 dst = (((((i64)ki * nk + kj) * nk + ki) * o + i) * o + j) * v * v + (i64)a * v + b;
        const double2 gv = g[dst];
        g[dst] = make_double2(gv.x + c * (xv.x * yv.x - xv.y * yv.y), gv.y + c * (xv.x * yv.y + xv.y * yv.x));
    }
}

hipError_t outer_oovv(void *g, const void *x, const void *y, double c, int nk, int o, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_outer_oovv, dim3(grid_for((i64)nk * nk * o * o * v * v)), dim3(256), 0, s, (double2 *)g,
                       (const double2 *)x, (const double2 *)y, c, nk, o, v);
    return hipGetLastError();
}

#define INST(T)                                                                                              \
    template hipError_t pp_in<T>(const void *, void *, KMesh, int, int, int, double, hipStream_t);             \
    template hipError_t add_inplace<T>(void *, const void *, i64, hipStream_t);                              \
    template hipError_t expand_ab<T>(const void *, void *, KMesh, int, int, int, double, hipStream_t);        \
    template hipError_t zero_fill<T>(void *, i64, hipStream_t);                                              \
    template hipError_t pair_transpose<T>(const void *, void *, int, int, int, hipStream_t);                                                                                              \
    template hipError_t tau_like<T>(const void *, const void *, const void *, void *, KMesh, int, int, int,  \
                                    double, int, hipStream_t);                                               \
    template hipError_t pp_out<T>(const void *, const void *, void *, const double *, KMesh, int, int, int,  \
                                  double, hipStream_t);                                                      \
    template hipError_t s1_out<T>(const void *, const void *, void *, const double *, int, int, int, int,    \
                                  hipStream_t);                                                              \
    template hipError_t chol_slice<T>(const void *, void *, int, int, int, int, int, int, int, double, int,  \
                                      hipStream_t);                                                          \
    template hipError_t one_body_slice<T>(const void *, void *, int, int, int, int, int, int, hipStream_t);  \
    template hipError_t axis_slice<T>(const void *, void *, int, int, int, int, int, int, int, int, hipStream_t); \
    template hipError_t rhs_to_block<double, T>(const void *, void *, int, i64, i64, double, hipStream_t);
INST(double)
INST(float)

}  // namespace lrcc
