// Streaming kernels of the response solver: batched inner products with a
// fixed reduction tree (bitwise reproducible for a given launch shape), batched
// axpy with one complex coefficient per right-hand side, and the orbital-energy
// denominator preconditioner (the Jacobi update of Sec. II.C with the
// denominators of Eq. D shifted by -omega).  Vectors use the caller layout
// [nrhs][...] with each right-hand side contiguous.
#include "common.hpp"
#include "solver.hpp"

#include <algorithm>

namespace lrcc {

namespace {
constexpr int DB = 256;
}

// Krylov vectors are kept in complex128 (double2) or, for the complex64 inner solves of the
// mixed refinement, in complex64 (float2); the arithmetic on them is complex128 either way.
static __device__ __forceinline__ double2 ld2(const double2 *p, i64 i) { return p[i]; }
static __device__ __forceinline__ double2 ld2(const float2 *p, i64 i) {
    const float2 v = p[i];
    return make_double2(v.x, v.y);
}
static __device__ __forceinline__ void st2(double2 *p, i64 i, double2 v) { p[i] = v; }
static __device__ __forceinline__ void st2(float2 *p, i64 i, double2 v) { p[i] = make_float2((float)v.x, (float)v.y); }

// part[r][b] = sum over the fixed chunk b of conj(u_r) * v_r
__global__ void __launch_bounds__(DB) k_dot_partial(const double2 *u, const double2 *v, i64 n, int nblk, double2 *part,
                                                     int conj_u) {
    __shared__ double sr[DB], si[DB];
    const int r = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const double2 *ur = u + (i64)r * n, *vr = v + (i64)r * n;
    double ar = 0, ai = 0;
    for (i64 i = (i64)b * DB + t; i < n; i += (i64)nblk * DB) {
        double2 x = ur[i];
        const double2 y = vr[i];
        if (conj_u) x.y = -x.y;
        ar += x.x * y.x - x.y * y.y;
        ai += x.x * y.y + x.y * y.x;
    }
    sr[t] = ar;
    si[t] = ai;
    __syncthreads();
    for (int s = DB / 2; s > 0; s >>= 1) {
        if (t < s) { sr[t] += sr[t + s]; si[t] += si[t + s]; }
        __syncthreads();
    }
    if (t == 0) part[(i64)r * nblk + b] = make_double2(sr[0], si[0]);
}

__global__ void k_dot_final(const double2 *part, int nblk, int R, double scale, double2 *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double ar = 0, ai = 0;
    for (int b = 0; b < nblk; ++b) { ar += part[(i64)r * nblk + b].x; ai += part[(i64)r * nblk + b].y; }
    out[r] = make_double2(scale * ar, scale * ai);
}

int dot_blocks(i64 n) {
    i64 b = (n + DB * 8 - 1) / (DB * 8);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t batched_dot(const void *u, const void *v, int R, i64 n, double scale, void *part, void *out, hipStream_t s,
                       int conj_u) {
    const int nblk = dot_blocks(n);
    hipLaunchKernelGGL(k_dot_partial, dim3(nblk, R), dim3(DB), 0, s, (const double2 *)u, (const double2 *)v, n, nblk,
                       (double2 *)part, conj_u);
    hipLaunchKernelGGL(k_dot_final, dim3((R + 63) / 64), dim3(64), 0, s, (const double2 *)part, nblk, R, scale,
                       (double2 *)out);
    return hipGetLastError();
}

// y_r = beta * y_r + alpha_r * x_r   (alpha: R complex values on the device)
__global__ void k_axpby(double2 *y, const double2 *x, const double2 *alpha, double beta, int R, i64 n) {
    const i64 N = (i64)R * n;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        const int r = (int)(t / n);
        const double2 a = alpha[r], xv = x[t];
        double2 yv = beta == 0.0 ? make_double2(0, 0) : y[t];
        yv.x = beta * yv.x + a.x * xv.x - a.y * xv.y;
        yv.y = beta * yv.y + a.x * xv.y + a.y * xv.x;
        y[t] = yv;
    }
}

// y_r = beta * y_r + alpha_r * x_r on Krylov-vector storage (complex128 or complex64)
template <typename V>
__global__ void k_basis_axpby(V *y, const V *x, const double2 *alpha, double beta, int R, i64 n) {
    const i64 N = (i64)R * n;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        const int r = (int)(t / n);
        const double2 a = alpha[r], xv = ld2(x, t);
        double2 yv = beta == 0.0 ? make_double2(0, 0) : ld2(y, t);
        yv.x = beta * yv.x + a.x * xv.x - a.y * xv.y;
        yv.y = beta * yv.y + a.x * xv.y + a.y * xv.x;
        st2(y, t, yv);
    }
}

hipError_t basis_axpby(void *y, const void *x, const void *alpha, double beta, int R, i64 n, int f32, hipStream_t s) {
    i64 g = ((i64)R * n + 255) / 256;
    g = std::max<i64>(1, std::min<i64>(g, 262144));
    if (f32)
        hipLaunchKernelGGL(k_basis_axpby<float2>, dim3((unsigned)g), dim3(256), 0, s, (float2 *)y, (const float2 *)x,
                           (const double2 *)alpha, beta, R, n);
    else
        hipLaunchKernelGGL(k_basis_axpby<double2>, dim3((unsigned)g), dim3(256), 0, s, (double2 *)y,
                           (const double2 *)x, (const double2 *)alpha, beta, R, n);
    return hipGetLastError();
}

hipError_t batched_axpby(void *y, const void *x, const void *alpha, double beta, int R, i64 n, hipStream_t s) {
    i64 N = (i64)R * n;
    i64 g = (N + 255) / 256;
    if (g > 262144) g = 262144;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)g), dim3(256), 0, s, (double2 *)y, (const double2 *)x,
                       (const double2 *)alpha, beta, R, n);
    return hipGetLastError();
}

// singles: out[r][k][i][a] = in / (e_v[k][a] - e_o[k][i] - w_r)
// doubles: out[r][ki,kj,ka][i][j][a][b] = in / (e_v[ka][a] + e_v[kb][b] - e_o[ki][i] - e_o[kj][j] - w_r)
__global__ void k_precond(double2 *o1, double2 *o2, const double2 *i1, const double2 *i2, const double *eo,
                          const double *ev, const double *eo2, const double *ev2, const double *omega, KMesh km,
                          int R, int no, int nv) {
    const int nk = km.size();
    const i64 n1 = (i64)nk * no * nv, n2 = (i64)nk * nk * nk * no * no * nv * nv;
    const i64 N = (i64)R * (n1 + n2);
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        double d;
        double2 x;
        double2 *dst;
        if (t < (i64)R * n1) {
            const int r = (int)(t / n1);
            i64 q = t % n1;
            const int a = (int)(q % nv); q /= nv;
            const int i = (int)(q % no);
            const int k = (int)(q / no);
            d = ev[k * nv + a] - eo[k * no + i] - (omega ? omega[r] : 0.0);
            x = i1[t];
            dst = o1 + t;
        } else {
            const i64 u = t - (i64)R * n1;
            const int r = (int)(u / n2);
            i64 q = u % n2;
            const int b = (int)(q % nv); q /= nv;
            const int a = (int)(q % nv); q /= nv;
            const int j = (int)(q % no); q /= no;
            const int i = (int)(q % no); q /= no;
            const int ka = (int)(q % nk); q /= nk;
            const int kj = (int)(q % nk);
            const int ki = (int)(q / nk);
            const int kb = km.comb(ki, kj, ka);
            d = ev2[ka * nv + a] + ev2[kb * nv + b] - eo2[ki * no + i] - eo2[kj * no + j] - (omega ? omega[r] : 0.0);
            x = i2[u];
            dst = o2 + u;
        }
        if (fabs(d) < 1e-2) d = d < 0 ? -1e-2 : 1e-2;   // guard near-zero dressed denominators
        *dst = make_double2(x.x / d, x.y / d);
    }
}

hipError_t precond(void *o1, void *o2, const void *i1, const void *i2, const double *eo, const double *ev,
                   const double *eo2, const double *ev2, const double *omega, KMesh km, int R, int no, int nv,
                   hipStream_t s) {
    const int nk = km.size();
    const i64 N = (i64)R * ((i64)nk * no * nv + (i64)nk * nk * nk * no * no * nv * nv);
    i64 g = (N + 255) / 256;
    if (g > 262144) g = 262144;
    hipLaunchKernelGGL(k_precond, dim3((unsigned)g), dim3(256), 0, s, (double2 *)o1, (double2 *)o2,
                       (const double2 *)i1, (const double2 *)i2, eo, ev, eo2, ev2, omega, km, R, no, nv);
    return hipGetLastError();
}

// ------------------------------------------------------------------ packed Krylov vectors
// The doubles of every vector the solver handles are antisymmetric under (ki,i) <-> (kj,j) and
// (ka,a) <-> (kb,b) (the amplitudes of Eq. tx2, and the operator maps them to such), so the
// Krylov basis keeps one k block per orbit of those swaps: the blocks with ki <= kj and
// ka <= kb, whole, scaled by sqrt(w) with w = (full blocks in the orbit) / 4, so that the plain
// inner product of packed vectors equals the 1/4-weighted one of the full vectors.

int pack_tables(const KMesh &km, std::vector<int> &canon, std::vector<int> &map, std::vector<double> &scale) {
    const int nk = km.size();
    std::vector<int> pidx((size_t)nk * nk * nk, -1);
    canon.clear();
    scale.clear();
    map.assign((size_t)nk * nk * nk, 0);
    for (int ki = 0; ki < nk; ++ki)
        for (int kj = ki; kj < nk; ++kj)
            for (int ka = 0; ka < nk; ++ka) {
                const int kb = km.comb(ki, kj, ka);
                if (ka > kb) continue;
                const int f = (ki * nk + kj) * nk + ka;
                pidx[f] = (int)canon.size();
                canon.push_back(f);
                scale.push_back(std::sqrt((ki < kj ? 1.0 : 0.5) * (ka < kb ? 1.0 : 0.5)));
            }
    for (int ki = 0; ki < nk; ++ki)
        for (int kj = 0; kj < nk; ++kj)
            for (int ka = 0; ka < nk; ++ka) {
                const int kb = km.comb(ki, kj, ka);
                const int fc = (std::min(ki, kj) * nk + std::max(ki, kj)) * nk + std::min(ka, kb);
                map[(size_t)(ki * nk + kj) * nk + ka] = 4 * pidx[fc] + 2 * (ki > kj) + (ka > kb);
            }
    return (int)canon.size();
}

// singles: o1 = a1 - b1; doubles: o2[r][p] = scale[p] (a2 - b2)[r][canon[p]] (b may be null)
template <typename V>
__global__ void k_pack(V *o1, V *o2, const double2 *a1, const double2 *a2, const double2 *b1, const double2 *b2,
                       const int *canon, const double *scale, int R, i64 n1, int np, i64 blk, i64 n2) {
    const i64 n2p = (i64)np * blk, N1 = (i64)R * n1;
    const i64 N = N1 + (i64)R * n2p;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        if (t < N1) {
            double2 x = a1[t];
            if (b1) {
                const double2 y = b1[t];
                x.x -= y.x;
                x.y -= y.y;
            }
            st2(o1, t, x);
        } else {
            const i64 u = t - N1;
            const int r = (int)(u / n2p);
            const i64 q = u - (i64)r * n2p;
            const int p = (int)(q / blk);
            const i64 src = (i64)r * n2 + (i64)canon[p] * blk + (q - (i64)p * blk);
            double2 x = a2[src];
            if (b2) {
                const double2 y = b2[src];
                x.x -= y.x;
                x.y -= y.y;
            }
            const double sc = scale[p];
            st2(o2, u, make_double2(sc * x.x, sc * x.y));
        }
    }
}

hipError_t pack_vec(void *o1, void *o2p, const void *a1, const void *a2, const void *b1, const void *b2,
                    const PackMap &pm, int R, i64 n1, i64 blk, int f32, hipStream_t s) {
    const i64 n2 = (i64)pm.nfull * blk;
    const i64 N = (i64)R * (n1 + (i64)pm.np * blk);
    i64 g = (N + 255) / 256;
    if (g > 262144) g = 262144;
    const dim3 grid((unsigned)std::max<i64>(g, 1));
    if (f32)
        hipLaunchKernelGGL(k_pack<float2>, grid, dim3(256), 0, s, (float2 *)o1, (float2 *)o2p, (const double2 *)a1,
                           (const double2 *)a2, (const double2 *)b1, (const double2 *)b2, pm.canon, pm.scale, R, n1,
                           pm.np, blk, n2);
    else
        hipLaunchKernelGGL(k_pack<double2>, grid, dim3(256), 0, s, (double2 *)o1, (double2 *)o2p, (const double2 *)a1,
                           (const double2 *)a2, (const double2 *)b1, (const double2 *)b2, pm.canon, pm.scale, R, n1,
                           pm.np, blk, n2);
    return hipGetLastError();
}

// The preconditioned full vector of a packed one: doubles element (ki,kj,ka)(i,j,a,b) from the
// orbit's block at the swapped indices, with the sign of the swaps and 1/scale, both parts
// divided by the denominators of k_precond.
template <typename V>
__global__ void k_unpack_precond(double2 *o1, double2 *o2, const V *i1, const V *i2p, const int *map,
                                 const double *scale, const double *eo, const double *ev, const double *eo2,
                                 const double *ev2, const double *omega, KMesh km, int R, int no, int nv, int np) {
    const int nk = km.size();
    const i64 blk = (i64)no * no * nv * nv;
    const i64 n1 = (i64)nk * no * nv, n2 = (i64)nk * nk * nk * blk, n2p = (i64)np * blk;
    const i64 N = (i64)R * (n1 + n2);
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < N; t += (i64)gridDim.x * blockDim.x) {
        double d;
        double2 x;
        double2 *dst;
        if (t < (i64)R * n1) {
            const int r = (int)(t / n1);
            i64 q = t % n1;
            const int a = (int)(q % nv); q /= nv;
            const int i = (int)(q % no);
            const int k = (int)(q / no);
            d = ev[k * nv + a] - eo[k * no + i] - (omega ? omega[r] : 0.0);
            x = ld2(i1, t);
            dst = o1 + t;
        } else {
            const i64 u = t - (i64)R * n1;
            const int r = (int)(u / n2);
            i64 q = u % n2;
            const int b = (int)(q % nv); q /= nv;
            const int a = (int)(q % nv); q /= nv;
            const int j = (int)(q % no); q /= no;
            const int i = (int)(q % no); q /= no;
            const int f = (int)q;
            const int ka = f % nk, kj = (f / nk) % nk, ki = f / (nk * nk);
            const int kb = km.comb(ki, kj, ka);
            const int m = map[f], p = m >> 2;
            const bool fi = (m & 2) != 0, fa = (m & 1) != 0;
            const int ii = fi ? j : i, jj = fi ? i : j, aa = fa ? b : a, bb = fa ? a : b;
            const double2 y = ld2(i2p, (i64)r * n2p + (i64)p * blk + (((i64)ii * no + jj) * nv + aa) * nv + bb);
            const double sg = (fi != fa ? -1.0 : 1.0) / scale[p];
            x = make_double2(sg * y.x, sg * y.y);
            d = ev2[ka * nv + a] + ev2[kb * nv + b] - eo2[ki * no + i] - eo2[kj * no + j] - (omega ? omega[r] : 0.0);
            dst = o2 + u;
        }
        if (fabs(d) < 1e-2) d = d < 0 ? -1e-2 : 1e-2;   // guard near-zero dressed denominators
        *dst = make_double2(x.x / d, x.y / d);
    }
}

hipError_t unpack_precond(void *o1, void *o2, const void *i1, const void *i2p, const PackMap &pm, const double *eo,
                          const double *ev, const double *eo2, const double *ev2, const double *omega, KMesh km,
                          int R, int no, int nv, int f32, hipStream_t s) {
    const int nk = km.size();
    const i64 N = (i64)R * ((i64)nk * no * nv + (i64)nk * nk * nk * no * no * nv * nv);
    i64 g = (N + 255) / 256;
    if (g > 262144) g = 262144;
    const dim3 grid((unsigned)std::max<i64>(g, 1));
    if (f32)
        hipLaunchKernelGGL(k_unpack_precond<float2>, grid, dim3(256), 0, s, (double2 *)o1, (double2 *)o2,
                           (const float2 *)i1, (const float2 *)i2p, pm.map, pm.scale, eo, ev, eo2, ev2, omega, km, R,
                           no, nv, pm.np);
    else
        hipLaunchKernelGGL(k_unpack_precond<double2>, grid, dim3(256), 0, s, (double2 *)o1, (double2 *)o2,
                           (const double2 *)i1, (const double2 *)i2p, pm.map, pm.scale, eo, ev, eo2, ev2, omega, km,
                           R, no, nv, pm.np);
    return hipGetLastError();
}

// d[k][p] = Re F[k][p][p] for a k-diagonal complex matrix [nk][n][n]
__global__ void k_diag_real(const double2 *F, double *d, int nk, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nk * n) return;
    const int k = t / n, p = t % n;
    d[t] = F[((i64)k * n + p) * n + p].x;
}

hipError_t diag_real(const void *F, double *d, int nk, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_real, dim3((nk * n + 255) / 256), dim3(256), 0, s, (const double2 *)F, d, nk, n);
    return hipGetLastError();
}

// Y[r] = beta Y[r] + sum_i C[r][i] V[i] for R outputs from m basis vectors of length n
// (complex128; V and Y contiguous [m][n] and [R][n]; C on the device, [R][m])
__global__ void k_combine(double2 *Y, const double2 *V, const double2 *C, int R, int m, i64 n, double beta) {
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        for (int r = 0; r < R; ++r) {
            double2 acc = beta == 0.0 ? make_double2(0, 0) : Y[(i64)r * n + t];
            acc.x *= beta;
            acc.y *= beta;
            for (int i = 0; i < m; ++i) {
                const double2 c = C[r * m + i], v = V[(i64)i * n + t];
                acc.x += c.x * v.x - c.y * v.y;
                acc.y += c.x * v.y + c.y * v.x;
            }
            Y[(i64)r * n + t] = acc;
        }
    }
}

hipError_t combine(void *Y, const void *V, const void *C, int R, int m, i64 n, double beta, hipStream_t s) {
    const i64 g = std::min<i64>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_combine, dim3((unsigned)std::max<i64>(g, 1)), dim3(256), 0, s, (double2 *)Y,
                       (const double2 *)V, (const double2 *)C, R, m, n, beta);
    return hipGetLastError();
}

// ------------------------------------------------------------------ device-resident GMRES
// Vectors of one Krylov space: vector i, right-hand side r is (s + (i*R + r)*n1, d + (i*R + r)*n2).
// Inner products weight the doubles by dw (1/4 for full antisymmetric doubles, where every
// independent amplitude then counts once; 1 for packed doubles, which carry the weight).

namespace {
constexpr int MD = 256;        // threads of the multi-dot and multi-axpy kernels
constexpr int MDV = 8;         // basis vectors per multi-dot workgroup
}

// part[(r*k + i)*nblk + b] = sum over chunk b of conj(V_i[r]) w[r] (singles weight 1, doubles dw)
template <typename V>
__global__ void __launch_bounds__(MD) k_multidot_partial(const V *Vs, const V *Vd, const V *ws, const V *wd, int R,
                                                         i64 n1, i64 n2, int k, int nblk, double dw, double2 *part) {
    __shared__ double sr[MDV][MD], si[MDV][MD];
    const int b = blockIdx.x, r = blockIdx.y, i0 = blockIdx.z * MDV, t = threadIdx.x;
    const int nv = min(MDV, k - i0);
    double ar[MDV], ai[MDV];
#pragma unroll
    for (int q = 0; q < MDV; ++q) { ar[q] = 0; ai[q] = 0; }
    const i64 N = n1 + n2;
    for (i64 e = (i64)b * MD + t; e < N; e += (i64)nblk * MD) {
        const bool single = e < n1;
        const i64 off = single ? (i64)r * n1 + e : (i64)r * n2 + (e - n1);
        const double2 y = single ? ld2(ws, off) : ld2(wd, off);
        const double wt = single ? 1.0 : dw;
#pragma unroll
        for (int q = 0; q < MDV; ++q) {
            if (q < nv) {
                const i64 vo = single ? (i64)(i0 + q) * R * n1 + off : (i64)(i0 + q) * R * n2 + off;
                const double2 x = single ? ld2(Vs, vo) : ld2(Vd, vo);
                ar[q] += wt * (x.x * y.x + x.y * y.y);
                ai[q] += wt * (x.x * y.y - x.y * y.x);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < MDV; ++q) { sr[q][t] = ar[q]; si[q][t] = ai[q]; }
    __syncthreads();
    for (int st = MD / 2; st > 0; st >>= 1) {
        if (t < st)
#pragma unroll
            for (int q = 0; q < MDV; ++q) { sr[q][t] += sr[q][t + st]; si[q][t] += si[q][t + st]; }
        __syncthreads();
    }
    if (t < nv) part[((i64)r * k + i0 + t) * nblk + b] = make_double2(sr[t][0], si[t][0]);
}

// out[r*ostride + i] = sum_b part[(r*k + i)*nblk + b]  (fixed order)
__global__ void k_multidot_final(const double2 *part, int R, int k, int nblk, double2 *out, int ostride) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= R * k) return;
    const int r = q / k, i = q - r * k;
    double ar = 0, ai = 0;
    for (int b = 0; b < nblk; ++b) {
        const double2 x = part[(i64)q * nblk + b];
        ar += x.x;
        ai += x.y;
    }
    out[(i64)r * ostride + i] = make_double2(ar, ai);
}

int multidot_blocks(i64 n) {
    i64 b = (n + MD * 16 - 1) / (MD * 16);
    return (int)std::max<i64>(1, std::min<i64>(b, 512));
}

hipError_t multidot(const void *Vs, const void *Vd, const void *ws, const void *wd, int R, i64 n1, i64 n2, int k,
                    void *part, void *out, int ostride, double dw, int f32, hipStream_t s) {
    const int nblk = multidot_blocks(n1 + n2);
    const dim3 grid(nblk, R, (k + MDV - 1) / MDV);
    if (f32)
        hipLaunchKernelGGL(k_multidot_partial<float2>, grid, dim3(MD), 0, s, (const float2 *)Vs, (const float2 *)Vd,
                           (const float2 *)ws, (const float2 *)wd, R, n1, n2, k, nblk, dw, (double2 *)part);
    else
        hipLaunchKernelGGL(k_multidot_partial<double2>, grid, dim3(MD), 0, s, (const double2 *)Vs,
                           (const double2 *)Vd, (const double2 *)ws, (const double2 *)wd, R, n1, n2, k, nblk, dw,
                           (double2 *)part);
    hipLaunchKernelGGL(k_multidot_final, dim3((R * k + 63) / 64), dim3(64), 0, s, (const double2 *)part, R, k, nblk,
                       (double2 *)out, ostride);
    return hipGetLastError();
}

// w[r] = beta w[r] + sum_{i<k} c_r,i V_i[r], c_r,i = sign * C[r*cstride + i], zero where mask[r] == 0
// (mask may be null); singles and doubles in one launch (grid y = right-hand side)
template <typename V>
__global__ void __launch_bounds__(MD) k_multiaxpy(V *ws, V *wd, const V *Vs, const V *Vd, const double2 *C,
                                                  int cstride, double sign, const int *mask, double beta, int R, i64 n1,
                                                  i64 n2, int k) {
    __shared__ double2 c[64];
    const int r = blockIdx.y;
    const bool on = !mask || mask[r] != 0;
    for (int i = threadIdx.x; i < k; i += MD) {
        const double2 x = C[(i64)r * cstride + i];
        c[i] = on ? make_double2(sign * x.x, sign * x.y) : make_double2(0, 0);
    }
    __syncthreads();
    const i64 N = n1 + n2;
    for (i64 e = (i64)blockIdx.x * MD + threadIdx.x; e < N; e += (i64)gridDim.x * MD) {
        const bool single = e < n1;
        const i64 off = single ? (i64)r * n1 + e : (i64)r * n2 + (e - n1);
        V *wp = single ? ws + off : wd + off;
        double2 acc = beta == 0.0 ? make_double2(0, 0) : ld2(wp, 0);
        acc.x *= beta;
        acc.y *= beta;
        for (int i = 0; i < k; ++i) {
            const i64 vo = single ? (i64)i * R * n1 + off : (i64)i * R * n2 + off;
            const double2 x = single ? ld2(Vs, vo) : ld2(Vd, vo);
            acc.x += c[i].x * x.x - c[i].y * x.y;
            acc.y += c[i].x * x.y + c[i].y * x.x;
        }
        st2(wp, 0, acc);
    }
}

hipError_t multiaxpy(void *ws, void *wd, const void *Vs, const void *Vd, const void *C, int cstride, double sign,
                     const int *mask, double beta, int R, i64 n1, i64 n2, int k, int f32, hipStream_t s) {
    if (k > 64) return hipErrorInvalidValue;
    const i64 g = std::max<i64>(1, std::min<i64>((n1 + n2 + MD - 1) / MD, 4096));
    if (f32)
        hipLaunchKernelGGL(k_multiaxpy<float2>, dim3((unsigned)g, R), dim3(MD), 0, s, (float2 *)ws, (float2 *)wd,
                           (const float2 *)Vs, (const float2 *)Vd, (const double2 *)C, cstride, sign, mask, beta, R,
                           n1, n2, k);
    else
        hipLaunchKernelGGL(k_multiaxpy<double2>, dim3((unsigned)g, R), dim3(MD), 0, s, (double2 *)ws, (double2 *)wd,
                           (const double2 *)Vs, (const double2 *)Vd, (const double2 *)C, cstride, sign, mask, beta,
                           R, n1, n2, k);
    return hipGetLastError();
}

static __device__ double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
static __device__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
static __device__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Start of a GMRES cycle for right-hand side r (one thread each): beta = ||r0||, relative residual,
// active flag, g = (beta, 0, ...), and the scale 1/beta of the first basis vector.
__global__ void k_gmres_init(GmresState g, const double2 *beta2, double tol) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= g.R) return;
    const double b2 = beta2[r].x, bi = beta2[r].y;
    const bool fin = isfinite(b2) && isfinite(bi);
    const double beta = fin ? sqrt(fmax(0.0, b2)) : nan("");
    const double bn = g.bn[r];
    double rel = (!fin || !isfinite(bn)) ? nan("") : (bn > 0 ? beta / bn : 0.0);
    g.rel[r] = rel;
    for (int i = 0; i <= g.m; ++i) g.g[(i64)r * (g.m + 1) + i] = make_double2(i == 0 && fin ? beta : 0.0, 0.0);
    g.kr[r] = 0;
    const bool act = fin && rel > tol && beta > 0 && !g.sing[r];
    g.act[r] = act ? 1 : 0;
    g.scal[r] = make_double2(act ? 1.0 / beta : 0.0, 0.0);
}

// Arnoldi step j for right-hand side r: column j of the Hessenberg matrix from the two
// Gram-Schmidt passes, the previous Givens rotations applied to it, a new rotation, the residual
// estimate, and the scale 1/h_{j+1,j} of the next basis vector.  A pivot at or below `sing_pivot`
// (> 0 only in complex128) marks the right-hand side singular and stops it.
__global__ void k_gmres_step(GmresState g, int j, const double2 *h1, const double2 *h2, const double2 *hn2, double tol,
                             double sing_pivot) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= g.R) return;
    const int m = g.m, ld = m + 1;
    double2 *H = g.H + (i64)r * (m + 1) * m, *cs = g.cs + (i64)r * m, *sn = g.sn + (i64)r * m;
    double2 *gg = g.g + (i64)r * ld;
    if (!g.act[r]) {
        g.scal[r] = make_double2(0, 0);
        return;
    }
    for (int i = 0; i <= j; ++i) {
        const double2 a = h1[(i64)r * ld + i], b = h2 ? h2[(i64)r * ld + i] : make_double2(0, 0);
        H[i * m + j] = make_double2(a.x + b.x, a.y + b.y);
    }
    const double n2 = hn2[r].x;
    if (!isfinite(n2) || !isfinite(hn2[r].y)) {
        g.rel[r] = nan("");
        g.act[r] = 0;
        g.scal[r] = make_double2(0, 0);
        return;
    }
    const double hn = sqrt(fmax(0.0, n2));
    H[(j + 1) * m + j] = make_double2(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const double2 a = H[i * m + j], b = H[(i + 1) * m + j];
        const double2 t0 = cmul(cconj(cs[i]), a), t1 = cmul(cconj(sn[i]), b);
        const double2 u0 = cmul(sn[i], a), u1 = cmul(cs[i], b);
        H[i * m + j] = make_double2(t0.x + t1.x, t0.y + t1.y);
        H[(i + 1) * m + j] = make_double2(u1.x - u0.x, u1.y - u0.y);
    }
    const double2 a = H[j * m + j], b = H[(j + 1) * m + j];
    const double den = sqrt(cabs2(a) + cabs2(b));
    if (sing_pivot > 0 && den <= sing_pivot) {
        g.sing[r] = 1;
        g.act[r] = 0;
        g.scal[r] = make_double2(0, 0);
        return;
    }
    cs[j] = den > 0 ? make_double2(a.x / den, a.y / den) : make_double2(1, 0);
    sn[j] = den > 0 ? make_double2(b.x / den, b.y / den) : make_double2(0, 0);
    H[j * m + j] = make_double2(den, 0);
    H[(j + 1) * m + j] = make_double2(0, 0);
    const double2 gj = gg[j];
    gg[j] = cmul(cconj(cs[j]), gj);
    const double2 ng = cmul(sn[j], gj);
    gg[j + 1] = make_double2(-ng.x, -ng.y);
    g.kr[r] = j + 1;
    const double bn = g.bn[r];
    const double rel = bn > 0 ? sqrt(cabs2(gg[j + 1])) / bn : 0.0;
    g.rel[r] = rel;
    const bool act = !(rel <= tol || hn == 0 || isnan(rel));
    g.act[r] = act ? 1 : 0;
    g.scal[r] = make_double2(act && hn > 0 ? 1.0 / hn : 0.0, 0.0);
}

// End of a cycle: y = H^-1 g on the first kr[r] steps (back substitution), coefficients y[r][i].
__global__ void k_gmres_solve(GmresState g, double2 *y) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= g.R) return;
    const int m = g.m, k = g.kr[r];
    const double2 *H = g.H + (i64)r * (m + 1) * m, *gg = g.g + (i64)r * (m + 1);
    double2 *yr = y + (i64)r * (m + 1);
    for (int i = 0; i <= m; ++i) yr[i] = make_double2(0, 0);
    for (int i = k - 1; i >= 0; --i) {
        double2 acc = gg[i];
        for (int l = i + 1; l < k; ++l) {
            const double2 t = cmul(H[i * m + l], yr[l]);
            acc.x -= t.x;
            acc.y -= t.y;
        }
        const double2 d = H[i * m + i];
        const double dd = cabs2(d);
        yr[i] = dd > 0 ? make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd)
                       : make_double2(0, 0);
    }
}

// rel[r] -> status words for the host: (rel, act, sing) packed per right-hand side
__global__ void k_gmres_status(GmresState g, double *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= g.R) return;
    out[3 * r] = g.rel[r];
    out[3 * r + 1] = g.act[r];
    out[3 * r + 2] = g.sing[r];
}

hipError_t gmres_init(const GmresState &g, const void *beta2, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_init, dim3((g.R + 63) / 64), dim3(64), 0, s, g, (const double2 *)beta2, tol);
    return hipGetLastError();
}
hipError_t gmres_step(const GmresState &g, int j, const void *h1, const void *h2, const void *hn2, double tol,
                      double sing_pivot, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_step, dim3((g.R + 63) / 64), dim3(64), 0, s, g, j, (const double2 *)h1,
                       (const double2 *)h2, (const double2 *)hn2, tol, sing_pivot);
    return hipGetLastError();
}
hipError_t gmres_solve(const GmresState &g, void *y, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_solve, dim3((g.R + 63) / 64), dim3(64), 0, s, g, (double2 *)y);
    return hipGetLastError();
}
hipError_t gmres_status(const GmresState &g, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_status, dim3((g.R + 63) / 64), dim3(64), 0, s, g, out);
    return hipGetLastError();
}

// per-right-hand-side norms^2 into out[r] (as complex, real part) via the multi-dot of w with itself
hipError_t selfdot(const void *ws, const void *wd, int R, i64 n1, i64 n2, void *part, void *out, double dw, int f32,
                   hipStream_t s) {
    // V_0 = w with a one-vector "space": stride arguments make vector 0 the vector itself
    return multidot(ws, wd, ws, wd, R, n1, n2, 1, part, out, 1, dw, f32, s);
}

}  // namespace lrcc
