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

}  // namespace lrcc
