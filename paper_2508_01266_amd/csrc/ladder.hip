// Particle-particle ladder with the integral block rebuilt in LDS.
//
//   Z[ki,kj,ka][r][a][b] += alpha * sum_ke sum_{e,f} Y[ki,kj,ke][r][e][f] * W(ka,kb,ke)[e,f][a,b]
//   W(ka,kb,ke)[e,f][a,b] = sum_Q La[ka][ke][Q][a][e] * Lb[kb][kf][Q][b][f]
// with kb = ki+kj-ka, kf = ki+kj-ke and r = (rhs, i, j).  This is the vvvv term
// of Eq. tx2 (the (1/2Nk) tbar_IJ^EF W_ABEF contraction) with the integrals
// never stored: each 16x64 (ef)x(ab) tile of W is built in LDS as a
// (a,e)x(b,f) rank-naux MFMA product of two Cholesky slices and immediately
// consumed by the row tile.
#include "common.hpp"

namespace lrcc {

template <typename T> struct MfmaL;
template <> struct MfmaL<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct MfmaL<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

namespace {
constexpr int LTM = 64;              // rows (rhs,i,j) per tile
constexpr int TA = 8, TB = 8;        // (a,b) tile: 64 columns
constexpr int TE = 4, TF = 4;        // (e,f) tile: 16 K values
constexpr int LTN = TA * TB, LTK = TE * TF;
constexpr int QC = 16;               // Cholesky vectors per LDS chunk
constexpr int NTL = 256;
}

template <typename T>
__global__ void __launch_bounds__(NTL) ladder_kernel(LadderArgs p) {
    typedef typename Cx<T>::type C2;
    typedef typename MfmaL<T>::v4 v4;
    // LDS: rebuilt W tile, Y tile, Cholesky chunks
    __shared__ T Wr[LTK][LTN], Wi[LTK][LTN];
    __shared__ T Yr[LTK][LTM], Yi[LTK][LTM];
    __shared__ T Pr[QC][TA * TE], Pi[QC][TA * TE];   // rows (a,e)
    __shared__ T Qr[QC][TB * TF], Qi[QC][TB * TF];   // cols (b,f)

    const int nk = p.nk, o = p.o, v = p.v, naux = p.naux;
    const int M = p.nrhs * o * o;
    const int tilesM = (M + LTM - 1) / LTM;
    const int tilesA = (v + TA - 1) / TA;
    const int mt = blockIdx.x % tilesM;
    const int rest = blockIdx.x / tilesM;
    const int a0 = (rest % tilesA) * TA;
    const int b0 = (rest / tilesA) * TB;
    const int blk = blockIdx.y;                       // (ki,kj,ka)
    const int ki = blk / (nk * nk), kj = (blk / nk) % nk, ka = blk % nk;
    const int kb = p.km.comb(ki, kj, ka);
    const int m0 = mt * LTM;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const i64 vv = (i64)v * v;
    const i64 blk4 = (i64)M * vv;                     // elements per (ki,kj,k) block

    const C2 *Y = reinterpret_cast<const C2 *>(p.Y);
    const C2 *La = reinterpret_cast<const C2 *>(p.La);
    const C2 *Lb = reinterpret_cast<const C2 *>(p.Lb);
    C2 *Z = reinterpret_cast<C2 *>(p.Z);

    v4 accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { accr[i][j] = v4{0, 0, 0, 0}; acci[i][j] = v4{0, 0, 0, 0}; }

    // rebuild sub-tile owned by this wave: rows (a,e) 16*(wave&1).., cols (b,f) 16*(wave>>1)..
    const int rw = 16 * (wave & 1), cw = 16 * (wave >> 1);

    for (int ke = 0; ke < nk; ++ke) {
        const int kf = p.km.comb(ki, kj, ke);
        const C2 *Yb = Y + ((i64)(ki * nk + kj) * nk + ke) * blk4;
        const C2 *Lab = La + (i64)(ka * nk + ke) * naux * vv;
        const C2 *Lbb = Lb + (i64)(kb * nk + kf) * naux * vv;
        for (int e0 = 0; e0 < v; e0 += TE) {
            for (int f0 = 0; f0 < v; f0 += TF) {
                // ---- rebuild W tile: G[(a,e)][(b,f)] = sum_Q La[Q][a][e] Lb[Q][b][f]
                v4 gr = v4{0, 0, 0, 0}, gi = v4{0, 0, 0, 0};
                for (int q0 = 0; q0 < naux; q0 += QC) {
                    // 2 * QC * 32 complex loads; 256 threads -> 4 each
                    for (int idx = tid; idx < 2 * QC * 32; idx += NTL) {
                        const int which = idx / (QC * 32);
                        const int rem = idx % (QC * 32);
                        const int q = rem / 32, c = rem % 32;
                        const int x = c / 4, y = c % 4;      // (a or b, e or f)
                        C2 val; val.x = 0; val.y = 0;
                        if (which == 0) {
                            const int a = a0 + x, e = e0 + y;
                            if (q0 + q < naux && a < v && e < v) val = Lab[(i64)(q0 + q) * vv + (i64)a * v + e];
                            Pr[q][c] = val.x; Pi[q][c] = val.y;
                        } else {
                            const int b = b0 + x, f = f0 + y;
                            if (q0 + q < naux && b < v && f < v) val = Lbb[(i64)(q0 + q) * vv + (i64)b * v + f];
                            Qr[q][c] = val.x; Qi[q][c] = val.y;
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int kk = 0; kk < QC; kk += 4) {
                        const int kr = kk + (lane >> 4), c = lane & 15;
                        const T xr = Pr[kr][rw + c], xi = Pi[kr][rw + c];
                        const T yr = Qr[kr][cw + c], yi = Qi[kr][cw + c];
                        gr = MfmaL<T>::mma(xr, yr, gr);
                        gr = MfmaL<T>::mma(-xi, yi, gr);
                        gi = MfmaL<T>::mma(xr, yi, gi);
                        gi = MfmaL<T>::mma(xi, yr, gi);
                    }
                    __syncthreads();
                }
                // scatter G sub-tile into W[(e,f)][(a,b)]
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ae = rw + MfmaL<T>::row(lane, r);
                    const int bf = cw + (lane & 15);
                    const int a = ae / 4, e = ae % 4, b = bf / 4, f = bf % 4;
                    Wr[e * TF + f][a * TB + b] = gr[r];
                    Wi[e * TF + f][a * TB + b] = gi[r];
                }
                // ---- Y tile: rows m0.., K = (e,f)
                for (int idx = tid; idx < LTM * LTK; idx += NTL) {
                    const int kk = idx % LTK, m = idx / LTK;
                    const int e = e0 + kk / TF, f = f0 + kk % TF;
                    C2 val; val.x = 0; val.y = 0;
                    if (m0 + m < M && e < v && f < v) val = Yb[(i64)(m0 + m) * vv + (i64)e * v + f];
                    Yr[kk][m] = val.x; Yi[kk][m] = val.y;
                }
                __syncthreads();
#pragma unroll
                for (int kk = 0; kk < LTK; kk += 4) {
                    const int kr = kk + (lane >> 4), c = lane & 15;
                    T ar[2], ai[2], br[2], bi[2];
#pragma unroll
                    for (int i = 0; i < 2; ++i) { ar[i] = Yr[kr][wm + 16 * i + c]; ai[i] = Yi[kr][wm + 16 * i + c]; }
#pragma unroll
                    for (int j = 0; j < 2; ++j) { br[j] = Wr[kr][wn + 16 * j + c]; bi[j] = Wi[kr][wn + 16 * j + c]; }
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            accr[i][j] = MfmaL<T>::mma(ar[i], br[j], accr[i][j]);
                            accr[i][j] = MfmaL<T>::mma(-ai[i], bi[j], accr[i][j]);
                            acci[i][j] = MfmaL<T>::mma(ar[i], bi[j], acci[i][j]);
                            acci[i][j] = MfmaL<T>::mma(ai[i], br[j], acci[i][j]);
                        }
                }
                __syncthreads();
            }
        }
    }

    // epilogue: Z block (ki,kj,ka) rows m, cols (a,b)
    C2 *Zb = Z + ((i64)(ki * nk + kj) * nk + ka) * blk4;
    const T al = (T)p.alpha;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + MfmaL<T>::row(lane, r);
                const int c = wn + 16 * j + (lane & 15);
                const int a = a0 + c / TB, b = b0 + c % TB;
                if (m < M && a < v && b < v) {
                    const i64 off = (i64)m * vv + (i64)a * v + b;
                    C2 o2 = Zb[off];
                    o2.x += al * accr[i][j][r];
                    o2.y += al * acci[i][j][r];
                    Zb[off] = o2;
                }
            }
}


// Large-batch variant: 256 rows per workgroup (8 waves in a 4x2 grid, each a
// 64x32 sub-tile), so every rebuilt W tile serves 4x more rows and the
// rebuild costs naux/256 of the product instead of naux/64.  The four 16x16
// blocks of the (a,e)x(b,f) rebuild are split over wave pairs by halves of the
// Cholesky range and summed through LDS.
namespace {
constexpr int BTM = 256;
constexpr int NTB = 512;
}

template <typename T>
__global__ void __launch_bounds__(NTB) ladder_kernel_big(LadderArgs p) {
    typedef typename Cx<T>::type C2;
    typedef typename MfmaL<T>::v4 v4;
    __shared__ T Wr[LTK][LTN], Wi[LTK][LTN];
    __shared__ T Yr[LTK][BTM], Yi[LTK][BTM];
    __shared__ T Pr[2][QC][TA * TE], Pi[2][QC][TA * TE];
    __shared__ T Qr[2][QC][TB * TF], Qi[2][QC][TB * TF];
    __shared__ T Gr[4][64][4], Gi[4][64][4];   // partial rebuild blocks of waves 4..7

    const int nk = p.nk, o = p.o, v = p.v, naux = p.naux;
    const int M = p.nrhs * o * o;
    const int tilesM = (M + BTM - 1) / BTM;
    const int tilesA = (v + TA - 1) / TA;
    const int mt = blockIdx.x % tilesM;
    const int rest = blockIdx.x / tilesM;
    const int a0 = (rest % tilesA) * TA;
    const int b0 = (rest / tilesA) * TB;
    const int blk = blockIdx.y;
    const int ki = blk / (nk * nk), kj = (blk / nk) % nk, ka = blk % nk;
    const int kb = p.km.comb(ki, kj, ka);
    const int m0 = mt * BTM;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 3) * 64, wn = (wave >> 2) * 32;
    const i64 vv = (i64)v * v;
    const i64 blk4 = (i64)M * vv;

    const C2 *Y = reinterpret_cast<const C2 *>(p.Y);
    const C2 *La = reinterpret_cast<const C2 *>(p.La);
    const C2 *Lb = reinterpret_cast<const C2 *>(p.Lb);
    C2 *Z = reinterpret_cast<C2 *>(p.Z);

    v4 accr[4][2], acci[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { accr[i][j] = v4{0, 0, 0, 0}; acci[i][j] = v4{0, 0, 0, 0}; }

    // rebuild block of this wave (waves w and w+4 share block w&3, halves of the Q chunks)
    const int gb = wave & 3, half = wave >> 2;
    const int rw = 16 * (gb & 1), cw = 16 * (gb >> 1);

    for (int ke = 0; ke < nk; ++ke) {
        const int kf = p.km.comb(ki, kj, ke);
        const C2 *Yb = Y + ((i64)(ki * nk + kj) * nk + ke) * blk4;
        const C2 *Lab = La + (i64)(ka * nk + ke) * naux * vv;
        const C2 *Lbb = Lb + (i64)(kb * nk + kf) * naux * vv;
        for (int e0 = 0; e0 < v; e0 += TE) {
            for (int f0 = 0; f0 < v; f0 += TF) {
                v4 gr = v4{0, 0, 0, 0}, gi = v4{0, 0, 0, 0};
                for (int q0 = 0; q0 < naux; q0 += 2 * QC) {
                    // two Cholesky chunks: chunk h covers [q0 + h*QC, q0 + (h+1)*QC)
                    for (int idx = tid; idx < 2 * 2 * QC * 32; idx += NTB) {
                        const int h = idx / (2 * QC * 32);
                        const int rem0 = idx % (2 * QC * 32);
                        const int which = rem0 / (QC * 32);
                        const int rem = rem0 % (QC * 32);
                        const int q = rem / 32, cc = rem % 32;
                        const int x = cc / 4, y = cc % 4;
                        const int qq = q0 + h * QC + q;
                        C2 val; val.x = 0; val.y = 0;
                        if (which == 0) {
                            const int a = a0 + x, e = e0 + y;
                            if (qq < naux && a < v && e < v) val = Lab[(i64)qq * vv + (i64)a * v + e];
                            Pr[h][q][cc] = val.x; Pi[h][q][cc] = val.y;
                        } else {
                            const int b = b0 + x, f = f0 + y;
                            if (qq < naux && b < v && f < v) val = Lbb[(i64)qq * vv + (i64)b * v + f];
                            Qr[h][q][cc] = val.x; Qi[h][q][cc] = val.y;
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int kk = 0; kk < QC; kk += 4) {
                        const int kr = kk + (lane >> 4), c = lane & 15;
                        const T xr = Pr[half][kr][rw + c], xi = Pi[half][kr][rw + c];
                        const T yr = Qr[half][kr][cw + c], yi = Qi[half][kr][cw + c];
                        gr = MfmaL<T>::mma(xr, yr, gr);
                        gr = MfmaL<T>::mma(-xi, yi, gr);
                        gi = MfmaL<T>::mma(xr, yi, gi);
                        gi = MfmaL<T>::mma(xi, yr, gi);
                    }
                    __syncthreads();
                }
                if (half == 1) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) { Gr[gb][lane][r] = gr[r]; Gi[gb][lane][r] = gi[r]; }
                }
                __syncthreads();
                if (half == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int ae = rw + MfmaL<T>::row(lane, r);
                        const int bf = cw + (lane & 15);
                        const int a = ae / 4, e = ae % 4, b = bf / 4, f = bf % 4;
                        Wr[e * TF + f][a * TB + b] = gr[r] + Gr[gb][lane][r];
                        Wi[e * TF + f][a * TB + b] = gi[r] + Gi[gb][lane][r];
                    }
                }
                for (int idx = tid; idx < BTM * LTK; idx += NTB) {
                    const int kk = idx % LTK, m = idx / LTK;
                    const int e = e0 + kk / TF, f = f0 + kk % TF;
                    C2 val; val.x = 0; val.y = 0;
                    if (m0 + m < M && e < v && f < v) val = Yb[(i64)(m0 + m) * vv + (i64)e * v + f];
                    Yr[kk][m] = val.x; Yi[kk][m] = val.y;
                }
                __syncthreads();
#pragma unroll
                for (int kk = 0; kk < LTK; kk += 4) {
                    const int kr = kk + (lane >> 4), c = lane & 15;
                    T ar[4], ai[4], br[2], bi[2];
#pragma unroll
                    for (int i = 0; i < 4; ++i) { ar[i] = Yr[kr][wm + 16 * i + c]; ai[i] = Yi[kr][wm + 16 * i + c]; }
#pragma unroll
                    for (int j = 0; j < 2; ++j) { br[j] = Wr[kr][wn + 16 * j + c]; bi[j] = Wi[kr][wn + 16 * j + c]; }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            accr[i][j] = MfmaL<T>::mma(ar[i], br[j], accr[i][j]);
                            accr[i][j] = MfmaL<T>::mma(-ai[i], bi[j], accr[i][j]);
                            acci[i][j] = MfmaL<T>::mma(ar[i], bi[j], acci[i][j]);
                            acci[i][j] = MfmaL<T>::mma(ai[i], br[j], acci[i][j]);
                        }
                }
                __syncthreads();
            }
        }
    }

    C2 *Zb = Z + ((i64)(ki * nk + kj) * nk + ka) * blk4;
    const T al = (T)p.alpha;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + MfmaL<T>::row(lane, r);
                const int c = wn + 16 * j + (lane & 15);
                const int a = a0 + c / TB, b = b0 + c % TB;
                if (m < M && a < v && b < v) {
                    const i64 off = (i64)m * vv + (i64)a * v + b;
                    C2 o2 = Zb[off];
                    o2.x += al * accr[i][j][r];
                    o2.y += al * acci[i][j][r];
                    Zb[off] = o2;
                }
            }
}

static bool use_big(const LadderArgs &a) { return a.nrhs * a.o * a.o >= 192; }

// Antisymmetry-packed large-batch variant.  With Y antisymmetric in (e,f) and
// the result antisymmetric in (a,b):
//   sum_{e,f} Y^{ef} K_{abef} = sum_{(ke,e) < (kf,f)} Y^{ef} (K_{abef} - K_{abfe}),
// so only the unique input pairs contribute, and only the unique output pairs
// (ka,a) < (kb,b) are formed; they are written with weight 2*alpha so that the
// final P(ij)P(ab) assembly reproduces the full ladder (the (b,a) partners are
// left to the antisymmetriser).  Each 16x64 W tile is rebuilt in LDS as the
// difference of two rank-naux products, one per 16x16 block per wave.
namespace {
constexpr int NTP = 512;
}

template <typename T>
__global__ void __launch_bounds__(NTP) ladder_kernel_packed(LadderArgs p) {
    typedef typename Cx<T>::type C2;
    typedef typename MfmaL<T>::v4 v4;
    __shared__ T Wr[LTK][LTN], Wi[LTK][LTN];
    __shared__ T Yr[LTK][BTM], Yi[LTK][BTM];
    // Cholesky chunks: [0] La(ka,ke)[a][e], [1] Lb(kb,kf)[b][f], [2] La(ka,kf)[a][f], [3] Lb(kb,ke)[b][e]
    __shared__ T Lr[4][QC][32], Li[4][QC][32];
    __shared__ T Gr[4][64][4], Gi[4][64][4];   // second products of waves 4..7

    const int nk = p.nk, o = p.o, v = p.v, naux = p.naux;
    const int M = p.nrhs * o * o;
    const int tilesM = (M + BTM - 1) / BTM;
    const int tilesA = (v + TA - 1) / TA;
    const int mt = blockIdx.x % tilesM;
    const int rest = blockIdx.x / tilesM;
    const int ta = rest % tilesA, tb = rest / tilesA;
    const int a0 = ta * TA, b0 = tb * TB;
    const int blk = blockIdx.y;
    const int ki = blk / (nk * nk), kj = (blk / nk) % nk, ka = blk % nk;
    const int kb = p.km.comb(ki, kj, ka);
    // unique output pairs only
    if (ka > kb || (ka == kb && ta > tb)) return;
    const bool diag_out = (ka == kb);
    const int m0 = mt * BTM;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 3) * 64, wn = (wave >> 2) * 32;
    const i64 vv = (i64)v * v;
    const i64 blk4 = (i64)M * vv;

    const C2 *Y = reinterpret_cast<const C2 *>(p.Y);
    const C2 *La = reinterpret_cast<const C2 *>(p.La);
    const C2 *Lb = reinterpret_cast<const C2 *>(p.Lb);
    C2 *Z = reinterpret_cast<C2 *>(p.Z);

    v4 accr[4][2], acci[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { accr[i][j] = v4{0, 0, 0, 0}; acci[i][j] = v4{0, 0, 0, 0}; }

    const int gb = wave & 3, second = wave >> 2;
    const int rw = 16 * (gb & 1), cw = 16 * (gb >> 1);

    for (int ke = 0; ke < nk; ++ke) {
        const int kf = p.km.comb(ki, kj, ke);
        if (ke > kf) continue;
        const bool diag_in = (ke == kf);
        const C2 *Yb = Y + ((i64)(ki * nk + kj) * nk + ke) * blk4;
        const C2 *L0 = La + (i64)(ka * nk + ke) * naux * vv;   // [a][e]
        const C2 *L1 = Lb + (i64)(kb * nk + kf) * naux * vv;   // [b][f]
        const C2 *L2 = La + (i64)(ka * nk + kf) * naux * vv;   // [a][f]
        const C2 *L3 = Lb + (i64)(kb * nk + ke) * naux * vv;   // [b][e]
        for (int e0 = 0; e0 < v; e0 += TE) {
            for (int f0 = diag_in ? (e0 / TF) * TF : 0; f0 < v; f0 += TF) {
                // rebuild: waves 0-3 G1[(a,e)][(b,f)] = sum La(ka,ke)[a][e] Lb(kb,kf)[b][f],
                //          waves 4-7 G2[(a,f)][(b,e)] = sum La(ka,kf)[a][f] Lb(kb,ke)[b][e]
                v4 gr = v4{0, 0, 0, 0}, gi = v4{0, 0, 0, 0};
                for (int q0 = 0; q0 < naux; q0 += QC) {
                    for (int idx = tid; idx < 4 * QC * 32; idx += NTP) {
                        const int which = idx / (QC * 32);
                        const int rem = idx % (QC * 32);
                        const int q = rem / 32, cc = rem % 32;
                        const int x = cc / 4, y = cc % 4;
                        const int qq = q0 + q;
                        C2 val; val.x = 0; val.y = 0;
                        const int r0 = (which == 0 || which == 2) ? a0 + x : b0 + x;
                        const int c0 = (which == 0 || which == 3) ? e0 + y : f0 + y;
                        const C2 *src = which == 0 ? L0 : which == 1 ? L1 : which == 2 ? L2 : L3;
                        if (qq < naux && r0 < v && c0 < v) val = src[(i64)qq * vv + (i64)r0 * v + c0];
                        Lr[which][q][cc] = val.x; Li[which][q][cc] = val.y;
                    }
                    __syncthreads();
                    const int ra = second ? 2 : 0, rb = second ? 3 : 1;
#pragma unroll
                    for (int kk = 0; kk < QC; kk += 4) {
                        const int kr = kk + (lane >> 4), c = lane & 15;
                        const T xr = Lr[ra][kr][rw + c], xi = Li[ra][kr][rw + c];
                        const T yr = Lr[rb][kr][cw + c], yi = Li[rb][kr][cw + c];
                        gr = MfmaL<T>::mma(xr, yr, gr);
                        gr = MfmaL<T>::mma(-xi, yi, gr);
                        gi = MfmaL<T>::mma(xr, yi, gi);
                        gi = MfmaL<T>::mma(xi, yr, gi);
                    }
                    __syncthreads();
                }
                // G2 block gb of wave gb+4 holds rows (a,f) and cols (b,e); it is needed at
                // W[(e,f)][(a,b)] -= G2[(a,f)][(b,e)]: exchange through LDS in W coordinates
                if (second) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) { Gr[gb][lane][r] = gr[r]; Gi[gb][lane][r] = gi[r]; }
                }
                __syncthreads();
                if (!second) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int ae = rw + MfmaL<T>::row(lane, r);
                        const int bf = cw + (lane & 15);
                        const int a = ae / 4, e = ae % 4, b = bf / 4, f = bf % 4;
                        Wr[e * TF + f][a * TB + b] = gr[r];
                        Wi[e * TF + f][a * TB + b] = gi[r];
                    }
                }
                __syncthreads();
                if (second) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        // this wave's G2 element: row (a, f') = rw + row(lane,r), col (b, e') = cw + lane%16
                        const int af = rw + MfmaL<T>::row(lane, r);
                        const int be = cw + (lane & 15);
                        const int a = af / 4, f = af % 4, b = be / 4, e = be % 4;
                        Wr[e * TF + f][a * TB + b] -= Gr[gb][lane][r];
                        Wi[e * TF + f][a * TB + b] -= Gi[gb][lane][r];
                    }
                }
                // Y tile with the unique-pair mask of the input
                for (int idx = tid; idx < BTM * LTK; idx += NTP) {
                    const int kk = idx % LTK, m = idx / LTK;
                    const int e = e0 + kk / TF, f = f0 + kk % TF;
                    C2 val; val.x = 0; val.y = 0;
                    if (m0 + m < M && e < v && f < v && (!diag_in || e < f))
                        val = Yb[(i64)(m0 + m) * vv + (i64)e * v + f];
                    Yr[kk][m] = val.x; Yi[kk][m] = val.y;
                }
                __syncthreads();
#pragma unroll
                for (int kk = 0; kk < LTK; kk += 4) {
                    const int kr = kk + (lane >> 4), c = lane & 15;
                    T ar[4], ai[4], br[2], bi[2];
#pragma unroll
                    for (int i = 0; i < 4; ++i) { ar[i] = Yr[kr][wm + 16 * i + c]; ai[i] = Yi[kr][wm + 16 * i + c]; }
#pragma unroll
                    for (int j = 0; j < 2; ++j) { br[j] = Wr[kr][wn + 16 * j + c]; bi[j] = Wi[kr][wn + 16 * j + c]; }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            accr[i][j] = MfmaL<T>::mma(ar[i], br[j], accr[i][j]);
                            accr[i][j] = MfmaL<T>::mma(-ai[i], bi[j], accr[i][j]);
                            acci[i][j] = MfmaL<T>::mma(ar[i], bi[j], acci[i][j]);
                            acci[i][j] = MfmaL<T>::mma(ai[i], br[j], acci[i][j]);
                        }
                }
                __syncthreads();
            }
        }
    }

    C2 *Zb = Z + ((i64)(ki * nk + kj) * nk + ka) * blk4;
    const T al = (T)(2.0 * p.alpha);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + MfmaL<T>::row(lane, r);
                const int c = wn + 16 * j + (lane & 15);
                const int a = a0 + c / TB, b = b0 + c % TB;
                if (m < M && a < v && b < v && (!diag_out || a < b)) {
                    const i64 off = (i64)m * vv + (i64)a * v + b;
                    C2 o2 = Zb[off];
                    o2.x += al * accr[i][j][r];
                    o2.y += al * acci[i][j][r];
                    Zb[off] = o2;
                }
            }
}


// Pipelined antisymmetry-packed variant (same arithmetic as ladder_kernel_packed):
// WM x WN waves over a BM x 64 output tile, BM = 64 WM rows, so the rank-naux
// integral rebuild (eight 16x16 blocks per step, one per wave of the first eight)
// is amortised over more rows: its cost relative to the main product is
// 2 Naux / BM.  Global loads run one stage ahead in registers: the Y tile of a
// step is fetched while its integral tile is rebuilt, each Cholesky chunk while
// the previous one is multiplied, and the first chunk of the next step while the
// current step's main product runs.  The load maps are hoisted: every load of a
// thread has the same position inside its block.
template <typename T, int WM, int WN, int QCH>
__device__ __forceinline__ void ladder_pipe_tile(const LadderArgs &p, const int bx, const int blk) {
    typedef typename Cx<T>::type C2;
    typedef typename MfmaL<T>::v4 v4;
    constexpr int FM = 4;                          // 16-row blocks per wave
    constexpr int FN = LTN / (WN * 16);            // 16-column blocks per wave
    constexpr int BM = WM * FM * 16;               // rows per tile
    constexpr int NT = WM * WN * 64;               // threads per workgroup
    constexpr int YPT = BM * LTK / NT;             // Y elements per thread per step
    constexpr int LPT = 4 * QCH * 32 / NT;         // Cholesky elements per thread per chunk
    static_assert(WM * WN >= 8, "eight waves rebuild the integral tile");
    // the rebuild forms complex64 products as three real matrix-core products (complex128,
    // and the main product in both precisions, keep four)
    constexpr bool kGauss = sizeof(T) == 4;
    static_assert(YPT * NT == BM * LTK && LPT * NT == 4 * QCH * 32, "even loads");
    constexpr int PY = 16, PL = 16, PW = sizeof(T) == 8 ? 9 : 17;
    __shared__ T Wr[LTK][LTN + PW], Wi[LTK][LTN + PW];
    __shared__ T Yr[LTK][BM + PY], Yi[LTK][BM + PY];
    __shared__ T Lr[4][QCH][32 + PL], Li[4][QCH][32 + PL];

    const int nk = p.nk, v = p.v, naux = p.naux, o = p.o;
    const int M = p.nrhs * o * o;                  // rows of one (ki, kj, k) block of Y and Z
    const bool rows_packed = p.pack_rows != 0;
    const int tilesM = ((rows_packed ? p.mrows : M) + BM - 1) / BM;
    const int tilesA = (v + TA - 1) / TA;
    const int mt = bx % tilesM;
    const int rest = bx / tilesM;
    const int ta = rest % tilesA, tb = rest / tilesA;
    const int a0 = ta * TA, b0 = tb * TB;
    // block: (K = ki + kj, ka) over the unique rows of class K (rows_packed), else (ki, kj, ka)
    int K, ka, ki = 0, kj = 0;
    if (rows_packed) {
        K = blk / nk;
        ka = blk % nk;
    } else {
        ki = blk / (nk * nk);
        kj = (blk / nk) % nk;
        ka = blk % nk;
        K = p.km.sum3(1, ki, 1, kj, 0, 0);
    }
    const int kb = p.km.sub(K, ka);
    if (ka > kb || (ka == kb && ta > tb)) return;
    const bool diag_out = (ka == kb);
    const int P = o * (o - 1) / 2;
    const int Mr = rows_packed ? ladder_class_rows(p, K) : M;   // rows of this block
    const int m0 = mt * BM;
    if (m0 >= Mr) return;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave % WM) * FM * 16, wn = (wave / WM) * FN * 16;
    const i64 vv = (i64)v * v;
    const i64 blk4 = (i64)M * vv;
    const C2 *Y = reinterpret_cast<const C2 *>(p.Y);
    const C2 *La = reinterpret_cast<const C2 *>(p.La);
    const C2 *Lb = reinterpret_cast<const C2 *>(p.Lb);
    C2 *Z = reinterpret_cast<C2 *>(p.Z);
    const int gb = wave & 3, second = (wave >> 2) & 1;
    const bool rebuilder = WM * WN == 8 || wave < 8;   // compile-time true with eight waves
    // row table of the tile, in rows of vv elements: (ki * nk + kj) * nk * M (the row's block, the
    // third momentum added per step) + (rhs * o + i) * o + j; -1 past the end.  Class rows: the unique
    // rows of block (ki, kj) for every ki <= kj with ki + kj = K, in increasing ki: all (rhs, i, j)
    // when ki < kj, the o(o-1)/2 pairs i < j per right-hand side when ki == kj
    __shared__ int rowtab[BM];
    for (int t = tid; t < BM; t += NT) {
        int m = m0 + t, ro = -1;
        if (m < Mr) {
            if (rows_packed) {
                int bi = 0, bj = 0;
                for (int k = 0; k < nk; ++k) {
                    const int kk = p.km.sub(K, k);
                    if (k > kk) continue;
                    const int cnt = k < kk ? M : p.nrhs * P;
                    if (m < cnt) { bi = k; bj = kk; break; }
                    m -= cnt;
                }
                int r0 = m;
                if (bi == bj) {
                    const int r = m / P;
                    int q = m - r * P, i = 0;
                    while (q >= o - 1 - i) { q -= o - 1 - i; ++i; }
                    r0 = (r * o + i) * o + i + 1 + q;
                }
                ro = (bi * nk + bj) * nk * M + r0;
            } else {
                ro = (ki * nk + kj) * nk * M + m;
            }
        }
        rowtab[t] = ro;
    }
    __syncthreads();
    const int rw = 16 * (gb & 1), cw = 16 * (gb >> 1);

    // steps (ke <= kf, e0, f0 >= e0 when ke == kf); the step after `s`, or ke = nk when done
    auto kf_of = [&](int ke) { return p.km.sub(K, ke); };
    auto first_valid = [&](int ke) {
        while (ke < nk && ke > kf_of(ke)) ++ke;
        return ke;
    };
    auto advance = [&](int &ke, int &e0, int &f0) {
        f0 += TF;
        if (f0 >= v) {
            e0 += TE;
            if (e0 >= v) { ke = first_valid(ke + 1); e0 = 0; }
            f0 = (ke < nk && ke == kf_of(ke)) ? (e0 / TF) * TF : 0;
        }
    };

    // every load of a thread sits at the same in-block position: the maps are hoisted
    static_assert(NT % LTK == 0 && ((QCH * 32) % NT == 0 || NT % (QCH * 32) == 0), "load maps");
    const int ykk = tid % LTK, ym = tid / LTK;
    const int ye = ykk / TF, yf = ykk % TF;
    const int lx = (tid % 32) / 4, ly = tid % 4;
    // Cholesky load q: matrix lwhich(q), vector row lrow(q) of the chunk
    auto lwhich = [&](int q) {
        if constexpr ((QCH * 32) % NT == 0) return (q * NT) / (QCH * 32);
        else return (tid % NT) / (QCH * 32) + q * (NT / (QCH * 32));
    };
    auto lrow = [&](int q) {
        if constexpr ((QCH * 32) % NT == 0) return ((q * NT) % (QCH * 32) + tid) / 32;
        else return (tid % (QCH * 32)) / 32;
    };

    C2 lv[LPT], yv[YPT];
    auto load_chunk = [&](int ke, int e0, int f0, int q0) {
        const int kf = kf_of(ke);
        const C2 *L0 = La + (i64)(ka * nk + ke) * naux * vv;
        const C2 *L1 = Lb + (i64)(kb * nk + kf) * naux * vv;
        const C2 *L2 = La + (i64)(ka * nk + kf) * naux * vv;
        const C2 *L3 = Lb + (i64)(kb * nk + ke) * naux * vv;
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int which = lwhich(q);
            const int qq = q0 + lrow(q);
            const int r0 = (which == 0 || which == 2) ? a0 + lx : b0 + lx;
            const int c0 = (which == 0 || which == 3) ? e0 + ly : f0 + ly;
            const C2 *src = which == 0 ? L0 : which == 1 ? L1 : which == 2 ? L2 : L3;
            C2 val; val.x = 0; val.y = 0;
            if (qq < naux && r0 < v && c0 < v) val = src[(i64)qq * vv + (i64)r0 * v + c0];
            lv[q] = val;
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            Lr[lwhich(q)][lrow(q)][tid % 32] = lv[q].x;
            Li[lwhich(q)][lrow(q)][tid % 32] = lv[q].y;
        }
    };
    auto load_y = [&](int ke, int e0, int f0) {
        const bool diag_in = ke == kf_of(ke);
        const int e = e0 + ye, f = f0 + yf;
        const bool ok = e < v && f < v && (!diag_in || e < f);
        const C2 *Yb = Y + (i64)ke * blk4 + (i64)e * v + f;
#pragma unroll
        for (int q = 0; q < YPT; ++q) {
            const int ro = rowtab[ym + q * (NT / LTK)];
            C2 val; val.x = 0; val.y = 0;
            if (ok && ro >= 0) val = Yb[(i64)ro * vv];
            yv[q] = val;
        }
    };

    v4 accr[FM][FN], acci[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) { accr[i][j] = v4{0, 0, 0, 0}; acci[i][j] = v4{0, 0, 0, 0}; }

    int ke = first_valid(0), e0 = 0, f0 = 0;
    if (ke < nk) load_chunk(ke, e0, f0, 0);
    while (ke < nk) {
        load_y(ke, e0, f0);
        // rebuild: waves 0-3 G1[(a,e)][(b,f)] = sum La(ka,ke)[a][e] Lb(kb,kf)[b][f],
        //          waves 4-7 G2[(a,f)][(b,e)] = sum La(ka,kf)[a][f] Lb(kb,ke)[b][e]
        // complex64: three real products per complex one (Gauss): with k1 = yr (xr + xi),
        // k2 = xr (yi - yr), k3 = xi (yr + yi): re = k1 - k3, im = k1 + k2
        v4 gr = v4{0, 0, 0, 0}, gi = v4{0, 0, 0, 0}, g3 = v4{0, 0, 0, 0};
        const int ra = second ? 2 : 0, rb = second ? 3 : 1;
        for (int q0 = 0; q0 < naux; q0 += QCH) {
            store_chunk();
            __syncthreads();
            if (q0 + QCH < naux) load_chunk(ke, e0, f0, q0 + QCH);
#pragma unroll 2
            for (int kk = 0; kk < (rebuilder ? QCH : 0); kk += 4) {
                const int kr = kk + (lane >> 4), c = lane & 15;
                const T xr = Lr[ra][kr][rw + c], xi = Li[ra][kr][rw + c];
                const T yr = Lr[rb][kr][cw + c], yi = Li[rb][kr][cw + c];
                if constexpr (kGauss) {
                    gr = MfmaL<T>::mma(xr + xi, yr, gr);
                    gi = MfmaL<T>::mma(xr, yi - yr, gi);
                    g3 = MfmaL<T>::mma(xi, yr + yi, g3);
                } else {
                    gr = MfmaL<T>::mma(xr, yr, gr);
                    gr = MfmaL<T>::mma(-xi, yi, gr);
                    gi = MfmaL<T>::mma(xr, yi, gi);
                    gi = MfmaL<T>::mma(xi, yr, gi);
                }
            }
            __syncthreads();
        }
        if constexpr (kGauss) {
            gi = gr + gi;
            gr = gr - g3;
        }
        // W[(e,f)][(a,b)] = G1[(a,e)][(b,f)] - G2[(a,f)][(b,e)]: the G1 waves write, then the G2 waves subtract
        if (rebuilder && !second) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ae = rw + MfmaL<T>::row(lane, r);
                const int bf = cw + (lane & 15);
                Wr[(ae % 4) * TF + bf % 4][(ae / 4) * TB + bf / 4] = gr[r];
                Wi[(ae % 4) * TF + bf % 4][(ae / 4) * TB + bf / 4] = gi[r];
            }
        }
        __syncthreads();
        if (rebuilder && second) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int af = rw + MfmaL<T>::row(lane, r);
                const int be = cw + (lane & 15);
                Wr[(be % 4) * TF + af % 4][(af / 4) * TB + be / 4] -= gr[r];
                Wi[(be % 4) * TF + af % 4][(af / 4) * TB + be / 4] -= gi[r];
            }
        }
#pragma unroll
        for (int q = 0; q < YPT; ++q) {
            Yr[ykk][ym + q * (NT / LTK)] = yv[q].x;
            Yi[ykk][ym + q * (NT / LTK)] = yv[q].y;
        }
        __syncthreads();
        advance(ke, e0, f0);
        if (ke < nk) load_chunk(ke, e0, f0, 0);
#pragma unroll
        for (int kk = 0; kk < LTK; kk += 4) {
            const int kr = kk + (lane >> 4), c = lane & 15;
            T ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) { ar[i] = Yr[kr][wm + 16 * i + c]; ai[i] = Yi[kr][wm + 16 * i + c]; }
#pragma unroll
            for (int j = 0; j < FN; ++j) { br[j] = Wr[kr][wn + 16 * j + c]; bi[j] = Wi[kr][wn + 16 * j + c]; }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    accr[i][j] = MfmaL<T>::mma(ar[i], br[j], accr[i][j]);
                    accr[i][j] = MfmaL<T>::mma(-ai[i], bi[j], accr[i][j]);
                    acci[i][j] = MfmaL<T>::mma(ar[i], bi[j], acci[i][j]);
                    acci[i][j] = MfmaL<T>::mma(ai[i], br[j], acci[i][j]);
                }
        }
        __syncthreads();
    }

    C2 *Zb = Z + (i64)ka * blk4;
    // unique (a, b) outputs carry 2 alpha, and unique rows a further 2: the P(ij)P(ab) assembly
    // reproduces the partners from the antisymmetry
    const T al = (T)((rows_packed ? 4.0 : 2.0) * p.alpha);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ro = rowtab[wm + 16 * i + MfmaL<T>::row(lane, r)];
                const int c = wn + 16 * j + (lane & 15);
                const int a = a0 + c / TB, b = b0 + c % TB;
                if (ro >= 0 && a < v && b < v && (!diag_out || a < b)) {
                    const i64 off = (i64)ro * vv + (i64)a * v + b;
                    C2 o2 = Zb[off];
                    o2.x += al * accr[i][j][r];
                    o2.y += al * acci[i][j][r];
                    Zb[off] = o2;
                }
            }
}

// Workgroups are dealt to the eight XCDs round-robin by linear id, and each XCD has its own L2.
// order 1: the 1D grid is read as (XCD c = id % 8, slot s = id / 8); slot s of XCD c runs row tile
// s % tilesM of group G = (s / tilesM) * 8 + c, a group being one (k block, a/b tile): the row
// tiles of a group share the Cholesky chunks of every step (147 KB at Naux = 144) in one L2, and
// groups (with their early exits: non-unique blocks and tiles, rows past a diagonal block's end)
// are spread evenly over the XCDs.  order 0: x = row tile + tilesM * a/b tile, y = k block.
constexpr int kXcd = 8;

template <typename T, int WM, int WN, int QCH>
__global__ void __launch_bounds__(WM * WN * 64) ladder_kernel_pipe(LadderArgs p) {
    if (p.order == 1) {
        constexpr int BM = WM * 4 * 16;
        const int tilesM = ((p.pack_rows ? p.mrows : p.nrhs * p.o * p.o) + BM - 1) / BM;
        const int tAB = ((p.v + TA - 1) / TA) * ((p.v + TB - 1) / TB);
        const int groups = (p.pack_rows ? p.nk * p.nk : p.nk * p.nk * p.nk) * tAB;
        const int g = blockIdx.x, c = g % kXcd, s = g / kXcd;
        const int G = (s / tilesM) * kXcd + c;
        if (G >= groups) return;
        ladder_pipe_tile<T, WM, WN, QCH>(p, s % tilesM + tilesM * (G % tAB), G / tAB);
    } else {
        ladder_pipe_tile<T, WM, WN, QCH>(p, blockIdx.x, blockIdx.y);
    }
}

// Persistent form over several ladders (chains of different shapes): every
// workgroup takes (ladder, k block, tile) items from one atomic counter until
// the queue is empty.  The ladders are ordered by decreasing cost per item, so
// the expensive tiles start first and the cheap ones fill the tail.
template <typename T, int WM, int WN, int QCH>
__global__ void __launch_bounds__(WM * WN * 64) ladder_kernel_pipe_group(LadderGroup g) {
    __shared__ long long item_s;

    while (true) {
        if (threadIdx.x == 0) item_s = (long long)atomicAdd(g.counter, 1u);
        __syncthreads();
        const long long item = item_s;
        __syncthreads();
        if (item >= g.total) break;
        int d = 0;
        while (d + 1 < g.n && g.start[d + 1] <= item) ++d;
        const LadderArgs p = g.args[d];
        const long long local = item - g.start[d];
        const long long ntile = g.tiles[d];
        ladder_pipe_tile<T, WM, WN, QCH>(p, (int)(local % ntile), (int)(local / ntile));
    }
}

__global__ void k_zero_counter(unsigned *c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0u;
}

// launch shape of the pipelined kernel per precision: complex64 384-row tiles of
// 12 waves (three per SIMD, 168 registers each) with 24-vector Cholesky chunks,
// complex128 256-row tiles of 8 waves with 8-vector chunks, sized to the register
// file and LDS
template <typename T> struct PipeCfg;
template <> struct PipeCfg<float> { static constexpr int WM = 6, WN = 2, QCH = 24, BM = 384; };
template <> struct PipeCfg<double> { static constexpr int WM = 4, WN = 2, QCH = 8, BM = 256; };

// The launch arguments of the pipelined kernel with the largest class's row count filled in.
LadderArgs ladder_prepared(const LadderArgs &a) {
    LadderArgs b = a;
    b.mrows = 0;
    if (b.pack_rows)
        for (int K = 0; K < b.km.size(); ++K) b.mrows = std::max(b.mrows, ladder_class_rows(b, K));
    return b;
}

int ladder_rows_max(const LadderArgs &a) { return ladder_prepared(a).mrows; }

// (row tiles, blocks) of the pipelined kernel's grid
template <typename T>
static void pipe_grid(const LadderArgs &b, long long &tilesM, long long &blocks) {
    const long long rows = b.pack_rows ? b.mrows : (long long)b.nrhs * b.o * b.o;
    tilesM = (rows + PipeCfg<T>::BM - 1) / PipeCfg<T>::BM;
    blocks = (long long)b.nk * b.nk * (b.pack_rows ? 1 : b.nk);
}

template <typename T>
hipError_t launch_ladder(const LadderArgs &a, hipStream_t s) {
    const int M = a.nrhs * a.o * a.o;
    const int tA = (a.v + TA - 1) / TA, tB = (a.v + TB - 1) / TB;
    if (a.packed == 2) {
        typedef PipeCfg<T> C;
        const LadderArgs b = ladder_prepared(a);
        // row offsets are 32-bit in units of v*v elements
        if ((long long)b.nk * b.nk * b.nk * M >= (1LL << 31)) return hipErrorInvalidValue;
        long long tilesMp, blocks;
        pipe_grid<T>(b, tilesMp, blocks);
        const long long groups = blocks * tA * tB;
        dim3 gp((unsigned)(tilesMp * tA * tB), (unsigned)blocks);
        if (b.order == 1) gp = dim3((unsigned)(kXcd * tilesMp * ((groups + kXcd - 1) / kXcd)), 1);
        hipLaunchKernelGGL((ladder_kernel_pipe<T, C::WM, C::WN, C::QCH>), gp, dim3(C::WM * C::WN * 64), 0, s, b);
    } else if (use_big(a)) {
        const int tilesM = (M + BTM - 1) / BTM;
        dim3 grid(tilesM * tA * tB, a.nk * a.nk * a.nk);
        if (a.packed) hipLaunchKernelGGL(ladder_kernel_packed<T>, grid, dim3(NTP), 0, s, a);
        else hipLaunchKernelGGL(ladder_kernel_big<T>, grid, dim3(NTB), 0, s, a);
    } else {
        const int tilesM = (M + LTM - 1) / LTM;
        dim3 grid(tilesM * tA * tB, a.nk * a.nk * a.nk);
        hipLaunchKernelGGL(ladder_kernel<T>, grid, dim3(NTL), 0, s, a);
    }
    return hipGetLastError();
}

template <typename T>
long long ladder_group_tiles(const LadderArgs &a, long long *blocks) {
    const LadderArgs b = ladder_prepared(a);
    const int tA = (a.v + TA - 1) / TA, tB = (a.v + TB - 1) / TB;
    long long tilesM, nb;
    pipe_grid<T>(b, tilesM, nb);
    if (blocks) *blocks = nb;
    return tilesM * tA * tB;
}

template <typename T>
hipError_t launch_ladder_group(const LadderGroup &g, int nblocks, hipStream_t s) {
    typedef PipeCfg<T> C;
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, g.counter);
    hipLaunchKernelGGL((ladder_kernel_pipe_group<T, C::WM, C::WN, C::QCH>), dim3(nblocks), dim3(C::WM * C::WN * 64), 0, s, g);
    return hipGetLastError();
}

template long long ladder_group_tiles<double>(const LadderArgs &, long long *);
template long long ladder_group_tiles<float>(const LadderArgs &, long long *);
template hipError_t launch_ladder_group<double>(const LadderGroup &, int, hipStream_t);
template hipError_t launch_ladder_group<float>(const LadderGroup &, int, hipStream_t);

double ladder_flop_count(const LadderArgs &a, bool fp64, bool mfma) {
    const int M = a.nrhs * a.o * a.o;
    const bool pipe = a.packed == 2;
    const bool big = pipe || use_big(a);
    const int tm = pipe ? (fp64 ? PipeCfg<double>::BM : PipeCfg<float>::BM) : big ? BTM : LTM;
    const double tilesM = (M + tm - 1) / tm;
    const int tA = (a.v + TA - 1) / TA, tB = (a.v + TB - 1) / TB, tE = (a.v + TE - 1) / TE, tF = (a.v + TF - 1) / TF;
    const int qc = pipe ? (fp64 ? PipeCfg<double>::QCH : PipeCfg<float>::QCH) : (big && !a.packed) ? 2 * QC : QC;
    const double qpad = (double)((a.naux + qc - 1) / qc) * qc;
    const double main_step = 8.0 * tm * LTN * LTK, rebuild_step = 8.0 * (TA * TE) * (TB * TF) * qpad;
    if (!(big && a.packed)) {
        const double steps = (double)a.nk * a.nk * a.nk * tilesM * tA * tB * a.nk * tE * tF;
        return steps * (main_step + rebuild_step);
    }
    // packed: count the unique output tiles and unique input tiles actually visited, at 8 real
    // flops per complex product formed; in real matrix-core flops (mfma) the complex64
    // pipelined kernel's rebuild products count 6
    const double rb = (mfma && pipe && !fp64) ? 0.75 : 1.0;
    const int nk = a.nk;
    const bool rows = pipe && a.pack_rows;
    // blocks: momentum classes K = ki + kj with the unique rows of all their (ki <= kj) pairs, or
    // every (ki, kj) pair with all its rows
    double steps = 0;
    for (int K = 0; K < nk; ++K)
        for (int ki = 0; ki < (rows ? 1 : nk); ++ki) {
            const int kj = a.km.sub(K, ki);
            const double tiles = rows ? (double)((ladder_class_rows(a, K) + tm - 1) / tm) : tilesM;
            for (int ka = 0; ka < nk; ++ka) {
                const int kb = a.km.sub(K, ka);
                if (ka > kb) continue;
                const double out = ka == kb ? tA * (tA + 1) / 2.0 : (double)tA * tB;
                double in = 0;
                for (int ke = 0; ke < nk; ++ke) {
                    const int kf = a.km.sub(K, ke);
                    if (ke > kf) continue;
                    in += ke == kf ? tE * (tE + 1) / 2.0 : (double)tE * tF;
                }
                steps += out * in * tiles;
            }
            (void)kj;
        }
    return steps * (main_step + 2.0 * rb * rebuild_step);
}

double ladder_executed_flops(const LadderArgs &a, bool fp64) { return ladder_flop_count(a, fp64, false); }
double ladder_mfma_flops(const LadderArgs &a, bool fp64) { return ladder_flop_count(a, fp64, true); }

template hipError_t launch_ladder<double>(const LadderArgs &, hipStream_t);
template hipError_t launch_ladder<float>(const LadderArgs &, hipStream_t);

}  // namespace lrcc
