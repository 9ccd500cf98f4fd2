// Batched strided complex GEMM on the gfx950 matrix cores.
//
// A complex product is four real MFMA products on split real/imaginary
// planes staged in LDS: Cre += Are*Bre - Aim*Bim, Cim += Are*Bim + Aim*Bre.
// Tile 64x64x16 (complex), 256 threads = 4 waves in a 2x2 grid, each wave a
// 32x32 sub-tile of 2x2 MFMA 16x16x4 blocks.  Operand addresses use the
// two-level index splits of GemmArgs so that k-blocked tensors are read in
// place (no permute passes); the thread->element map of each tile load runs
// along the unit-stride index when one exists, for coalesced loads.
#include "common.hpp"

namespace lrcc {

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output row of accumulator register r held by `lane` (column = lane % 16)
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int TM = 64, TN = 64, TK = 16, NT = 256;

template <typename T>
__global__ void __launch_bounds__(NT) gemm_kernel(GemmArgs g) {
    typedef typename Cx<T>::type C2;
    typedef typename Mfma<T>::v4 v4;
    __shared__ T Ar[TK][TM], Ai[TK][TM], Br[TK][TN], Bi[TK][TN];

    const int job = blockIdx.y;
    const int tilesM = (g.M + TM - 1) / TM;
    const int m0 = (blockIdx.x % tilesM) * TM;
    const int n0 = (blockIdx.x / tilesM) * TN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;

    const C2 *A = reinterpret_cast<const C2 *>(g.A);
    const C2 *B = reinterpret_cast<const C2 *>(g.B);
    C2 *C = reinterpret_cast<C2 *>(g.C);

    // thread -> tile element maps (4 elements of A and 4 of B per thread)
    const bool aM = g.aMfast != 0;
    const bool bN = g.bNfast != 0;
    int am[4], ak[4], bk[4], bn[4];
    i64 arow[4], bcol[4];
    bool aok[4], bok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int idx = tid + NT * q;
        if (aM) { am[q] = idx % TM; ak[q] = idx / TM; } else { ak[q] = idx % TK; am[q] = idx / TK; }
        if (bN) { bn[q] = idx % TN; bk[q] = idx / TN; } else { bk[q] = idx % TK; bn[q] = idx / TK; }
        int gm = m0 + am[q], gn = n0 + bn[q];
        aok[q] = gm < g.M;
        bok[q] = gn < g.N;
        arow[q] = aok[q] ? split_off(gm, g.sm, g.Am) : 0;
        bcol[q] = bok[q] ? split_off(gn, g.sn, g.Bn) : 0;
    }

    v4 accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { accr[i][j] = v4{0, 0, 0, 0}; acci[i][j] = v4{0, 0, 0, 0}; }

    const int sb = g.segBeg[job], se = g.segBeg[job + 1];
    for (int s = sb; s < se; ++s) {
        const C2 *As = A + g.segA[s];
        const C2 *Bs = B + g.segB[s];
        for (int k0 = 0; k0 < g.K; k0 += TK) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int gk = k0 + ak[q];
                C2 v;
                if (aok[q] && gk < g.K) {
                    v = As[arow[q] + split_off(gk, g.sk, g.Ak)];
                } else { v.x = 0; v.y = 0; }
                Ar[ak[q]][am[q]] = v.x;
                Ai[ak[q]][am[q]] = v.y;
                gk = k0 + bk[q];
                C2 w;
                if (bok[q] && gk < g.K) {
                    w = Bs[bcol[q] + split_off(gk, g.sk, g.Bk)];
                } else { w.x = 0; w.y = 0; }
                Br[bk[q]][bn[q]] = w.x;
                Bi[bk[q]][bn[q]] = w.y;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < TK; kk += 4) {
                const int kr = kk + (lane >> 4), c = lane & 15;
                T ar[2], ai[2], br[2], bi[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) { ar[i] = Ar[kr][wm + 16 * i + c]; ai[i] = Ai[kr][wm + 16 * i + c]; }
#pragma unroll
                for (int j = 0; j < 2; ++j) { br[j] = Br[kr][wn + 16 * j + c]; bi[j] = Bi[kr][wn + 16 * j + c]; }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        accr[i][j] = Mfma<T>::mma(ar[i], br[j], accr[i][j]);
                        accr[i][j] = Mfma<T>::mma(-ai[i], bi[j], accr[i][j]);
                        acci[i][j] = Mfma<T>::mma(ar[i], bi[j], acci[i][j]);
                        acci[i][j] = Mfma<T>::mma(ai[i], br[j], acci[i][j]);
                    }
            }
            __syncthreads();
        }
    }

    const T alr = (T)g.alpha_re, ali = (T)g.alpha_im;
    C2 *Cj = C + g.offC[job];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int gm = m0 + wm + 16 * i + Mfma<T>::row(lane, r);
                int gn = n0 + wn + 16 * j + (lane & 15);
                if (gm < g.M && gn < g.N) {
                    i64 off = split_off(gm, g.sm, g.Cm) + split_off(gn, g.sn, g.Cn);
                    T xr = accr[i][j][r], xi = acci[i][j][r];
                    T vr = alr * xr - ali * xi, vi = alr * xi + ali * xr;
                    if (g.beta) { C2 o = Cj[off]; vr += o.x; vi += o.y; }
                    C2 w; w.x = vr; w.y = vi;
                    Cj[off] = w;
                }
            }
}

template <typename T>
hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
    if (g.njobs <= 0 || g.M <= 0 || g.N <= 0) return hipSuccess;
    const int tilesM = (g.M + TM - 1) / TM, tilesN = (g.N + TN - 1) / TN;
    // grid.y is limited to 65535: launch the job list in chunks
    for (int j0 = 0; j0 < g.njobs; j0 += 65535) {
        GemmArgs c = g;
        c.njobs = (g.njobs - j0 < 65535) ? g.njobs - j0 : 65535;
        c.offC = g.offC + j0;
        c.segBeg = g.segBeg + j0;
        dim3 grid(tilesM * tilesN, c.njobs);
        hipLaunchKernelGGL(gemm_kernel<T>, grid, dim3(NT), 0, s, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_gemm<double>(const GemmArgs &, hipStream_t);
template hipError_t launch_gemm<float>(const GemmArgs &, hipStream_t);

}  // namespace lrcc
