// Batched strided complex GEMM on the gfx950 matrix cores.
//
// A complex product is four real MFMA products on split real/imaginary
// planes staged in LDS: Cre += Are*Bre - Aim*Bim, Cim += Are*Bim + Aim*Bre.
// 256 threads = 4 waves; each wave owns a WTM x WTN sub-tile of 16x16x4 MFMA
// blocks.  Tile shapes: 64x64 (default), 128x128 (complex64, large M and N)
// and 128x64 (complex128, large M).  Operand addresses use the three-level
// index splits of GemmArgs so that k-blocked tensors are read in place (no
// permute passes); the thread->element map of each tile load runs along the
// unit-stride index when one exists, for coalesced loads.
#include "common.hpp"

#include <algorithm>
#include <vector>

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

constexpr int TK = 16, NT = 256;

// G3: complex products from three real matrix-core products (Gauss' method:
// k1 = br (ar + ai), k2 = ar (bi - br), k3 = ai (br + bi); re = k1 - k3, im = k1 + k2)
template <typename T, int TM, int TN, int WTM, int WTN, int KIND, bool G3 = false>
__global__ void __launch_bounds__(NT) gemm_kernel(GemmArgs g) {
    typedef typename Cx<T>::type C2;
    typedef typename Mfma<T>::v4 v4;
    constexpr int WGM = TM / WTM;            // waves along M
    constexpr int FM = WTM / 16, FN = WTN / 16;
    constexpr int LA = TM * TK / NT, LB = TK * TN / NT;
    static_assert((TM / WTM) * (TN / WTN) == 4, "4 waves per block");
    // rows padded so that K-fast tile stores (16 lanes along K) and the MFMA operand
    // reads (4 K rows x 16 lanes) fall into distinct LDS banks
    constexpr int PAD = sizeof(T) == 8 ? 9 : 17;
    __shared__ T Ar[TK][TM + PAD], Ai[TK][TM + PAD], Br[TK][TN + PAD], Bi[TK][TN + PAD];

    const int job = blockIdx.y;
    const int split = blockIdx.z;
    const int tilesM = (g.M + TM - 1) / TM;
    const int m0 = (blockIdx.x % tilesM) * TM;
    const int n0 = (blockIdx.x / tilesM) * TN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave % WGM) * WTM, wn = (wave / WGM) * WTN;

    const C2 *A = reinterpret_cast<const C2 *>(g.A);
    const C2 *B = reinterpret_cast<const C2 *>(g.B);
    C2 *C = reinterpret_cast<C2 *>(g.C);

    const bool aM = g.aMfast != 0;
    const bool bN = g.bNfast != 0;
    int am[LA], ak[LA], bk[LB], bn[LB];
    // operand offsets inside a segment's blocks fit in 32 bits (checked when the GEMM is recorded)
    const int ak0 = (int)g.Ak.s[0], ak1 = (int)g.Ak.s[1], ak2 = (int)g.Ak.s[2];
    const int bk0 = (int)g.Bk.s[0], bk1 = (int)g.Bk.s[1], bk2 = (int)g.Bk.s[2];
    int arow[LA], bcol[LB];
    bool aok[LA], bok[LB];
#pragma unroll
    for (int q = 0; q < LA; ++q) {
        const int idx = tid + NT * q;
        if (aM) { am[q] = idx % TM; ak[q] = idx / TM; } else { ak[q] = idx % TK; am[q] = idx / TK; }
        const int gm = m0 + am[q];
        aok[q] = gm < g.M;
        arow[q] = aok[q] ? split_off32(gm, g.sm, (int)g.Am.s[0], (int)g.Am.s[1], (int)g.Am.s[2]) : 0;
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
        const int idx = tid + NT * q;
        if (bN) { bn[q] = idx % TN; bk[q] = idx / TN; } else { bk[q] = idx % TK; bn[q] = idx / TK; }
        const int gn = n0 + bn[q];
        bok[q] = gn < g.N;
        bcol[q] = bok[q] ? split_off32(gn, g.sn, (int)g.Bn.s[0], (int)g.Bn.s[1], (int)g.Bn.s[2]) : 0;
    }

    v4 accr[FM][FN], acci[FM][FN], acc3[G3 ? FM : 1][G3 ? FN : 1];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) { accr[i][j] = v4{0, 0, 0, 0}; acci[i][j] = v4{0, 0, 0, 0}; }
    if constexpr (G3) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc3[i][j] = v4{0, 0, 0, 0};
    }

    const int sb = g.segBeg[job], se = g.segBeg[job + 1];
    const int ksteps = (g.K + TK - 1) / TK;
    const i64 nsteps = (i64)(se - sb) * ksteps;
    const int tbeg = (int)(nsteps * split / g.ksplit), tend = (int)(nsteps * (split + 1) / g.ksplit);
    // software pipeline: the global loads of step t+1 are issued into registers
    // before the matrix-core work of step t
    C2 va[LA], vb[LB];
    auto fetch = [&](int t) {
        const int s = sb + t / ksteps, k0 = (t % ksteps) * TK;
        const C2 *As = A + g.segA[s];
        const C2 *Bs = B + g.segB[s];
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const int gk = k0 + ak[q];
            if (aok[q] && gk < g.K) va[q] = As[arow[q] + split_off32<(KIND >= 2)>(gk, g.sk, ak0, ak1, ak2)];
            else { va[q].x = 0; va[q].y = 0; }
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int gk = k0 + bk[q];
            if (bok[q] && gk < g.K) vb[q] = Bs[bcol[q] + split_off32<(KIND >= 2)>(gk, g.sk, bk0, bk1, bk2)];
            else { vb[q].x = 0; vb[q].y = 0; }
        }
    };
    if (tbeg < tend) fetch(tbeg);
    for (int t = tbeg; t < tend; ++t) {
#pragma unroll
        for (int q = 0; q < LA; ++q) { Ar[ak[q]][am[q]] = va[q].x; Ai[ak[q]][am[q]] = va[q].y; }
#pragma unroll
        for (int q = 0; q < LB; ++q) { Br[bk[q]][bn[q]] = vb[q].x; Bi[bk[q]][bn[q]] = vb[q].y; }
        __syncthreads();
        if (t + 1 < tend) fetch(t + 1);
#pragma unroll
        for (int kk = 0; kk < TK; kk += 4) {
            const int kr = kk + (lane >> 4), c = lane & 15;
            T ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) { ar[i] = Ar[kr][wm + 16 * i + c]; ai[i] = Ai[kr][wm + 16 * i + c]; }
#pragma unroll
            for (int j = 0; j < FN; ++j) { br[j] = Br[kr][wn + 16 * j + c]; bi[j] = Bi[kr][wn + 16 * j + c]; }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if constexpr (G3) {
                        accr[i][j] = Mfma<T>::mma(ar[i] + ai[i], br[j], accr[i][j]);
                        acci[i][j] = Mfma<T>::mma(ar[i], bi[j] - br[j], acci[i][j]);
                        acc3[i][j] = Mfma<T>::mma(ai[i], br[j] + bi[j], acc3[i][j]);
                    } else {
                        accr[i][j] = Mfma<T>::mma(ar[i], br[j], accr[i][j]);
                        accr[i][j] = Mfma<T>::mma(-ai[i], bi[j], accr[i][j]);
                        acci[i][j] = Mfma<T>::mma(ar[i], bi[j], acci[i][j]);
                        acci[i][j] = Mfma<T>::mma(ai[i], br[j], acci[i][j]);
                    }
                }
        }
        __syncthreads();
    }
    if constexpr (G3) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                acci[i][j] = accr[i][j] + acci[i][j];
                accr[i][j] = accr[i][j] - acc3[i][j];
            }
    }

    if (g.ksplit > 1) {
        // raw partial sums, reduced by k_gemm_reduce
        C2 *Pj = reinterpret_cast<C2 *>(g.part) + ((i64)split * g.njobs_all + g.job0 + job) * g.M * g.N;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gm = m0 + wm + 16 * i + Mfma<T>::row(lane, r);
                    const int gn = n0 + wn + 16 * j + (lane & 15);
                    if (gm < g.M && gn < g.N) {
                        C2 w; w.x = accr[i][j][r]; w.y = acci[i][j][r];
                        Pj[(i64)gm * g.N + gn] = w;
                    }
                }
        return;
    }
    const T js = g.jscale ? (T)g.jscale[g.job0 + job] : (T)1;
    const T alr = js * (T)g.alpha_re, ali = js * (T)g.alpha_im;
    C2 *Cj = C + g.offC[job];
    i64 coff[FN];
    bool cok[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int gn = n0 + wn + 16 * j + (lane & 15);
        cok[j] = gn < g.N;
        coff[j] = cok[j] ? split_off(gn, g.sn, g.Cn) : 0;
    }
    // Output rows in groups of EG fragment rows.  With beta all reads of C in a group are
    // issued, unconditionally, before its first write: a write may alias a later read as far
    // as the compiler knows, so read-add-write element by element would wait out one memory
    // round trip per element, which bounds the short-K products.
    constexpr int EG = 1;
#pragma unroll
    for (int i0 = 0; i0 < FM; i0 += EG) {
        i64 roff[EG][4];
        bool rok[EG][4];
#pragma unroll
        for (int ii = 0; ii < EG; ++ii)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * (i0 + ii) + Mfma<T>::row(lane, r);
                rok[ii][r] = gm < g.M;
                roff[ii][r] = rok[ii][r] ? split_off(gm, g.sm, g.Cm) : 0;
            }
        C2 old[EG][FN][4];
        if (g.beta) {
#pragma unroll
            for (int ii = 0; ii < EG; ++ii)
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r)   // (0, 0) of the block stands in for outside elements
                        old[ii][j][r] = Cj[rok[ii][r] && cok[j] ? roff[ii][r] + coff[j] : 0];
        }
#pragma unroll
        for (int ii = 0; ii < EG; ++ii)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (!(rok[ii][r] && cok[j])) continue;
                    const T xr = accr[i0 + ii][j][r], xi = acci[i0 + ii][j][r];
                    T vr = alr * xr - ali * xi, vi = alr * xi + ali * xr;
                    if (g.beta) { vr += old[ii][j][r].x; vi += old[ii][j][r].y; }
                    C2 w; w.x = vr; w.y = vi;
                    Cj[roff[ii][r] + coff[j]] = w;
                }
    }
}

template <typename T, int TM, int TN, int WTM, int WTN, bool G3 = false>
hipError_t launch_shape(const GemmArgs &g, hipStream_t s) {
    const int tilesM = (g.M + TM - 1) / TM, tilesN = (g.N + TN - 1) / TN;
    // grid.y is limited to 65535: launch the job list in chunks
    for (int j0 = 0; j0 < g.njobs; j0 += 65535) {
        GemmArgs c = g;
        c.njobs = (g.njobs - j0 < 65535) ? g.njobs - j0 : 65535;
        c.offC = g.offC + j0;
        c.segBeg = g.segBeg + j0;
        c.job0 = j0;
        dim3 grid(tilesM * tilesN, c.njobs, g.ksplit);
        // KIND 2 (generic) and 3 (ladder): the reduction index is a triangle split
        if (g.sk.tri && g.kind == 1)
            hipLaunchKernelGGL((gemm_kernel<T, TM, TN, WTM, WTN, 3, G3>), grid, dim3(NT), 0, s, c);
        else if (g.sk.tri) hipLaunchKernelGGL((gemm_kernel<T, TM, TN, WTM, WTN, 2, G3>), grid, dim3(NT), 0, s, c);
        else if (g.kind == 1) hipLaunchKernelGGL((gemm_kernel<T, TM, TN, WTM, WTN, 1, G3>), grid, dim3(NT), 0, s, c);
        else hipLaunchKernelGGL((gemm_kernel<T, TM, TN, WTM, WTN, 0, G3>), grid, dim3(NT), 0, s, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// C[job](m, n) = alpha * sum_split part[split][job][m][n] (+ C), splits summed in order
template <typename T>
__global__ void k_gemm_reduce(GemmArgs g) {
    typedef typename Cx<T>::type C2;
    const C2 *P = reinterpret_cast<const C2 *>(g.part);
    C2 *C = reinterpret_cast<C2 *>(g.C);
    const i64 per = (i64)g.M * g.N, n = (i64)g.njobs * per;
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        const int job = (int)(t / per);
        const T js = g.jscale ? (T)g.jscale[job] : (T)1;
        const T alr = js * (T)g.alpha_re, ali = js * (T)g.alpha_im;
        const int gm = (int)((t % per) / g.N), gn = (int)(t % g.N);
        T xr = 0, xi = 0;
        for (int z = 0; z < g.ksplit; ++z) {
            const C2 v = P[(i64)z * n + t];
            xr += v.x;
            xi += v.y;
        }
        T vr = alr * xr - ali * xi, vi = alr * xi + ali * xr;
        const i64 off = g.offC[job] + split_off(gm, g.sm, g.Cm) + split_off(gn, g.sn, g.Cn);
        if (g.beta) { C2 o = C[off]; vr += o.x; vi += o.y; }
        C2 w; w.x = vr; w.y = vi;
        C[off] = w;
    }
}

int gemm_shape(const GemmArgs &g, bool fp64) {
    if (g.shape >= 0) return g.shape;
    if (g.M <= 16 && g.N >= 128) return 2;
    if (g.M >= 128 && g.N >= 128) return 1;
    if (fp64 && g.M >= 128 && g.N >= 64) return 1;
    return 0;
}

std::vector<int> gemm_candidates(const GemmArgs &g, bool fp64) {
    GemmArgs h = g;
    h.shape = -1;
    std::vector<int> c{gemm_shape(h, fp64)};
    // complex64 large tiles also come with three real products per complex one (4)
    const int others[5] = {0, 1, 3, 4, 2};
    const int cap = fp64 ? 3 : 4;
    for (int s : others) {
        if ((int)c.size() == cap) break;
        if ((s == 3 || s == 4) && fp64) continue;   // complex128 large tile is already 128x64
        if (s == 4 && (g.M < 128 || g.N < 128)) continue;
        if (s == 2 && g.M > 32) continue;         // small-M tile only for short M
        if (s != 0 && g.M < 64 && s != 2) continue;
        if (std::find(c.begin(), c.end(), s) == c.end()) c.push_back(s);
    }
    return c;
}

template <typename T>
hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
    if (g.njobs <= 0 || g.M <= 0 || g.N <= 0) return hipSuccess;
    constexpr bool f64 = sizeof(T) == 8;
    hipError_t e;
    switch (gemm_shape(g, f64)) {
    case 1:
        if constexpr (f64) e = launch_shape<T, 128, 64, 64, 32>(g, s);
        else e = launch_shape<T, 128, 128, 64, 64>(g, s);
        break;
    case 2: e = launch_shape<T, 16, 256, 16, 64>(g, s); break;
    case 3:   // complex64 only: 128x64 tiles with three real products per complex one
        e = launch_shape<T, 128, 64, 64, 32, !f64>(g, s);
        break;
    case 4:   // complex64 only: 128x128 tiles with three real products per complex one
        if constexpr (f64) e = launch_shape<T, 128, 64, 64, 32>(g, s);
        else e = launch_shape<T, 128, 128, 64, 64, true>(g, s);
        break;
    default: e = launch_shape<T, 64, 64, 32, 32>(g, s); break;
    }
    if (e != hipSuccess || g.ksplit <= 1) return e;
    const i64 n = (i64)g.njobs * g.M * g.N;
    const unsigned blocks = (unsigned)std::min<i64>((n + 255) / 256, 65535);
    hipLaunchKernelGGL(k_gemm_reduce<T>, dim3(blocks), dim3(256), 0, s, g);
    return hipGetLastError();
}

template hipError_t launch_gemm<double>(const GemmArgs &, hipStream_t);
template hipError_t launch_gemm<float>(const GemmArgs &, hipStream_t);

}  // namespace lrcc
