// Internal declarations shared by the HIP kernels and the host planner.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

namespace lrcc {

typedef long long i64;

// Planning without a device: allocations return placeholder addresses, no
// copies or launches happen, and every recorded GEMM is bounds-checked.
extern bool g_dry_run;


// Real type -> interleaved complex type used in device memory.
template <typename T> struct Cx;
template <> struct Cx<double> { typedef double2 type; };
template <> struct Cx<float> { typedef float2 type; };

// Three-level split of a GEMM index: idx = (i0*d1 + i1)*d2 + i2 and the
// address contribution is i0*s[0] + i1*s[1] + i2*s[2] (units: complex elements).
struct Split {
    int d1, d2;
};
struct Strides {
    i64 s[3];
};
__host__ __device__ inline i64 split_off(int idx, Split sp, Strides st) {
    const int q = idx / sp.d2;
    return (i64)(q / sp.d1) * st.s[0] + (i64)(q % sp.d1) * st.s[1] + (i64)(idx % sp.d2) * st.s[2];
}

// One strided complex GEMM over a list of output blocks ("jobs").
// For job j: C_j[m][n] = beta*C_j[m][n] + alpha * sum_{s in segs(j)} sum_k A_s[m][k] B_s[k][n]
//   A_s[m][k] = A + segA[s] + off(m; sm, Am) + off(k; sk, Ak)
//   B_s[k][n] = B + segB[s] + off(k; sk, Bk) + off(n; sn, Bn)
//   C_j[m][n] = C + offC[j] + off(m; sm, Cm) + off(n; sn, Cn)
struct GemmArgs {
    const void *A, *B;
    void *C;
    int M, N, K;
    Split sm, sn, sk;
    Strides Am, Ak, Bk, Bn, Cm, Cn;
    int aMfast, bNfast;  // tile-load thread maps: 1 = run along m (resp. n)
    int shape;           // tile shape: -1 automatic, 0 = 64x64, 1 = large (128x128 complex64, 128x64
                         // complex128), 2 = 16x256 (small M)
    int alt;             // autotuner candidate: 0 = heuristic shape, 1 = the alternative shape
    double alpha_re, alpha_im;
    int beta;
    const i64 *offC;
    const int *segBeg;   // njobs + 1
    const i64 *segA, *segB;
    int njobs;
    int job0;            // index of the first job of this launch in the full job list
    int njobs_all;       // length of the full job list
    // split-K: ksplit > 1 partitions each job's (segment, K) steps into ksplit ranges; each writes its
    // partial product to part[split][job][M][N] (dense) and a second kernel sums the ranges in order
    // and applies alpha/beta (deterministic, no atomics)
    int ksplit;
    void *part;
    const float *jscale; // per-job multiplier of alpha (full job list), or null
    int kind;            // 0 generic, 1 stored-integral ladder (a separate kernel symbol for profiling)
};

template <typename T>
hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);
int gemm_shape(const GemmArgs &g, bool fp64);

// Ladder: sigma2[ki,kj,ka][R][i][j][a][b] += alpha * sum_{ke} sum_{e,f}
//   Y[ki,kj,ke][R][i][j][e][f] * sum_Q La[ka][ke][Q][a][e] * Lb[kb][kf][Q][b][f]
struct LadderArgs {
    const void *Y;       // [nk^3][R][o][o][v][v]
    const void *La;      // [nk][nk][naux][v][v]
    const void *Lb;      // [nk][nk][naux][v][v]
    void *Z;             // output, same layout as Y (accumulated)
    int nk, nrhs, o, v, naux;
    double alpha;
    int packed;          // 1: Y antisymmetric in (e,f); form only unique (e,f) and (a,b) pairs
};
template <typename T>
hipError_t launch_ladder(const LadderArgs &a, hipStream_t s);
// real flops the ladder kernel executes (tile padding and LDS rebuild included)
double ladder_executed_flops(const LadderArgs &a);

}  // namespace lrcc
