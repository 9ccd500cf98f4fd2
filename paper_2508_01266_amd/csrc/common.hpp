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

// Device-memory arena: between arena_begin and arena_end, dev_alloc hands out 256-byte-aligned
// pieces of [base, base + size) instead of calling hipMalloc (LRCC_E_OOM past the end), and
// dev_free ignores pointers inside any registered arena.
void arena_register(void *base, size_t size);
void arena_begin(void *base, size_t size);
void arena_end();
size_t arena_used();
bool arena_active();
bool in_arena(const void *p);
// The static device array of the no-allocation entry point on device `dev` (its address from
// hipGetSymbolAddress, taken once per device with that device current) and its size.
void *noalloc_scratch(int dev, size_t *bytes);


// Crystal-momentum mesh Z_n0 x Z_n1 x Z_n2: momentum is conserved modulo a
// reciprocal-lattice vector (Eq. momentum), so k points add componentwise,
// each component modulo its own extent.  A point is stored by its flat index
// (j0 * n1 + j1) * n2 + j2; the 1D chain of the paper is the mesh (nk, 1, 1),
// whose flat index is the plain k index, and takes a single-modulus path.
struct KMesh {
    int n0 = 1, n1 = 1, n2 = 1;
    __host__ __device__ int size() const { return n0 * n1 * n2; }
    __host__ __device__ bool chain() const { return n1 == 1 && n2 == 1; }
    // flat index of sa*a + sb*b + sc*c (signs -1, 0 or +1)
    __host__ __device__ int sum3(int sa, int a, int sb, int b, int sc, int c) const {
        if (chain()) {
            const int r = (sa * a + sb * b + sc * c) % n0;
            return r < 0 ? r + n0 : r;
        }
        const int a2 = a % n2, b2 = b % n2, c2 = c % n2;
        const int a1 = (a / n2) % n1, b1 = (b / n2) % n1, c1 = (c / n2) % n1;
        const int a0 = a / (n1 * n2), b0 = b / (n1 * n2), c0 = c / (n1 * n2);
        int r0 = (sa * a0 + sb * b0 + sc * c0) % n0;
        int r1 = (sa * a1 + sb * b1 + sc * c1) % n1;
        int r2 = (sa * a2 + sb * b2 + sc * c2) % n2;
        r0 += r0 < 0 ? n0 : 0;
        r1 += r1 < 0 ? n1 : 0;
        r2 += r2 < 0 ? n2 : 0;
        return (r0 * n1 + r1) * n2 + r2;
    }
    // a + b - c: the fourth momentum of a conserving quartet
    __host__ __device__ int comb(int a, int b, int c) const { return sum3(1, a, 1, b, -1, c); }
    __host__ __device__ int sub(int a, int b) const { return sum3(1, a, -1, b, 0, 0); }
};

// Real type -> interleaved complex type used in device memory.
template <typename T> struct Cx;
template <> struct Cx<double> { typedef double2 type; };
template <> struct Cx<float> { typedef float2 type; };

// Three-level split of a GEMM index: idx = (i0*d1 + i1)*d2 + i2 and the
// address contribution is i0*s[0] + i1*s[1] + i2*s[2] (units: complex elements).
// The divisions use multiply-high magic numbers (exact for 0 <= idx < 2^31):
// x / d = (x * m) >> (31 + l) with l = ceil(log2 d), m = ceil(2^(31+l) / d); set by
// split_magic before a launch.
// Triangle split (tri = n > 1, made by tri_split): (i1, i2) runs over the n(n-1)/2 pairs
// p < q of an n x n block, packed as a d1 x d2 rectangle by pairing row r of the strict
// upper triangle with a complementary row (n even: rows r and n-1-r, d1 = n/2, d2 = n-1;
// n odd: rows r and n-2-r, d1 = (n-1)/2, d2 = n); the contribution is
// i0*s[0] + p*s[1] + q*s[2].
struct Split {
    int d1, d2;
    unsigned m1 = 0, m2 = 0;   // magic multipliers for d1, d2
    int l1 = 0, l2 = 0;        // their shifts
    int tri = 0;               // n of a triangle split, 0 for a plain one
};
inline Split tri_split(int n) {
    Split s{(n & 1) ? (n - 1) / 2 : n / 2, (n & 1) ? n : n - 1};
    s.tri = n;
    return s;
}
// pair (p, q), p < q, of the packed position (r, c) of a triangle split of n
__host__ __device__ inline void tri_pair(int r, int c, int n, int &p, int &q) {
    if (c < n - 1 - r) {
        p = r;
        q = r + 1 + c;
    } else {
        p = n - 1 - (n & 1) - r;
        q = c + 1 - (n & 1);
    }
}
struct Strides {
    i64 s[3];
};
inline void div_magic(int d, unsigned &m, int &l) {
    l = 0;
    while ((1LL << l) < d) ++l;
    m = (unsigned)(((1ULL << (31 + l)) + (unsigned long long)d - 1) / (unsigned long long)d);
}
inline Split split_magic(Split s) {
    div_magic(s.d1, s.m1, s.l1);
    div_magic(s.d2, s.m2, s.l2);
    return s;
}
__host__ __device__ inline int fdiv(int x, unsigned m, int l) {
    return (int)(((unsigned long long)(unsigned)x * m) >> (31 + l));
}
// 32-bit form for offsets inside one operand block (bounded on the host)
// TRI: the split may be a triangle split (checked at run time); false: a plain split (the
// GEMM's reduction index inside its K loop, where the check would cost every load)
template <bool TRI = true>
__host__ __device__ inline int split_off32(int idx, Split sp, int s0, int s1, int s2) {
    const int q = fdiv(idx, sp.m2, sp.l2);
    const int q0 = fdiv(q, sp.m1, sp.l1);
    int i1 = q - q0 * sp.d1, i2 = idx - q * sp.d2;
    if (TRI && sp.tri) tri_pair(i1, i2, sp.tri, i1, i2);
    return q0 * s0 + i1 * s1 + i2 * s2;
}
__host__ __device__ inline i64 split_off(int idx, Split sp, Strides st) {
    const int q = fdiv(idx, sp.m2, sp.l2);
    const int q0 = fdiv(q, sp.m1, sp.l1);
    int i1 = q - q0 * sp.d1, i2 = idx - q * sp.d2;
    if (sp.tri) tri_pair(i1, i2, sp.tri, i1, i2);
    return (i64)q0 * st.s[0] + (i64)i1 * st.s[1] + (i64)i2 * st.s[2];
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
                         // complex128), 2 = 16x256 (small M), 3 = 128x64 (complex64), 4 = 128x128
                         // (complex64); 3 and 4 form complex products from three real products
    int alt;             // unused (kept zero)
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
    int kind;            // 0 generic, 1 ladder over integral blocks (a separate kernel symbol for
                         // profiling); the launcher takes instances 2 (generic) and 3 (ladder) when
                         // sk is a triangle split
};

template <typename T>
hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);
int gemm_shape(const GemmArgs &g, bool fp64);
// tile shapes the autotuner tries for g (the heuristic one first, at most 3, 4 in complex64)
std::vector<int> gemm_candidates(const GemmArgs &g, bool fp64);

// Ladder: sigma2[ki,kj,ka][R][i][j][a][b] += alpha * sum_{ke} sum_{e,f}
//   Y[ki,kj,ke][R][i][j][e][f] * sum_Q La[ka][ke][Q][a][e] * Lb[kb][kf][Q][b][f]
struct LadderArgs {
    const void *Y;       // [nk^3][R][o][o][v][v]
    const void *La;      // [nk][nk][naux][v][v]
    const void *Lb;      // [nk][nk][naux][v][v]
    void *Z;             // output, same layout as Y (accumulated)
    int nk, nrhs, o, v, naux;   // nk = km.size()
    double alpha;
    int packed;          // Y antisymmetric in (e,f): form only unique (e,f) and (a,b) pairs
                         // (1: 256-row kernel, 2: pipelined kernel); 0: full ranges
    int pack_rows;       // with packed == 2: Y and the result are also antisymmetric in the row pair
                         // (i,j) and Z goes through P(ij)P(ab) afterwards, so only the unique rows
                         // (ki,i) < (kj,j) are formed (blocks ki > kj skipped, i < j when ki == kj)
                         // and written with a further factor 2
    int order;           // pipelined kernel: 1 = XCD-grouped tile order (the row tiles of one
                         // (block, a/b tile) run on one XCD), 0 = row tile fastest in the grid
    int mrows;           // pipelined kernel with pack_rows: rows of the largest momentum class (set
                         // by the launcher; see ladder_class_rows)
    KMesh km;            // k mesh of the blocks
};
// With pack_rows the pipelined kernel's row tiles run over momentum classes: class K holds the
// unique rows of every block (ki, kj) with ki <= kj and ki + kj = K (all of them share the
// integral tiles of a step), block after block in increasing ki.
__host__ __device__ inline int ladder_class_rows(const LadderArgs &p, int K) {
    const int nk = p.km.size(), P = p.o * (p.o - 1) / 2;
    int rows = 0;
    for (int ki = 0; ki < nk; ++ki) {
        const int kj = p.km.sub(K, ki);
        if (ki < kj) rows += p.nrhs * p.o * p.o;
        else if (ki == kj) rows += p.nrhs * P;
    }
    return rows;
}
template <typename T>
hipError_t launch_ladder(const LadderArgs &a, hipStream_t s);

// Several pipelined packed ladders in one persistent launch (device-resident tables):
// ladder d owns items [start[d], start[d+1]); item = k block * tiles[d] + tile.
struct LadderGroup {
    const LadderArgs *args;
    const long long *start;   // n + 1 prefix sums
    const long long *tiles;   // tiles per k block of each ladder
    int n;
    long long total;
    unsigned *counter;        // work-queue counter (zeroed by the launcher on the stream)
};
template <typename T>
long long ladder_group_tiles(const LadderArgs &a, long long *blocks);
// the pipelined kernel's arguments with mrows filled in, and that row count
LadderArgs ladder_prepared(const LadderArgs &a);
int ladder_rows_max(const LadderArgs &a);
// the pipelined kernel is used from this many rows in the largest momentum class on
constexpr int kPipeMinRows = 128;
template <typename T>
hipError_t launch_ladder_group(const LadderGroup &g, int nblocks, hipStream_t s);
// real flops the ladder kernel executes (tile padding and LDS rebuild included)
double ladder_executed_flops(const LadderArgs &a, bool fp64);
// the same launch in real matrix-core flops (complex products formed from three real
// products count 6)
double ladder_mfma_flops(const LadderArgs &a, bool fp64);

}  // namespace lrcc
