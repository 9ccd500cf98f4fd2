// Host-side planner: k-blocked tensors and their contractions as GEMM job lists.
#pragma once
#include <array>
#include <complex>
#include <functional>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "common.hpp"

namespace lrcc {

// A momentum-conserving tensor stored as dense blocks (Sec. II.A, Eq. momentum).
// Indices have class 'o' or 'v'.  Four-index tensors obey
// sg[0] k0 + sg[1] k1 + sg[2] k2 + sg[3] k3 = 0 on the k mesh km and are stored as
// [k0][k1][k2] blocks (k3 implied); two-index tensors are k-diagonal, [k0]
// blocks.  An optional right-hand-side axis of extent nR sits at the start of
// every block: block = [R][d0][d1]...  Elements are interleaved complex.
struct KT {
    void *p = nullptr;
    std::string cls;
    int sg[4] = {1, 1, -1, -1};
    int nR = 0;
    int nk = 0, no = 0, nv = 0;   // nk = km.size()
    KMesh km;
    int nidx() const { return (int)cls.size(); }
    int ext(int d) const { return cls[d] == 'o' ? no : nv; }
    i64 inner() const {
        i64 e = nR > 0 ? nR : 1;
        for (int d = 0; d < nidx(); ++d) e *= ext(d);
        return e;
    }
    i64 nblocks() const {
        i64 b = 1;
        for (int d = 0; d < nidx() - 1; ++d) b *= nk;
        return b;
    }
    i64 count() const { return inner() * nblocks(); }
};

struct LrccError : std::runtime_error {
    int code;
    LrccError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// Event timing of recorded launches: pairs of events recorded on the launch
// stream around every op with a given tag (and around whole program runs).
enum { TAG_NONE = 0, TAG_LADDER = 1, TAG_PROGRAM = 2, TAG_BUILD = 3, NTAGS = 4 };
struct Profiler {
    bool on = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    std::vector<hipEvent_t> pool;
    hipEvent_t ev();
    void record(int tag, hipEvent_t a, hipEvent_t b) { marks.push_back({tag, {a, b}}); }
    // sums (ms, count) per tag, recycles the events
    void read(double *ms, long long *cnt);
    ~Profiler();
};

// A tunable launch of a recorded program: the op index and a setter for its
// variant (candidate 0 or 1).
struct Tunable {
    size_t op;
    int ncand;                           // number of valid candidates
    std::function<void(int)> set;
};

// A recorded sequence of device launches plus the device memory it owns.
struct Program {
    std::vector<std::function<hipError_t(hipStream_t)>> ops;
    std::vector<int> tags;  // per op (TAG_NONE unless set by tag_last)
    std::vector<std::string> names;  // per op, for the per-op timing report
    void name_last(const std::string &n) {
        names.resize(ops.size());
        names.back() = n;
    }
    std::vector<Tunable> tunables;
    bool tuned = false;
    std::string tune_key;
    // Time every tunable op under each candidate (full program runs, so the
    // recomputed outputs stay valid) and keep the fastest per op.
    hipError_t autotune(hipStream_t s, std::vector<int> &choice);
    void apply(const std::vector<int> &choice);
    std::vector<void *> owned;
    i64 flops = 0;       // executed real flops of the recorded GEMMs and ladder
    i64 last_flops = 0;  // executed flops of the op recorded last
    i64 tag_flops[NTAGS] = {0, 0, 0, 0};
    void tag_last(int t) {
        tags.resize(ops.size(), TAG_NONE);
        tags.back() = t;
        tag_flops[t] += last_flops;
    }
    hipError_t run(hipStream_t s, Profiler *prof = nullptr);
    hipError_t run_range(hipStream_t s, size_t begin, size_t end);
    // the recorded GEMM launches (op index -> arguments as tuned, precision, executed flops)
    struct GemmOp {
        std::shared_ptr<GemmArgs> args;
        bool fp64;
        i64 flops;
    };
    std::map<size_t, GemmOp> gemm_ops;
    // real flops of the matrix-core instructions of the GEMM launches with tag t: 8 per complex
    // multiply-add formed, 6 for the tiles that form complex products from three real ones
    double tag_mfma_flops(int t) const;
    // ladder path of a sigma program: 1 integrals rebuilt in LDS, 2 stored blocks, 3 blocks built
    // one momentum class at a time (0: no ladder term)
    int ladder_path = 0;
    // the rebuild-in-LDS ladder launch of a sigma program (for multi-chain launches)
    std::shared_ptr<LadderArgs> ladder_args;
    size_t ladder_op = (size_t)-1;
    // Replay through a HIP graph captured on first use for this key (the
    // pointers the recorded launches read); `s` must not be the null stream.
    typedef std::array<const void *, 5> GraphKey;
    std::map<GraphKey, hipGraphExec_t> graphs;
    hipError_t run_graph(hipStream_t s, const GraphKey &key);
    void drop_graphs();
    void *alloc(size_t bytes);
    ~Program();
};

// C[cl] (+)= alpha * sum A[al] B[bl]; labels are one character per index, 'R'
// for the right-hand-side axis (first in a label string when present).
// pack: label pairs ("pq" per pair, at most one pair per GEMM index group) over which
// the launches run on unique pairs only: momentum blocks k_p <= k_q, and p < q inside the
// diagonal blocks k_p = k_q (triangle splits).  A summed pair must be antisymmetric in both
// operands (factor 2).  An output pair leaves C defined only on those unique pairs (the
// others are not written; with accumulate false C is zeroed first): with factor 2 for a
// consumer that antisymmetrises C in the pair, or with its true values when the pair's first
// label is in `exact`, for a consumer that reads C through the same packing.
template <typename T>
void contract(Program &P, const KT &C, const std::string &cl, const KT &A, const std::string &al, const KT &B,
              const std::string &bl, std::complex<double> alpha, bool accumulate = true,
              const std::string &pack = "", const std::string &exact = "");

// Raw strided GEMM with explicit job/segment lists (host vectors are uploaded).
// sizeA/B/C are the element counts of the operands: every address the GEMM can
// form is checked against them before the launch is recorded.
// jscale (optional, one per job) multiplies alpha job by job.
template <typename T>
void raw_gemm(Program &P, GemmArgs g, const std::vector<i64> &offC, const std::vector<int> &segBeg,
              const std::vector<i64> &segA, const std::vector<i64> &segB, i64 sizeA, i64 sizeB, i64 sizeC,
              const std::vector<float> &jscale = {});

// Placeholder-or-real device allocation honouring g_dry_run.
void *dev_alloc(size_t bytes);
void dev_free(void *p);

}  // namespace lrcc
