// k-blocked contraction planner.  For a contraction C += alpha * A.B of
// momentum-conserving block tensors it enumerates the allowed crystal-momentum
// assignments (Eq. momentum: every two-electron block satisfies
// k_p + k_q = k_r + k_s, so only Nk^3 of Nk^4 blocks exist and each free
// k-sum of the paper's equations becomes a sum over segments), groups the
// result by output block, and describes the dense block products as one
// strided batched GEMM whose index groups read the blocks in place.
#include "plan.hpp"
#include "elem.hpp"

#include <algorithm>
#include <memory>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>

namespace lrcc {

bool g_dry_run = false;

namespace {
std::uintptr_t g_fake_next = 0x100000;
}

namespace {
struct ArenaState {
    char *base = nullptr;
    size_t size = 0, used = 0;
};
ArenaState g_arena;                                   // active arena (base null: none)
std::vector<std::pair<const char *, size_t>> g_arenas;   // every registered arena range
}

void arena_register(void *base, size_t size) { g_arenas.push_back({(const char *)base, size}); }
void arena_begin(void *base, size_t size) { g_arena = ArenaState{(char *)base, size, 0}; }
void arena_end() { g_arena = ArenaState{}; }
size_t arena_used() { return g_arena.used; }
bool arena_active() { return g_arena.base != nullptr; }
bool in_arena(const void *p) {
    for (const auto &a : g_arenas)
        if ((const char *)p >= a.first && (const char *)p < a.first + a.second) return true;
    return false;
}

double Program::tag_mfma_flops(int t) const {
    double f = 0;
    for (const auto &kv : gemm_ops) {
        if (kv.first >= tags.size() || tags[kv.first] != t) continue;
        const int sh = gemm_shape(*kv.second.args, kv.second.fp64);
        const bool g3 = !kv.second.fp64 && (sh == 3 || sh == 4);
        f += (double)kv.second.flops * (g3 ? 0.75 : 1.0);
    }
    return f;
}

void *dev_alloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (g_arena.base) {
        const size_t need = (bytes + 255) / 256 * 256;
        if (g_arena.used + need > g_arena.size)
            throw LrccError(4, "the work tensors need more than the " + std::to_string(g_arena.size) +
                                   "-byte static device array");
        void *p = g_arena.base + g_arena.used;
        g_arena.used += need;
        return p;
    }
    if (g_dry_run) {
        void *p = reinterpret_cast<void *>(g_fake_next);
        g_fake_next += (bytes + 4095) / 4096 * 4096 + 4096;
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        throw LrccError(4, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void dev_free(void *p) {
    if (!g_dry_run && p && !in_arena(p)) {
        hipError_t e = hipFree(p);
        (void)e;
    }
}

void *Program::alloc(size_t bytes) {
    void *p = dev_alloc(bytes);
    owned.push_back(p);
    return p;
}

Program::~Program() {
    drop_graphs();
    for (void *p : owned) dev_free(p);
}

void Program::drop_graphs() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
}

hipError_t Program::run_graph(hipStream_t s, const GraphKey &key) {
    auto it = graphs.find(key);
    if (it == graphs.end()) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t er = run(s, nullptr);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(s, &graph);
        if (er != hipSuccess) return er;
        if (e != hipSuccess) return e;
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        it = graphs.emplace(key, exec).first;
    }
    return hipGraphLaunch(it->second, s);
}

hipError_t Program::run_range(hipStream_t s, size_t begin, size_t end) {
    for (size_t i = begin; i < end && i < ops.size(); ++i) {
        hipError_t e = ops[i](s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t Program::run(hipStream_t s, Profiler *prof) {
    tags.resize(ops.size(), TAG_NONE);
    const bool timed = prof && prof->on;
    hipEvent_t p0 = nullptr, p1 = nullptr;
    if (timed) {
        p0 = prof->ev();
        p1 = prof->ev();
        hipError_t e = hipEventRecord(p0, s);
        if (e != hipSuccess) return e;
    }
    // LRCC_OP_TIMES: time every op of a profiled run and print one line per op
    static const bool per_op = std::getenv("LRCC_OP_TIMES") != nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> opev;
    if (timed && per_op) names.resize(ops.size());
    for (size_t i = 0; i < ops.size(); ++i) {
        hipEvent_t a = nullptr, b = nullptr;
        if (timed && per_op) {
            hipEvent_t x = prof->ev(), y = prof->ev();
            opev.push_back({x, y});
            (void)hipEventRecord(x, s);
            hipError_t e = ops[i](s);
            if (e != hipSuccess) return e;
            (void)hipEventRecord(y, s);
            if (tags[i] != TAG_NONE) prof->record(tags[i], x, y);   // the profile owns these two
            continue;
        }
        if (timed && tags[i] != TAG_NONE) {
            a = prof->ev();
            b = prof->ev();
            hipError_t e = hipEventRecord(a, s);
            if (e != hipSuccess) return e;
        }
        hipError_t e = ops[i](s);
        if (e != hipSuccess) return e;
        if (a) {
            e = hipEventRecord(b, s);
            if (e != hipSuccess) return e;
            prof->record(tags[i], a, b);
        }
    }
    if (timed) {
        hipError_t e = hipEventRecord(p1, s);
        if (e != hipSuccess) return e;
        prof->record(TAG_PROGRAM, p0, p1);
    }
    if (!opev.empty()) {
        (void)hipEventSynchronize(opev.back().second);
        for (size_t i = 0; i < opev.size(); ++i) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, opev[i].first, opev[i].second);
            std::fprintf(stderr, "[lrcc-op] %4zu %10.3f ms  %s\n", i, ms, names[i].c_str());
            if (tags[i] != TAG_NONE) continue;
            prof->pool.push_back(opev[i].first);
            prof->pool.push_back(opev[i].second);
        }
    }
    return hipSuccess;
}

void Program::apply(const std::vector<int> &choice) {
    for (size_t i = 0; i < tunables.size() && i < choice.size(); ++i)
        tunables[i].set(std::min(choice[i], tunables[i].ncand - 1));
    tuned = true;
}

hipError_t Program::autotune(hipStream_t s, std::vector<int> &choice) {
    const size_t nt = tunables.size();
    int maxc = 1;
    for (auto &tu : tunables) maxc = std::max(maxc, tu.ncand);
    std::vector<std::vector<float>> t(maxc, std::vector<float>(nt, 1e30f));
    std::vector<hipEvent_t> ev(2 * nt);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) return hipErrorUnknown;
    hipError_t err = hipSuccess;
    for (int cand = 0; cand < maxc && err == hipSuccess; ++cand) {
        for (auto &tu : tunables) tu.set(std::min(cand, tu.ncand - 1));
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {  // first run warms caches and code
            size_t k = 0;
            for (size_t i = 0; i < ops.size(); ++i) {
                const bool timed = k < nt && tunables[k].op == i;
                if (timed) (void)hipEventRecord(ev[2 * k], s);
                err = ops[i](s);
                if (err != hipSuccess) break;
                if (timed) { (void)hipEventRecord(ev[2 * k + 1], s); ++k; }
            }
            if (err == hipSuccess) err = hipStreamSynchronize(s);
            if (rep == 1 && err == hipSuccess)
                for (size_t k2 = 0; k2 < nt; ++k2) {
                    float ms = 0;
                    if (hipEventElapsedTime(&ms, ev[2 * k2], ev[2 * k2 + 1]) == hipSuccess) t[cand][k2] = ms;
                }
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    choice.assign(nt, 0);
    for (size_t k = 0; k < nt; ++k)
        for (int cnd = 1; cnd < tunables[k].ncand; ++cnd)
            if (t[cnd][k] < t[choice[k]][k]) choice[k] = cnd;
    if (std::getenv("LRCC_VERBOSE"))
        for (size_t k = 0; k < nt; ++k) {
            const size_t op = tunables[k].op;
            std::fprintf(stderr, "[lrcc] autotune op %zu (%s):", op, op < names.size() ? names[op].c_str() : "");
            for (int cnd = 0; cnd < tunables[k].ncand; ++cnd) std::fprintf(stderr, " %.3f", t[cnd][k]);
            std::fprintf(stderr, " ms -> %d\n", choice[k]);
        }
    apply(choice);
    return err;
}

hipEvent_t Profiler::ev() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) throw LrccError(5, "hipEventCreate failed");
    return e;
}

void Profiler::read(double *ms, long long *cnt) {
    for (int t = 0; t < NTAGS; ++t) { ms[t] = 0; cnt[t] = 0; }
    for (auto &m : marks) {
        float x = 0;
        if (hipEventSynchronize(m.second.second) != hipSuccess ||
            hipEventElapsedTime(&x, m.second.first, m.second.second) != hipSuccess)
            throw LrccError(5, "event timing failed");
        ms[m.first] += x;
        cnt[m.first] += 1;
        pool.push_back(m.second.first);
        pool.push_back(m.second.second);
    }
    marks.clear();
}

Profiler::~Profiler() {
    for (auto &m : marks) { pool.push_back(m.second.first); pool.push_back(m.second.second); }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

namespace {

struct TInfo {
    const KT *t;
    std::string lab;
    bool hasR;
    std::vector<i64> stride;   // per label position
    std::vector<int> extent;
};

TInfo info(const KT &t, const std::string &lab) {
    TInfo r;
    r.t = &t;
    r.lab = lab;
    r.hasR = !lab.empty() && lab[0] == 'R';
    const int nl = (int)lab.size();
    if (r.hasR != (t.nR > 0)) throw LrccError(1, "label/rhs mismatch for tensor labels " + lab);
    if (nl - (r.hasR ? 1 : 0) != t.nidx()) throw LrccError(1, "label count mismatch: " + lab);
    r.extent.resize(nl);
    for (int p = 0; p < nl; ++p) r.extent[p] = (r.hasR && p == 0) ? t.nR : t.ext(p - (r.hasR ? 1 : 0));
    r.stride.assign(nl, 1);
    for (int p = nl - 2; p >= 0; --p) r.stride[p] = r.stride[p + 1] * r.extent[p + 1];
    return r;
}

int pos(const TInfo &t, char c) {
    size_t p = t.lab.find(c);
    return p == std::string::npos ? -1 : (int)p;
}

// Split the label set into maximal runs adjacent (same order) in both tensors,
// ordered by position in `q`.
std::vector<std::vector<char>> chains(std::vector<char> set, const TInfo &p, const TInfo &q) {
    std::sort(set.begin(), set.end(), [&](char a, char b) { return pos(q, a) < pos(q, b); });
    std::vector<std::vector<char>> out;
    for (char c : set) {
        if (!out.empty()) {
            char prev = out.back().back();
            if (pos(q, c) == pos(q, prev) + 1 && pos(p, c) == pos(p, prev) + 1) {
                out.back().push_back(c);
                continue;
            }
        }
        out.push_back({c});
    }
    return out;
}

// Order index groups by decreasing stride in the operand x (read from HBM), so
// that its smallest-stride group is the innermost level of the GEMM index.
std::vector<std::vector<char>> by_stride(std::vector<std::vector<char>> ch, const TInfo &x) {
    std::stable_sort(ch.begin(), ch.end(), [&](const std::vector<char> &a, const std::vector<char> &b) {
        return x.stride[pos(x, a.back())] > x.stride[pos(x, b.back())];
    });
    return ch;
}

void make_split(const std::vector<std::vector<char>> &ch, const TInfo &x, const TInfo &y, Split &sp,
                Strides &sx, Strides &sy, int &total, const std::string &what) {
    if (ch.size() > 3) throw LrccError(1, "contraction needs more than 3 index groups in " + what);
    std::vector<int> ext;
    std::vector<i64> stx, sty;
    for (auto &c : ch) {
        int e = 1;
        for (char l : c) e *= x.extent[pos(x, l)];
        ext.push_back(e);
        stx.push_back(x.stride[pos(x, c.back())]);
        sty.push_back(y.stride[pos(y, c.back())]);
    }
    while (ext.size() < 3) {
        ext.insert(ext.begin(), 1);
        stx.insert(stx.begin(), 0);
        sty.insert(sty.begin(), 0);
    }
    sp.d1 = ext[1];
    sp.d2 = ext[2];
    total = ext[0] * ext[1] * ext[2];
    for (int i = 0; i < 3; ++i) { sx.s[i] = stx[i]; sy.s[i] = sty[i]; }
}

// block index of tensor t for per-label momenta; -1 if the momenta violate t's rule
i64 block_of(const TInfo &t, const std::map<char, int> &k) {
    const KT &T = *t.t;
    const int nk = T.nk;
    const int off = t.hasR ? 1 : 0;
    std::vector<int> ks;
    for (int d = 0; d < T.nidx(); ++d) ks.push_back(k.at(t.lab[off + d]));
    if (T.nidx() == 2) {
        if (ks[0] != ks[1]) return -1;
        return ks[0];
    }
    // the fourth momentum implied by the first three must be the given one
    const int k3 = T.km.sum3(-T.sg[3] * T.sg[0], ks[0], -T.sg[3] * T.sg[1], ks[1], -T.sg[3] * T.sg[2], ks[2]);
    if (k3 != ks[3]) return -1;
    return ((i64)ks[0] * nk + ks[1]) * nk + ks[2];
}

}  // namespace

namespace {
// largest offset a split forms (strides are non-negative; a triangle split of n reaches the pair
// (n-2, n-1))
i64 max_off(int total, Split sp, Strides st) {
    if (total <= 0) return 0;
    const int e0 = total / (sp.d1 * sp.d2);
    const int m1 = sp.tri ? sp.tri - 2 : sp.d1 - 1, m2 = sp.tri ? sp.tri - 1 : sp.d2 - 1;
    return (i64)(e0 - 1) * st.s[0] + (i64)m1 * st.s[1] + (i64)m2 * st.s[2];
}

// A triangle split must visit every pair p < q of its n x n block exactly once (checked once per n).
void check_tri(const Split &sp) {
    if (!sp.tri) return;
    static std::set<int> ok;
    if (ok.count(sp.tri)) return;
    const int n = sp.tri;
    if (n < 2 || sp.d1 * sp.d2 != n * (n - 1) / 2) throw LrccError(1, "bad triangle split");
    std::vector<char> seen((size_t)n * n, 0);
    for (int r = 0; r < sp.d1; ++r)
        for (int c = 0; c < sp.d2; ++c) {
            int p, q;
            tri_pair(r, c, n, p, q);
            if (!(0 <= p && p < q && q < n) || seen[(size_t)p * n + q]++) throw LrccError(1, "bad triangle split");
        }
    ok.insert(n);
}
}  // namespace

template <typename T>
void raw_gemm(Program &P, GemmArgs g, const std::vector<i64> &offC, const std::vector<int> &segBeg,
              const std::vector<i64> &segA, const std::vector<i64> &segB, i64 sizeA, i64 sizeB, i64 sizeC,
              const std::vector<float> &jscale) {
    g.njobs = (int)offC.size();
    if (g.njobs == 0) return;
    if (!jscale.empty() && jscale.size() != offC.size()) throw LrccError(1, "per-job scale list of the wrong length");
    // every address formed by the kernel stays inside the operands
    if (g.M <= 0 || g.N <= 0) return;                // no outputs
    if (g.M % (g.sm.d1 * g.sm.d2) || g.N % (g.sn.d1 * g.sn.d2) || g.K % (g.sk.d1 * g.sk.d2))
        throw LrccError(1, "GEMM split does not divide its dimension");
    check_tri(g.sm);
    check_tri(g.sn);
    check_tri(g.sk);
    for (const Strides *st : {&g.Am, &g.Ak, &g.Bk, &g.Bn, &g.Cm, &g.Cn})
        for (int i = 0; i < 3; ++i)
            if (st->s[i] < 0) throw LrccError(1, "negative GEMM stride");
    const i64 mA = max_off(g.M, g.sm, g.Am) + max_off(g.K, g.sk, g.Ak);
    const i64 mB = max_off(g.K, g.sk, g.Bk) + max_off(g.N, g.sn, g.Bn);
    const i64 mC = max_off(g.M, g.sm, g.Cm) + max_off(g.N, g.sn, g.Cn);
    if (mA >= (i64)INT32_MAX || mB >= (i64)INT32_MAX)
        throw LrccError(1, "GEMM operand block offsets exceed 32 bits");
    if ((int)segBeg.size() != g.njobs + 1 || segBeg.back() != (int)segA.size() || segA.size() != segB.size())
        throw LrccError(1, "inconsistent GEMM job lists");
    for (size_t s = 0; s < segA.size(); ++s)
        if (segA[s] < 0 || segA[s] + mA >= sizeA || segB[s] < 0 || segB[s] + mB >= sizeB)
            throw LrccError(1, "GEMM operand access out of bounds");
    for (i64 o : offC)
        if (o < 0 || o + mC >= sizeC) throw LrccError(1, "GEMM output access out of bounds");
    i64 *dOff = (i64 *)P.alloc(offC.size() * sizeof(i64));
    int *dBeg = (int *)P.alloc(segBeg.size() * sizeof(int));
    i64 *dA = (i64 *)P.alloc(std::max<size_t>(1, segA.size()) * sizeof(i64));
    i64 *dB = (i64 *)P.alloc(std::max<size_t>(1, segB.size()) * sizeof(i64));
    if (!g_dry_run) {
        bool ok = hipMemcpy(dOff, offC.data(), offC.size() * sizeof(i64), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(dBeg, segBeg.data(), segBeg.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
        if (!segA.empty())
            ok = ok && hipMemcpy(dA, segA.data(), segA.size() * sizeof(i64), hipMemcpyHostToDevice) == hipSuccess;
        if (!segB.empty())
            ok = ok && hipMemcpy(dB, segB.data(), segB.size() * sizeof(i64), hipMemcpyHostToDevice) == hipSuccess;
        if (!ok) throw LrccError(5, "upload of GEMM job lists failed");
    }
    g.jscale = nullptr;
    if (!jscale.empty()) {
        float *dS = (float *)P.alloc(jscale.size() * sizeof(float));
        if (!g_dry_run && hipMemcpy(dS, jscale.data(), jscale.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            throw LrccError(5, "upload of GEMM job scales failed");
        g.jscale = dS;
    }
    g.offC = dOff;
    g.segBeg = dBeg;
    g.segA = dA;
    g.segB = dB;
    g.njobs_all = g.njobs;
    g.job0 = 0;
    g.sm = split_magic(g.sm);
    g.sn = split_magic(g.sn);
    g.sk = split_magic(g.sk);
    g.alt = 0;
    // split-K when the job x tile grid cannot fill the chip but the jobs have long reductions
    {
        const i64 tn = g.M <= 16 ? (g.N + 255) / 256 : (g.N + 63) / 64;
        const i64 tiles = (i64)g.njobs * ((g.M + 63) / 64) * tn;
        const i64 steps = (i64)segA.size() * ((g.K + 15) / 16) / g.njobs;  // average per job
        i64 ks = 1;
        if (tiles < 1024 && steps >= 64) {
            ks = std::min<i64>({(2048 + tiles - 1) / tiles, steps / 16, (i64)256});
            while (ks > 1 && ks * g.njobs * (i64)g.M * g.N * (i64)sizeof(T) * 2 > ((i64)256 << 20)) ks /= 2;
        }
        g.ksplit = (int)std::max<i64>(1, ks);
        g.part = g.ksplit > 1 ? P.alloc((size_t)g.ksplit * g.njobs * g.M * g.N * sizeof(T) * 2) : nullptr;
    }
    P.last_flops = 8LL * g.M * g.N * g.K * (i64)segA.size();
    P.flops += P.last_flops;
    auto gp = std::make_shared<GemmArgs>(g);
    P.ops.push_back([gp](hipStream_t s) { return launch_gemm<T>(*gp, s); });
    P.gemm_ops[P.ops.size() - 1] = Program::GemmOp{gp, sizeof(T) == 8, P.last_flops};
    // candidates: tile shapes, the heuristic one first
    const std::vector<int> cand = gemm_candidates(g, sizeof(T) == 8);
    P.tunables.push_back({P.ops.size() - 1, (int)cand.size(), [gp, cand](int c) { gp->shape = c == 0 ? -1 : cand[c]; }});
}

// momenta of every label of C's block cb (the fourth from C's conservation rule)
void job_momenta(const KT &C, const TInfo &tc, const std::string &cl, i64 cb, std::map<char, int> &k) {
    const int nk = C.nk, off = tc.hasR ? 1 : 0;
    if (C.nidx() == 2) {
        k[cl[off]] = (int)cb;
        k[cl[off + 1]] = (int)cb;
        return;
    }
    const int k0 = (int)(cb / (nk * nk)), k1 = (int)((cb / nk) % nk), k2 = (int)(cb % nk);
    k[cl[off]] = k0;
    k[cl[off + 1]] = k1;
    k[cl[off + 2]] = k2;
    k[cl[off + 3]] = C.km.sum3(-C.sg[3] * C.sg[0], k0, -C.sg[3] * C.sg[1], k1, -C.sg[3] * C.sg[2], k2);
}

// contract() over unique antisymmetric pairs: one launch per combination of diagonal /
// off-diagonal momentum blocks of the packed pairs (their index groups then differ in size)
template <typename T>
void contract_packed(Program &P, const KT &C, const std::string &cl, const KT &A, const std::string &al,
                     const KT &B, const std::string &bl, std::complex<double> alpha, bool accumulate,
                     const std::string &pack, const std::string &exact, const GemmArgs &g0, const TInfo &ta,
                     const TInfo &tb, const TInfo &tc,
                     const std::vector<char> &Ml, const std::vector<char> &Nl, const std::vector<char> &Kl,
                     const std::vector<char> &sum_k, const std::string &what) {
    struct Pair {
        char p, q;
        int grp;   // 0: M (C and A), 1: N (C and B), 2: K (A and B)
    };
    std::vector<Pair> pk;
    if (pack.size() % 2) throw LrccError(1, "pack needs label pairs: " + what);
    auto has = [](const std::vector<char> &v, char c) { return std::find(v.begin(), v.end(), c) != v.end(); };
    for (size_t i = 0; i < pack.size(); i += 2) {
        const char p = pack[i], q = pack[i + 1];
        int grp = -1;
        if (has(Ml, p) && has(Ml, q)) grp = 0;
        else if (has(Nl, p) && has(Nl, q)) grp = 1;
        else if (has(Kl, p) && has(Kl, q)) grp = 2;
        if (grp < 0) throw LrccError(1, std::string("packed pair ") + p + q + " not in one index group: " + what);
        for (const Pair &o : pk)
            if (o.grp == grp) throw LrccError(1, "two packed pairs in one index group: " + what);
        pk.push_back({p, q, grp});
    }
    // the triangle form of a group holding a pair: (others, p, q), the other labels forming one run
    // adjacent (same order) in both tensors, so that they index as one level
    auto tri_group = [&](const Pair &pr, const std::vector<char> &labels, const TInfo &x, const TInfo &y, Split &sp,
                         Strides &sx, Strides &sy, int &total) {
        std::vector<char> rest;
        for (char c : labels)
            if (c != pr.p && c != pr.q) rest.push_back(c);
        std::sort(rest.begin(), rest.end(), [&](char a, char b) { return pos(x, a) < pos(x, b); });
        for (size_t i = 1; i < rest.size(); ++i)
            if (pos(x, rest[i]) != pos(x, rest[i - 1]) + 1 || pos(y, rest[i]) != pos(y, rest[i - 1]) + 1)
                throw LrccError(1, "packed pair whose other labels are not one adjacent run: " + what);
        const int n = x.extent[pos(x, pr.p)];
        if (x.extent[pos(x, pr.q)] != n || n < 2) throw LrccError(1, "packed pair of unequal or short extents: " + what);
        sp = tri_split(n);
        int ext = 1;
        for (char c : rest) ext *= x.extent[pos(x, c)];
        const i64 rx = rest.empty() ? 0 : x.stride[pos(x, rest.back())], ry = rest.empty() ? 0 : y.stride[pos(y, rest.back())];
        sx = Strides{{rx, x.stride[pos(x, pr.p)], x.stride[pos(x, pr.q)]}};
        sy = Strides{{ry, y.stride[pos(y, pr.p)], y.stride[pos(y, pr.q)]}};
        total = ext * (n * (n - 1) / 2);
    };
    const int np = (int)pk.size(), nk = C.nk;
    i64 nsum = 1;
    for (size_t i = 0; i < sum_k.size(); ++i) nsum *= nk;
    // jobs and segments per variant (bit i set: pair i on its diagonal momentum blocks)
    std::vector<std::vector<i64>> offC(1 << np), segA(1 << np), segB(1 << np);
    std::vector<std::vector<int>> segBeg(1 << np, std::vector<int>{0});
    for (i64 cb = 0; cb < C.nblocks(); ++cb) {
        std::map<char, int> k;
        job_momenta(C, tc, cl, cb, k);
        int jbits = 0;
        bool skip = false;
        for (int i = 0; i < np; ++i) {
            if (pk[i].grp == 2) continue;
            const int kp = k.at(pk[i].p), kq = k.at(pk[i].q);
            if (kp > kq) skip = true;
            if (kp == kq) jbits |= 1 << i;
        }
        if (skip) continue;
        std::vector<size_t> before(1 << np);
        for (int m = 0; m < (1 << np); ++m) before[m] = segA[m].size();
        for (i64 sidx = 0; sidx < nsum; ++sidx) {
            i64 q = sidx;
            for (char c : sum_k) { k[c] = (int)(q % nk); q /= nk; }
            const i64 ba = block_of(ta, k), bb = block_of(tb, k);
            if (ba < 0 || bb < 0) continue;
            int bits = jbits;
            bool sk = false;
            for (int i = 0; i < np; ++i) {
                if (pk[i].grp != 2) continue;
                const int kp = k.at(pk[i].p), kq = k.at(pk[i].q);
                if (kp > kq) sk = true;
                if (kp == kq) bits |= 1 << i;
            }
            if (sk) continue;
            segA[bits].push_back(ba * A.inner());
            segB[bits].push_back(bb * B.inner());
        }
        for (int m = 0; m < (1 << np); ++m) {
            if (segA[m].size() == before[m]) continue;
            offC[m].push_back(cb * C.inner());
            segBeg[m].push_back((int)segA[m].size());
        }
    }
    if (!accumulate) {
        // the packed launches write C in parts: clear it once, then accumulate
        void *cp = C.p;
        const i64 n = C.count();
        P.ops.push_back([cp, n](hipStream_t s) { return zero_fill<T>(cp, n, s); });
    }
    for (int m = 0; m < (1 << np); ++m) {
        if (offC[m].empty()) continue;
        // a pair over a single index has no p < q: its diagonal blocks contribute nothing
        bool empty = false;
        for (int i = 0; i < np; ++i) {
            const TInfo &x = pk[i].grp == 1 ? tb : ta;
            if ((m >> i & 1) && x.extent[pos(x, pk[i].p)] < 2) empty = true;
        }
        if (empty) continue;
        GemmArgs g = g0;
        g.beta = 1;
        double f = 1;
        for (const Pair &pr : pk)
            if (pr.grp == 2 || exact.find(pr.p) == std::string::npos) f *= 2;
        g.alpha_re = alpha.real() * f;
        g.alpha_im = alpha.imag() * f;
        for (int i = 0; i < np; ++i) {
            if (!(m >> i & 1)) continue;
            if (pk[i].grp == 0) tri_group(pk[i], Ml, ta, tc, g.sm, g.Am, g.Cm, g.M);
            else if (pk[i].grp == 1) tri_group(pk[i], Nl, tb, tc, g.sn, g.Bn, g.Cn, g.N);
            else tri_group(pk[i], Kl, ta, tb, g.sk, g.Ak, g.Bk, g.K);
        }
        g.aMfast = (g.Am.s[2] == 1) || (g.Ak.s[2] != 1);
        g.bNfast = (g.Bn.s[2] == 1) || (g.Bk.s[2] != 1);
        raw_gemm<T>(P, g, offC[m], segBeg[m], segA[m], segB[m], A.count(), B.count(), C.count());
        char nm[200];
        std::snprintf(nm, sizeof nm, "gemm %s packed %s (diagonal mask %d) M=%d N=%d K=%d jobs=%zu segs=%zu",
                      what.c_str(), pack.c_str(), m, g.M, g.N, g.K, offC[m].size(), segA[m].size());
        P.name_last(nm);
    }
}

template <typename T>
void contract(Program &P, const KT &C, const std::string &cl, const KT &A, const std::string &al, const KT &B,
              const std::string &bl, std::complex<double> alpha, bool accumulate, const std::string &pack,
              const std::string &exact) {
    // the GEMM stores run along its N index: put the output's unit-stride index there
    // (operand order does not change a complex product)
    if (al.find(cl.back()) != std::string::npos && bl.find(cl.back()) == std::string::npos) {
        contract<T>(P, C, cl, B, bl, A, al, alpha, accumulate, pack, exact);
        return;
    }
    TInfo tc = info(C, cl), ta = info(A, al), tb = info(B, bl);
    const std::string what = cl + " <- " + al + " * " + bl;
    std::vector<char> Ml, Nl, Kl, free_k, sum_k;
    std::string all = cl + al + bl;
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    for (char c : all) {
        const bool inC = pos(tc, c) >= 0, inA = pos(ta, c) >= 0, inB = pos(tb, c) >= 0;
        if (inC && inA && !inB) Ml.push_back(c);
        else if (inC && inB && !inA) Nl.push_back(c);
        else if (inA && inB && !inC) Kl.push_back(c);
        else throw LrccError(1, std::string("label '") + c + "' must appear in exactly two operands: " + what);
        if (c != 'R') (inC ? free_k : sum_k).push_back(c);
    }
    GemmArgs g{};
    g.shape = -1;
    g.A = A.p;
    g.B = B.p;
    g.C = C.p;
    make_split(by_stride(chains(Ml, ta, tc), ta), ta, tc, g.sm, g.Am, g.Cm, g.M, what);
    {
        // N groups by decreasing stride in B, or in C when the reduction is short (the output
        // traffic then dominates and the small operand B stays in cache)
        i64 kext = 1;
        for (char c : Kl) kext *= ta.extent[pos(ta, c)];
        for (size_t i = 0; i < sum_k.size(); ++i) kext *= C.nk;
        make_split(by_stride(chains(Nl, tb, tc), kext <= 64 && !tb.hasR ? tc : tb), tb, tc, g.sn, g.Bn, g.Cn, g.N, what);
    }
    {
        // K: make the unit-stride group innermost for whichever operand has one (A first)
        auto kc = chains(Kl, tb, ta);
        bool a_unit = false;
        for (auto &c : kc) a_unit = a_unit || ta.stride[pos(ta, c.back())] == 1;
        make_split(a_unit ? by_stride(kc, ta) : by_stride(kc, tb), ta, tb, g.sk, g.Ak, g.Bk, g.K, what);
    }
    g.aMfast = (g.Am.s[2] == 1) || (g.Ak.s[2] != 1);
    g.bNfast = (g.Bn.s[2] == 1) || (g.Bk.s[2] != 1);
    g.alpha_re = alpha.real();
    g.alpha_im = alpha.imag();
    g.beta = accumulate ? 1 : 0;
    if (!pack.empty()) {
        contract_packed<T>(P, C, cl, A, al, B, bl, alpha, accumulate, pack, exact, g, ta, tb, tc, Ml, Nl, Kl, sum_k,
                           what);
        return;
    }

    const int nk = C.nk;
    std::vector<i64> offC, segA, segB;
    std::vector<int> segBeg{0};
    const i64 nblkC = C.nblocks();
    i64 nsum = 1;
    for (size_t i = 0; i < sum_k.size(); ++i) nsum *= nk;
    for (i64 cb = 0; cb < nblkC; ++cb) {
        std::map<char, int> k;
        const int off = tc.hasR ? 1 : 0;
        if (C.nidx() == 2) {
            k[cl[off]] = (int)cb;
            k[cl[off + 1]] = (int)cb;
        } else {
            int k0 = (int)(cb / (nk * nk)), k1 = (int)((cb / nk) % nk), k2 = (int)(cb % nk);
            k[cl[off]] = k0;
            k[cl[off + 1]] = k1;
            k[cl[off + 2]] = k2;
            k[cl[off + 3]] = C.km.sum3(-C.sg[3] * C.sg[0], k0, -C.sg[3] * C.sg[1], k1, -C.sg[3] * C.sg[2], k2);
        }
        const size_t before = segA.size();
        for (i64 sidx = 0; sidx < nsum; ++sidx) {
            i64 q = sidx;
            for (char c : sum_k) { k[c] = (int)(q % nk); q /= nk; }
            const i64 ba = block_of(ta, k), bb = block_of(tb, k);
            if (ba < 0 || bb < 0) continue;
            segA.push_back(ba * A.inner());
            segB.push_back(bb * B.inner());
        }
        if (segA.size() == before && accumulate) continue;  // nothing to add to this block
        offC.push_back(cb * C.inner());
        segBeg.push_back((int)segA.size());
    }
    if (std::getenv("LRCC_PLAN_DUMP")) {
        const double pad = 8.0 * ((g.M + 63) / 64 * 64.0) * ((g.N + 63) / 64 * 64.0) * ((g.K + 15) / 16 * 16.0) * segA.size();
        std::fprintf(stderr, "gemm %-28s M=%-7d N=%-7d K=%-6d jobs=%-5zu segs=%-6zu alg=%.3e padded=%.3e\n",
                     what.c_str(), g.M, g.N, g.K, offC.size(), segA.size(), 8.0 * g.M * g.N * g.K * segA.size(), pad);
    }
    raw_gemm<T>(P, g, offC, segBeg, segA, segB, A.count(), B.count(), C.count());
    char nm[160];
    std::snprintf(nm, sizeof nm, "gemm %s M=%d N=%d K=%d jobs=%zu segs=%zu", what.c_str(), g.M, g.N, g.K,
                  offC.size(), segA.size());
    P.name_last(nm);
}

template void contract<double>(Program &, const KT &, const std::string &, const KT &, const std::string &,
                               const KT &, const std::string &, std::complex<double>, bool, const std::string &,
                               const std::string &);
template void contract<float>(Program &, const KT &, const std::string &, const KT &, const std::string &,
                              const KT &, const std::string &, std::complex<double>, bool, const std::string &,
                              const std::string &);
template void raw_gemm<double>(Program &, GemmArgs, const std::vector<i64> &, const std::vector<int> &,
                               const std::vector<i64> &, const std::vector<i64> &, i64, i64, i64,
                               const std::vector<float> &);
template void raw_gemm<float>(Program &, GemmArgs, const std::vector<i64> &, const std::vector<int> &,
                              const std::vector<i64> &, const std::vector<i64> &, i64, i64, i64,
                              const std::vector<float> &);

}  // namespace lrcc
