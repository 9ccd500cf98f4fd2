// Context, input validation, the amplitude-dependent Jacobian blocks and the
// sigma program (the CCSD Jacobian applied to perturbed amplitudes), plus the
// C ABI of include/lrcc.h.
//
// Internally everything is in supercell ("crystal") normalisation: the
// integrals are built from L/sqrt(Nk), and the paper-normalised T2, X2 (Nk
// times the crystal amplitudes, each free k-sum of Eqs. t1-tx2 carrying 1/Nk)
// are divided by Nk on entry and sigma2 multiplied by Nk on exit.  In this
// normalisation the k-blocked equations are the molecular spin-orbital ones
// restricted to momentum-allowed blocks (Sec. II.A: collective indices).
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <complex>
#include <cstring>
#include <array>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lrcc.h"
#include "common.hpp"
#include "elem.hpp"
#include "plan.hpp"
#include "solver.hpp"
#include "eig.hpp"
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <algorithm>

using namespace lrcc;
typedef std::complex<double> cd;

#define HIPCHK(x)                                                                                    \
    do {                                                                                             \
        hipError_t e_ = (x);                                                                         \
        if (e_ != hipSuccess) throw LrccError(LRCC_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

struct DevMem {
    std::vector<void *> ptrs;
    bool dry = false;
    void *get(size_t bytes) {
        dry = g_dry_run;
        void *p = dev_alloc(bytes);
        ptrs.push_back(p);
        return p;
    }
    void release() {
        if (!dry)
            for (void *p : ptrs) dev_free(p);   // (pieces of a static arena are not freed)
        ptrs.clear();
    }
    ~DevMem() { release(); }
};

// Amplitude-dependent state of one precision.
template <typename T>
struct State {
    DevMem mem;
    KT fov, t1, t2, tau;
    KT g_oovv, g_ooov, g_ovov, g_ovvv, g_ovoo;
    KT Fae, Fmi, Fme, Fbe, Fmj, Fg, Wp, Wbar, R, S, U, H, G2;
    void *La = nullptr, *Lb = nullptr;      // dressed virtual Cholesky slices (ladder)
    void *LaT = nullptr, *LbT = nullptr;    // pair-transposed copies (adjoint ladder)
    void *d_o1 = nullptr, *d_v1 = nullptr, *d_o2 = nullptr, *d_v2 = nullptr;  // preconditioner diagonals
    void *Wst = nullptr;                    // stored antisymmetrised ladder integrals (null: rebuild in LDS)
    bool ready = false;
};

}  // namespace

struct lrcc_ctx {
    int dev = 0;
    mutable std::string err;
    // bumped whenever recorded programs or the buffers they read are rebuilt (new Hamiltonian,
    // k mesh or amplitude-dependent state); groups of chains compare it to rebuild their tables
    unsigned long long gen = 0;
    int nk = 0, no = 0, nv = 0, naux = 0, n = 0;
    KMesh km;                                  // k mesh (a 1D chain unless set by lrcc_set_kmesh)
    bool km_set = false;
    bool ham = false, amp = false;
    DevMem hmem;          // Hamiltonian-level device memory (f64)
    void *fock = nullptr, *Ls = nullptr, *Lcs = nullptr;
    KT g_oooo, g_ooov, g_oovv, g_ovov, g_ovvo, g_ovvv, g_ovoo;
    State<double> s64;
    State<float> s32;
    // sigma programs keyed by (precision, nrhs)
    std::map<std::pair<int, int>, std::unique_ptr<Program>> progs;
    std::map<std::pair<int, int>, std::unique_ptr<DevMem>> progmem;
    // run-time bindings read by the recorded programs
    const void *io_x1 = nullptr, *io_x2 = nullptr;
    void *io_y1 = nullptr, *io_y2 = nullptr;
    const double *io_omega = nullptr;
    // host-API staging buffers
    DevMem stage;
    size_t stage_b1 = 0, stage_b2 = 0, stage_nrhs = 0;   // capacities of the staging buffers
    void *st_x1 = nullptr, *st_x2 = nullptr, *st_y1 = nullptr, *st_y2 = nullptr, *st_om = nullptr;
    // scratch of the vector-Jacobian product entry (grown on demand)
    DevMem vjpmem;
    i64 vjp_n1 = 0, vjp_n2 = 0;                // capacities (complex elements) of vj1/vw1 and vj2/vw2
    void *vj1 = nullptr, *vj2 = nullptr, *vw1 = nullptr, *vw2 = nullptr;
    Profiler prof;
    bool use_graphs = false;
    bool pack_ladder = true;                   // antisymmetry-packed forward ladder for large batches
    bool pack_pairs = true;                    // hole-hole products of the forward sigma on unique pairs
    int ladder_mode = 0;                       // 0: automatic (3 if one class of blocks fits, else 1);
                                               // 1: rebuild integrals in LDS; 2: stored integral blocks;
                                               // 3: blocks of one momentum class at a time, per sigma
    std::vector<int> wslot;                    // (ka, kb, ke) -> slot of the stored blocks, -1 if not stored
    int nwslot = 0;
    std::vector<int> wcls;                     // (ka, kb, ke) -> slot within its class ka + kb, -1 if none
    int ncls_slots = 0;                        // most slots of one class
    bool autotune = false;
    hipStream_t own_stream = nullptr;          // non-null stream for solver work (graph capture)
    std::unique_ptr<Program> pre64, pre32;     // amplitude-dependent blocks (f64) and their f32 copies
    // pre64 op ranges that form R_iabf and subtract it from H_abej: skipped by the lean
    // precompute, whose H lacks the R part (the lean sigma forms that term from x1 directly)
    std::vector<std::pair<size_t, size_t>> pre64_lean_skip;
    // pre64 op ranges of U_ianf and of the t2 term of W-bar (into its first-layout buffer pre64_Wraw):
    // both linear in t2 alone.  With lin_on, the lean precompute replaces them by B(T) + lin_eps B(y)
    // from the buffers linU_* / linW_* (filled at T once per F evaluation and at y per direction).
    std::pair<size_t, size_t> pre64_U{0, 0}, pre64_Wt{0, 0};
    void *pre64_Wraw = nullptr;
    i64 n_U = 0, n_Wraw = 0;
    void *linU_T = nullptr, *linU_y = nullptr, *linW_T = nullptr, *linW_y = nullptr, *lin_tmp = nullptr;
    bool lin_T_ready = false, lin_on = false;
    double lin_eps = 0;
    void *eps_o = nullptr, *eps_v = nullptr;   // diagonal of fock per k (preconditioner)
    DevMem solmem;                             // solver work vectors
    bool lam_valid = false;
    void *dip = nullptr;                       // [3][nk][n][n] device copy
    State<double> xs[3];                       // one-body perturbation operators (dipole axes)
    std::unique_ptr<Program> prex[3], prog_xi, prog_grad;
    DevMem amem;                               // alpha pipeline buffers
    void *lam1 = nullptr, *lam2 = nullptr, *xi1 = nullptr, *xi2 = nullptr, *gb1 = nullptr, *gb2 = nullptr;
    void *ybuf = nullptr, *ubuf = nullptr;     // E'' helper vectors [nk][o][v]
    std::unique_ptr<Program> prog_epp;
    // last polarizability solve
    int nfreq = 0, nrhs_sol = 0;
    std::vector<int> axes;
    std::vector<double> alpha;                 // [nfreq][3][3] complex
    DevMem solv;                               // solutions x of the last solve
    void *sol1 = nullptr, *sol2 = nullptr;
    size_t sol_bytes = 0;
    std::vector<double> last_omega;            // frequencies of the last solve
    // one-body densities of amplitude-space vectors (dipole gradients)
    DevMem gmem;
    KT dT1, dT2;                               // amplitudes the density programs read (crystal)
    std::map<int, std::unique_ptr<Program>> dens;
    std::map<int, std::unique_ptr<DevMem>> densmem;
    // initial guesses of the next lrcc_solve, keyed by (axis, ifreq, sign): device [n1 + n2] complex
    std::map<std::array<int, 3>, std::unique_ptr<DevMem>> guess;
};

static std::string g_create_err;

namespace {

KT make_kt(lrcc_ctx *c, const char *cls, void *p, int nR = 0, std::initializer_list<int> sg = {1, 1, -1, -1}) {
    KT t;
    t.p = p;
    t.cls = cls;
    t.nR = nR;
    t.nk = c->nk;
    t.km = c->km;
    t.no = c->no;
    t.nv = c->nv;
    int i = 0;
    for (int s : sg) t.sg[i++] = s;
    if (t.nidx() == 2) { t.sg[0] = 1; t.sg[1] = -1; }
    return t;
}

template <typename T>
KT alloc_kt(lrcc_ctx *c, DevMem &m, const char *cls, int nR = 0, std::initializer_list<int> sg = {1, 1, -1, -1}) {
    KT t = make_kt(c, cls, nullptr, nR, sg);
    t.p = m.get(t.count() * 2 * sizeof(T));
    return t;
}

// <pq||rs> = (pr|qs) - (ps|qr),  (pr|qs) = sum_Q Ls[kp][kr][Q][p][r] Lcs[kq][ks][Q][q][s]
// (Ls = L/sqrt(Nk), Lcs[k1][k2][Q][p][q] = conj(L[k2][k1][Q][q][p])/sqrt(Nk)), scaled by `scale`.
void build_eri(lrcc_ctx *c, Program &P, const KT &out, double scale) {
    const int nk = c->nk, n = c->n, naux = c->naux;
    auto off = [&](char cl) { return cl == 'o' ? 0 : c->no; };
    const i64 Lblk = (i64)naux * n * n;
    std::vector<i64> str(4);
    str[3] = 1;
    for (int d = 2; d >= 0; --d) str[d] = str[d + 1] * out.ext(d + 1);
    for (int pass = 0; pass < 2; ++pass) {
        // pass 0: Coulomb (pr|qs): M=(p,r) from Ls[kp][kr], N=(q,s) from Lcs[kq][ks]
        // pass 1: exchange -(ps|qr): M=(p,s) from Ls[kp][ks], N=(q,r) from Lcs[kq][kr]
        const int mi = pass == 0 ? 2 : 3, ni = pass == 0 ? 3 : 2;
        GemmArgs g{};
        g.shape = -1;
        g.A = c->Ls;
        g.B = c->Lcs;
        g.C = out.p;
        g.M = out.ext(0) * out.ext(mi);
        g.N = out.ext(1) * out.ext(ni);
        g.K = naux;
        g.sm = Split{out.ext(0), out.ext(mi)};
        g.Am = Strides{{0, n, 1}};
        g.Cm = Strides{{0, str[0], str[mi]}};
        g.sn = Split{out.ext(1), out.ext(ni)};
        g.Bn = Strides{{0, n, 1}};
        g.Cn = Strides{{0, str[1], str[ni]}};
        g.sk = Split{1, naux};
        g.Ak = Strides{{0, 0, (i64)n * n}};
        g.Bk = Strides{{0, 0, (i64)n * n}};
        g.aMfast = 1;
        g.bNfast = 1;
        g.alpha_re = pass == 0 ? scale : -scale;
        g.alpha_im = 0;
        g.beta = pass;
        std::vector<i64> offC, segA, segB;
        std::vector<int> beg{0};
        for (int k0 = 0; k0 < nk; ++k0)
            for (int k1 = 0; k1 < nk; ++k1)
                for (int k2 = 0; k2 < nk; ++k2) {
                    const int k3 = c->km.comb(k0, k1, k2);
                    const int km = pass == 0 ? k2 : k3, kn = pass == 0 ? k3 : k2;
                    offC.push_back((((i64)k0 * nk + k1) * nk + k2) * out.inner());
                    segA.push_back((i64)(k0 * nk + km) * Lblk + (i64)off(out.cls[0]) * n + off(out.cls[mi]));
                    segB.push_back((i64)(k1 * nk + kn) * Lblk + (i64)off(out.cls[1]) * n + off(out.cls[ni]));
                    beg.push_back((int)segA.size());
                }
        raw_gemm<double>(P, g, offC, beg, segA, segB, (i64)nk * nk * Lblk, (i64)nk * nk * Lblk, out.count());
    }
}

template <typename T>
void kt_copy(Program &P, const KT &dst, const KT &src) {
    void *d = dst.p;
    const void *s = src.p;
    size_t bytes = src.count() * 2 * sizeof(T);
    P.ops.push_back([=](hipStream_t st) { return hipMemcpyAsync(d, s, bytes, hipMemcpyDeviceToDevice, st); });
}

// Dressing of the virtual Cholesky slice for the ladder (t1-transformed integrals):
//   out[k1][k2][Q][a][e] -= sum_m t1[k1][m][a] src[k1][k2][Q][m][o+e]
// where out already holds src[k1][k2][Q][o+a][o+e].
void build_dressing(lrcc_ctx *c, Program &P, void *slice_src, void *out, const void *t1) {
    // slice_src: full scaled Cholesky array [nk][nk][naux][n][n]; out already holds the vv slice
    const int nk = c->nk, n = c->n, naux = c->naux, o = c->no, v = c->nv;
    GemmArgs g{};
        g.shape = -1;
    g.A = t1;
    g.B = slice_src;
    g.C = out;
    g.M = v;
    g.N = v;
    g.K = o;
    g.sm = Split{1, v};
    g.Am = Strides{{0, 0, 1}};
    g.Cm = Strides{{0, 0, v}};
    g.sk = Split{1, o};
    g.Ak = Strides{{0, 0, v}};
    g.Bk = Strides{{0, 0, n}};
    g.sn = Split{1, v};
    g.Bn = Strides{{0, 0, 1}};
    g.Cn = Strides{{0, 0, 1}};
    g.aMfast = 1;
    g.bNfast = 1;
    g.alpha_re = -1;
    g.beta = 1;
    std::vector<i64> offC, segA, segB;
    std::vector<int> beg{0};
    for (int k1 = 0; k1 < nk; ++k1)
        for (int k2 = 0; k2 < nk; ++k2)
            for (int q = 0; q < naux; ++q) {
                offC.push_back((((i64)k1 * nk + k2) * naux + q) * v * v);
                segA.push_back((i64)k1 * o * v);
                segB.push_back((((i64)k1 * nk + k2) * naux + q) * n * n + o);
                beg.push_back((int)segA.size());
            }
    raw_gemm<double>(P, g, offC, beg, segA, segB, (i64)nk * o * v, (i64)nk * nk * naux * n * n,
                     (i64)nk * nk * naux * v * v);
}

// Stored ladder integrals.  For the unique momentum pairs ka <= kb (output) and
// ke <= kf (input; kb, kf implied by ka + kb = ke + kf):
//   W'(ka,kb,ke)[e][f][a][b] = s (K(ka,ke,kb,kf)[a][e][b][f] - K(ka,kf,kb,ke)[a][f][b][e]),
//   K(k1,k2,k3,k4)[a][e][b][f] = sum_Q La[k1][k2][Q][a][e] Lb[k3][k4][Q][b][f],
// with s = 1/2 when ke == kf and 1 otherwise, so that for Y antisymmetric in
// (e,f) the ladder of every output block is sum over ke <= kf of Y(ke) W'.
// The blocks of one momentum class K = ka + kb (the outputs of the row pairs ki + kj = K)
// also get slots numbered within the class, for the class-at-a-time ladder (mode 3).
void ladder_slots(lrcc_ctx *c) {
    const int nk = c->nk;
    c->wslot.assign((size_t)nk * nk * nk, -1);
    c->wcls.assign((size_t)nk * nk * nk, -1);
    std::vector<int> per(nk, 0);
    int n = 0;
    for (int ka = 0; ka < nk; ++ka)
        for (int kb = ka; kb < nk; ++kb)
            for (int ke = 0; ke < nk; ++ke) {
                const int kf = c->km.comb(ka, kb, ke);
                if (ke > kf) continue;
                const size_t at = ((size_t)ka * nk + kb) * nk + ke;
                c->wslot[at] = n++;
                c->wcls[at] = per[c->km.sum3(1, ka, 1, kb, 0, 0)]++;
            }
    c->nwslot = n;
    c->ncls_slots = *std::max_element(per.begin(), per.end());
}

// Momentum class of a pair: k1 + k2.
static int kclass(const lrcc_ctx *c, int k1, int k2) { return c->km.sum3(1, k1, 1, k2, 0, 0); }

// Ladder path of a sigma program: 2 stored blocks (Wst set), 3 blocks built one momentum class at a
// time, 1 integrals rebuilt in LDS.  Mode 0 (automatic) takes 3 when one class of blocks of
// elem_bytes per element takes at most an eighth of the free device memory, else 1; inside the
// static array of the no-allocation entry point it takes 1 (the array is small).
static int ladder_path(lrcc_ctx *c, const void *Wst, size_t elem_bytes) {
    if (Wst) return 2;
    if (c->ladder_mode == 3) return 3;
    if (c->ladder_mode != 0 || arena_active()) return 1;
    if (g_dry_run) return 3;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return 1;
    const size_t v2 = (size_t)c->nv * c->nv;
    return (size_t)c->ncls_slots * v2 * v2 * elem_bytes <= fr / 8 ? 3 : 1;
}

// Slot of block (ka, kb, ke) in an integral-block array: the global slot (cls0 < 0), or, in the
// array of the momentum classes cls0, cls0 + 1, ... (ncls_slots blocks each), the slot within its
// class after those of the classes before it.
static i64 block_slot(const lrcc_ctx *c, int cls0, int ka, int kb, int ke) {
    const size_t at = ((size_t)ka * c->nk + kb) * c->nk + ke;
    if (cls0 < 0) return c->wslot[at];
    return c->wcls[at] < 0 ? -1 : (i64)(kclass(c, ka, kb) - cls0) * c->ncls_slots + c->wcls[at];
}
// whether momentum class k is in [cls0, cls0 + ncls) (every class for cls0 < 0)
static bool in_classes(int k, int cls0, int ncls) { return cls0 < 0 || (k >= cls0 && k < cls0 + ncls); }

// Momentum classes per batch of the class-built ladder (mode 3): as many as fit in an eighth of
// the free device memory, at most 2 GiB (one class at least; every sigma program holds its own).
static int class_batch(lrcc_ctx *c, size_t elem_bytes) {
    const size_t v2 = (size_t)c->nv * c->nv, per = (size_t)c->ncls_slots * v2 * v2 * elem_bytes;
    size_t fr = 0, tot = 0;
    if (g_dry_run) return std::min(c->nk, 2);      // plan checks: several batches, the last ragged
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return 1;
    const size_t budget = std::min(fr / 8, (size_t)2 << 30);
    return (int)std::max<size_t>(1, std::min<size_t>(c->nk, budget / std::max<size_t>(per, 1)));
}

// cls0 < 0: every unique block into its slot of W (nwslot blocks); cls0 >= 0: the blocks of the
// momentum classes cls0 .. cls0 + ncls - 1 into their slots of a class array (block_slot).
template <typename T>
void build_wstore(lrcc_ctx *c, Program &P, const void *La, const void *Lb, void *W, int cls0 = -1, int ncls = 0,
                  int tag = TAG_NONE) {
    const int nk = c->nk, v = c->nv, naux = c->naux;
    const i64 vv = (i64)v * v, v4 = vv * vv, lsz = (i64)nk * nk * naux * vv;
    for (int part = 0; part < 2; ++part) {
        GemmArgs g{};
        g.shape = -1;
        g.A = La;
        g.B = Lb;
        g.C = W;
        g.M = (int)vv;
        g.N = (int)vv;
        g.K = naux;
        g.sk = Split{1, naux};
        g.Ak = Strides{{0, 0, vv}};
        g.Bk = Strides{{0, 0, vv}};
        g.sm = Split{v, v};
        g.sn = Split{v, v};
        if (part == 0) {
            // rows (a, e), columns (f, b):  + La(ka,ke)[a][e] Lb(kb,kf)[b][f]
            g.Am = Strides{{0, v, 1}};
            g.Cm = Strides{{0, v, vv * v}};
            g.Bn = Strides{{0, 1, v}};
            g.Cn = Strides{{0, vv, 1}};
            g.alpha_re = 1.0;
            g.beta = 0;
        } else {
            // rows (a, f), columns (e, b):  - La(ka,kf)[a][f] Lb(kb,ke)[b][e]
            g.Am = Strides{{0, v, 1}};
            g.Cm = Strides{{0, v, vv}};
            g.Bn = Strides{{0, 1, v}};
            g.Cn = Strides{{0, vv * v, 1}};
            g.alpha_re = -1.0;
            g.beta = 1;
        }
        g.aMfast = 1;
        g.bNfast = 1;
        std::vector<i64> offC, segA, segB;
        std::vector<int> beg{0};
        std::vector<float> js;
        for (int ka = 0; ka < nk; ++ka)
            for (int kb = ka; kb < nk; ++kb)
                for (int ke = 0; ke < nk; ++ke) {
                    const int kf = c->km.comb(ka, kb, ke);
                    if (!in_classes(kclass(c, ka, kb), cls0, ncls)) continue;
                    const i64 sl = block_slot(c, cls0, ka, kb, ke);
                    if (sl < 0) continue;
                    offC.push_back(sl * v4);
                    const int k2 = part == 0 ? ke : kf, k4 = part == 0 ? kf : ke;
                    segA.push_back(((i64)ka * nk + k2) * naux * vv);
                    segB.push_back(((i64)kb * nk + k4) * naux * vv);
                    beg.push_back((int)segA.size());
                    js.push_back(ke == kf ? 0.5f : 1.0f);
                }
        raw_gemm<T>(P, g, offC, beg, segA, segB, lsz, lsz, (i64)(cls0 < 0 ? c->nwslot : ncls * c->ncls_slots) * v4, js);
        if (tag != TAG_NONE) P.tag_last(tag);
        P.name_last(part == 0 ? "ladder integrals (direct)" : "ladder integrals (exchange)");
    }
}

// Whether the ladder integrals are stored (ladder mode 2; the plan check covers
// that path too).  Mode 2 refuses blocks that would take more than half of the
// free device memory.
bool store_ladder(lrcc_ctx *c, size_t elem_bytes, size_t also) {
    if (g_dry_run) return c->ladder_mode != 3;
    if (c->ladder_mode != 2) return false;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return false;
    const size_t bytes = (size_t)c->nwslot * c->nv * c->nv * c->nv * c->nv * elem_bytes;
    if (bytes + also > fr / 2) throw LrccError(LRCC_E_OOM, "stored ladder integrals do not fit in device memory");
    return true;
}

template <typename T>
void convert_kt(Program &P, State<float> &dst_state, KT &dst, const KT &src, lrcc_ctx *c) {
    dst = src;
    dst.p = dst_state.mem.get(src.count() * 2 * sizeof(float));
    void *d = dst.p;
    const void *s = src.p;
    i64 n = src.count();
    P.ops.push_back([=](hipStream_t st) { return convert_f64_f32(s, d, n, st); });
}

// ---------------------------------------------------------------- precompute
// Allocate the amplitude-dependent state and record the programs that compute it
// from the device amplitudes (run again whenever the amplitudes change).
void build_state(lrcc_ctx *c) {
    const int nk = c->nk, o = c->no, v = c->nv, n = c->n, naux = c->naux;
    State<double> &S = c->s64;
    S.mem.release();
    c->s32.mem.release();
    S.ready = c->s32.ready = false;
    c->progs.clear();
    c->progmem.clear();
    ++c->gen;
    DevMem &m = S.mem;
    auto Pp = std::make_unique<Program>();
    Program &P = *Pp;

    S.t1 = alloc_kt<double>(c, m, "ov");
    S.t2 = alloc_kt<double>(c, m, "oovv");
    S.fov = alloc_kt<double>(c, m, "ov");
    KT foo = alloc_kt<double>(c, m, "oo"), fvv = alloc_kt<double>(c, m, "vv");
    void *fock = c->fock;
    {
        void *a = S.fov.p, *b = foo.p, *d = fvv.p;
        P.ops.push_back([=](hipStream_t s) { return one_body_slice<double>(fock, a, nk, n, 0, o, o, v, s); });
        P.ops.push_back([=](hipStream_t s) { return one_body_slice<double>(fock, b, nk, n, 0, o, 0, o, s); });
        P.ops.push_back([=](hipStream_t s) { return one_body_slice<double>(fock, d, nk, n, o, v, o, v, s); });
    }
    S.g_oovv = c->g_oovv; S.g_ooov = c->g_ooov; S.g_ovov = c->g_ovov; S.g_ovvv = c->g_ovvv; S.g_ovoo = c->g_ovoo;
    const KT &oovv = c->g_oovv, &ooov = c->g_ooov, &ovvv = c->g_ovvv, &ovvo = c->g_ovvo, &oooo = c->g_oooo;

    S.tau = alloc_kt<double>(c, m, "oovv");
    KT tt = alloc_kt<double>(c, m, "oovv");
    {
        void *t1p = S.t1.p, *t2p = S.t2.p, *tau = S.tau.p, *ttp = tt.p;
        const KMesh km = c->km;
        P.ops.push_back([=](hipStream_t s) { return tau_like<double>(t1p, t2p, t1p, tau, km, 1, o, v, 0.5, 0, s); });
        P.ops.push_back([=](hipStream_t s) { return tau_like<double>(t1p, t2p, t1p, ttp, km, 1, o, v, 0.25, 0, s); });
    }
    const KT &t1 = S.t1, &t2 = S.t2, &tau = S.tau;
    // F intermediates (full Fock matrix; the diagonal stays inside, Eq. D is only the preconditioner)
    S.Fae = alloc_kt<double>(c, m, "vv");
    kt_copy<double>(P, S.Fae, fvv);
    contract<double>(P, S.Fae, "ae", S.fov, "me", t1, "ma", -0.5);
    contract<double>(P, S.Fae, "ae", t1, "mf", ovvv, "mafe", 1.0);
    contract<double>(P, S.Fae, "ae", tt, "mnaf", oovv, "mnef", -0.5);
    S.Fmi = alloc_kt<double>(c, m, "oo");
    kt_copy<double>(P, S.Fmi, foo);
    contract<double>(P, S.Fmi, "mi", t1, "ie", S.fov, "me", 0.5);
    contract<double>(P, S.Fmi, "mi", t1, "ne", ooov, "mnie", 1.0);
    contract<double>(P, S.Fmi, "mi", tt, "inef", oovv, "mnef", 0.5);
    S.Fme = alloc_kt<double>(c, m, "ov");
    kt_copy<double>(P, S.Fme, S.fov);
    contract<double>(P, S.Fme, "me", t1, "nf", oovv, "mnef", 1.0);
    // Fg_me = sum_nf t_nf <mn||ef> (the t1 t1 part of the X-derivative of Fae and Fmi)
    S.Fg = alloc_kt<double>(c, m, "ov");
    contract<double>(P, S.Fg, "me", t1, "nf", oovv, "mnef", 1.0, false);
    S.Fbe = alloc_kt<double>(c, m, "vv");
    kt_copy<double>(P, S.Fbe, S.Fae);
    contract<double>(P, S.Fbe, "be", t1, "mb", S.Fme, "me", -0.5);
    S.Fmj = alloc_kt<double>(c, m, "oo");
    kt_copy<double>(P, S.Fmj, S.Fmi);
    contract<double>(P, S.Fmj, "mj", t1, "je", S.Fme, "me", 0.5);
    // W'_mnij = <mn||ij> + P(ij) t_je <mn||ie> + 1/2 tau_ijef <mn||ef>
    S.Wp = alloc_kt<double>(c, m, "oooo");
    kt_copy<double>(P, S.Wp, oooo);
    contract<double>(P, S.Wp, "mnij", t1, "je", ooov, "mnie", 1.0);
    contract<double>(P, S.Wp, "mnji", t1, "je", ooov, "mnie", -1.0);
    contract<double>(P, S.Wp, "mnij", tau, "ijef", oovv, "mnef", 0.5);
    // Wbar_mbej = <mb||ej> + t_jf <mb||ef> - t_nb <mn||ej> - (t_jnfb + t_jf t_nb) <mn||ef>
    S.Wbar = alloc_kt<double>(c, m, "ovvo");
    kt_copy<double>(P, S.Wbar, ovvo);
    contract<double>(P, S.Wbar, "mbej", t1, "jf", ovvv, "mbef", 1.0);
    contract<double>(P, S.Wbar, "mbej", t1, "nb", ooov, "mnje", 1.0);
    c->pre64_Wraw = S.Wbar.p;
    c->n_Wraw = S.Wbar.count();
    c->pre64_Wt.first = P.ops.size();
    contract<double>(P, S.Wbar, "mbej", t2, "jnfb", oovv, "mnef", -1.0);
    c->pre64_Wt.second = P.ops.size();
    KT ytmp = alloc_kt<double>(c, m, "oovo");
    contract<double>(P, ytmp, "mnej", t1, "jf", oovv, "mnef", 1.0, false);
    contract<double>(P, S.Wbar, "mbej", t1, "nb", ytmp, "mnej", -1.0);
    {
        // ring layout [m][e][b][j]: the (b,j) columns of the ring product become contiguous
        KT wr = alloc_kt<double>(c, m, "ovvo", 0, {1, -1, 1, -1});
        const int ext[4] = {o, v, v, o}, perm[4] = {0, 2, 1, 3}, sg[4] = {1, -1, 1, -1};
        void *src = S.Wbar.p, *dst = wr.p;
        const KMesh km = c->km;
        P.ops.push_back([=](hipStream_t s) { return permute4(src, dst, km, ext, perm, sg, s); });
        S.Wbar = wr;
    }
    // R_iabf = sum_me t_imae <mb||ef>   (k_i + k_f = k_a + k_b)
    c->pre64_lean_skip.clear();
    S.R = alloc_kt<double>(c, m, "ovvv", 0, {1, -1, -1, 1});
    const size_t r_begin = P.ops.size();
    contract<double>(P, S.R, "iabf", t2, "imae", ovvv, "mbef", 1.0, false);
    c->pre64_lean_skip.push_back({r_begin, P.ops.size()});
    // U_ianf = sum_me t_imae <mn||ef>   (k_i + k_f = k_a + k_n)
    S.U = alloc_kt<double>(c, m, "ovov", 0, {1, -1, -1, 1});
    c->n_U = S.U.count();
    c->pre64_U.first = P.ops.size();
    contract<double>(P, S.U, "ianf", t2, "imae", oovv, "mnef", 1.0, false);
    c->pre64_U.second = P.ops.size();
    // The doubles terms linear in x1 that share a contraction pattern are summed here, once per set
    // of amplitudes, so that each pattern costs one product over all (i, j, a, b) per sigma (the
    // final P(ij)P(ab) antisymmetrisation makes a term and its (i <-> j) image with opposite
    // sign equivalent):
    //   S_ijan = sum_me t_imae <mn||ej> + sum_f t_jf U_ianf + 1/4 sum_ef tau_ijef <an||ef>,
    //     entering as - S_ijan x_nb (the former S, Yp and Q / 4 terms);
    S.S = alloc_kt<double>(c, m, "oovo");
    contract<double>(P, S.S, "ijan", t2, "imae", ooov, "mnje", -1.0, false);
    contract<double>(P, S.S, "ijan", t1, "jf", S.U, "ianf", 1.0);
    contract<double>(P, S.S, "ijan", tau, "ijef", ovvv, "naef", -0.25);
    //   H_abej = 1/2 <ab||ej> - sum_m t_ma <mb||ej> - R_jabe, entering as x_ie H_abej (the R
    //     term R_iabf x_jf is minus its own (i <-> j) image, R_jabf x_if);
    S.H = alloc_kt<double>(c, m, "vvvo");
    build_eri(c, P, S.H, 0.5);
    contract<double>(P, S.H, "abej", t1, "ma", ovvo, "mbej", -1.0);
    {
        KT rp = alloc_kt<double>(c, m, "vvvo");
        const int ext[4] = {o, v, v, v}, perm[4] = {1, 2, 3, 0}, sg[4] = {1, 1, -1, -1};
        const void *src = S.R.p;
        void *dst = rp.p, *h = S.H.p;
        const i64 n = rp.count();
        const KMesh km = c->km;
        const size_t h_begin = P.ops.size();
        P.ops.push_back([=](hipStream_t s) { return permute4(src, dst, km, ext, perm, sg, s); });
        P.ops.push_back([=](hipStream_t s) { return scale_copy(dst, dst, -1.0, 0.0, n, s); });
        P.ops.push_back([=](hipStream_t s) { return add_inplace<double>(h, dst, n, s); });
        c->pre64_lean_skip.push_back({h_begin, P.ops.size()});
    }
    //   G2_ijbm = sum_e t_ie <mb||ej> + 1/2 <mb||ij>, entering as - G2_ijbm x_ma.
    S.G2 = alloc_kt<double>(c, m, "oovo");
    {
        const int ext[4] = {o, v, o, o}, perm[4] = {2, 3, 1, 0}, sg[4] = {1, 1, -1, -1};
        const void *src = c->g_ovoo.p;
        void *dst = S.G2.p;
        const i64 n = S.G2.count();
        const KMesh km = c->km;
        P.ops.push_back([=](hipStream_t s) { return permute4(src, dst, km, ext, perm, sg, s); });
        P.ops.push_back([=](hipStream_t s) { return scale_copy(dst, dst, 0.5, 0.0, n, s); });
    }
    contract<double>(P, S.G2, "ijbm", t1, "ie", ovvo, "mbej", 1.0);
    // t1-dressed virtual Cholesky slices for the ladder
    const i64 lvv = (i64)nk * nk * naux * v * v;
    S.La = m.get(lvv * 16);
    S.Lb = m.get(lvv * 16);
    {
        void *Ls = c->Ls, *Lcs = c->Lcs, *La = S.La, *Lb = S.Lb;
        P.ops.push_back([=](hipStream_t s) { return chol_slice<double>(Ls, La, nk, naux, n, o, v, o, v, 1.0, 0, s); });
        P.ops.push_back([=](hipStream_t s) { return chol_slice<double>(Lcs, Lb, nk, naux, n, o, v, o, v, 1.0, 0, s); });
        build_dressing(c, P, Ls, La, S.t1.p);
        build_dressing(c, P, Lcs, Lb, S.t1.p);
    }
    ladder_slots(c);
    const size_t wbytes32 = (size_t)c->nwslot * v * v * v * v * 8;
    if (store_ladder(c, 16, wbytes32)) {
        S.Wst = m.get((size_t)c->nwslot * v * v * v * v * 16);
        build_wstore<double>(c, P, S.La, S.Lb, S.Wst);
    }
    // preconditioner: diagonals of the dressed one-body blocks (F_mi, F_ae for singles,
    // Fbar_mj, Fbar_be for doubles) in place of the bare orbital energies of Eq. D
    S.d_o1 = m.get((size_t)nk * o * 8); S.d_v1 = m.get((size_t)nk * v * 8);
    S.d_o2 = m.get((size_t)nk * o * 8); S.d_v2 = m.get((size_t)nk * v * 8);
    {
        void *a = S.Fmi.p, *b = S.Fae.p, *cc = S.Fmj.p, *d = S.Fbe.p;
        double *da = (double *)S.d_o1, *db = (double *)S.d_v1, *dc = (double *)S.d_o2, *dd = (double *)S.d_v2;
        P.ops.push_back([=](hipStream_t s) { return diag_real(a, da, nk, o, s); });
        P.ops.push_back([=](hipStream_t s) { return diag_real(b, db, nk, v, s); });
        P.ops.push_back([=](hipStream_t s) { return diag_real(cc, dc, nk, o, s); });
        P.ops.push_back([=](hipStream_t s) { return diag_real(d, dd, nk, v, s); });
    }
    S.LaT = m.get(lvv * 16);
    S.LbT = m.get(lvv * 16);
    {
        void *La = S.La, *Lb = S.Lb, *LaT = S.LaT, *LbT = S.LbT;
        P.ops.push_back([=](hipStream_t s) { return pair_transpose<double>(La, LaT, nk, naux, v, s); });
        P.ops.push_back([=](hipStream_t s) { return pair_transpose<double>(Lb, LbT, nk, naux, v, s); });
    }
    c->pre64 = std::move(Pp);
    S.ready = true;

    // single-precision copies of everything the sigma reads
    State<float> &F = c->s32;
    auto P2p = std::make_unique<Program>();
    Program &P2 = *P2p;
    auto cv = [&](KT &d, const KT &s) { convert_kt<float>(P2, F, d, s, c); };
    cv(F.fov, S.fov); cv(F.t1, S.t1); cv(F.t2, S.t2); cv(F.tau, S.tau);
    cv(F.g_oovv, S.g_oovv); cv(F.g_ooov, S.g_ooov); cv(F.g_ovov, S.g_ovov); cv(F.g_ovvv, S.g_ovvv);
    cv(F.g_ovoo, S.g_ovoo);
    cv(F.Fae, S.Fae); cv(F.Fmi, S.Fmi); cv(F.Fme, S.Fme); cv(F.Fbe, S.Fbe); cv(F.Fmj, S.Fmj);
    cv(F.Fg, S.Fg); cv(F.Wp, S.Wp); cv(F.Wbar, S.Wbar); cv(F.R, S.R); cv(F.S, S.S); cv(F.U, S.U);
    cv(F.H, S.H); cv(F.G2, S.G2);
    F.La = F.mem.get(lvv * 8);
    F.Lb = F.mem.get(lvv * 8);
    F.LaT = F.mem.get(lvv * 8);
    F.LbT = F.mem.get(lvv * 8);
    for (int w = 0; w < 4; ++w) {
        void *a = w == 0 ? S.La : w == 1 ? S.Lb : w == 2 ? S.LaT : S.LbT;
        void *fa = w == 0 ? F.La : w == 1 ? F.Lb : w == 2 ? F.LaT : F.LbT;
        P2.ops.push_back([=](hipStream_t s) { return convert_f64_f32(a, fa, lvv, s); });
    }
    if (store_ladder(c, 8, 0)) {
        F.Wst = F.mem.get(wbytes32);
        build_wstore<float>(c, P2, F.La, F.Lb, F.Wst);
    }
    c->pre32 = std::move(P2p);
    F.ready = true;
}

// Upload T1, T2 (paper normalisation; T2 -> crystal by 1/Nk) into the state.
void upload_amplitudes(lrcc_ctx *c, const double *t1h, const double *t2h) {
    State<double> &S = c->s64;
    HIPCHK(hipMemcpy(S.t1.p, t1h, S.t1.count() * 16, hipMemcpyHostToDevice));
    std::vector<double> tmp(S.t2.count() * 2);
    std::memcpy(tmp.data(), t2h, tmp.size() * sizeof(double));
    for (auto &x : tmp) x /= c->nk;
    HIPCHK(hipMemcpy(S.t2.p, tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice));
}

bool tune_lookup(const std::string &key, std::vector<int> &choice);
void tune_store(const std::string &key, const std::vector<int> &choice);

// With autotuning on, the first run of an amplitude-dependent program picks its GEMM tiles (the
// programs recompute every block from the amplitudes, so repeated runs leave the same values).
static void tune_pre(lrcc_ctx *c, Program *p, const char *which, hipStream_t st) {
    if (!c->autotune || p->tuned || p->tunables.empty() || g_dry_run) return;
    char b[160];
    std::snprintf(b, sizeof b, "v9,%s,%d,%d,%d,%d,ladder%d,mesh%dx%dx%d", which, c->nk, c->no, c->nv, c->naux,
                  c->ladder_mode, c->km.n0, c->km.n1, c->km.n2);
    std::vector<int> choice;
    if (tune_lookup(b, choice)) {
        p->apply(choice);
        return;
    }
    HIPCHK(p->autotune(st, choice));
    tune_store(b, choice);
}

// Recompute every amplitude-dependent block from the device amplitudes.
// lean: the complex128 blocks without R_iabf (H_abej then lacks its R part), for the lean sigma
// programs only; a later full run restores every block.
void run_precompute(lrcc_ctx *c, bool fp32, hipStream_t st = nullptr, bool lean = false) {
    static const bool timed = std::getenv("LRCC_PRE_TIMES") != nullptr;   // per-op timing report
    tune_pre(c, c->pre64.get(), "pre64", st);
    if (fp32) tune_pre(c, c->pre32.get(), "pre32", st);
    if (lean) {
        // skipped ranges (kind 0) and, with lin_on, the blocks linear in t2 formed from their parts
        // at T and along y (kind 1: U, kind 2: the t2 term of W-bar)
        std::vector<std::tuple<size_t, size_t, int>> segs;
        for (const auto &r : c->pre64_lean_skip) segs.emplace_back(r.first, r.second, 0);
        if (c->lin_on) {
            segs.emplace_back(c->pre64_U.first, c->pre64_U.second, 1);
            segs.emplace_back(c->pre64_Wt.first, c->pre64_Wt.second, 2);
        }
        std::sort(segs.begin(), segs.end());
        const State<double> &S = c->s64;
        size_t at = 0;
        for (const auto &g : segs) {
            HIPCHK(c->pre64->run_range(st, at, std::get<0>(g)));
            if (std::get<2>(g) == 1) {
                HIPCHK(scale_copy(S.U.p, c->linU_y, c->lin_eps, 0.0, c->n_U, st));
                HIPCHK(add_inplace<double>(S.U.p, c->linU_T, c->n_U, st));
            } else if (std::get<2>(g) == 2) {
                HIPCHK(scale_copy(c->lin_tmp, c->linW_y, c->lin_eps, 0.0, c->n_Wraw, st));
                HIPCHK(add_inplace<double>(c->pre64_Wraw, c->lin_tmp, c->n_Wraw, st));
                HIPCHK(add_inplace<double>(c->pre64_Wraw, c->linW_T, c->n_Wraw, st));
            }
            at = std::get<1>(g);
        }
        HIPCHK(c->pre64->run_range(st, at, c->pre64->ops.size()));
        if (fp32) HIPCHK(c->pre32->run(st));
        HIPCHK(hipStreamSynchronize(st));
        return;
    }
    c->lin_T_ready = c->lin_on = false;   // the parts at T belong to the amplitudes they were taken at
    if (timed) {
        const bool was = c->prof.on;
        c->prof.on = true;
        HIPCHK(c->pre64->run(st, &c->prof));
        HIPCHK(hipStreamSynchronize(st));
        double ms[NTAGS];
        long long cnt[NTAGS];
        c->prof.read(ms, cnt);
        c->prof.on = was;
    } else
        HIPCHK(c->pre64->run(st));
    if (fp32) HIPCHK(c->pre32->run(st));
    HIPCHK(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------- sigma program
// The Jacobian product is recorded once as a list of symbolic operations, each
// linear in exactly one X-dependent ("active") tensor.  The forward program
// executes the list; the adjoint program (transpose Jacobian, the operator of
// the lambda equations l1, l2 and of the gradients) runs the list backwards,
// propagating cotangents through the transposed contractions.
struct SymOp {
    enum Kind { CON, COPY, TAU, LADDER } kind;
    KT C, A, B;
    std::string cl, al, bl;
    cd alpha = 1.0;
    bool acc = true;
    bool actA = false, actB = false;
    std::string pack;   // forward product: antisymmetric label pairs run on unique pairs (contract)
    std::string exact;  // of those, the output pairs written with their true values
    std::string tpack;  // the same for the transposed product of the active operand
};

struct SigmaGraph {
    std::vector<SymOp> ops;
    std::vector<KT> active;  // active[0] = x1, active[1] = x2, then intermediates
    KT x1, x2, Z, s1;
};

// Term sets of record_sigma: the full Jacobian; the lean one, without the term -x_ie R_jabe (for
// the blocks of the lean precompute, whose H_abej lacks R); that term alone.
enum SigmaTerms { TERMS_ALL = 0, TERMS_LEAN = 1, TERMS_R = 2 };

template <typename T>
SigmaGraph record_sigma(lrcc_ctx *c, State<T> &S, int R, DevMem &wm, bool full = true, int terms = TERMS_ALL) {
    SigmaGraph G;
    auto A = [&](const char *cls, std::initializer_list<int> sg = {1, 1, -1, -1}) {
        KT t = alloc_kt<T>(c, wm, cls, R, sg);
        G.active.push_back(t);
        return t;
    };
    auto is_act = [&](const KT &t) {
        for (auto &a : G.active)
            if (a.p == t.p) return true;
        return false;
    };
    auto con = [&](const KT &C, const char *cl, const KT &Aa, const char *al, const KT &Bb, const char *bl,
                   cd alpha, bool acc = true, const char *pack = "", const char *exact = "",
                   const char *tpack = "") {
        SymOp op;
        op.kind = SymOp::CON;
        op.C = C; op.A = Aa; op.B = Bb;
        op.cl = cl; op.al = al; op.bl = bl;
        op.alpha = alpha;
        op.acc = acc;
        op.pack = pack;
        op.exact = exact;
        op.tpack = tpack;
        op.actA = is_act(Aa);
        op.actB = is_act(Bb);
        if (op.actA == op.actB) throw LrccError(LRCC_E_ARG, std::string("term not linear in X: ") + cl);
        G.ops.push_back(op);
    };
    auto copy = [&](const KT &C, const KT &Aa) {
        SymOp op;
        op.kind = SymOp::COPY;
        op.C = C; op.A = Aa; op.actA = true;
        G.ops.push_back(op);
    };
    KT x1 = A("ov"), x2 = A("oovv"), dtau = A("oovv"), Z = A("oovv"), s1 = A("ov");
    KT dFae = A("vv"), dFmi = A("oo"), dFme = A("ov"), dFbe = A("vv"), dFmj = A("oo");
    KT Zmn = A("oooo"), Vx = A("oooo"), Yx = A("oovo");
    G.x1 = x1; G.x2 = x2; G.Z = Z; G.s1 = s1;
    if (terms == TERMS_R) {
        // -x_ie R_jabe = -sum_mf t_jmaf Q_ibmf, Q_ibmf = sum_e x_ie <mb||fe> (k_i + k_f = k_b + k_m):
        // linear in t2, so its change along a direction y of the amplitudes is this term with t2 = y2
        KT Q = A("ovov", {1, -1, -1, 1});
        con(Q, "Ribmf", x1, "Rie", S.g_ovvv, "mbfe", 1.0, false);
        con(Z, "Rijab", S.t2, "jmaf", Q, "Ribmf", -1.0, false);
        return G;
    }
    if (full) {
        SymOp op;
        op.kind = SymOp::TAU;
        op.C = dtau; op.A = x1; op.B = x2; op.actA = op.actB = true;
        G.ops.push_back(op);
    }
    const KT &t1 = S.t1, &t2 = S.t2;
    // X-dependent one-body intermediates (derivatives of F_ae, F_mi, F_me).  The doubles parts
    // -(x2 + dtau) <mn||ef> / 4 of dFae (and +1/4 of dFmi) are written as one product with dtau,
    // -dtau <mn||ef> / 2, plus the x1 t1 part of dtau contracted in closed form:
    // sum_mnf (dtau - x2)_mnaf <mn||ef> = 2 sum_m (x_ma Fg_me + t_ma dFme_me).
    if (full) con(dFme, "Rme", x1, "Rnf", S.g_oovv, "mnef", 1.0, false);
    con(dFae, "Rae", x1, "Rma", S.fov, "me", -0.5, false);
    if (full) {
        con(dFae, "Rae", x1, "Rmf", S.g_ovvv, "mafe", 1.0);
        con(dFae, "Rae", dtau, "Rmnaf", S.g_oovv, "mnef", -0.5, true, "mn", "", "mn");
        con(dFae, "Rae", x1, "Rma", S.Fg, "me", 0.5);
        con(dFae, "Rae", t1, "ma", dFme, "Rme", 0.5);
    }
    con(dFmi, "Rmi", x1, "Rie", S.fov, "me", 0.5, false);
    if (full) {
        con(dFmi, "Rmi", x1, "Rne", S.g_ooov, "mnie", 1.0);
        con(dFmi, "Rmi", dtau, "Rinef", S.g_oovv, "mnef", 0.5, true, "ef");
        con(dFmi, "Rmi", x1, "Rie", S.Fg, "me", -0.5);
        con(dFmi, "Rmi", t1, "ie", dFme, "Rme", -0.5);
    }
    // singles (operator part of Eq. tx1)
    con(s1, "Ria", x1, "Rie", S.Fae, "ae", 1.0, false);
    con(s1, "Ria", t1, "ie", dFae, "Rae", 1.0);
    con(s1, "Ria", x1, "Rma", S.Fmi, "mi", -1.0);
    con(s1, "Ria", t1, "ma", dFmi, "Rmi", -1.0);
    con(s1, "Ria", x2, "Rimae", S.Fme, "me", 1.0);
    if (full) {
        con(s1, "Ria", t2, "imae", dFme, "Rme", 1.0);
        con(s1, "Ria", x1, "Rnf", S.g_ovov, "naif", -1.0);
        con(s1, "Ria", x2, "Rimef", S.g_ovvv, "maef", -0.5, true, "ef", "", "ef");
        con(s1, "Ria", x2, "Rmnae", S.g_ooov, "nmie", 0.5, true, "mn", "", "mn");
    }
    // dressed one-body derivatives entering the doubles
    copy(dFbe, dFae);
    con(dFbe, "Rbe", x1, "Rmb", S.Fme, "me", -0.5);
    if (full) con(dFbe, "Rbe", t1, "mb", dFme, "Rme", -0.5);
    copy(dFmj, dFmi);
    con(dFmj, "Rmj", x1, "Rje", S.Fme, "me", 0.5);
    if (full) con(dFmj, "Rmj", t1, "je", dFme, "Rme", 0.5);
    // doubles (operator part of Eq. tx2): Z collects every term, sigma2 = P(ij)P(ab) Z.
    // Terms antisymmetric in both pairs enter with 1/4, in one pair with 1/2.  Products whose
    // operands are antisymmetric in a summed pair, or whose output pair reaches sigma2 (or the
    // transposed output) only antisymmetrised, run on unique pairs (pack / transposed pack: see
    // contract); dtau_bar's (e, f) pair is read unsymmetrised and is never packed.
    con(Z, "Rijab", x2, "Rijae", S.Fbe, "be", 0.5, false);
    con(Z, "Rijab", t2, "ijae", dFbe, "Rbe", 0.5);
    con(Z, "Rijab", x2, "Rimab", S.Fmj, "mj", -0.5, true, "ab", "", "ab");
    con(Z, "Rijab", t2, "imab", dFmj, "Rmj", -0.5, true, "ab", "", "ab");
    if (!full) return G;  // one-body (perturbation) operator: no two-electron terms
    {
        SymOp op;
        op.kind = SymOp::LADDER;
        op.C = Z; op.A = dtau; op.alpha = 0.25; op.actA = true;
        G.ops.push_back(op);
    }
    // hole-hole terms: Z += Zmn t2 / 16 + Vx tau / 8, Vx_ijmn = x_je <mn||ie> - (i <-> j).
    // With tau_mnab = t2_mnab + t_ma t_nb - t_mb t_na, Vx tau / 8 is Vx t2 / 8 plus a part
    // antisymmetric in (a, b), which P(ab) turns into Vx_ijmn t_ma t_nb / 4: the t2 parts share
    // one product with (Zmn + 2 Vx), and the t1 t1 part joins the Yx t1 product below
    // (Yx -= Vx t1 / 4), so no product over all (i, j, a, b) is spent on it.
    // Every operand of these three products is antisymmetric in each of its index pairs, and
    // Z enters sigma2 only through P(ij)P(ab): the forward products run on unique pairs (ij, mn,
    // ef, ab), Zmn being defined on the unique (ij, mn) pairs that its one consumer reads.
    // Transposed: dtau_bar is read by the transposed tau step alone, which antisymmetrises its rows
    // (ij); Z_bar is antisymmetric in both pairs; Zmn_bar is also read in full by the transposes of
    // the x1 terms, so it stays complete.
    con(Zmn, "Rijmn", dtau, "Rijef", S.g_oovv, "mnef", 1.0, false, "ijmnef", "im", "ijmn");
    con(Zmn, "Rijmn", x1, "Rje", S.g_ooov, "mnie", 2.0);
    con(Zmn, "Rjimn", x1, "Rje", S.g_ooov, "mnie", -2.0);
    con(Z, "Rijab", Zmn, "Rijmn", t2, "mnab", 1.0 / 16, true, "ijabmn", "", "ab");
    con(Z, "Rijab", S.Wp, "mnij", dtau, "Rmnab", 1.0 / 8, true, "ijabmn", "", "mnij");
    con(Vx, "Rijmn", x1, "Rje", S.g_ooov, "mnie", 1.0, false);
    con(Vx, "Rjimn", x1, "Rje", S.g_ooov, "mnie", -1.0);
    // ring terms (P(ij)P(ab))
    con(Z, "Rijab", x2, "Rimae", S.Wbar, "mebj", 1.0);
    con(Z, "Rijab", S.S, "ijan", x1, "Rnb", -1.0);
    con(Yx, "Rijan", x1, "Rjf", S.U, "ianf", 1.0, false);
    con(Yx, "Rijan", Vx, "Rijmn", t1, "ma", -0.25);
    con(Z, "Rijab", Yx, "Rijan", t1, "nb", -1.0);
    con(Z, "Rijab", x1, "Rie", S.H, "abej", 1.0);   // with TERMS_LEAN, H lacks its R part
    con(Z, "Rijab", S.G2, "ijbm", x1, "Rma", -1.0);
    return G;
}

template <typename T>
LadderArgs ladder_args(lrcc_ctx *c, const void *Y, const void *La, const void *Lb, void *Z, int R, double alpha) {
    LadderArgs la{};
    la.Y = Y; la.La = La; la.Lb = Lb; la.Z = Z;
    la.nk = c->nk; la.nrhs = R; la.o = c->no; la.v = c->nv; la.naux = c->naux;
    la.km = c->km;
    la.alpha = alpha;
    return la;
}

// Ladder products over stored or class-built integral blocks W'(ka,kb,ke)[e][f][a][b] (ka <= kb,
// ke <= kf; the ke = kf blocks hold W'/2), for the row pairs ki <= kj of the momentum classes
// cls0 .. cls0 + ncls - 1 (all classes, global slots, for cls0 < 0).  Every index pair that the antisymmetry makes redundant is skipped: rows
// (r, i < j) of the diagonal blocks ki = kj, columns a < b of the blocks ka = kb and reduction
// terms e < f of the blocks ke = kf are addressed through triangle splits, so the launches form
// only unique (rows, outputs, inputs) products up to the off-diagonal blocks' own i >= j, a >= b,
// e >= f halves, which are the partners' values.  One launch per combination of diagonal and
// off-diagonal rows, columns and reduction blocks (they differ in M, N, K).
//  forward:   Z(ki,kj,ka)[rows][ab] += 4 alpha sum_{ke <= kf} Y(ki,kj,ke)[rows][ef] W'(ka,kb,ke)
//             (x2 more for ke = kf: the e < f terms of W'/2); the factor 4 = 2 for the (kj,ki) /
//             i > j partner rows and 2 for the (kb,ka) / a > b partner columns, which the
//             P(ij)P(ab) assembly reproduces from antisymmetry;
//  transpose: T(ki,kj,ke)[rows][ef] += 2 alpha sum_{ka <= kb} Zbar(ki,kj,ka)[rows][ab] W'(ka,kb,ke)^T
//             (x2 more for the e < f columns of ke = kf, whose e > f half stays zero); the ka = kb
//             terms a < b give the full-range sum of Zbar W'^T / 2; the rows carry 2 for their
//             partners, T is completed by expand_ab.
template <typename T>
void ladder_block_gemms(lrcc_ctx *c, Program &P, bool transpose, const void *A, const void *W, i64 wblocks,
                        void *C, i64 sizeA, i64 sizeC, int R, int cls0, int ncls, std::complex<double> alpha,
                        const char *name) {
    const int nk = c->nk, o = c->no, v = c->nv;
    const i64 vv = (i64)v * v, inner = (i64)R * o * o * vv;
    const i64 Po = (i64)o * (o - 1) / 2, Pv = (i64)v * (v - 1) / 2;
    for (int rdiag = 0; rdiag < 2; ++rdiag)
        for (int ndiag = 0; ndiag < 2; ++ndiag)
            for (int kdiag = 0; kdiag < 2; ++kdiag) {
                if ((rdiag && Po == 0) || ((ndiag || kdiag) && Pv == 0)) continue;
                GemmArgs g{};
                g.shape = -1;
                g.kind = 1;
                g.A = A;
                g.B = W;
                g.C = C;
                // rows (r, i, j): all o^2 of an off-diagonal pair, i < j of a diagonal one
                if (rdiag) {
                    g.M = (int)(R * Po);
                    g.sm = tri_split(o);
                    g.Am = g.Cm = Strides{{(i64)o * o * vv, (i64)o * vv, vv}};
                } else {
                    g.M = R * o * o;
                    g.sm = Split{1, g.M};
                    g.Am = g.Cm = Strides{{0, 0, vv}};
                }
                // columns: (a, b) forward, (e, f) transposed; reduction: the other pair
                const Split full{1, (int)vv}, tri = tri_split(v);
                g.N = (int)(ndiag ? Pv : vv);
                g.sn = ndiag ? tri : full;
                g.K = (int)(kdiag ? Pv : vv);
                g.sk = kdiag ? tri : full;
                const Strides pair_in_row = ndiag ? Strides{{0, v, 1}} : Strides{{0, 0, 1}};
                g.Cn = pair_in_row;
                g.Ak = kdiag ? Strides{{0, v, 1}} : Strides{{0, 0, 1}};
                if (!transpose) {
                    g.Bk = kdiag ? Strides{{0, v * vv, vv}} : Strides{{0, 0, vv}};
                    g.Bn = ndiag ? Strides{{0, v, 1}} : Strides{{0, 0, 1}};
                    g.bNfast = 1;
                } else {
                    g.Bk = kdiag ? Strides{{0, v, 1}} : Strides{{0, 0, 1}};
                    g.Bn = ndiag ? Strides{{0, v * vv, vv}} : Strides{{0, 0, vv}};
                    g.bNfast = 0;
                }
                g.aMfast = 0;
                const double f = transpose ? 2.0 * (ndiag ? 2.0 : 1.0) : 4.0 * (kdiag ? 2.0 : 1.0);
                g.alpha_re = alpha.real() * f;
                g.alpha_im = alpha.imag() * f;
                g.beta = 1;
                std::vector<i64> offC, segA, segB;
                std::vector<int> beg{0};
                for (int ki = 0; ki < nk; ++ki)
                    for (int kj = ki; kj < nk; ++kj) {
                        if ((ki == kj) != (rdiag == 1) || !in_classes(kclass(c, ki, kj), cls0, ncls)) continue;
                        // output blocks: ka <= kb forward, ke <= kf transposed; reduction: the other
                        for (int kn = 0; kn < nk; ++kn) {
                            const int kn2 = c->km.comb(ki, kj, kn);
                            if (kn > kn2 || (kn == kn2) != (ndiag == 1)) continue;
                            const size_t s0 = segA.size();
                            for (int kr = 0; kr < nk; ++kr) {
                                const int kr2 = c->km.comb(ki, kj, kr);
                                if (kr > kr2 || (kr == kr2) != (kdiag == 1)) continue;
                                const int ka = transpose ? kr : kn, kb = transpose ? kr2 : kn2;
                                const int ke = transpose ? kn : kr;
                                segA.push_back((((i64)ki * nk + kj) * nk + kr) * inner);
                                segB.push_back(block_slot(c, cls0, ka, kb, ke) * vv * vv);
                            }
                            if (segA.size() == s0) continue;
                            offC.push_back((((i64)ki * nk + kj) * nk + kn) * inner);
                            beg.push_back((int)segA.size());
                        }
                    }
                if (offC.empty()) continue;
                raw_gemm<T>(P, g, offC, beg, segA, segB, sizeA, wblocks * vv * vv, sizeC);
                P.tag_last(TAG_LADDER);
                P.name_last(name);
            }
}

template <typename T>
Program *build_sigma(lrcc_ctx *c, State<T> &S, int R, DevMem &wm, bool full = true, int terms = TERMS_ALL) {
    const int nk = c->nk, o = c->no, v = c->nv;
    auto P = new Program();
    SigmaGraph G = record_sigma<T>(c, S, R, wm, full, terms);
    const i64 nb3 = (i64)nk * nk * nk;
    KT x1 = G.x1, x2 = G.x2, Z = G.Z, s1 = G.s1;
    // caller layout -> internal (paper -> crystal normalisation for doubles)
    P->ops.push_back([=](hipStream_t s) { return rhs_to_block<double, T>(c->io_x1, x1.p, R, nk, (i64)o * v, 1.0, s); });
    P->ops.push_back([=](hipStream_t s) {
        return rhs_to_block<double, T>(c->io_x2, x2.p, R, nb3, (i64)o * o * v * v, 1.0 / nk, s);
    });
    for (const SymOp &op : G.ops) {
        switch (op.kind) {
        case SymOp::CON:
            contract<T>(*P, op.C, op.cl, op.A, op.al, op.B, op.bl, op.alpha, op.acc, c->pack_pairs ? op.pack : "",
                        op.exact);
            break;
        case SymOp::COPY:
            kt_copy<T>(*P, op.C, op.A);
            break;
        case SymOp::TAU: {
            void *t1p = S.t1.p, *xa = op.A.p, *xb = op.B.p, *out = op.C.p;
            const KMesh km = c->km;
            P->ops.push_back([=](hipStream_t s) { return tau_like<T>(xa, xb, t1p, out, km, R, o, v, 1.0, 1, s); });
            break;
        }
        case SymOp::LADDER: {
            const bool by_class = ladder_path(c, S.Wst, 2 * sizeof(T)) == 3 && S.La && S.Lb;
            P->ladder_path = S.Wst ? 2 : by_class ? 3 : 1;
            if (S.Wst || by_class) {
                // stored integrals: Z(ki,kj,ka) += alpha' sum_{ke <= kf} Y(ki,kj,ke) W'(ka,kb,ke) for the
                // unique pairs (ladder_block_gemms).  By class (mode 3): for each momentum class
                // K = ki + kj = ka + kb, the class's blocks W' are built into a scratch array of
                // ncls_slots blocks and consumed by that class's products before the next class
                const i64 vv = (i64)v * v;
                const int nb = by_class ? class_batch(c, 2 * sizeof(T)) : nk;
                const i64 wblocks = by_class ? (i64)nb * c->ncls_slots : c->nwslot;
                void *Wb = by_class ? P->alloc((size_t)wblocks * vv * vv * 2 * sizeof(T)) : S.Wst;
                for (int K0 = by_class ? 0 : -1; K0 < (by_class ? nk : 0); K0 += by_class ? nb : 1) {
                    const int ncl = by_class ? std::min(nb, nk - K0) : 0;
                    if (by_class) build_wstore<T>(c, *P, S.La, S.Lb, Wb, K0, ncl, TAG_BUILD);
                    ladder_block_gemms<T>(c, *P, false, op.A.p, Wb, wblocks, op.C.p, op.A.count(), op.C.count(), R,
                                          K0, ncl, op.alpha,
                                          by_class ? "ladder (class integrals)" : "ladder (stored integrals)");
                }
                break;
            }
            LadderArgs la = ladder_args<T>(c, op.A.p, S.La, S.Lb, op.C.p, R, op.alpha.real());
            // dtau is antisymmetric in (e,f): packed kernels; the pipelined one from 320 rows on
            // (its 384-row tiles would idle more than a sixth of their rows below)
            // dtau and the ladder term are antisymmetric in (i, j) too, and Z reaches sigma2 only
            // through P(ij)P(ab): the pipelined kernel forms the unique rows only, the rows of all
            // (ki <= kj) pairs with one ki + kj in one stream of tiles (they share the integrals);
            // it is used from kPipeMinRows rows per class on (below, its tiles would mostly idle)
            la.pack_rows = 1;
            la.order = 1;
            la.packed = c->pack_ladder ? (ladder_rows_max(la) >= kPipeMinRows ? 2 : 1) : 0;
            auto lp = std::make_shared<LadderArgs>(la);
            P->ops.push_back([lp](hipStream_t s) { return launch_ladder<T>(*lp, s); });
            P->ladder_args = lp;
            P->ladder_op = P->ops.size() - 1;
            // candidates: pipelined packed in XCD-grouped (0) or plain (1) tile order, 256-row
            // packed (2) or full-range (3) ladder
            P->tunables.push_back({P->ops.size() - 1, 4, [lp](int c) {
                lp->packed = c <= 1 ? 2 : c == 2 ? 1 : 0;
                lp->order = c == 0 ? 1 : 0;
            }});
            P->last_flops = (i64)ladder_executed_flops(la, sizeof(T) == 8);
            P->flops += P->last_flops;
            P->tag_last(TAG_LADDER);
            P->name_last("ladder");
            break;
        }
        }
    }
    // outputs in the caller layout: y = (A - omega) x, paper normalisation
    P->ops.push_back([=](hipStream_t s) { return s1_out<T>(s1.p, c->io_x1, c->io_y1, c->io_omega, nk, R, o, v, s); });
    P->ops.push_back([=](hipStream_t s) {
        return pp_out<T>(Z.p, c->io_x2, c->io_y2, c->io_omega, c->km, R, o, v, (double)nk, s);
    });
    return P;
}

// Transpose product y = (A - omega)^T z with respect to the pairing
// <u, v> = sum u1 v1 + 1/4 sum u2 v2 (amplitude arrays in the caller's normalisation).
// Reverse sweep of a recorded term list: every active tensor of G receives its cotangent for
// the output cotangent z = (*z1src, *z2src) (caller layout, read when the program runs), in
// the pairing <z, y> = sum z1 y1 + 1/4 sum z2 y2.  The active buffers of G hold cotangents
// afterwards (x1, x2: the transpose product before the final assembly).
template <typename T>
void emit_reverse_sweep(lrcc_ctx *c, State<T> &S, int R, const SigmaGraph &G, Program *P,
                        const void *const *z1src, const void *const *z2src);

template <typename T>
Program *build_sigma_adjoint(lrcc_ctx *c, State<T> &S, int R, DevMem &wm, bool full = true,
                             int terms = TERMS_ALL) {
    const int nk = c->nk, o = c->no, v = c->nv;
    auto P = new Program();
    SigmaGraph G = record_sigma<T>(c, S, R, wm, full, terms);
    emit_reverse_sweep<T>(c, S, R, G, P, &c->io_x1, &c->io_x2);
    KT x1 = G.x1, x2 = G.x2;
    // y1 = x1bar - omega z1 ; y2 = P(ij)P(ab) x2bar / Nk - omega z2
    P->ops.push_back([=](hipStream_t s) { return s1_out<T>(x1.p, c->io_x1, c->io_y1, c->io_omega, nk, R, o, v, s); });
    P->ops.push_back([=](hipStream_t s) {
        return pp_out<T>(x2.p, c->io_x2, c->io_y2, c->io_omega, c->km, R, o, v, 1.0 / nk, s);
    });
    return P;
}

template <typename T>
void emit_reverse_sweep(lrcc_ctx *c, State<T> &S, int R, const SigmaGraph &G, Program *P,
                        const void *const *z1src, const void *const *z2src) {
    const int nk = c->nk, o = c->no, v = c->nv;
    // adjoint buffer for every active tensor (the forward buffers are reused as adjoints)
    for (const KT &a : G.active) {
        void *p = a.p;
        i64 n = a.count();
        P->ops.push_back([=](hipStream_t s) { return zero_fill<T>(p, n, s); });
    }
    KT x1 = G.x1, x2 = G.x2, Z = G.Z, s1 = G.s1;
    // cotangent of the outputs: s1bar = z1, Zbar = (Nk/4) P(ij)P(ab) z2
    P->ops.push_back([=](hipStream_t s) { return rhs_to_block<double, T>(*z1src, s1.p, R, nk, (i64)o * v, 1.0, s); });
    P->ops.push_back([=](hipStream_t s) { return pp_in<T>(*z2src, Z.p, c->km, R, o, v, 0.25 * nk, s); });
    for (auto it = G.ops.rbegin(); it != G.ops.rend(); ++it) {
        const SymOp &op = *it;
        switch (op.kind) {
        case SymOp::CON: {
            const std::string tp = c->pack_pairs ? op.tpack : "";
            if (op.actA) contract<T>(*P, op.A, op.al, op.C, op.cl, op.B, op.bl, op.alpha, true, tp);
            if (op.actB) contract<T>(*P, op.B, op.bl, op.A, op.al, op.C, op.cl, op.alpha, true, tp);
            break;
        }
        case SymOp::COPY: {
            void *a = op.A.p, *cc = op.C.p;
            i64 n = op.A.count();
            P->ops.push_back([=](hipStream_t s) { return add_inplace<T>(a, cc, n, s); });
            break;
        }
        case SymOp::TAU: {
            // dtau = x2 + (x_ia t_jb + t_ia x_jb - x_ib t_ja - t_ib x_ja)
            void *a = op.B.p, *cc = op.C.p;
            i64 n = op.B.count();
            P->ops.push_back([=](hipStream_t s) { return add_inplace<T>(a, cc, n, s); });
            const KT &dt = op.C, &xx1 = op.A, &t1 = S.t1;
            contract<T>(*P, xx1, "Ria", dt, "Rijab", t1, "jb", 1.0, true);
            contract<T>(*P, xx1, "Rjb", dt, "Rijab", t1, "ia", 1.0, true);
            contract<T>(*P, xx1, "Rib", dt, "Rijab", t1, "ja", -1.0, true);
            contract<T>(*P, xx1, "Rja", dt, "Rijab", t1, "ib", -1.0, true);
            break;
        }
        case SymOp::LADDER: {
            const bool by_class = ladder_path(c, S.Wst, 2 * sizeof(T)) == 3 && S.La && S.Lb;
            P->ladder_path = S.Wst ? 2 : by_class ? 3 : 1;
            if (S.Wst || by_class) {
                // stored integrals, transposed (ladder_block_gemms): with Zbar antisymmetric in (a, b),
                //   dtau_bar(ki,kj,ke) = alpha [sum_{ka<kb} Zbar(ki,kj,ka) W'(ka,kb,ke)^T
                //                              + 1/2 sum_{ka=kb} Zbar(ki,kj,ka) W'(ka,ka,ke)^T]
                // for ke <= kf, into a zeroed scratch array; expand_ab adds it and its (e, f)-
                // antisymmetric (kf, ke) partner blocks to dtau_bar.  By class (mode 3): the blocks
                // of one momentum class at a time in a scratch array, as in the forward product
                const i64 vv = (i64)v * v, n = op.A.count();
                void *tmp = P->alloc((size_t)n * 2 * sizeof(T)), *dst = op.A.p;
                const int nb = by_class ? class_batch(c, 2 * sizeof(T)) : nk;
                const i64 wblocks = by_class ? (i64)nb * c->ncls_slots : c->nwslot;
                void *Wb = by_class ? P->alloc((size_t)wblocks * vv * vv * 2 * sizeof(T)) : S.Wst;
                const KMesh km = c->km;
                P->ops.push_back([tmp, n](hipStream_t s) { return zero_fill<T>(tmp, n, s); });
                for (int K0 = by_class ? 0 : -1; K0 < (by_class ? nk : 0); K0 += by_class ? nb : 1) {
                    const int ncl = by_class ? std::min(nb, nk - K0) : 0;
                    if (by_class) build_wstore<T>(c, *P, S.La, S.Lb, Wb, K0, ncl, TAG_BUILD);
                    ladder_block_gemms<T>(c, *P, true, op.C.p, Wb, wblocks, tmp, op.C.count(), n, R, K0, ncl, op.alpha,
                                          by_class ? "ladder (class integrals, transposed)"
                                                   : "ladder (stored integrals, transposed)");
                }
                P->ops.push_back([tmp, dst, km, R, o, v](hipStream_t s) {
                    return expand_ab<T>(tmp, dst, km, R, o, v, 1.0, s);
                });
                break;
            }
            LadderArgs la = ladder_args<T>(c, op.C.p, S.LaT, S.LbT, op.A.p, R, op.alpha.real());
            // Zbar is antisymmetric in both pairs (it is only read in the reverse pass) and so is
            // the transposed ladder; dtau_bar is read by the transposed tau step alone, which sums
            // the four pair placements: the pipelined kernel forms unique pairs and class rows from
            // kPipeMinRows rows per class on (below, the full-range kernel: the tiles would idle)
            la.pack_rows = 1;
            la.order = 1;
            if (!(c->pack_ladder && ladder_rows_max(la) >= kPipeMinRows)) la.pack_rows = 0;
            else la.packed = 2;
            P->ops.push_back([=](hipStream_t s) { return launch_ladder<T>(la, s); });
            P->last_flops = (i64)ladder_executed_flops(la, sizeof(T) == 8);
            P->flops += P->last_flops;
            P->tag_last(TAG_LADDER);
            P->name_last("ladder");
            break;
        }
        }
    }
}

// Autotuning cache: one line per program, "key choice0 choice1 ..." in a text
// file (the path in LRCC_TUNE_CACHE); the key is nk,o,v,naux,nrhs,precision,direction,ladder path.
std::string tune_key(lrcc_ctx *c, int prec, int R, bool adj, int variant, int path) {
    char b[128];
    // "v9": candidate semantics (GEMM: heuristic tile shape first, up to three, four in complex64;
    // ladder: four kernel/order variants); the ladder path (1 rebuilt in LDS, 2 stored, 3 built by
    // momentum class) changes the program's launches, so it is part of the key
    std::snprintf(b, sizeof b, "v9,%d,%d,%d,%d,%d,%s,%s%d,ladder%d", c->nk, c->no, c->nv, c->naux, R,
                  prec == LRCC_FP64 ? "f64" : "f32", adj ? "adjoint" : "forward", variant, path);
    if (!c->km.chain()) return std::string(b) + ",mesh" + std::to_string(c->km.n0) + "x" + std::to_string(c->km.n1) +
                               "x" + std::to_string(c->km.n2);
    return b;
}

bool tune_lookup(const std::string &key, std::vector<int> &choice) {
    const char *path = std::getenv("LRCC_TUNE_CACHE");
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[8192];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        if (l.compare(0, key.size() + 1, key + " ") != 0) continue;
        // the choices: whitespace-separated candidate indices after the key
        choice.clear();
        const char *q = l.c_str() + key.size();
        char *end = nullptr;
        for (long x = std::strtol(q, &end, 10); end != q; x = std::strtol(q, &end, 10)) {
            choice.push_back((int)x);
            q = end;
        }
        found = true;
    }
    std::fclose(f);
    return found;
}

void tune_store(const std::string &key, const std::vector<int> &choice) {
    const char *path = std::getenv("LRCC_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s", key.c_str());
    for (int x : choice) std::fprintf(f, " %d", x);
    std::fprintf(f, "\n");
    std::fclose(f);
}

// Run a recorded sigma program on the current io bindings, eagerly (timed if
// profiling) or through its captured graph.  With autotuning on, the first run
// of a program chooses its launch variants (or takes them from the cache).
hipError_t run_sigma(lrcc_ctx *c, Program *p, hipStream_t st) {
    if (c->autotune && !p->tuned) {
        std::vector<int> choice;
        if (tune_lookup(p->tune_key, choice)) {
            p->apply(choice);
        } else {
            hipError_t e = p->autotune(st, choice);
            if (e != hipSuccess) return e;
            tune_store(p->tune_key, choice);
        }
    }
    if (c->use_graphs && st != nullptr) {
        Program::GraphKey key{c->io_x1, c->io_x2, c->io_y1, c->io_y2, c->io_omega};
        return p->run_graph(st, key);
    }
    return p->run(st, &c->prof);
}

// variant 0: the CCSD Jacobian; variant 1+x: the Jacobian of the one-body
// perturbation residual for dipole axis x (Fock matrix -> mu_x, no two-electron part);
// kLeanSigma: the CCSD Jacobian (complex128) without the term -x_ie R_jabe, on the blocks of the
// lean precompute; kRTermSigma: that term alone (complex128).
constexpr int kLeanSigma = -1, kRTermSigma = -2;
Program *sigma_program(lrcc_ctx *c, int prec, int R, bool adjoint = false, int variant = 0) {
    auto key = std::make_pair(variant * 4 + prec * 2 + (adjoint ? 1 : 0), R);
    auto it = c->progs.find(key);
    if (it != c->progs.end()) return it->second.get();
    auto mem = std::make_unique<DevMem>();
    Program *p;
    if (variant == kLeanSigma || variant == kRTermSigma) {
        if (prec != LRCC_FP64) throw LrccError(LRCC_E_ARG, "the lean sigma is FP64 only");
        const int terms = variant == kLeanSigma ? TERMS_LEAN : TERMS_R;
        p = adjoint ? build_sigma_adjoint<double>(c, c->s64, R, *mem, true, terms)
                    : build_sigma<double>(c, c->s64, R, *mem, true, terms);
    } else if (variant > 0) {
        if (prec != LRCC_FP64) throw LrccError(LRCC_E_ARG, "perturbation operators are FP64 only");
        State<double> &X = c->xs[variant - 1];
        p = adjoint ? build_sigma_adjoint<double>(c, X, R, *mem, false) : build_sigma<double>(c, X, R, *mem, false);
    } else if (!adjoint)
        p = prec == LRCC_FP64 ? build_sigma<double>(c, c->s64, R, *mem) : build_sigma<float>(c, c->s32, R, *mem);
    else
        p = prec == LRCC_FP64 ? build_sigma_adjoint<double>(c, c->s64, R, *mem)
                              : build_sigma_adjoint<float>(c, c->s32, R, *mem);
    p->tune_key = tune_key(c, prec, R, adjoint, variant, p->ladder_path);
    c->progs[key].reset(p);
    c->progmem[key] = std::move(mem);
    return p;
}


// ---------------------------------------------------------------- response solver
// Batched right-preconditioned restarted GMRES (one Krylov space per right-hand
// side, all advanced together so that each step is one multi-RHS sigma launch),
// and FP32-inner / FP64-residual iterative refinement.  Inner products weight
// the doubles by 1/4 so that every independent amplitude counts once.
struct Vecs {
    void *s = nullptr, *d = nullptr;  // singles [R][n1], doubles [R][n2] (complex128, caller layout)
};

struct SolveCtx {
    lrcc_ctx *c;
    int R;
    i64 n1, n2;
    hipStream_t st;
    const double *omega;  // device
    void *part = nullptr, *dout = nullptr, *alpha = nullptr;  // reduction / coefficient scratch
    int nsig64 = 0, nsig32 = 0;
    long long rhs_sig = 0;
    bool adjoint = false;
    std::vector<cd> dot(const Vecs &u, const Vecs &v) {
        std::vector<cd> a(R), b(R);
        HIPCHK(batched_dot(u.s, v.s, R, n1, 1.0, part, dout, st));
        HIPCHK(hipMemcpyAsync(a.data(), dout, R * 16, hipMemcpyDeviceToHost, st));
        HIPCHK(batched_dot(u.d, v.d, R, n2, 0.25, part, dout, st));
        HIPCHK(hipMemcpyAsync(b.data(), dout, R * 16, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int r = 0; r < R; ++r) a[r] += b[r];
        return a;
    }
    // NaN for a non-finite inner product, so that a NaN or Inf anywhere in a right-hand side
    // can never look converged
    std::vector<double> norm(const Vecs &u) {
        auto d = dot(u, u);
        std::vector<double> n(R);
        for (int r = 0; r < R; ++r)
            n[r] = std::isfinite(d[r].real()) && std::isfinite(d[r].imag())
                       ? std::sqrt(std::max(0.0, d[r].real()))
                       : std::numeric_limits<double>::quiet_NaN();
        return n;
    }
    // y = beta y + a_r x
    void axpby(const Vecs &y, const Vecs &x, const std::vector<cd> &a, double beta) {
        HIPCHK(hipMemcpyAsync(alpha, a.data(), R * 16, hipMemcpyHostToDevice, st));
        HIPCHK(batched_axpby(y.s, x.s, alpha, beta, R, n1, st));
        HIPCHK(batched_axpby(y.d, x.d, alpha, beta, R, n2, st));
        HIPCHK(hipStreamSynchronize(st));  // alpha buffer is reused by the next call
    }
    void copy(const Vecs &y, const Vecs &x) {
        HIPCHK(hipMemcpyAsync(y.s, x.s, R * n1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(y.d, x.d, R * n2 * 16, hipMemcpyDeviceToDevice, st));
    }
    void zero(const Vecs &y) {
        HIPCHK(hipMemsetAsync(y.s, 0, R * n1 * 16, st));
        HIPCHK(hipMemsetAsync(y.d, 0, R * n2 * 16, st));
    }
    // out = M^-1 in for a Krylov-space vector in with packed doubles (complex64 storage for f32)
    void unpack_prec(const Vecs &out, const Vecs &in, const PackMap &pm, int f32) {
        const State<double> &T = c->s64;
        HIPCHK(unpack_precond(out.s, out.d, in.s, in.d, pm, (const double *)T.d_o1, (const double *)T.d_v1,
                              (const double *)T.d_o2, (const double *)T.d_v2, omega, c->km, R, c->no, c->nv, f32,
                              st));
    }
    // y = (A - omega) x
    void op(const Vecs &y, const Vecs &x, int precision) {
        Program *p = sigma_program(c, precision, R, adjoint);
        c->io_x1 = x.s; c->io_x2 = x.d; c->io_y1 = y.s; c->io_y2 = y.d; c->io_omega = omega;
        HIPCHK(run_sigma(c, p, st));
        (precision == LRCC_FP64 ? nsig64 : nsig32)++;
        rhs_sig += R;
    }
};

// Largest element, NaN if any element is NaN (std::max_element skips NaN).
static double max_nan(const std::vector<double> &v) {
    double m = v.empty() ? 0.0 : -std::numeric_limits<double>::infinity();
    for (double x : v) {
        if (std::isnan(x)) return x;
        m = std::max(m, x);
    }
    return m;
}

// ||r|| / ||b||; NaN when either is not finite (0 for a zero right-hand side)
static double rel_res(double rn, double bn) {
    if (!std::isfinite(rn) || !std::isfinite(bn)) return std::numeric_limits<double>::quiet_NaN();
    return bn > 0 ? rn / bn : 0.0;
}

// Hessenberg pivots below this (after the Givens rotation) mean that (A - omega), right-
// preconditioned by the dressed diagonal (D - omega)^-1 (which scales it to O(1)), maps a
// unit direction of the Krylov space to zero to working precision: singular at that frequency.
constexpr double kSingularPivot = 1e-12;

// LRCC_VERBOSE set: progress lines of the solvers on stderr.
static bool verbose() {
    static int v = std::getenv("LRCC_VERBOSE") ? 1 : 0;
    return v != 0;
}

// Device workspace of the batched GMRES: a contiguous Krylov basis with packed doubles (one k
// block per antisymmetry orbit, PackMap; vector i of right-hand side r at (Vs + (i R + r) n1,
// Vd + (i R + r) n2) with n2 the packed length; complex128, or complex64 for the inner solves of
// the mixed refinement), the Hessenberg/Givens state of every right-hand
// side, the Gram-Schmidt coefficients and a pinned status buffer.  With graphs on, every Arnoldi
// step j is captured once (unpacking preconditioner, sigma, packing, two Gram-Schmidt passes (one
// in complex64), norm, rotation, normalisation, status copy) and replayed for later cycles and
// refinement steps of the same solve.
struct GmresWork {
    int R = 0, m = 0;
    i64 n1 = 0, n2 = 0;   // singles and packed doubles per right-hand side
    i64 blk = 0;          // elements of one doubles k block (o o v v)
    int f32 = 0;          // Krylov vectors stored in complex64 (the complex64 inner solves), else complex128
    size_t vb = 16;       // bytes per stored complex element
    PackMap pm;
    void *Vs = nullptr, *Vd = nullptr;
    GmresState g{};
    void *h1 = nullptr, *h2 = nullptr, *hn2 = nullptr, *beta2 = nullptr, *y = nullptr, *part = nullptr;
    void *ones = nullptr, *minus = nullptr;    // R complex 1 and -1 (axpby coefficients)
    void *stat_d = nullptr;                    // [3R] device status
    double *stat_h = nullptr;                  // [3R] pinned host status
    // (precision, j, tolerance) -> captured Arnoldi step (the tolerance is baked into the rotation
    // kernel's arguments, and the inner tolerance of the mixed path changes between refinements)
    std::map<std::tuple<int, int, double>, hipGraphExec_t> steps;
    Vecs vec(int i) const {
        Vecs v;
        v.s = (char *)Vs + (size_t)i * R * n1 * vb;
        v.d = (char *)Vd + (size_t)i * R * n2 * vb;
        return v;
    }
    ~GmresWork() {
        for (auto &kv : steps) (void)hipGraphExecDestroy(kv.second);
        if (stat_h) (void)hipHostFree(stat_h);
    }
};

// Packed length of the doubles of one right-hand side (PackMap) for the context's k mesh.
i64 packed_doubles(const lrcc_ctx *c) {
    std::vector<int> canon, map;
    std::vector<double> scale;
    return (i64)pack_tables(c->km, canon, map, scale) * c->no * c->no * c->nv * c->nv;
}

void gmres_alloc(lrcc_ctx *c, GmresWork &W, int R, int m, i64 n1, int f32, hipStream_t st) {
    DevMem &M = c->solmem;
    std::vector<int> canon, map;
    std::vector<double> scale;
    W.pm.np = pack_tables(c->km, canon, map, scale);
    W.pm.nfull = (int)map.size();
    W.blk = (i64)c->no * c->no * c->nv * c->nv;
    const i64 n2 = (i64)W.pm.np * W.blk;
    W.R = R; W.m = m; W.n1 = n1; W.n2 = n2;
    W.f32 = f32;
    W.vb = f32 ? 8 : 16;
    int *canon_d = (int *)M.get(canon.size() * sizeof(int)), *map_d = (int *)M.get(map.size() * sizeof(int));
    double *scale_d = (double *)M.get(scale.size() * sizeof(double));
    W.pm.canon = canon_d;
    W.pm.map = map_d;
    W.pm.scale = scale_d;
    W.Vs = M.get((size_t)(m + 1) * R * n1 * W.vb);
    W.Vd = M.get((size_t)(m + 1) * R * n2 * W.vb);
    W.g.R = R;
    W.g.m = m;
    W.g.H = (double2 *)M.get((size_t)R * (m + 1) * m * 16);
    W.g.cs = (double2 *)M.get((size_t)R * m * 16);
    W.g.sn = (double2 *)M.get((size_t)R * m * 16);
    W.g.g = (double2 *)M.get((size_t)R * (m + 1) * 16);
    W.g.scal = (double2 *)M.get((size_t)R * 16);
    W.g.bn = (double *)M.get((size_t)R * 8);
    W.g.rel = (double *)M.get((size_t)R * 8);
    W.g.act = (int *)M.get((size_t)R * 4);
    W.g.kr = (int *)M.get((size_t)R * 4);
    W.g.sing = (int *)M.get((size_t)R * 4);
    W.h1 = M.get((size_t)R * (m + 1) * 16);
    W.h2 = M.get((size_t)R * (m + 1) * 16);
    W.hn2 = M.get((size_t)R * 16);
    W.beta2 = M.get((size_t)R * 16);
    W.y = M.get((size_t)R * (m + 1) * 16);
    W.part = M.get((size_t)R * (m + 1) * multidot_blocks(n1 + n2) * 16);   // [R][m+1][blocks] partial sums
    W.ones = M.get((size_t)R * 16);
    W.minus = M.get((size_t)R * 16);
    W.stat_d = M.get((size_t)R * 3 * 8);
    if (g_dry_run) return;
    HIPCHK(hipMemcpyAsync(canon_d, canon.data(), canon.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(map_d, map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(scale_d, scale.data(), scale.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipHostMalloc((void **)&W.stat_h, (size_t)R * 3 * 8, hipHostMallocDefault));
    std::vector<cd> one(R, cd(1.0, 0.0)), mone(R, cd(-1.0, 0.0));
    HIPCHK(hipMemcpyAsync(W.ones, one.data(), (size_t)R * 16, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(W.minus, mone.data(), (size_t)R * 16, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
}

// Status of every right-hand side after the last cycle start or Arnoldi step (one host sync).
struct GmresStatus {
    std::vector<double> rel;
    std::vector<int> act, sing;
};
GmresStatus gmres_read(const GmresWork &W, hipStream_t st, bool launch = true) {
    if (launch) {
        HIPCHK(gmres_status(W.g, (double *)W.stat_d, st));
        HIPCHK(hipMemcpyAsync(W.stat_h, W.stat_d, (size_t)W.R * 3 * 8, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    GmresStatus s;
    s.rel.resize(W.R);
    s.act.resize(W.R);
    s.sing.resize(W.R);
    for (int r = 0; r < W.R; ++r) {
        s.rel[r] = W.stat_h[3 * r];
        s.act[r] = (int)W.stat_h[3 * r + 1];
        s.sing[r] = (int)W.stat_h[3 * r + 2];
    }
    return s;
}

// One Arnoldi step j on the device: z = M^-1 V_j (unpacked), w = (A - omega) z, V_{j+1} = w packed,
// classical Gram-Schmidt of V_{j+1} against V_0..V_j twice (the second pass restores
// orthogonality lost to rounding), the column of H and its Givens rotation (k_gmres_step),
// V_{j+1} /= h_{j+1,j}, and the status words copied to the pinned host buffer.  Right-hand sides
// that stopped keep their basis (masked).
hipError_t arnoldi_step(SolveCtx &S, GmresWork &W, int j, int precision, double tol, const Vecs &w, const Vecs &z,
                        bool eager_sigma) {
    lrcc_ctx *c = S.c;
    const int R = W.R;
    const i64 n1 = W.n1, n2 = W.n2;
    const Vecs vj = W.vec(j), vn = W.vec(j + 1);
    const State<double> &T = c->s64;
    hipStream_t st = S.st;
    hipError_t e;
    e = unpack_precond(z.s, z.d, vj.s, vj.d, W.pm, (const double *)T.d_o1, (const double *)T.d_v1,
                       (const double *)T.d_o2, (const double *)T.d_v2, S.omega, c->km, R, c->no, c->nv, W.f32, st);
    if (e != hipSuccess) return e;
    Program *p = sigma_program(c, precision, R, S.adjoint);
    c->io_x1 = z.s; c->io_x2 = z.d; c->io_y1 = w.s; c->io_y2 = w.d; c->io_omega = S.omega;
    e = eager_sigma ? run_sigma(c, p, st) : p->run(st);
    if (e != hipSuccess) return e;
    e = pack_vec(vn.s, vn.d, w.s, w.d, nullptr, nullptr, W.pm, R, n1, W.blk, W.f32, st);
    if (e != hipSuccess) return e;
    // classical Gram-Schmidt with one re-orthogonalisation; the complex64 inner solves of the
    // refinement (to a relative 1e-5 or so, corrected by the complex128 residual) take one pass
    const int passes = precision == LRCC_FP32 ? 1 : 2;
    for (int pass = 0; pass < passes; ++pass) {
        void *h = pass == 0 ? W.h1 : W.h2;
        e = multidot(W.Vs, W.Vd, vn.s, vn.d, R, n1, n2, j + 1, W.part, h, W.m + 1, 1.0, W.f32, st);
        if (e != hipSuccess) return e;
        e = multiaxpy(vn.s, vn.d, W.Vs, W.Vd, h, W.m + 1, -1.0, W.g.act, 1.0, R, n1, n2, j + 1, W.f32, st);
        if (e != hipSuccess) return e;
    }
    e = selfdot(vn.s, vn.d, R, n1, n2, W.part, W.hn2, 1.0, W.f32, st);
    if (e != hipSuccess) return e;
    e = gmres_step(W.g, j, W.h1, passes == 2 ? W.h2 : nullptr, W.hn2, tol, precision == LRCC_FP64 ? kSingularPivot : 0.0,
                   st);
    if (e != hipSuccess) return e;
    e = basis_axpby(vn.s, vn.s, W.g.scal, 0.0, R, n1, W.f32, st);
    if (e != hipSuccess) return e;
    e = basis_axpby(vn.d, vn.d, W.g.scal, 0.0, R, n2, W.f32, st);
    if (e != hipSuccess) return e;
    e = gmres_status(W.g, (double *)W.stat_d, st);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(W.stat_h, W.stat_d, (size_t)R * 3 * 8, hipMemcpyDeviceToHost, st);
}

// GMRES on (A - omega) x = b starting from x (in/out), all right-hand sides advanced together
// (each step one multi-RHS sigma launch), the Krylov state on the device.  Stops when every
// right-hand side reaches ||r|| <= tol ||b|| (or stopped: singular, non-finite) or after
// max_apply operator applications.  Returns per-RHS relative residual estimates.
std::vector<double> gmres(SolveCtx &S, GmresWork &W, const Vecs &b, const Vecs &x, int precision, double tol,
                          int max_apply, const Vecs &w, const Vecs &z, bool x_is_zero,
                          std::vector<bool> *singular = nullptr) {
    lrcc_ctx *c = S.c;
    const int R = S.R, m = W.m;
    const i64 n1 = S.n1, n2p = W.n2;
    hipStream_t st = S.st;
    // ||b|| once; the singular flags start clear
    {
        auto bn = S.norm(b);
        HIPCHK(hipMemcpyAsync(W.g.bn, bn.data(), (size_t)R * 8, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemsetAsync(W.g.sing, 0, (size_t)R * sizeof(int), st));   // never inside a captured step
        HIPCHK(hipStreamSynchronize(st));
    }
    std::vector<double> rel(R, 0.0);
    std::vector<bool> sing(R, false);
    int applied = 0;
    bool first = true;
    auto done = [&]() {
        if (singular) *singular = sing;
        return rel;
    };
    const Vecs v0 = W.vec(0);
    while (true) {
        // r = b - A x packed into V_0, its norm, the cycle's initial state on the device
        if (!(first && x_is_zero)) {
            S.op(w, x, precision);
            ++applied;
            HIPCHK(pack_vec(v0.s, v0.d, b.s, b.d, w.s, w.d, W.pm, R, n1, W.blk, W.f32, st));
        } else {
            HIPCHK(pack_vec(v0.s, v0.d, b.s, b.d, nullptr, nullptr, W.pm, R, n1, W.blk, W.f32, st));
        }
        first = false;
        HIPCHK(selfdot(v0.s, v0.d, R, n1, n2p, W.part, W.beta2, 1.0, W.f32, st));
        HIPCHK(gmres_init(W.g, W.beta2, tol, st));
        GmresStatus gs = gmres_read(W, st);
        bool all = true, nonfinite = false;
        for (int r = 0; r < R; ++r) {
            rel[r] = gs.rel[r];
            sing[r] = gs.sing[r] != 0;
            if (!(rel[r] <= tol) && !sing[r]) all = false;
            if (std::isnan(rel[r])) nonfinite = true;
        }
        if (verbose())
            std::fprintf(stderr, "[lrcc] gmres %s%s R=%d applied=%d max rel residual %.3e\n",
                         precision == LRCC_FP64 ? "fp64" : "fp32", S.adjoint ? " adjoint" : "", R, applied,
                         max_nan(rel));
        // a non-finite residual cannot recover: stop at once (the caller reports it)
        if (all || nonfinite || applied >= max_apply) return done();
        HIPCHK(basis_axpby(v0.s, v0.s, W.g.scal, 0.0, R, n1, W.f32, st));
        HIPCHK(basis_axpby(v0.d, v0.d, W.g.scal, 0.0, R, n2p, W.f32, st));
        int j = 0;
        for (; j < m && applied < max_apply; ++j) {
            // graph replay of the step once the sigma program has been tuned (the first run of a
            // program may autotune, which times launches and cannot be captured)
            Program *p = sigma_program(c, precision, R, S.adjoint);
            const bool graph = c->use_graphs && st != nullptr && (!c->autotune || p->tuned) && !c->prof.on;
            if (graph) {
                auto key = std::make_tuple(precision, j, tol);
                auto it = W.steps.find(key);
                if (it == W.steps.end()) {
                    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                    hipError_t er = arnoldi_step(S, W, j, precision, tol, w, z, false);
                    hipGraph_t gr = nullptr;
                    hipError_t ee = hipStreamEndCapture(st, &gr);
                    HIPCHK(er);
                    HIPCHK(ee);
                    hipGraphExec_t ex = nullptr;
                    hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(gr);
                    HIPCHK(ei);
                    it = W.steps.emplace(key, ex).first;
                }
                HIPCHK(hipGraphLaunch(it->second, st));
            } else {
                HIPCHK(arnoldi_step(S, W, j, precision, tol, w, z, true));
            }
            (precision == LRCC_FP64 ? S.nsig64 : S.nsig32)++;
            S.rhs_sig += R;
            ++applied;
            GmresStatus gs2 = gmres_read(W, st, false);
            bool any = false;
            for (int r = 0; r < R; ++r) {
                if (gs2.sing[r]) sing[r] = true;
                rel[r] = gs2.rel[r];
                any = any || gs2.act[r];
            }
            if (!any) { ++j; break; }
        }
        // x += M^-1 sum_i y_i V_i with y = H^-1 g per right-hand side; the sum goes to slot j,
        // whose vector V_j is not in the span the solution takes (and the next cycle restarts)
        HIPCHK(gmres_solve(W.g, W.y, st));
        const Vecs u = W.vec(j);
        HIPCHK(multiaxpy(u.s, u.d, W.Vs, W.Vd, W.y, m + 1, 1.0, nullptr, 0.0, R, n1, n2p, j, W.f32, st));
        S.unpack_prec(z, u, W.pm, W.f32);
        HIPCHK(batched_axpby(x.s, z.s, W.ones, 1.0, R, n1, st));
        HIPCHK(batched_axpby(x.d, z.d, W.ones, 1.0, R, S.n2, st));
        x_is_zero = false;
        if (applied >= max_apply) {
            HIPCHK(hipStreamSynchronize(st));
            return done();  // estimates from the rotations
        }
        bool open = false;
        for (int r = 0; r < R; ++r) open = open || !sing[r];
        if (!open) {
            HIPCHK(hipStreamSynchronize(st));
            return done();
        }
    }
}

// Solve (A - omega_r) x_r = b_r (or the transpose).  x holds the initial guess; x_is_zero
// saves the product with a zero guess.  On return rep.converged is 1 only if every relative
// residual is finite and <= tol; *singular (if given) is set when FP64 GMRES met a zero
// pivot on a right-hand side that did not converge.
void solve_response(lrcc_ctx *c, int R, const double *omega_dev, const Vecs &b, const Vecs &x,
                    const lrcc_solve_opts &o, lrcc_solve_report &rep, hipStream_t st, bool adjoint = false,
                    bool x_is_zero = false, bool *singular = nullptr) {
    auto t0 = std::chrono::steady_clock::now();
    SolveCtx S;
    S.c = c; S.R = R; S.st = st; S.omega = omega_dev; S.adjoint = adjoint;
    S.n1 = (i64)c->nk * c->no * c->nv;
    S.n2 = (i64)c->nk * c->nk * c->nk * c->no * c->no * c->nv * c->nv;
    const bool mixed = o.precision == LRCC_FP32;
    const i64 n2p = packed_doubles(c);
    const size_t per = (size_t)R * (S.n1 + S.n2) * 16;     // a full work vector
    // a Krylov vector (packed doubles): complex64 for the inner solves of the mixed refinement, whose
    // tolerance (1e-5 by default) is far above complex64 rounding
    const size_t perk = (size_t)R * (S.n1 + n2p) * (mixed ? 8 : 16);
    const int nwork = 2 + (mixed ? 2 : 0);
    c->solmem.release();
    int m = o.krylov;
    if (m <= 0) {
        // subspace size from the free device memory (85% of it, the rest left for the few
        // single-vector buffers of the alpha contraction), between 4 and 60 vectors
        size_t fr = 0, tot = 0;
        if (!g_dry_run) HIPCHK(hipMemGetInfo(&fr, &tot));
        const long long fit = (long long)((0.85 * (double)fr - (double)(per * nwork)) / (double)perk) - 1;
        m = (int)std::max(4LL, std::min(60LL, fit));
    }
    m = std::min(m, 60);   // the Gram-Schmidt kernels take at most 64 basis vectors
    const size_t need = perk * (m + 1) + per * nwork + (size_t)R * (dot_blocks(S.n2) + 4) * 16 * 2 +
                        (size_t)R * ((m + 1) * multidot_blocks(S.n1 + n2p) + 4 * (m + 2) + (size_t)(m + 1) * m) * 16;
    if (o.mem_cap_bytes > 0 && need > (size_t)o.mem_cap_bytes)
        throw LrccError(LRCC_E_OOM, "solver work vectors exceed the memory cap");
    GmresWork W;
    gmres_alloc(c, W, R, m, S.n1, mixed ? 1 : 0, st);
    auto mk = [&]() { Vecs v; v.s = c->solmem.get((size_t)R * S.n1 * 16); v.d = c->solmem.get((size_t)R * S.n2 * 16); return v; };
    Vecs w = mk(), z = mk();
    S.part = c->solmem.get((size_t)R * dot_blocks(S.n2) * 16);
    S.dout = c->solmem.get((size_t)R * 16);
    S.alpha = c->solmem.get((size_t)R * 16);
    std::vector<double> rel;
    std::vector<bool> sing;
    rep = lrcc_solve_report{};
    if (!mixed) {
        rel = gmres(S, W, b, x, LRCC_FP64, o.tol, o.max_iter, w, z, x_is_zero, &sing);
        rep.outer = 1;
    } else {
        Vecs r = mk(), dx = mk();
        auto bn = S.norm(b);
        for (int it = 0; it < o.max_outer; ++it) {
            // FP64 residual r = b - (A - w) x (r = b for a zero first guess)
            S.copy(r, b);
            if (it > 0 || !x_is_zero) {
                S.op(w, x, LRCC_FP64);
                S.axpby(r, w, std::vector<cd>(R, cd(-1.0, 0.0)), 1.0);
            }
            auto rn = S.norm(r);
            rel.assign(R, 0.0);
            bool all = true, nonfinite = false;
            for (int q = 0; q < R; ++q) {
                rel[q] = rel_res(rn[q], bn[q]);
                if (!(rel[q] <= o.tol)) all = false;
                if (std::isnan(rel[q])) nonfinite = true;
            }
            rep.outer = it + 1;
            const double worst = max_nan(rel);
            if (verbose())
                std::fprintf(stderr, "[lrcc] refinement step %d: max rel residual %.3e (krylov %d)\n", it, worst, m);
            if (all || nonfinite) break;
            // FP32 correction solve (A - w) dx = r to inner_tol, or only as far as the
            // outer tolerance still needs (with a 10x margin) on the last step
            const double itol = std::max(o.inner_tol, std::min(0.5, 0.1 * o.tol / worst));
            S.zero(dx);
            gmres(S, W, r, dx, LRCC_FP32, itol, 4 * m, w, z, true);
            S.axpby(x, dx, std::vector<cd>(R, cd(1.0, 0.0)), 1.0);
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    c->solmem.release();   // the Krylov space is not needed after the solve (W's captured steps go with it)
    rep.sigma_fp64 = S.nsig64;
    rep.sigma_fp32 = S.nsig32;
    rep.rhs_sigmas = S.rhs_sig;
    rep.max_rel_residual = max_nan(rel);
    rep.converged = rep.max_rel_residual <= o.tol;   // false for NaN
    if (singular) {
        *singular = false;
        for (size_t q = 0; q < sing.size(); ++q) *singular = *singular || (sing[q] && !(rel[q] <= o.tol));
    }
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Status for an unconverged solve: LRCC_E_SINGULAR after a zero pivot, else LRCC_E_NOCONV,
// with the residual (or its non-finiteness) in the message.
[[noreturn]] void throw_unconverged(const char *what, const lrcc_solve_report &rep, bool singular) {
    if (singular)
        throw LrccError(LRCC_E_SINGULAR, std::string(what) + ": the response operator is singular at this "
                                                             "frequency (zero Krylov pivot)");
    if (std::isnan(rep.max_rel_residual))
        throw LrccError(LRCC_E_NOCONV, std::string(what) + ": non-finite residual (NaN or Inf in the "
                                                           "right-hand side or the iterates)");
    throw LrccError(LRCC_E_NOCONV, std::string(what) + " did not converge: relative residual " +
                                       std::to_string(rep.max_rel_residual));
}

void default_opts(lrcc_solve_opts &o) {
    o.tol = 1e-10;
    o.max_iter = 400;
    o.krylov = 0;
    o.precision = LRCC_FP64;
    o.inner_tol = 1e-5;
    o.max_outer = 30;
    o.mem_cap_bytes = 0;
    o.reuse_lambda = 1;
}


// ---------------------------------------------------------------- polarizability
// alpha_XY(w) per cell from the symmetric linear-response function (Eq. lrf):
//   alpha = -1/(2 Nk) C^{+-w} [eta^X t^Y(w) + eta^Y t^X(-w) + F(t^X(-w), t^Y(w))],
//   C^{+-w} g(w) = g(w) + conj(g(-w)),
// with (A - w) t^X(w) = -xi^X (Eqs. rhs, tx1, tx2), A^T lambda = -dE/dT
// (Eqs. l1, l2), eta^X = A_X^T lambda + dE_X/dT for the one-body perturbation
// operator of axis X, and F(x, y) = d2 L / dT dT [x, y] of the Lagrangian
// L = E + <lambda, Omega>.  F is evaluated as the exact 5-point derivative of
// A(T + e y)^T lambda (A is cubic in T) plus the energy's second derivative.
// All pairings are bilinear: <u, w> = sum u1 w1 + 1/4 sum u2 w2.
void ensure_alpha_programs(lrcc_ctx *c) {
    if (c->prog_xi) return;
    const int nk = c->nk, o = c->no, v = c->nv, n = c->n;
    State<double> &S = c->s64;
    const i64 n1 = (i64)nk * o * v, n2 = (i64)nk * nk * nk * o * o * v * v;
    DevMem &m = c->amem;
    c->lam1 = m.get(n1 * 16); c->lam2 = m.get(n2 * 16);
    c->xi1 = m.get(3 * n1 * 16); c->xi2 = m.get(3 * n2 * 16);
    c->gb1 = m.get(n1 * 16); c->gb2 = m.get(n2 * 16);
    c->ybuf = m.get(n1 * 16); c->ubuf = m.get(n1 * 16);
    // one-body perturbation states: F-type intermediates of the residual with f -> mu_x, v -> 0
    for (int x = 0; x < 3; ++x) {
        State<double> &X = c->xs[x];
        DevMem &xm = X.mem;
        auto P = std::make_unique<Program>();
        X.t1 = S.t1; X.t2 = S.t2; X.tau = S.tau;
        X.fov = alloc_kt<double>(c, xm, "ov");
        KT foo = alloc_kt<double>(c, xm, "oo"), fvv = alloc_kt<double>(c, xm, "vv");
        const void *dx = (const char *)c->dip + (size_t)x * nk * n * n * 16;
        {
            void *a = X.fov.p, *b = foo.p, *d = fvv.p;
            P->ops.push_back([=](hipStream_t s) { return axis_slice<double>(dx, a, 1, nk, n, 0, o, o, v, 0, s); });
            P->ops.push_back([=](hipStream_t s) { return axis_slice<double>(dx, b, 1, nk, n, 0, o, 0, o, 0, s); });
            P->ops.push_back([=](hipStream_t s) { return axis_slice<double>(dx, d, 1, nk, n, o, v, o, v, 0, s); });
        }
        const KT &t1 = S.t1;
        X.Fae = alloc_kt<double>(c, xm, "vv");
        kt_copy<double>(*P, X.Fae, fvv);
        contract<double>(*P, X.Fae, "ae", X.fov, "me", t1, "ma", -0.5);
        X.Fmi = alloc_kt<double>(c, xm, "oo");
        kt_copy<double>(*P, X.Fmi, foo);
        contract<double>(*P, X.Fmi, "mi", t1, "ie", X.fov, "me", 0.5);
        X.Fme = X.fov;
        X.Fbe = alloc_kt<double>(c, xm, "vv");
        kt_copy<double>(*P, X.Fbe, X.Fae);
        contract<double>(*P, X.Fbe, "be", t1, "mb", X.Fme, "me", -0.5);
        X.Fmj = alloc_kt<double>(c, xm, "oo");
        kt_copy<double>(*P, X.Fmj, X.Fmi);
        contract<double>(*P, X.Fmj, "mj", t1, "je", X.Fme, "me", 0.5);
        X.ready = true;
        c->prex[x] = std::move(P);
    }
    // xi^X for all three axes (caller layout, per-cell normalisation): Eq. rhs in the
    // standard <mu| exp(-T) X exp(T) |HF> form
    {
        auto P = std::make_unique<Program>();
        const int R = 3;
        KT Xoo = alloc_kt<double>(c, m, "oo", R), Xov = alloc_kt<double>(c, m, "ov", R);
        KT Xvv = alloc_kt<double>(c, m, "vv", R), s1 = alloc_kt<double>(c, m, "ov", R);
        KT Y = alloc_kt<double>(c, m, "vv", R), Fx = alloc_kt<double>(c, m, "vv", R), Gx = alloc_kt<double>(c, m, "oo", R);
        KT Z = alloc_kt<double>(c, m, "oovv", R);
        const void *dip = c->dip;
        {
            void *a = Xoo.p, *b = Xov.p, *d = Xvv.p, *e = s1.p;
            P->ops.push_back([=](hipStream_t s) { return axis_slice<double>(dip, a, 3, nk, n, 0, o, 0, o, 0, s); });
            P->ops.push_back([=](hipStream_t s) { return axis_slice<double>(dip, b, 3, nk, n, 0, o, o, v, 0, s); });
            P->ops.push_back([=](hipStream_t s) { return axis_slice<double>(dip, d, 3, nk, n, o, v, o, v, 0, s); });
            // driver X_ai stored as [k][x][i][a]
            P->ops.push_back([=](hipStream_t s) { return axis_slice<double>(dip, e, 3, nk, n, 0, o, o, v, 1, s); });
        }
        const KT &t1 = S.t1, &t2 = S.t2;
        contract<double>(*P, s1, "Ria", t2, "ikac", Xov, "Rkc", 1.0);
        contract<double>(*P, Y, "Rac", t1, "ka", Xov, "Rkc", 1.0, false);
        contract<double>(*P, s1, "Ria", t1, "ic", Y, "Rac", -1.0);
        contract<double>(*P, s1, "Ria", t1, "ic", Xvv, "Rac", 1.0);
        contract<double>(*P, s1, "Ria", t1, "ka", Xoo, "Rki", -1.0);
        kt_copy<double>(*P, Fx, Xvv);
        contract<double>(*P, Fx, "Rbc", t1, "kb", Xov, "Rkc", -1.0);
        kt_copy<double>(*P, Gx, Xoo);
        contract<double>(*P, Gx, "Rkj", t1, "jc", Xov, "Rkc", 1.0);
        contract<double>(*P, Z, "Rijab", t2, "ijac", Fx, "Rbc", 0.5, false);
        contract<double>(*P, Z, "Rijab", t2, "ikab", Gx, "Rkj", -0.5);
        void *xi1 = c->xi1, *xi2 = c->xi2;
        P->ops.push_back([=](hipStream_t s) { return s1_out<double>(s1.p, nullptr, xi1, nullptr, nk, R, o, v, s); });
        const KMesh km = c->km;
        P->ops.push_back([=](hipStream_t s) { return pp_out<double>(Z.p, nullptr, xi2, nullptr, km, R, o, v, (double)nk, s); });
        c->prog_xi = std::move(P);
    }
    // right-hand side of the lambda equations: -(S^-1 dE/dT) = -(f_ia + <ij||ab> t_jb, <ij||ab>/Nk)
    {
        auto P = std::make_unique<Program>();
        KT g1 = alloc_kt<double>(c, m, "ov");
        kt_copy<double>(*P, g1, S.fov);
        contract<double>(*P, g1, "ia", S.g_oovv, "ijab", S.t1, "jb", 1.0);
        void *gb1 = c->gb1, *gb2 = c->gb2, *ov = S.g_oovv.p;
        P->ops.push_back([=](hipStream_t s) { return scale_copy(gb1, g1.p, -1.0, 0.0, n1, s); });
        P->ops.push_back([=](hipStream_t s) { return scale_copy(gb2, ov, -1.0 / nk, 0.0, n2, s); });
        c->prog_grad = std::move(P);
    }
    // second derivative of the energy: u_ia = sum_jb <ij||ab> y_jb
    {
        auto P = std::make_unique<Program>();
        KT y = make_kt(c, "ov", c->ybuf), u = make_kt(c, "ov", c->ubuf);
        contract<double>(*P, u, "ia", S.g_oovv, "ijab", y, "jb", 1.0, false);
        c->prog_epp = std::move(P);
    }
}

// eta^X = A_X^T lambda + (X_ov, 0) for dipole axis x (caller layout, one vector)
void eta_vector(lrcc_ctx *c, int x, const Vecs &out, hipStream_t st) {
    const int nk = c->nk, no = c->no, nv = c->nv, n = c->n;
    HIPCHK(c->prex[x]->run(st));
    Program *p = sigma_program(c, LRCC_FP64, 1, true, 1 + x);
    c->io_x1 = c->lam1; c->io_x2 = c->lam2; c->io_y1 = out.s; c->io_y2 = out.d; c->io_omega = nullptr;
    HIPCHK(p->run(st));
    const void *dx = (const char *)c->dip + (size_t)x * nk * n * n * 16;
    HIPCHK(axis_slice<double>(dx, c->ubuf, 1, nk, n, 0, no, no, nv, 0, st));
    HIPCHK(add_inplace<double>(out.s, c->ubuf, (i64)nk * no * nv, st));
}

// F(., y) = d/de [A(T + e y)^T lambda] + E''(., y): the gradient in x of the
// bilinear F(x, y) of the response function.  A is cubic in T, so the 5-point
// derivative is exact; y is in caller layout (per-cell normalisation).  Leaves
// the device amplitudes shifted: the caller restores them from (T1, T2) and
// re-runs the amplitude-dependent blocks when all stencils are done.
// With p0 = A(T)^T lambda at the unshifted amplitudes (the same for every y), three
// shifted points suffice: p'(0) = (6 p(h) - 2 p(-h) - p(2h) - 3 p(0)) / (6h) is exact for
// the cubic p(e) = A(T + e y)^T lambda.  The stencil runs on the lean transpose (lean blocks,
// without the term -x_ie R_jabe, and p0 without it, from lambda_product); that term, linear
// in t2, adds its exact derivative once per direction.
void f_vector(lrcc_ctx *c, SolveCtx &D, const Vecs &y, const Vecs &Fy, const Vecs &q, const void *T1,
              const void *T2, hipStream_t st, const Vecs *p0 = nullptr) {
    const int nk = c->nk;
    const i64 n1 = D.n1, n2 = D.n2;
    State<double> &S = c->s64;
    const i64 nt1 = S.t1.count(), nt2 = S.t2.count();
    // shifted points: the lean blocks and the matching transpose program (one vector)
    Program *adj = sigma_program(c, LRCC_FP64, 1, true, kLeanSigma);
    const double coef5[4] = {1.0 / 12.0, -8.0 / 12.0, 8.0 / 12.0, -1.0 / 12.0};
    const int shift5[4] = {-2, -1, 1, 2};
    const double coef3[3] = {-2.0 / 6.0, 6.0 / 6.0, -1.0 / 6.0};
    const int shift3[3] = {-1, 1, 2};
    const int npt = p0 ? 3 : 4;
    const double *coef = p0 ? coef3 : coef5;
    const int *shift = p0 ? shift3 : shift5;
    // step: |h y| about 1e-2 in the rms sense
    cd yy = 0;
    {
        SolveCtx N = D;
        N.R = 1;
        yy = N.dot(y, y)[0];
    }
    const double rms = std::sqrt(std::max(yy.real(), 1e-300) / (double)(n1 + n2 / 4));
    const double h = 1e-2 / rms;
    if (p0) {
        std::vector<cd> w0(1, cd(-3.0 / (6.0 * h), 0.0));
        HIPCHK(hipMemcpy(D.alpha, w0.data(), 16, hipMemcpyHostToDevice));
        HIPCHK(batched_axpby(Fy.s, p0->s, D.alpha, 0.0, 1, n1, st));
        HIPCHK(batched_axpby(Fy.d, p0->d, D.alpha, 0.0, 1, n2, st));
        HIPCHK(hipStreamSynchronize(st));
    } else {
        HIPCHK(hipMemsetAsync(Fy.s, 0, n1 * 16, st));
        HIPCHK(hipMemsetAsync(Fy.d, 0, n2 * 16, st));
    }
    // The term -x_ie R_jabe of the transpose is linear in t2 and depends on nothing else that
    // moves: its part of the derivative is the term with t2 = y2 (crystal normalisation y2 / Nk),
    // formed once; the stencil points run the lean transpose without it.
    {
        Program *rt = sigma_program(c, LRCC_FP64, 1, true, kRTermSigma);
        HIPCHK(scale_copy(S.t2.p, y.d, 1.0 / nk, 0.0, nt2, st));
        c->io_x1 = c->lam1; c->io_x2 = c->lam2; c->io_y1 = q.s; c->io_y2 = q.d; c->io_omega = nullptr;
        HIPCHK(rt->run(st));
        HIPCHK(add_inplace<double>(Fy.s, q.s, n1, st));
        HIPCHK(add_inplace<double>(Fy.d, q.d, n2, st));
    }
    // U_ianf and the t2 term of W-bar are linear in t2 alone: their parts along y (t2 = y2 / Nk still
    // in place), once; each stencil point then forms B(T) + e B(y) instead of building B
    if (c->lin_T_ready) {
        HIPCHK(c->pre64->run_range(st, c->pre64_U.first, c->pre64_U.second));
        HIPCHK(hipMemcpyAsync(c->linU_y, S.U.p, (size_t)c->n_U * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(zero_fill<double>(c->pre64_Wraw, c->n_Wraw, st));
        HIPCHK(c->pre64->run_range(st, c->pre64_Wt.first, c->pre64_Wt.second));
        HIPCHK(hipMemcpyAsync(c->linW_y, c->pre64_Wraw, (size_t)c->n_Wraw * 16, hipMemcpyDeviceToDevice, st));
    }
    c->lin_on = c->lin_T_ready;   // without the parts at T the stencil points build both blocks
    for (int k = 0; k < npt; ++k) {
        // T' = T + shift*h*y  (T2 stored in crystal normalisation: y2 / Nk)
        HIPCHK(hipMemcpyAsync(S.t1.p, T1, nt1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(S.t2.p, T2, nt2 * 16, hipMemcpyDeviceToDevice, st));
        std::vector<cd> a1(1, cd(shift[k] * h, 0.0)), a2(1, cd(shift[k] * h / nk, 0.0));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(D.alpha, a1.data(), 16, hipMemcpyHostToDevice));
        HIPCHK(batched_axpby(S.t1.p, y.s, D.alpha, 1.0, 1, nt1, st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(D.alpha, a2.data(), 16, hipMemcpyHostToDevice));
        HIPCHK(batched_axpby(S.t2.p, y.d, D.alpha, 1.0, 1, nt2, st));
        const auto tp0 = std::chrono::steady_clock::now();
        c->lin_eps = shift[k] * h;
        run_precompute(c, false, st, true);
        const auto tp1 = std::chrono::steady_clock::now();
        c->io_x1 = c->lam1; c->io_x2 = c->lam2; c->io_y1 = q.s; c->io_y2 = q.d; c->io_omega = nullptr;
        HIPCHK(adj->run(st));
        std::vector<cd> w(1, cd(coef[k] / h, 0.0));
        HIPCHK(hipStreamSynchronize(st));
        if (verbose())
            std::fprintf(stderr, "[lrcc] F stencil point %d: blocks %.2f ms, transpose product %.2f ms\n", k,
                         std::chrono::duration<double, std::milli>(tp1 - tp0).count(),
                         std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp1).count());
        HIPCHK(hipMemcpy(D.alpha, w.data(), 16, hipMemcpyHostToDevice));
        HIPCHK(batched_axpby(Fy.s, q.s, D.alpha, 1.0, 1, n1, st));
        HIPCHK(batched_axpby(Fy.d, q.d, D.alpha, 1.0, 1, n2, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    c->lin_on = false;
    // energy part: sum <ij||ab> x_ia y_jb
    HIPCHK(hipMemcpyAsync(c->ybuf, y.s, n1 * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(c->prog_epp->run(st));
    HIPCHK(add_inplace<double>(Fy.s, c->ubuf, n1, st));
}

// p0 = A(T)^T lambda without the term -x_ie R_jabe (the lean transpose of the F stencils) at the
// current amplitudes, shared by every F stencil: the full product minus that term; q is scratch.
void lambda_product(lrcc_ctx *c, const Vecs &p0, const Vecs &q, hipStream_t st) {
    const i64 n1 = (i64)c->nk * c->no * c->nv, n2 = (i64)c->nk * c->nk * c->nk * c->no * c->no * c->nv * c->nv;
    Program *adj = sigma_program(c, LRCC_FP64, 1, true);
    c->io_x1 = c->lam1; c->io_x2 = c->lam2; c->io_y1 = p0.s; c->io_y2 = p0.d; c->io_omega = nullptr;
    HIPCHK(adj->run(st));
    Program *rt = sigma_program(c, LRCC_FP64, 1, true, kRTermSigma);
    c->io_y1 = q.s; c->io_y2 = q.d;
    HIPCHK(rt->run(st));
    HIPCHK(scale_copy(q.s, q.s, -1.0, 0.0, n1, st));
    HIPCHK(scale_copy(q.d, q.d, -1.0, 0.0, n2, st));
    HIPCHK(add_inplace<double>(p0.s, q.s, n1, st));
    HIPCHK(add_inplace<double>(p0.d, q.d, n2, st));
    // the blocks linear in t2 alone at T, for the lean precompute of the stencil points: U as the
    // full precompute left it, the t2 term of W-bar formed alone in its (scratch) first-layout buffer
    const State<double> &S = c->s64;
    if (!c->linU_T) {
        c->linU_T = c->amem.get((size_t)c->n_U * 16);
        c->linU_y = c->amem.get((size_t)c->n_U * 16);
        c->linW_T = c->amem.get((size_t)c->n_Wraw * 16);
        c->linW_y = c->amem.get((size_t)c->n_Wraw * 16);
        c->lin_tmp = c->amem.get((size_t)c->n_Wraw * 16);
    }
    HIPCHK(hipMemcpyAsync(c->linU_T, S.U.p, (size_t)c->n_U * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(zero_fill<double>(c->pre64_Wraw, c->n_Wraw, st));
    HIPCHK(c->pre64->run_range(st, c->pre64_Wt.first, c->pre64_Wt.second));
    HIPCHK(hipMemcpyAsync(c->linW_T, c->pre64_Wraw, (size_t)c->n_Wraw * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    c->lin_T_ready = true;
}

// The density programs' amplitude copies are filled from the context's amplitudes by
// whole-array copies: refuse a mismatch (a state left from another shape) instead of
// writing past them.
void check_density_shape(lrcc_ctx *c) {
    const State<double> &S = c->s64;
    if (c->dT1.count() != S.t1.count() || c->dT2.count() != S.t2.count() || c->dT1.nk != c->nk ||
        c->dT1.no != c->no || c->dT1.nv != c->nv)
        throw LrccError(LRCC_E_STATE, "density buffers do not match the current amplitude shape");
}

// One-body density of R amplitude-space vectors a (caller layout, per-cell
// normalisation) with respect to the perturbation operator of Eq. rhs:
//   D_r[k][p][q] = d <a_r, xi^V> / d V[k][p][q]     (pairing sum a1 xi1 + 1/4 sum a2 xi2)
// at the amplitudes in (dT1, dT2).  xi^V is linear in V; the program is the
// transpose of the xi program term by term.  Reads io_x1/io_x2, writes
// io_y1 = D [R][nk][n][n].
Program *dens_program(lrcc_ctx *c, int R) {
    auto it = c->dens.find(R);
    if (it != c->dens.end()) return it->second.get();
    const int nk = c->nk, o = c->no, v = c->nv, n = c->n;
    if (!c->dT1.p) {
        c->dT1 = alloc_kt<double>(c, c->gmem, "ov");
        c->dT2 = alloc_kt<double>(c, c->gmem, "oovv");
    }
    check_density_shape(c);
    auto mem = std::make_unique<DevMem>();
    DevMem &m = *mem;
    auto P = std::make_unique<Program>();
    const KT &t1 = c->dT1, &t2 = c->dT2;
    KT a1 = alloc_kt<double>(c, m, "ov", R), Zb = alloc_kt<double>(c, m, "oovv", R);
    KT Fb = alloc_kt<double>(c, m, "vv", R), Gb = alloc_kt<double>(c, m, "oo", R), Yb = alloc_kt<double>(c, m, "vv", R);
    KT Xov = alloc_kt<double>(c, m, "ov", R), Xvv = alloc_kt<double>(c, m, "vv", R), Xoo = alloc_kt<double>(c, m, "oo", R);
    lrcc_ctx *cc = c;
    {
        void *pa = a1.p, *pz = Zb.p;
        P->ops.push_back([=](hipStream_t s) { return rhs_to_block<double, double>(cc->io_x1, pa, R, nk, (i64)o * v, 1.0, s); });
        // xi2 = Nk P(ij)P(ab) Z and the pairing weight 1/4: Z-bar = (Nk/4) P(ij)P(ab) a2
        P->ops.push_back([=](hipStream_t s) { return pp_in<double>(cc->io_x2, pz, cc->km, R, o, v, 0.25 * nk, s); });
    }
    // Z = 1/2 t2_ijac Fx_bc - 1/2 t2_ikab Gx_kj
    contract<double>(*P, Fb, "Rbc", Zb, "Rijab", t2, "ijac", 0.5, false);
    contract<double>(*P, Gb, "Rkj", Zb, "Rijab", t2, "ikab", -0.5, false);
    // singles: s1 = t2_ikac X_kc - t1_ic (t1_ka X_kc) + t1_ic X_ac - t1_ka X_ki + X_ai
    contract<double>(*P, Xov, "Rkc", a1, "Ria", t2, "ikac", 1.0, false);
    contract<double>(*P, Yb, "Rac", a1, "Ria", t1, "ic", -1.0, false);
    contract<double>(*P, Xov, "Rkc", Yb, "Rac", t1, "ka", 1.0);
    // Fx_bc = X_bc - t1_kb X_kc ; Gx_kj = X_kj + t1_jc X_kc
    contract<double>(*P, Xov, "Rkc", Fb, "Rbc", t1, "kb", -1.0);
    contract<double>(*P, Xov, "Rkc", Gb, "Rkj", t1, "jc", 1.0);
    kt_copy<double>(*P, Xvv, Fb);
    contract<double>(*P, Xvv, "Rac", a1, "Ria", t1, "ic", 1.0);
    kt_copy<double>(*P, Xoo, Gb);
    contract<double>(*P, Xoo, "Rki", a1, "Ria", t1, "ka", -1.0);
    {
        void *poo = Xoo.p, *pov = Xov.p, *pvv = Xvv.p, *pa = a1.p;
        P->ops.push_back([=](hipStream_t s) { return axis_scatter(poo, cc->io_y1, R, nk, n, 0, o, 0, o, 0, s); });
        P->ops.push_back([=](hipStream_t s) { return axis_scatter(pov, cc->io_y1, R, nk, n, 0, o, o, v, 0, s); });
        P->ops.push_back([=](hipStream_t s) { return axis_scatter(pvv, cc->io_y1, R, nk, n, o, v, o, v, 0, s); });
        P->ops.push_back([=](hipStream_t s) { return axis_scatter(pa, cc->io_y1, R, nk, n, 0, o, o, v, 1, s); });
    }
    Program *raw = P.get();
    c->dens[R] = std::move(P);
    c->densmem[R] = std::move(mem);
    return raw;
}

void solve_alpha(lrcc_ctx *c, unsigned axis_mask, int nfreq, const double *omega, const lrcc_solve_opts &o,
                 lrcc_solve_report &rep) {
    auto t0 = std::chrono::steady_clock::now();
    const int nk = c->nk, no = c->no, nv = c->nv, n = c->n;
    const i64 n1 = (i64)nk * no * nv, n2 = (i64)nk * nk * nk * no * no * nv * nv;
    ensure_alpha_programs(c);
    if (!c->own_stream) HIPCHK(hipStreamCreate(&c->own_stream));
    hipStream_t st = c->own_stream;
    double ph[3] = {0, 0, 0}, t_last = 0;
    auto phase = [&](int k, const char *what) {
        (void)hipStreamSynchronize(st);
        const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        ph[k] = t - t_last;
        t_last = t;
        if (verbose()) std::fprintf(stderr, "[lrcc] alpha: %s done at %.2f s\n", what, t);
    };
    // axes with a non-zero dipole (the paper skips vanishing components, Sec. II.B)
    std::vector<int> axes;
    {
        std::vector<double> d((size_t)3 * nk * n * n * 2);
        HIPCHK(hipMemcpy(d.data(), c->dip, d.size() * 8, hipMemcpyDeviceToHost));
        for (int x = 0; x < 3; ++x) {
            if (!(axis_mask & (1u << x))) continue;
            double mx = 0;
            for (size_t i = 0; i < (size_t)nk * n * n * 2; ++i) mx = std::max(mx, std::fabs(d[(size_t)x * nk * n * n * 2 + i]));
            if (mx > 1e-14) axes.push_back(x);
        }
    }
    const int nax = (int)axes.size();
    c->axes = axes;
    c->nfreq = nfreq;
    c->last_omega.assign(omega, omega + nfreq);
    c->alpha.assign((size_t)nfreq * 9 * 2, 0.0);
    rep = lrcc_solve_report{};
    if (nax == 0 || nfreq == 0) return;
    DevMem tmp;
    auto vec = [&](int R) { Vecs v; v.s = tmp.get((size_t)R * n1 * 16); v.d = tmp.get((size_t)R * n2 * 16); return v; };
    auto sub = [&](const Vecs &v, int r) { Vecs u; u.s = (char *)v.s + (size_t)r * n1 * 16; u.d = (char *)v.d + (size_t)r * n2 * 16; return u; };
    SolveCtx D;  // for bilinear dots
    D.c = c; D.R = 1; D.n1 = n1; D.n2 = n2; D.st = st;
    D.part = tmp.get((size_t)dot_blocks(n2) * 16 * 2);
    D.dout = tmp.get(32);
    D.alpha = tmp.get(32);
    auto bdot = [&](const Vecs &u, const Vecs &v) {
        cd a, b;
        HIPCHK(batched_dot(u.s, v.s, 1, n1, 1.0, D.part, D.dout, st, 0));
        HIPCHK(hipMemcpy(&a, D.dout, 16, hipMemcpyDeviceToHost));
        HIPCHK(batched_dot(u.d, v.d, 1, n2, 0.25, D.part, D.dout, st, 0));
        HIPCHK(hipMemcpy(&b, D.dout, 16, hipMemcpyDeviceToHost));
        return a + b;
    };
    void *zero_om = tmp.get(8 * 2);
    HIPCHK(hipMemset(zero_om, 0, 16));
    lrcc_solve_report r1{};
    Vecs lam{c->lam1, c->lam2};
    // lambda (once per set of amplitudes)
    if (!o.reuse_lambda) c->lam_valid = false;
    long long extra_rhs_sig = 0;
    if (!c->lam_valid) {
        HIPCHK(c->prog_grad->run(st));
        HIPCHK(hipMemset(c->lam1, 0, n1 * 16));
        HIPCHK(hipMemset(c->lam2, 0, n2 * 16));
        Vecs b{c->gb1, c->gb2};
        // one right-hand side: launch-latency bound, so complex128 throughout (the complex64
        // corrections only add refinement steps here)
        lrcc_solve_opts ol = o;
        ol.precision = LRCC_FP64;
        bool sing = false;
        solve_response(c, 1, (const double *)zero_om, b, lam, ol, r1, st, true, true, &sing);
        if (!r1.converged) {
            rep = r1;
            throw_unconverged("lambda equations", r1, sing);
        }
        c->lam_valid = true;
    }
    phase(0, "lambda");
    // perturbation vectors and the batched response solve: rhs r = (j*2 + sign)*nax + a
    HIPCHK(c->prog_xi->run(st));
    const int R = nfreq * 2 * nax;
    c->solv.release();
    c->sol1 = c->solv.get((size_t)R * n1 * 16);
    c->sol2 = c->solv.get((size_t)R * n2 * 16);
    Vecs X{c->sol1, c->sol2};
    Vecs B = vec(R);
    std::vector<double> om(R);
    for (int j = 0; j < nfreq; ++j)
        for (int sg = 0; sg < 2; ++sg)
            for (int a = 0; a < nax; ++a) {
                const int r = (j * 2 + sg) * nax + a;
                om[r] = sg == 0 ? omega[j] : -omega[j];
                Vecs xi{(char *)c->xi1 + (size_t)axes[a] * n1 * 16, (char *)c->xi2 + (size_t)axes[a] * n2 * 16};
                Vecs br = sub(B, r);
                HIPCHK(scale_copy(br.s, xi.s, -1.0, 0.0, n1, st));
                HIPCHK(scale_copy(br.d, xi.d, -1.0, 0.0, n2, st));
            }
    void *dom = tmp.get((size_t)R * 8);
    HIPCHK(hipMemcpy(dom, om.data(), R * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(X.s, 0, (size_t)R * n1 * 16));
    HIPCHK(hipMemset(X.d, 0, (size_t)R * n2 * 16));
    // initial guesses (lrcc_set_guess) for the solved axes and frequencies; all are consumed
    bool guessed = false;
    for (const auto &gs : c->guess) {
        const int ax = gs.first[0], j = gs.first[1], sg = gs.first[2];
        const int a = (int)(std::find(axes.begin(), axes.end(), ax) - axes.begin());
        if (a >= nax || j >= nfreq) continue;
        const Vecs dst = sub(X, (j * 2 + (sg > 0 ? 0 : 1)) * nax + a);
        const char *src = (const char *)gs.second->ptrs[0];
        HIPCHK(hipMemcpyAsync(dst.s, src, (size_t)n1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(dst.d, src + (size_t)n1 * 16, (size_t)n2 * 16, hipMemcpyDeviceToDevice, st));
        guessed = true;
    }
    HIPCHK(hipStreamSynchronize(st));
    c->guess.clear();
    lrcc_solve_report r2{};
    bool sing = false;
    solve_response(c, R, (const double *)dom, B, X, o, r2, st, false, !guessed, &sing);
    c->nrhs_sol = R;
    if (!r2.converged) {
        rep = r2;
        rep.sigma_fp64 += r1.sigma_fp64;
        rep.sigma_fp32 += r1.sigma_fp32;
        rep.rhs_sigmas += r1.rhs_sigmas;
        c->nfreq = 0;   // no polarizability from unconverged amplitudes
        throw_unconverged("response equations", r2, sing);
    }
    // eta^X = A_X^T lambda + (X_ov, 0)
    std::vector<Vecs> eta(nax);
    for (int a = 0; a < nax; ++a) {
        eta[a] = vec(1);
        eta_vector(c, axes[a], eta[a], st);
    }
    phase(1, "response");
    // eta . t for every axis and solution
    std::vector<cd> et((size_t)nax * R);
    for (int a = 0; a < nax; ++a)
        for (int r = 0; r < R; ++r) et[(size_t)a * R + r] = bdot(eta[a], sub(X, r));
    // F(t^X(-w), t^Y(+w)) by the exact stencil in T along y = t^Y(+w)
    std::vector<cd> Fv((size_t)nfreq * nax * nax);
    {
        State<double> &S = c->s64;
        const i64 nt1 = S.t1.count(), nt2 = S.t2.count();
        void *T1 = tmp.get(nt1 * 16), *T2 = tmp.get(nt2 * 16);
        HIPCHK(hipMemcpy(T1, S.t1.p, nt1 * 16, hipMemcpyDeviceToDevice));
        HIPCHK(hipMemcpy(T2, S.t2.p, nt2 * 16, hipMemcpyDeviceToDevice));
        Vecs Fy = vec(1), q = vec(1), p0 = vec(1);
        lambda_product(c, p0, q, st);
        ++extra_rhs_sig;
        for (int j = 0; j < nfreq; ++j)
            for (int b = 0; b < nax; ++b) {
                f_vector(c, D, sub(X, (j * 2 + 0) * nax + b), Fy, q, T1, T2, st, &p0);
                extra_rhs_sig += 3;
                for (int a = 0; a < nax; ++a) Fv[((size_t)j * nax + a) * nax + b] = bdot(Fy, sub(X, (j * 2 + 1) * nax + a));
            }
        HIPCHK(hipMemcpy(S.t1.p, T1, nt1 * 16, hipMemcpyDeviceToDevice));
        HIPCHK(hipMemcpy(S.t2.p, T2, nt2 * 16, hipMemcpyDeviceToDevice));
        run_precompute(c, true, st);
    }
    phase(2, "eta and F");
    // assemble alpha
    auto rid = [&](int j, int sg, int a) { return (j * 2 + sg) * nax + a; };
    for (int j = 0; j < nfreq; ++j)
        for (int a = 0; a < nax; ++a)
            for (int b = 0; b < nax; ++b) {
                // g(X,Y,+) = eta^X t^Y(w) + eta^Y t^X(-w) + F(t^X(-w), t^Y(w))
                cd gp = et[(size_t)a * R + rid(j, 0, b)] + et[(size_t)b * R + rid(j, 1, a)] + Fv[((size_t)j * nax + a) * nax + b];
                // g(X,Y,-) = eta^X t^Y(-w) + eta^Y t^X(w) + F(t^X(w), t^Y(-w)) ; F symmetric
                cd gm = et[(size_t)a * R + rid(j, 1, b)] + et[(size_t)b * R + rid(j, 0, a)] + Fv[((size_t)j * nax + b) * nax + a];
                cd al = -0.5 * (gp + std::conj(gm)) / (double)nk;
                const size_t idx = ((size_t)j * 9 + axes[a] * 3 + axes[b]) * 2;
                c->alpha[idx] = al.real();
                c->alpha[idx + 1] = al.imag();
            }
    rep.converged = 1;
    rep.outer = r2.outer;
    rep.sigma_fp64 = r1.sigma_fp64 + r2.sigma_fp64;
    rep.sigma_fp32 = r1.sigma_fp32 + r2.sigma_fp32;
    rep.max_rel_residual = std::max(r1.max_rel_residual, r2.max_rel_residual);
    rep.rhs_sigmas = r1.rhs_sigmas + r2.rhs_sigmas + extra_rhs_sig;
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < 3; ++k) rep.phase_seconds[k] = ph[k];
}


// ---------------------------------------------------------------- non-symmetric (lambda-bar) form of alpha
// With the perturbed multipliers lambda-bar^Y(s w) = (A + s w)^-T (eta^Y + F(., t^Y(s w)))
// (one batched transpose solve over all axes, frequencies and signs), the response
// function needs the amplitudes of one operator only:
//   g_XY(s w) = eta^X t^Y(s w) - <lambda-bar^Y(s w), xi^X>,
//   alpha_XY(w) = -1/(2 Nk) [g_XY(w) + conj(g_XY(-w))],
// which equals the symmetric form for exact solutions (the identity the two
// formulations share; it checks the F term and the transpose solver).
void alpha_lambda_bar(lrcc_ctx *c, const lrcc_solve_opts &o, double *out, lrcc_solve_report &rep) {
    auto t0 = std::chrono::steady_clock::now();
    const int nk = c->nk, no = c->no, nv = c->nv;
    const i64 n1 = (i64)nk * no * nv, n2 = (i64)nk * nk * nk * no * no * nv * nv;
    const auto &axes = c->axes;
    const int nax = (int)axes.size(), nfreq = c->nfreq;
    if (!c->lam_valid || !c->sol1 || c->nrhs_sol != nfreq * 2 * nax || nax == 0)
        throw LrccError(LRCC_E_STATE, "lrcc_solve must precede the lambda-bar form");
    hipStream_t st = c->own_stream;
    const int R = nfreq * 2 * nax;
    DevMem tmp;
    auto vec = [&](int r) { Vecs v; v.s = tmp.get((size_t)r * n1 * 16); v.d = tmp.get((size_t)r * n2 * 16); return v; };
    auto sub = [&](const Vecs &v, int r) { Vecs u; u.s = (char *)v.s + (size_t)r * n1 * 16; u.d = (char *)v.d + (size_t)r * n2 * 16; return u; };
    Vecs X{c->sol1, c->sol2};
    SolveCtx D;
    D.c = c; D.R = 1; D.n1 = n1; D.n2 = n2; D.st = st;
    D.part = tmp.get((size_t)dot_blocks(n2) * 16 * 2);
    D.dout = tmp.get(32);
    D.alpha = tmp.get(32);
    auto bdot = [&](const Vecs &u, const Vecs &v) {
        cd a, b;
        HIPCHK(batched_dot(u.s, v.s, 1, n1, 1.0, D.part, D.dout, st, 0));
        HIPCHK(hipMemcpy(&a, D.dout, 16, hipMemcpyDeviceToHost));
        HIPCHK(batched_dot(u.d, v.d, 1, n2, 0.25, D.part, D.dout, st, 0));
        HIPCHK(hipMemcpy(&b, D.dout, 16, hipMemcpyDeviceToHost));
        return a + b;
    };
    // right-hand sides, in the layout of the solutions: r = (j*2 + sign)*nax + a
    std::vector<Vecs> eta(nax);
    for (int a = 0; a < nax; ++a) { eta[a] = vec(1); eta_vector(c, axes[a], eta[a], st); }
    Vecs B = vec(R), Lb = vec(R);
    std::vector<double> om(R);
    {
        State<double> &S = c->s64;
        const i64 nt1 = S.t1.count(), nt2 = S.t2.count();
        void *T1 = tmp.get(nt1 * 16), *T2 = tmp.get(nt2 * 16);
        HIPCHK(hipMemcpyAsync(T1, S.t1.p, nt1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(T2, S.t2.p, nt2 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        Vecs q = vec(1), p0 = vec(1);
        lambda_product(c, p0, q, st);
        for (int j = 0; j < nfreq; ++j)
            for (int sg = 0; sg < 2; ++sg)
                for (int a = 0; a < nax; ++a) {
                    const int r = (j * 2 + sg) * nax + a;
                    // (A + s w)^T: the solver applies (A - omega_r)^T
                    om[r] = sg == 0 ? -c->last_omega[j] : c->last_omega[j];
                    Vecs b = sub(B, r);
                    f_vector(c, D, sub(X, r), b, q, T1, T2, st, &p0);
                    HIPCHK(add_inplace<double>(b.s, eta[a].s, n1, st));
                    HIPCHK(add_inplace<double>(b.d, eta[a].d, n2, st));
                }
        HIPCHK(hipMemcpyAsync(S.t1.p, T1, nt1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(S.t2.p, T2, nt2 * 16, hipMemcpyDeviceToDevice, st));
        run_precompute(c, true, st);
    }
    void *dom = tmp.get((size_t)R * 8);
    HIPCHK(hipMemcpy(dom, om.data(), R * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(Lb.s, 0, (size_t)R * n1 * 16));
    HIPCHK(hipMemset(Lb.d, 0, (size_t)R * n2 * 16));
    bool sing = false;
    solve_response(c, R, (const double *)dom, B, Lb, o, rep, st, true, true, &sing);
    if (!rep.converged) throw_unconverged("perturbed lambda equations", rep, sing);
    std::vector<double> al((size_t)nfreq * 9 * 2, 0.0);
    for (int j = 0; j < nfreq; ++j)
        for (int x = 0; x < nax; ++x)
            for (int y = 0; y < nax; ++y) {
                cd g[2];
                for (int sg = 0; sg < 2; ++sg) {
                    const int ry = (j * 2 + sg) * nax + y;
                    Vecs xi{(char *)c->xi1 + (size_t)axes[x] * n1 * 16, (char *)c->xi2 + (size_t)axes[x] * n2 * 16};
                    g[sg] = bdot(eta[x], sub(X, ry)) - bdot(sub(Lb, ry), xi);
                }
                const cd v = -0.5 * (g[0] + std::conj(g[1])) / (double)nk;
                const size_t idx = ((size_t)j * 9 + axes[x] * 3 + axes[y]) * 2;
                al[idx] = v.real();
                al[idx + 1] = v.imag();
            }
    std::memcpy(out, al.data(), al.size() * 8);
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------- dipole gradient of alpha
// alpha_XY(w) = -1/(2 Nk) [g(w) + conj(g(-w))],
//   g(w) = eta^X t^Y(w) + eta^Y t^X(-w) + F(t^X(-w), t^Y(w)),  t^Z(w) = -(A - w)^-1 xi^Z.
// It is bilinear in (mu_X, mu_Y) at fixed amplitudes and lambda.  Along a
// perturbation V of mu_X, with a = (A + w)^-T (eta^Y + F(., t^Y(w))):
//   d g(w) = eta^V t^Y(w) - <a, xi^V>,
// and symmetrically for mu_Y and for g(-w).  <a, xi^V> and eta^V t are linear
// in V: the density program gives them as one-body densities (eta^V t =
// d/de <lambda, xi^V(T + e t)> + V_ov t1, the derivative exact by central
// difference since xi is quadratic in T).  The conjugated g(-w) contributes
// conj(G[k][q][p]) for Hermitian V.
void alpha_dip_grad(lrcc_ctx *c, int j, int X, int Y, const lrcc_solve_opts &o, double *out) {
    const int nk = c->nk, no = c->no, nv = c->nv, n = c->n;
    const i64 n1 = (i64)nk * no * nv, n2 = (i64)nk * nk * nk * no * no * nv * nv;
    const auto &axes = c->axes;
    const int nax = (int)axes.size();
    if (j < 0 || j >= c->nfreq || (int)c->last_omega.size() != c->nfreq)
        throw LrccError(LRCC_E_ARG, "frequency index out of range of the last solve");
    const int ax = (int)(std::find(axes.begin(), axes.end(), X) - axes.begin());
    const int ay = (int)(std::find(axes.begin(), axes.end(), Y) - axes.begin());
    if (ax >= nax || ay >= nax) throw LrccError(LRCC_E_ARG, "axis not solved in the last solve (zero dipole or masked)");
    if (!c->lam_valid || !c->sol1 || c->nrhs_sol != c->nfreq * 2 * nax)
        throw LrccError(LRCC_E_STATE, "lrcc_solve must precede the gradient");
    hipStream_t st = c->own_stream;
    const double w = c->last_omega[j];
    DevMem tmp;
    auto vec = [&](int R) { Vecs v; v.s = tmp.get((size_t)R * n1 * 16); v.d = tmp.get((size_t)R * n2 * 16); return v; };
    auto sub = [&](const Vecs &v, int r) { Vecs u; u.s = (char *)v.s + (size_t)r * n1 * 16; u.d = (char *)v.d + (size_t)r * n2 * 16; return u; };
    Vecs sol{c->sol1, c->sol2};
    auto tsol = [&](int sg, int a) { return sub(sol, (j * 2 + sg) * nax + a); };  // sg 0: +w, 1: -w
    SolveCtx D;
    D.c = c; D.R = 1; D.n1 = n1; D.n2 = n2; D.st = st;
    D.part = tmp.get((size_t)dot_blocks(n2) * 16 * 2);
    D.dout = tmp.get(32);
    D.alpha = tmp.get(32);
    // the four adjoint right-hand sides (two when X == Y): slot, vector t, eta axis, solve frequency
    //   0: mu_X in g(w):  eta^Y + F(., t^Y(w)),   (A + w)^T       uses eta^V t^Y(w)
    //   1: mu_X in g(-w): eta^Y + F(., t^Y(-w)),  (A - w)^T       uses eta^V t^Y(-w)
    //   2: mu_Y in g(w):  eta^X + F(., t^X(-w)),  (A - w)^T       uses eta^V t^X(-w)
    //   3: mu_Y in g(-w): eta^X + F(., t^X(w)),   (A + w)^T       uses eta^V t^X(w)
    const bool same = X == Y;
    const int nb = same ? 2 : 4;
    Vecs tv[4] = {tsol(0, ay), tsol(1, ay), tsol(1, ax), tsol(0, ax)};
    const int eta_ax[4] = {Y, Y, X, X};
    const double wsolve[4] = {-w, w, w, -w};
    Vecs B = vec(nb), A = vec(nb);
    {
        Vecs etaY = vec(1), etaX = same ? etaY : vec(1);
        eta_vector(c, Y, etaY, st);
        if (!same) eta_vector(c, X, etaX, st);
        State<double> &S = c->s64;
        const i64 nt1 = S.t1.count(), nt2 = S.t2.count();
        void *T1 = tmp.get(nt1 * 16), *T2 = tmp.get(nt2 * 16);
        HIPCHK(hipMemcpyAsync(T1, S.t1.p, nt1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(T2, S.t2.p, nt2 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        Vecs q = vec(1), p0 = vec(1);
        lambda_product(c, p0, q, st);
        for (int b = 0; b < nb; ++b) {
            Vecs bb = sub(B, b);
            f_vector(c, D, tv[b], bb, q, T1, T2, st, &p0);
            HIPCHK(add_inplace<double>(bb.s, (eta_ax[b] == Y ? etaY : etaX).s, n1, st));
            HIPCHK(add_inplace<double>(bb.d, (eta_ax[b] == Y ? etaY : etaX).d, n2, st));
        }
        HIPCHK(hipMemcpyAsync(S.t1.p, T1, nt1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(S.t2.p, T2, nt2 * 16, hipMemcpyDeviceToDevice, st));
        run_precompute(c, true, st);
    }
    void *dom = tmp.get((size_t)nb * 8);
    HIPCHK(hipMemcpy(dom, wsolve, nb * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(A.s, 0, (size_t)nb * n1 * 16));
    HIPCHK(hipMemset(A.d, 0, (size_t)nb * n2 * 16));
    lrcc_solve_report r{};
    bool sing = false;
    solve_response(c, nb, (const double *)dom, B, A, o, r, st, true, true, &sing);
    if (!r.converged) throw_unconverged("adjoint response equations", r, sing);
    // densities: D_xi of the adjoint vectors at T, D_eta of the response vectors
    State<double> &S = c->s64;
    const i64 nt1 = S.t1.count(), nt2 = S.t2.count();
    const size_t nd = (size_t)nk * n * n;
    void *dd = tmp.get((size_t)nb * nd * 16);
    Program *dn = dens_program(c, nb), *d1 = dens_program(c, 1);   // (allocate dT1, dT2 on first use)
    check_density_shape(c);
    HIPCHK(hipMemcpyAsync(c->dT1.p, S.t1.p, nt1 * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(c->dT2.p, S.t2.p, nt2 * 16, hipMemcpyDeviceToDevice, st));
    c->io_x1 = A.s; c->io_x2 = A.d; c->io_y1 = dd;
    HIPCHK(dn->run(st));
    std::vector<cd> Dxi((size_t)nb * nd), Deta((size_t)nb * nd, 0.0), tmpd(nd);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(Dxi.data(), dd, Dxi.size() * 16, hipMemcpyDeviceToHost));
    std::vector<cd> t1h((size_t)n1);
    for (int b = 0; b < nb; ++b) {
        const Vecs &t = tv[b];
        cd yy = 0;
        {
            SolveCtx N = D;
            N.R = 1;
            yy = N.dot(t, t)[0];
        }
        const double rms = std::sqrt(std::max(yy.real(), 1e-300) / (double)(n1 + n2 / 4));
        const double h = 1e-2 / rms;
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            HIPCHK(hipMemcpyAsync(c->dT1.p, S.t1.p, nt1 * 16, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(c->dT2.p, S.t2.p, nt2 * 16, hipMemcpyDeviceToDevice, st));
            std::vector<cd> a1(1, cd(sgn * h, 0.0)), a2(1, cd(sgn * h / nk, 0.0));
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipMemcpy(D.alpha, a1.data(), 16, hipMemcpyHostToDevice));
            HIPCHK(batched_axpby(c->dT1.p, t.s, D.alpha, 1.0, 1, nt1, st));
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipMemcpy(D.alpha, a2.data(), 16, hipMemcpyHostToDevice));
            HIPCHK(batched_axpby(c->dT2.p, t.d, D.alpha, 1.0, 1, nt2, st));
            c->io_x1 = c->lam1; c->io_x2 = c->lam2; c->io_y1 = dd;
            HIPCHK(d1->run(st));
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipMemcpy(tmpd.data(), dd, nd * 16, hipMemcpyDeviceToHost));
            for (size_t e = 0; e < nd; ++e) Deta[(size_t)b * nd + e] += (sgn / (2.0 * h)) * tmpd[e];
        }
        // (V_ov, 0) part of eta: + V[k][i][o+a] t1[k][i][a]
        HIPCHK(hipMemcpy(t1h.data(), t.s, n1 * 16, hipMemcpyDeviceToHost));
        for (int k = 0; k < nk; ++k)
            for (int i = 0; i < no; ++i)
                for (int a = 0; a < nv; ++a)
                    Deta[(size_t)b * nd + ((size_t)k * n + i) * n + no + a] += t1h[((size_t)k * no + i) * nv + a];
    }
    // assemble: grad[Z][k][p][q] = -1/(2Nk) (G+[k][p][q] + conj(G-[k][q][p])), G = D_eta - D_xi
    std::vector<cd> g((size_t)3 * nd, 0.0);
    auto G = [&](int b, int k, int p, int qq) {
        const size_t e = (size_t)b * nd + ((size_t)k * n + p) * n + qq;
        return Deta[e] - Dxi[e];
    };
    const int slot_ax[2] = {X, Y};
    for (int sl = 0; sl < 2; ++sl) {
        // slot 0 (mu_X): vectors 0 (g(w)) and 1 (g(-w)); slot 1 (mu_Y): 2 and 3, or 1 and 0 when X == Y
        const int bp = sl == 0 ? 0 : (same ? 1 : 2), bm = sl == 0 ? 1 : (same ? 0 : 3);
        for (int k = 0; k < nk; ++k)
            for (int p = 0; p < n; ++p)
                for (int qq = 0; qq < n; ++qq)
                    g[(size_t)slot_ax[sl] * nd + ((size_t)k * n + p) * n + qq] +=
                        -0.5 / nk * (G(bp, k, p, qq) + std::conj(G(bm, k, qq, p)));
    }
    std::memcpy(out, g.data(), g.size() * 16);
}

// ---------------------------------------------------------------- Fock-matrix gradient of alpha
// Helpers: the one-body density of u at shifted amplitudes, and the vector
// Omega''[x, y] (second derivative of the residual along x and y).
//
// Shifted amplitudes T + sx x + sy y into the density program's copy (crystal T2).
void dens_shift(lrcc_ctx *c, SolveCtx &D, const Vecs *x, double sx, const Vecs *y, double sy, hipStream_t st) {
    check_density_shape(c);
    State<double> &S = c->s64;
    const i64 nt1 = S.t1.count(), nt2 = S.t2.count();
    const int nk = c->nk;
    HIPCHK(hipMemcpyAsync(c->dT1.p, S.t1.p, nt1 * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(c->dT2.p, S.t2.p, nt2 * 16, hipMemcpyDeviceToDevice, st));
    const Vecs *v[2] = {x, y};
    const double sc[2] = {sx, sy};
    for (int i = 0; i < 2; ++i) {
        if (!v[i]) continue;
        std::vector<cd> a1(1, cd(sc[i], 0.0)), a2(1, cd(sc[i] / nk, 0.0));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(D.alpha, a1.data(), 16, hipMemcpyHostToDevice));
        HIPCHK(batched_axpby(c->dT1.p, v[i]->s, D.alpha, 1.0, 1, nt1, st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(D.alpha, a2.data(), 16, hipMemcpyHostToDevice));
        HIPCHK(batched_axpby(c->dT2.p, v[i]->d, D.alpha, 1.0, 1, nt2, st));
    }
}

// D_xi(u; T + sx x + sy y) on the host, [nk][n][n]
std::vector<cd> density_at(lrcc_ctx *c, SolveCtx &D, const Vecs &u, const Vecs *x, double sx, const Vecs *y,
                           double sy, void *dd, hipStream_t st) {
    Program *d1 = dens_program(c, 1);
    dens_shift(c, D, x, sx, y, sy, st);
    c->io_x1 = u.s; c->io_x2 = u.d; c->io_y1 = dd;
    HIPCHK(d1->run(st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<cd> h((size_t)c->nk * c->n * c->n);
    HIPCHK(hipMemcpy(h.data(), dd, h.size() * 16, hipMemcpyDeviceToHost));
    return h;
}

double step_for(SolveCtx &D, const Vecs &t) {
    SolveCtx N = D;
    N.R = 1;
    const cd tt = N.dot(t, t)[0];
    const double rms = std::sqrt(std::max(tt.real(), 1e-300) / (double)(D.n1 + D.n2 / 4));
    return 1e-2 / rms;
}

// d/de D_xi(u; T + e t): exact central difference (xi is quadratic in T)
std::vector<cd> density_d1(lrcc_ctx *c, SolveCtx &D, const Vecs &u, const Vecs &t, void *dd, hipStream_t st) {
    const double h = step_for(D, t);
    auto p = density_at(c, D, u, &t, h, nullptr, 0, dd, st), m = density_at(c, D, u, &t, -h, nullptr, 0, dd, st);
    for (size_t e = 0; e < p.size(); ++e) p[e] = (p[e] - m[e]) / (2.0 * h);
    return p;
}

// d2/de dd D_xi(u; T + e x + d y): exact four-point mixed difference
std::vector<cd> density_d2(lrcc_ctx *c, SolveCtx &D, const Vecs &u, const Vecs &x, const Vecs &y, void *dd,
                           hipStream_t st) {
    const double hx = step_for(D, x), hy = step_for(D, y);
    auto pp = density_at(c, D, u, &x, hx, &y, hy, dd, st), pm = density_at(c, D, u, &x, hx, &y, -hy, dd, st);
    auto mp = density_at(c, D, u, &x, -hx, &y, hy, dd, st), mm = density_at(c, D, u, &x, -hx, &y, -hy, dd, st);
    for (size_t e = 0; e < pp.size(); ++e) pp[e] = (pp[e] - pm[e] - mp[e] + mm[e]) / (4.0 * hx * hy);
    return pp;
}

// out = Omega''[x, y] = d/de A(T + e x) y: the forward product is cubic in T, so the
// 5-point derivative is exact.  Leaves the amplitudes shifted (caller restores).
void omega2_vector(lrcc_ctx *c, SolveCtx &D, const Vecs &x, const Vecs &y, const Vecs &out, const Vecs &q,
                   const void *T1, const void *T2, hipStream_t st) {
    const int nk = c->nk;
    const i64 n1 = D.n1, n2 = D.n2;
    State<double> &S = c->s64;
    const i64 nt1 = S.t1.count(), nt2 = S.t2.count();
    Program *fwd = sigma_program(c, LRCC_FP64, 1, false);
    const double coef[4] = {1.0, -8.0, 8.0, -1.0};
    const int shift[4] = {-2, -1, 1, 2};
    const double h = step_for(D, x);
    HIPCHK(hipMemsetAsync(out.s, 0, n1 * 16, st));
    HIPCHK(hipMemsetAsync(out.d, 0, n2 * 16, st));
    for (int k = 0; k < 4; ++k) {
        HIPCHK(hipMemcpyAsync(S.t1.p, T1, nt1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(S.t2.p, T2, nt2 * 16, hipMemcpyDeviceToDevice, st));
        std::vector<cd> a1(1, cd(shift[k] * h, 0.0)), a2(1, cd(shift[k] * h / nk, 0.0));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(D.alpha, a1.data(), 16, hipMemcpyHostToDevice));
        HIPCHK(batched_axpby(S.t1.p, x.s, D.alpha, 1.0, 1, nt1, st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(D.alpha, a2.data(), 16, hipMemcpyHostToDevice));
        HIPCHK(batched_axpby(S.t2.p, x.d, D.alpha, 1.0, 1, nt2, st));
        run_precompute(c, false, st);
        c->io_x1 = y.s; c->io_x2 = y.d; c->io_y1 = q.s; c->io_y2 = q.d; c->io_omega = nullptr;
        HIPCHK(fwd->run(st));
        std::vector<cd> wv(1, cd(coef[k] / (12.0 * h), 0.0));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(D.alpha, wv.data(), 16, hipMemcpyHostToDevice));
        HIPCHK(batched_axpby(out.s, q.s, D.alpha, 1.0, 1, n1, st));
        HIPCHK(batched_axpby(out.d, q.d, D.alpha, 1.0, 1, n2, st));
        HIPCHK(hipStreamSynchronize(st));
    }
}

// d alpha_XY(w_j) / d f at fixed amplitudes, lambda re-solved (it depends on f).
// Every f-dependence is linear (the residual is linear in f), with the one-body
// part of the residual being xi^f(T) (quadratic in T).  With a the transpose
// solutions of the dipole gradient and z = A^-1 w, w = A_X t^Y + A_Y t^X(-w) +
// Omega''[t^X(-w), t^Y(w)] (the lambda-sensitivity of eta and F):
//   d g(w) = - <a_Y, dA t^Y(w)> - <a_X, dA t^X(-w)> - <lambda, dA z> - <dg, z>
//            + <lambda, dOmega''[t^X(-w), t^Y(w)]>,     dg = (df_ov, 0),
// where <u, dA t> = d/de D_xi(u; T + e t) . df and the last term is the mixed
// second derivative of D_xi(lambda; .) . df.  g(-w) likewise, conjugated.
// The adjoint vectors of a polarizability gradient at frequency index j (shared by the Fock and
// Cholesky gradients): the four transpose solutions
//   A[0] = (A + w)^-T (eta^Y + F(., t^Y(w))),   A[1] = (A - w)^-T (eta^Y + F(., t^Y(-w))),
//   A[2] = (A - w)^-T (eta^X + F(., t^X(-w))),  A[3] = (A + w)^-T (eta^X + F(., t^X(w))),
// and the lambda sensitivities Z[sg] = A^-1 w(sg), w(+) = Omega''[t^X(-w), t^Y(w)] + A_X t^Y(w)
// + A_Y t^X(-w) (w(-) with w -> -w).  Allocated in tmp; D is a one-vector dot context.
struct GradAdjoints {
    Vecs A, Z;
    int ax = 0, ay = 0, nax = 0;
};

GradAdjoints grad_adjoints(lrcc_ctx *c, int j, int X, int Y, const lrcc_solve_opts &o, DevMem &tmp, SolveCtx &D) {
    const int nk = c->nk, no = c->no, nv = c->nv;
    const i64 n1 = (i64)nk * no * nv, n2 = (i64)nk * nk * nk * no * no * nv * nv;
    const auto &axes = c->axes;
    const int nax = (int)axes.size();
    if (j < 0 || j >= c->nfreq || (int)c->last_omega.size() != c->nfreq)
        throw LrccError(LRCC_E_ARG, "frequency index out of range of the last solve");
    const int ax = (int)(std::find(axes.begin(), axes.end(), X) - axes.begin());
    const int ay = (int)(std::find(axes.begin(), axes.end(), Y) - axes.begin());
    if (ax >= nax || ay >= nax) throw LrccError(LRCC_E_ARG, "axis not solved in the last solve (zero dipole or masked)");
    if (!c->lam_valid || !c->sol1 || c->nrhs_sol != c->nfreq * 2 * nax)
        throw LrccError(LRCC_E_STATE, "lrcc_solve must precede the gradient");
    hipStream_t st = c->own_stream;
    const double w = c->last_omega[j];
    auto vec = [&](int R) { Vecs v; v.s = tmp.get((size_t)R * n1 * 16); v.d = tmp.get((size_t)R * n2 * 16); return v; };
    auto sub = [&](const Vecs &v, int r) { Vecs u; u.s = (char *)v.s + (size_t)r * n1 * 16; u.d = (char *)v.d + (size_t)r * n2 * 16; return u; };
    Vecs sol{c->sol1, c->sol2};
    auto tsol = [&](int sg, int a) { return sub(sol, (j * 2 + sg) * nax + a); };  // sg 0: +w, 1: -w
    D.c = c; D.R = 1; D.n1 = n1; D.n2 = n2; D.st = st;
    D.part = tmp.get((size_t)dot_blocks(n2) * 16 * 2);
    D.dout = tmp.get(32);
    D.alpha = tmp.get(32);
    (void)dens_program(c, 1);   // allocates the density program's amplitude copy
    Vecs tv[4] = {tsol(0, ay), tsol(1, ay), tsol(1, ax), tsol(0, ax)};
    const bool same = X == Y;
    const double wsolve[4] = {-w, w, w, -w};
    GradAdjoints G;
    G.ax = ax; G.ay = ay; G.nax = nax;
    Vecs B = vec(4), W = vec(2);
    G.A = vec(4);
    G.Z = vec(2);
    {
        Vecs etaY = vec(1), etaX = same ? etaY : vec(1);
        eta_vector(c, Y, etaY, st);
        if (!same) eta_vector(c, X, etaX, st);
        State<double> &S = c->s64;
        const i64 nt1 = S.t1.count(), nt2 = S.t2.count();
        void *T1 = tmp.get(nt1 * 16), *T2 = tmp.get(nt2 * 16);
        HIPCHK(hipMemcpyAsync(T1, S.t1.p, nt1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(T2, S.t2.p, nt2 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        Vecs q = vec(1), p0 = vec(1);
        lambda_product(c, p0, q, st);
        for (int b = 0; b < 4; ++b) {
            Vecs bb = sub(B, b);
            f_vector(c, D, tv[b], bb, q, T1, T2, st, &p0);
            const Vecs &e = b < 2 ? etaY : etaX;
            HIPCHK(add_inplace<double>(bb.s, e.s, n1, st));
            HIPCHK(add_inplace<double>(bb.d, e.d, n2, st));
        }
        // w(+) = Omega''[t^X(-w), t^Y(w)] + A_X t^Y(w) + A_Y t^X(-w);  w(-) with w -> -w
        for (int sg = 0; sg < 2; ++sg) {
            const Vecs tx = tsol(1 - sg, ax), ty = tsol(sg, ay);
            omega2_vector(c, D, tx, ty, sub(W, sg), q, T1, T2, st);
        }
        HIPCHK(hipMemcpyAsync(S.t1.p, T1, nt1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(S.t2.p, T2, nt2 * 16, hipMemcpyDeviceToDevice, st));
        run_precompute(c, true, st);
        for (int sg = 0; sg < 2; ++sg) {
            const Vecs tx = tsol(1 - sg, ax), ty = tsol(sg, ay);
            const int pa[2] = {X, Y};
            const Vecs vin[2] = {ty, tx};
            for (int k = 0; k < 2; ++k) {
                HIPCHK(c->prex[pa[k]]->run(st));
                Program *p = sigma_program(c, LRCC_FP64, 1, false, 1 + pa[k]);
                c->io_x1 = vin[k].s; c->io_x2 = vin[k].d; c->io_y1 = q.s; c->io_y2 = q.d; c->io_omega = nullptr;
                HIPCHK(p->run(st));
                HIPCHK(add_inplace<double>(sub(W, sg).s, q.s, n1, st));
                HIPCHK(add_inplace<double>(sub(W, sg).d, q.d, n2, st));
            }
        }
    }
    void *dom = tmp.get(4 * 8), *zom = tmp.get(2 * 8);
    HIPCHK(hipMemcpy(dom, wsolve, 4 * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(zom, 0, 2 * 8));
    HIPCHK(hipMemset(G.A.s, 0, (size_t)4 * n1 * 16));
    HIPCHK(hipMemset(G.A.d, 0, (size_t)4 * n2 * 16));
    HIPCHK(hipMemset(G.Z.s, 0, (size_t)2 * n1 * 16));
    HIPCHK(hipMemset(G.Z.d, 0, (size_t)2 * n2 * 16));
    lrcc_solve_report r{};
    bool sing = false;
    solve_response(c, 4, (const double *)dom, B, G.A, o, r, st, true, true, &sing);
    if (!r.converged) throw_unconverged("adjoint response equations", r, sing);
    solve_response(c, 2, (const double *)zom, W, G.Z, o, r, st, false, true, &sing);
    if (!r.converged) throw_unconverged("lambda-sensitivity equations", r, sing);
    return G;
}

void alpha_fock_grad(lrcc_ctx *c, int j, int X, int Y, const lrcc_solve_opts &o, double *out) {
    const int nk = c->nk, no = c->no, nv = c->nv, n = c->n;
    const i64 n1 = (i64)nk * no * nv, n2 = (i64)nk * nk * nk * no * no * nv * nv;
    hipStream_t st = c->own_stream;
    DevMem tmp;
    SolveCtx D;
    GradAdjoints GA = grad_adjoints(c, j, X, Y, o, tmp, D);
    const int ax = GA.ax, ay = GA.ay, nax = GA.nax;
    auto sub = [&](const Vecs &v, int r) { Vecs u; u.s = (char *)v.s + (size_t)r * n1 * 16; u.d = (char *)v.d + (size_t)r * n2 * 16; return u; };
    Vecs sol{c->sol1, c->sol2};
    auto tsol = [&](int sg, int a) { return sub(sol, (j * 2 + sg) * nax + a); };
    const Vecs &A = GA.A, &Z = GA.Z;
    // densities
    const size_t nd = (size_t)nk * n * n;
    void *dd = tmp.get(nd * 16);
    Vecs lam{c->lam1, c->lam2};
    std::vector<cd> G[2];
    std::vector<cd> zh((size_t)n1);
    for (int sg = 0; sg < 2; ++sg) {
        // sg 0: g(w) with a_X = A[0] along t^X(-w), a_Y = A[2] along t^Y(w)
        // sg 1: g(-w) with a_X = A[1] along t^X(w), a_Y = A[3] along t^Y(-w)
        const Vecs tx = tsol(1 - sg, ax), ty = tsol(sg, ay);
        const Vecs aX = sub(A, sg == 0 ? 0 : 1), aY = sub(A, sg == 0 ? 2 : 3);
        const Vecs zz = sub(Z, sg);
        auto d_ay = density_d1(c, D, aY, ty, dd, st);
        auto d_ax = density_d1(c, D, aX, tx, dd, st);
        auto d_lz = density_d1(c, D, lam, zz, dd, st);
        auto d_2 = density_d2(c, D, lam, tx, ty, dd, st);
        G[sg].assign(nd, 0.0);
        for (size_t e = 0; e < nd; ++e) G[sg][e] = -d_ay[e] - d_ax[e] - d_lz[e] + d_2[e];
        HIPCHK(hipMemcpy(zh.data(), zz.s, n1 * 16, hipMemcpyDeviceToHost));
        for (int k = 0; k < nk; ++k)
            for (int i = 0; i < no; ++i)
                for (int a = 0; a < nv; ++a)
                    G[sg][((size_t)k * n + i) * n + no + a] -= zh[((size_t)k * no + i) * nv + a];
    }
    std::vector<cd> g(nd);
    for (int k = 0; k < nk; ++k)
        for (int p = 0; p < n; ++p)
            for (int qq = 0; qq < n; ++qq)
                g[((size_t)k * n + p) * n + qq] =
                    -0.5 / nk * (G[0][((size_t)k * n + p) * n + qq] + std::conj(G[1][((size_t)k * n + qq) * n + p]));
    std::memcpy(out, g.data(), g.size() * 16);
}

// ---------------------------------------------------------------- gradient with respect to the Cholesky vectors
// alpha depends on the two-electron integrals through the Jacobian, the multipliers and the energy.
// With h any Hamiltonian parameter that enters the residual linearly (as f does) the derivative of
// g(w) at fixed amplitudes is
//   d g = dE''[tX(-w), tY(w)] + <lambda, dOmega''[tX(-w), tY(w)]> - <aY, dA tY(w)> - <aX, dA tX(-w)>
//         - <lambda, dA z> + <db, z>,
// (aX, aY, z as in the Fock gradient; b the right-hand side of the lambda equations).  Every term is
// a contraction of the parameter cotangent of the sigma, Gamma(u, t; T) = d <u, A(T) t> / dh, or a
// closed form in <ij||ab>: <u, dA t> = Gamma(u, t; T) . dh, and <lambda, dOmega''[x, y]> is the exact
// 4-point derivative of Gamma(lambda, y; T + e x) in e (A is cubic in T).  Gamma is obtained in
// three linear stages, all on the device: (1) the sigma's term list, run forward on t and backward on
// u, gives the cotangents of the blocks it reads (integral classes, amplitude-dependent blocks, the
// t1-dressed virtual Cholesky slices; the ladder's density D_ab,ef = sum_rij ubar_ijab dtau_ijef is
// formed one momentum block at a time and contracted with the other slice at once, never stored
// whole); (2) the amplitude-dependent blocks are linear in the integrals at fixed T, so their
// cotangents flow back to the integral classes (at the amplitudes of the evaluation point); (3) the
// classes are bilinear in the scaled Cholesky vectors, whose cotangents follow by transposed GEMMs.

// Cotangent buffers (complex128): the amplitude-dependent blocks the sigma reads (cleared for every
// evaluation point), the integral classes and the scaled Cholesky arrays (accumulated).
struct HamBar {
    DevMem mem;
    KT fov, Fae, Fmi, Fme, Fg, Fbe, Fmj, Wp, Wbar, S, U, H, G2;
    KT oooo, ooov, oovv, ovov, ovvo, ovvv, ovoo;
    void *La = nullptr, *Lb = nullptr;           // [nk][nk][naux][v][v]
    void *Ls = nullptr, *Lcs = nullptr;          // [nk][nk][naux][n][n]
    i64 nl = 0, nlvv = 0;
    std::vector<std::pair<void *, i64>> blocks, classes;   // (pointer, complex count) for clearing
};

void hambar_alloc(lrcc_ctx *c, HamBar &B) {
    const State<double> &S = c->s64;
    auto like = [&](KT &dst, const KT &src, std::vector<std::pair<void *, i64>> &list) {
        dst = src;
        dst.p = B.mem.get(src.count() * 16);
        list.push_back({dst.p, src.count()});
    };
    like(B.fov, S.fov, B.blocks); like(B.Fae, S.Fae, B.blocks); like(B.Fmi, S.Fmi, B.blocks);
    like(B.Fme, S.Fme, B.blocks); like(B.Fg, S.Fg, B.blocks); like(B.Fbe, S.Fbe, B.blocks);
    like(B.Fmj, S.Fmj, B.blocks); like(B.Wp, S.Wp, B.blocks); like(B.Wbar, S.Wbar, B.blocks);
    like(B.S, S.S, B.blocks); like(B.U, S.U, B.blocks); like(B.H, S.H, B.blocks); like(B.G2, S.G2, B.blocks);
    like(B.oooo, c->g_oooo, B.classes); like(B.ooov, c->g_ooov, B.classes); like(B.oovv, c->g_oovv, B.classes);
    like(B.ovov, c->g_ovov, B.classes); like(B.ovvo, c->g_ovvo, B.classes); like(B.ovvv, c->g_ovvv, B.classes);
    like(B.ovoo, c->g_ovoo, B.classes);
    B.nlvv = (i64)c->nk * c->nk * c->naux * c->nv * c->nv;
    B.nl = (i64)c->nk * c->nk * c->naux * c->n * c->n;
    B.La = B.mem.get(B.nlvv * 16);
    B.Lb = B.mem.get(B.nlvv * 16);
    B.blocks.push_back({B.La, B.nlvv});
    B.blocks.push_back({B.Lb, B.nlvv});
    B.Ls = B.mem.get(B.nl * 16);
    B.Lcs = B.mem.get(B.nl * 16);
    B.classes.push_back({B.Ls, B.nl});
    B.classes.push_back({B.Lcs, B.nl});
}

void hambar_clear(const std::vector<std::pair<void *, i64>> &list, hipStream_t st) {
    for (const auto &e : list) HIPCHK(zero_fill<double>(e.first, e.second, st));
}

// the cotangent buffer of a tensor the sigma reads, or null for amplitudes (t1, t2, tau)
const KT *bar_of(lrcc_ctx *c, const HamBar &B, const KT &t) {
    const State<double> &S = c->s64;
    const std::pair<const void *, const KT *> map[] = {
        {S.fov.p, &B.fov}, {S.Fae.p, &B.Fae}, {S.Fmi.p, &B.Fmi}, {S.Fme.p, &B.Fme}, {S.Fg.p, &B.Fg},
        {S.Fbe.p, &B.Fbe}, {S.Fmj.p, &B.Fmj}, {S.Wp.p, &B.Wp}, {S.Wbar.p, &B.Wbar}, {S.S.p, &B.S},
        {S.U.p, &B.U}, {S.H.p, &B.H}, {S.G2.p, &B.G2}, {c->g_oovv.p, &B.oovv}, {c->g_ooov.p, &B.ooov},
        {c->g_ovov.p, &B.ovov}, {c->g_ovvv.p, &B.ovvv}};
    for (const auto &m : map)
        if (m.first == t.p) return m.second;
    if (t.p == S.t1.p || t.p == S.t2.p || t.p == S.tau.p) return nullptr;
    throw LrccError(LRCC_E_STATE, "parameter gradient: the sigma reads a block without a cotangent");
}

// One complex128 GEMM job: C[m][n] (+)= alpha sum_k A[m][k] B[k][n] with two-level index splits.
void gemm1(Program &P, const void *A, i64 offA, i64 sizeA, const void *Bm, i64 offB, i64 sizeB, void *C, i64 offC,
           i64 sizeC, Split sm, Strides Am, Strides Cm, Split sn, Strides Bn, Strides Cn, Split sk, Strides Ak,
           Strides Bk, double alpha, int beta) {
    GemmArgs g{};
    g.shape = -1;
    g.A = A;
    g.B = Bm;
    g.C = C;
    g.M = sm.d1 * sm.d2;
    g.N = sn.d1 * sn.d2;
    g.K = sk.d1 * sk.d2;
    g.sm = sm; g.Am = Am; g.Cm = Cm;
    g.sn = sn; g.Bn = Bn; g.Cn = Cn;
    g.sk = sk; g.Ak = Ak; g.Bk = Bk;
    g.aMfast = 1;
    g.bNfast = 1;
    g.alpha_re = alpha;
    g.beta = beta;
    raw_gemm<double>(P, g, {offC}, {0, 1}, {offA}, {offB}, sizeA, sizeB, sizeC);
}

// Cotangents of the ladder slices: with Z += alpha sum Y W(La, Lb) (full index ranges, as the
// full-range kernel forms it) and the cotangent Zbar of Z, per momentum block (ki, kj, ka, ke)
//   D[(a,b),(e,f)] = sum_{r,i,j} Zbar[ki,kj,ka][r][i][j][a][b] Y[ki,kj,ke][r][i][j][e][f],
//   Labar[ka][ke][Q][a][e] += alpha sum_{b,f} D Lb[kb][kf][Q][b][f],
//   Lbbar[kb][kf][Q][b][f] += alpha sum_{a,e} D La[ka][ke][Q][a][e];
// D (v^4) lives in one scratch block, rebuilt for every momentum block.
void ladder_param_vjp(lrcc_ctx *c, Program &P, const KT &Y, const KT &Zb, double alpha, const void *La,
                      const void *Lb, void *Lab, void *Lbb, int R) {
    const int nk = c->nk, o = c->no, v = c->nv, naux = c->naux;
    const i64 vv = (i64)v * v, v3 = vv * v, blk = (i64)R * o * o * vv, nl = (i64)nk * nk * naux * vv;
    void *D = P.alloc((size_t)vv * vv * 16);
    const i64 nD = vv * vv;
    for (int ki = 0; ki < nk; ++ki)
        for (int kj = 0; kj < nk; ++kj)
            for (int ka = 0; ka < nk; ++ka) {
                const int kb = c->km.comb(ki, kj, ka);
                for (int ke = 0; ke < nk; ++ke) {
                    const int kf = c->km.comb(ki, kj, ke);
                    const i64 oz = (((i64)ki * nk + kj) * nk + ka) * blk, oy = (((i64)ki * nk + kj) * nk + ke) * blk;
                    // D[m=(a,b)][n=(e,f)] = sum_k Zbar[k][m] Y[k][n], k = (r, i, j)
                    gemm1(P, Zb.p, oz, Zb.count(), Y.p, oy, Y.count(), D, 0, nD,
                          Split{1, (int)vv}, Strides{{0, 0, 1}}, Strides{{0, 0, vv}},
                          Split{1, (int)vv}, Strides{{0, 0, 1}}, Strides{{0, 0, 1}},
                          Split{1, (int)(R * o * o)}, Strides{{0, 0, vv}}, Strides{{0, 0, vv}}, 1.0, 0);
                    // Labar[ka][ke][Q][(a,e)] += alpha sum_{(b,f)} D[a][b][e][f] Lb[kb][kf][Q][b][f]
                    const i64 oae = ((i64)ka * nk + ke) * naux * vv, obf = ((i64)kb * nk + kf) * naux * vv;
                    gemm1(P, D, 0, nD, Lb, obf, nl, Lab, oae, nl,
                          Split{v, v}, Strides{{0, v3, v}}, Strides{{0, v, 1}},
                          Split{1, naux}, Strides{{0, 0, vv}}, Strides{{0, 0, vv}},
                          Split{v, v}, Strides{{0, vv, 1}}, Strides{{0, v, 1}}, alpha, 1);
                    // Lbbar[kb][kf][Q][(b,f)] += alpha sum_{(a,e)} D[a][b][e][f] La[ka][ke][Q][a][e]
                    gemm1(P, D, 0, nD, La, oae, nl, Lbb, obf, nl,
                          Split{v, v}, Strides{{0, vv, 1}}, Strides{{0, v, 1}},
                          Split{1, naux}, Strides{{0, 0, vv}}, Strides{{0, 0, vv}},
                          Split{v, v}, Strides{{0, v3, v}}, Strides{{0, v, 1}}, alpha, 1);
                }
            }
}

// Program: Gamma(u, t; T) accumulated into the block cotangents of B.  Reads t from io_x1/io_x2
// and u from io_y1/io_y2 (caller layouts, one vector each, per-cell normalisation).
Program *build_param_vjp(lrcc_ctx *c, HamBar &B, DevMem &wm) {
    State<double> &S = c->s64;
    const int nk = c->nk, o = c->no, v = c->nv, R = 1;
    auto P = new Program();
    SigmaGraph Gf = record_sigma<double>(c, S, R, wm);   // forward values
    SigmaGraph Ga = record_sigma<double>(c, S, R, wm);   // cotangents
    // forward: the only active operands paired with Hamiltonian blocks are x1, x2 and dtau
    {
        KT x1 = Gf.x1, x2 = Gf.x2;
        P->ops.push_back([=](hipStream_t s) { return rhs_to_block<double, double>(c->io_x1, x1.p, R, nk, (i64)o * v, 1.0, s); });
        P->ops.push_back([=](hipStream_t s) {
            return rhs_to_block<double, double>(c->io_x2, x2.p, R, (i64)nk * nk * nk, (i64)o * o * v * v, 1.0 / nk, s);
        });
        const SymOp &tau = Gf.ops.at(0);
        if (tau.kind != SymOp::TAU) throw LrccError(LRCC_E_STATE, "parameter gradient: unexpected term list");
        void *t1p = S.t1.p, *xa = tau.A.p, *xb = tau.B.p, *out = tau.C.p;
        const KMesh km = c->km;
        P->ops.push_back([=](hipStream_t s) { return tau_like<double>(xa, xb, t1p, out, km, R, o, v, 1.0, 1, s); });
    }
    emit_reverse_sweep<double>(c, S, R, Ga, P, (const void *const *)&c->io_y1, (const void *const *)&c->io_y2);
    auto fwd_ok = [&](const KT &a) { return a.p == Gf.x1.p || a.p == Gf.x2.p || a.p == Gf.ops[0].C.p; };
    for (size_t q = 0; q < Gf.ops.size(); ++q) {
        const SymOp &f = Gf.ops[q], &a = Ga.ops[q];
        if (f.kind == SymOp::CON) {
            const KT &act = f.actA ? f.A : f.B, &par = f.actA ? f.B : f.A;
            const std::string &al = f.actA ? f.al : f.bl, &pl = f.actA ? f.bl : f.al;
            const KT *pb = bar_of(c, B, par);
            if (!pb) continue;
            if (!fwd_ok(act)) throw LrccError(LRCC_E_STATE, "parameter gradient: forward value missing");
            contract<double>(*P, *pb, pl, act, al, a.C, a.cl, f.alpha, true);
        } else if (f.kind == SymOp::LADDER) {
            ladder_param_vjp(c, *P, f.A, a.C, f.alpha.real(), S.La, S.Lb, B.La, B.Lb, R);
        }
    }
    return P;
}

// The integrals' cotangent flowing to the scaled Cholesky arrays: for a class array
// g[k0][k1][k2][d0][d1][d2][d3] = scale [sum_Q Ls[k0][k2][Q][d0][d2] Lcs[k1][k3][Q][d1][d3]
//                                        - sum_Q Ls[k0][k3][Q][d0][d3] Lcs[k1][k2][Q][d1][d2]]
// (as built for the stored classes), Lsbar and Lcsbar += the transposed products with gbar.
void eri_vjp(lrcc_ctx *c, Program &P, const KT &gb, double scale, void *Lsb, void *Lcsb) {
    const int nk = c->nk, n = c->n, naux = c->naux;
    auto off = [&](char cl) { return cl == 'o' ? 0 : c->no; };
    const i64 Lblk = (i64)naux * n * n, nl = (i64)nk * nk * Lblk, nn = (i64)n * n;
    i64 str[4];
    str[3] = 1;
    for (int d = 2; d >= 0; --d) str[d] = str[d + 1] * gb.ext(d + 1);
    for (int pass = 0; pass < 2; ++pass) {
        const int mi = pass == 0 ? 2 : 3, ni = pass == 0 ? 3 : 2;
        const double sc = pass == 0 ? scale : -scale;
        for (int side = 0; side < 2; ++side) {
            // side 0: Lsbar[k0][km][Q][d0][dmi] += sc sum_{d1,dni} gbar Lcs[k1][kn][Q][d1][dni]
            // side 1: Lcsbar[k1][kn][Q][d1][dni] += sc sum_{d0,dmi} gbar Ls[k0][km][Q][d0][dmi]
            const int r0 = side == 0 ? 0 : 1, r1 = side == 0 ? mi : ni;     // output index dims of gbar
            const int s0 = side == 0 ? 1 : 0, s1 = side == 0 ? ni : mi;     // summed index dims of gbar
            GemmArgs g{};
            g.shape = -1;
            g.A = gb.p;
            g.B = side == 0 ? c->Lcs : c->Ls;
            g.C = side == 0 ? Lsb : Lcsb;
            g.M = gb.ext(r0) * gb.ext(r1);
            g.N = naux;
            g.K = gb.ext(s0) * gb.ext(s1);
            g.sm = Split{gb.ext(r0), gb.ext(r1)};
            g.Am = Strides{{0, str[r0], str[r1]}};
            g.Cm = Strides{{0, n, 1}};
            g.sn = Split{1, naux};
            g.Bn = Strides{{0, 0, nn}};
            g.Cn = Strides{{0, 0, nn}};
            g.sk = Split{gb.ext(s0), gb.ext(s1)};
            g.Ak = Strides{{0, str[s0], str[s1]}};
            g.Bk = Strides{{0, n, 1}};
            g.aMfast = 0;
            g.bNfast = 0;
            g.alpha_re = sc;
            g.beta = 1;
            // jobs: output Cholesky blocks; segments: the class blocks feeding them
            std::map<std::pair<int, int>, std::vector<std::pair<i64, i64>>> jobs;
            for (int k0 = 0; k0 < nk; ++k0)
                for (int k1 = 0; k1 < nk; ++k1)
                    for (int k2 = 0; k2 < nk; ++k2) {
                        const int k3 = c->km.comb(k0, k1, k2);
                        const int km = pass == 0 ? k2 : k3, kn = pass == 0 ? k3 : k2;
                        const i64 ga = (((i64)k0 * nk + k1) * nk + k2) * gb.inner();
                        if (side == 0)
                            jobs[{k0, km}].push_back({ga, (i64)(k1 * nk + kn) * Lblk + (i64)off(gb.cls[1]) * n + off(gb.cls[ni])});
                        else
                            jobs[{k1, kn}].push_back({ga, (i64)(k0 * nk + km) * Lblk + (i64)off(gb.cls[0]) * n + off(gb.cls[mi])});
                    }
            std::vector<i64> offC, segA, segB;
            std::vector<int> beg{0};
            for (const auto &j : jobs) {
                const char cr0 = gb.cls[r0], cr1 = gb.cls[r1];
                offC.push_back((i64)(j.first.first * nk + j.first.second) * Lblk + (i64)off(cr0) * n + off(cr1));
                for (const auto &sg : j.second) {
                    segA.push_back(sg.first);
                    segB.push_back(sg.second);
                }
                beg.push_back((int)segA.size());
            }
            raw_gemm<double>(P, g, offC, beg, segA, segB, gb.count(), nl, nl);
        }
    }
}

// Program: the block cotangents of B flow back to the integral classes and the scaled Cholesky
// arrays at the context's current amplitudes (the reverse of the amplitude-dependent blocks).
Program *build_state_reverse(lrcc_ctx *c, HamBar &B, DevMem &wm) {
    State<double> &S = c->s64;
    const int nk = c->nk, o = c->no, v = c->nv, n = c->n, naux = c->naux;
    auto P = new Program();
    const KT &t1 = S.t1, &t2 = S.t2, &tau = S.tau;
    const KMesh km = c->km;
    // tilde tau (tau with half the t1 t1 part), as in the forward blocks
    KT tt = alloc_kt<double>(c, wm, "oovv");
    {
        void *t1p = t1.p, *t2p = t2.p, *ttp = tt.p;
        P->ops.push_back([=](hipStream_t s) { return tau_like<double>(t1p, t2p, t1p, ttp, km, 1, o, v, 0.25, 0, s); });
    }
    auto zero = [&](const KT &t) {
        void *p = t.p;
        const i64 cnt = t.count();
        P->ops.push_back([=](hipStream_t s) { return zero_fill<double>(p, cnt, s); });
    };
    auto add = [&](const KT &dst, const KT &src, double a) {
        void *d = dst.p;
        const void *sp = src.p;
        const i64 cnt = src.count();
        void *tmp = a == 1.0 ? nullptr : P->alloc((size_t)cnt * 16);
        P->ops.push_back([=](hipStream_t s) {
            if (!tmp) return add_inplace<double>(d, sp, cnt, s);
            hipError_t e = scale_copy(tmp, sp, a, 0.0, cnt, s);
            return e != hipSuccess ? e : add_inplace<double>(d, tmp, cnt, s);
        });
    };
    // dst += a * permute4(src) (dst in the output layout of the permutation)
    auto padd = [&](const KT &dst, const KT &src, std::array<int, 4> ext, std::array<int, 4> perm, double a) {
        KT tmp = dst;
        tmp.p = P->alloc((size_t)dst.count() * 16);
        const void *sp = src.p;
        void *tp = tmp.p;
        const std::array<int, 4> sg{dst.sg[0], dst.sg[1], dst.sg[2], dst.sg[3]};
        P->ops.push_back([=](hipStream_t s) { return permute4(sp, tp, km, ext.data(), perm.data(), sg.data(), s); });
        add(dst, tmp, a);
    };
    // G2_ijbm = 1/2 permute(ovoo) + t_ie <mb||ej>
    contract<double>(*P, B.ovvo, "mbej", t1, "ie", B.G2, "ijbm", 1.0);
    padd(B.ovoo, B.G2, {o, o, v, o}, {3, 2, 0, 1}, 0.5);
    // H_abej = 1/2 <ab||ej> - t_ma <mb||ej> - permute(R)
    eri_vjp(c, *P, B.H, 0.5, B.Ls, B.Lcs);
    contract<double>(*P, B.ovvo, "mbej", t1, "ma", B.H, "abej", -1.0);
    KT Rb = alloc_kt<double>(c, wm, "ovvv", 0, {1, -1, -1, 1});
    zero(Rb);
    padd(Rb, B.H, {v, v, v, o}, {3, 0, 1, 2}, -1.0);
    // S_ijan = -t_imae <mn||je> + t_jf U_ianf - 1/4 tau_ijef <na||ef>
    contract<double>(*P, B.ooov, "mnje", t2, "imae", B.S, "ijan", -1.0);
    contract<double>(*P, B.U, "ianf", t1, "jf", B.S, "ijan", 1.0);
    contract<double>(*P, B.ovvv, "naef", tau, "ijef", B.S, "ijan", -0.25);
    // U_ianf = t_imae <mn||ef> ; R_iabf = t_imae <mb||ef>
    contract<double>(*P, B.oovv, "mnef", t2, "imae", B.U, "ianf", 1.0);
    contract<double>(*P, B.ovvv, "mbef", t2, "imae", Rb, "iabf", 1.0);
    // Wbar (ring layout [m][e][b][j]) = permute of Wbar0 (ovvo):
    //   Wbar0 = <mb||ej> + t_jf <mb||ef> + t_nb <mn||je> - t_jnfb <mn||ef> - t_nb (t_jf <mn||ef>)
    KT W0 = alloc_kt<double>(c, wm, "ovvo");
    zero(W0);
    padd(W0, B.Wbar, {o, v, v, o}, {0, 2, 1, 3}, 1.0);
    add(B.ovvo, W0, 1.0);
    contract<double>(*P, B.ovvv, "mbef", t1, "jf", W0, "mbej", 1.0);
    contract<double>(*P, B.ooov, "mnje", t1, "nb", W0, "mbej", 1.0);
    contract<double>(*P, B.oovv, "mnef", t2, "jnfb", W0, "mbej", -1.0);
    KT yb = alloc_kt<double>(c, wm, "oovo");
    contract<double>(*P, yb, "mnej", t1, "nb", W0, "mbej", -1.0, false);
    contract<double>(*P, B.oovv, "mnef", t1, "jf", yb, "mnej", 1.0);
    // W'_mnij = <mn||ij> + P(ij) t_je <mn||ie> + 1/2 tau_ijef <mn||ef>
    add(B.oooo, B.Wp, 1.0);
    contract<double>(*P, B.ooov, "mnie", t1, "je", B.Wp, "mnij", 1.0);
    contract<double>(*P, B.ooov, "mnie", t1, "je", B.Wp, "mnji", -1.0);
    contract<double>(*P, B.oovv, "mnef", tau, "ijef", B.Wp, "mnij", 0.5);
    // Fbar_mj = F_mi + 1/2 t_je F_me ; Fbar_be = F_ae - 1/2 t_mb F_me (accumulated into copies)
    KT Fmi = B.Fmi, Fae = B.Fae, Fme = B.Fme;
    add(Fmi, B.Fmj, 1.0);
    contract<double>(*P, Fme, "me", t1, "je", B.Fmj, "mj", 0.5);
    add(Fae, B.Fbe, 1.0);
    contract<double>(*P, Fme, "me", t1, "mb", B.Fbe, "be", -0.5);
    // Fg_me = t_nf <mn||ef> ; F_me = f_me + t_nf <mn||ef>
    contract<double>(*P, B.oovv, "mnef", t1, "nf", B.Fg, "me", 1.0);
    contract<double>(*P, B.oovv, "mnef", t1, "nf", Fme, "me", 1.0);
    // F_mi = f_mi + 1/2 t_ie f_me + t_ne <mn||ie> + 1/2 ttau_inef <mn||ef>
    contract<double>(*P, B.ooov, "mnie", t1, "ne", Fmi, "mi", 1.0);
    contract<double>(*P, B.oovv, "mnef", tt, "inef", Fmi, "mi", 0.5);
    // F_ae = f_ae - 1/2 f_me t_ma + t_mf <ma||fe> - 1/2 ttau_mnaf <mn||ef>
    contract<double>(*P, B.ovvv, "mafe", t1, "mf", Fae, "ae", 1.0);
    contract<double>(*P, B.oovv, "mnef", tt, "mnaf", Fae, "ae", -0.5);
    // dressed virtual slices: La = Ls_vv - t1 . Ls_ov, Lb = Lcs_vv - t1 . Lcs_ov
    for (int w = 0; w < 2; ++w) {
        const void *lb = w == 0 ? B.La : B.Lb;
        void *dst = w == 0 ? B.Ls : B.Lcs;
        P->ops.push_back([=](hipStream_t s) { return slice_add(lb, dst, nk, naux, n, o, v, o, v, s); });
        // dst[k1][k2][Q][m][o+e] += - sum_a t1[k1][m][a] lb[k1][k2][Q][a][e]
        GemmArgs g{};
        g.shape = -1;
        g.A = t1.p;
        g.B = lb;
        g.C = dst;
        g.M = o;
        g.N = v;
        g.K = v;
        g.sm = Split{1, o};
        g.Am = Strides{{0, 0, v}};
        g.Cm = Strides{{0, 0, n}};
        g.sk = Split{1, v};
        g.Ak = Strides{{0, 0, 1}};
        g.Bk = Strides{{0, 0, v}};
        g.sn = Split{1, v};
        g.Bn = Strides{{0, 0, 1}};
        g.Cn = Strides{{0, 0, 1}};
        g.aMfast = 0;
        g.bNfast = 1;
        g.alpha_re = -1.0;
        g.beta = 1;
        std::vector<i64> offC, segA, segB;
        std::vector<int> beg{0};
        for (int k1 = 0; k1 < nk; ++k1)
            for (int k2 = 0; k2 < nk; ++k2)
                for (int q = 0; q < naux; ++q) {
                    offC.push_back((((i64)k1 * nk + k2) * naux + q) * n * n + o);
                    segA.push_back((i64)k1 * o * v);
                    segB.push_back((((i64)k1 * nk + k2) * naux + q) * v * v);
                    beg.push_back((int)segA.size());
                }
        raw_gemm<double>(*P, g, offC, beg, segA, segB, (i64)nk * o * v, B.nlvv, B.nl);
    }
    return P;
}

// Program: the integral classes' cotangents flow to the scaled Cholesky arrays.
Program *build_class_reverse(lrcc_ctx *c, HamBar &B) {
    auto P = new Program();
    for (const KT *g : {&B.oooo, &B.ooov, &B.oovv, &B.ovov, &B.ovvo, &B.ovvv, &B.ovoo})
        eri_vjp(c, *P, *g, 1.0, B.Ls, B.Lcs);
    return P;
}

// d alpha_XY(w_j) / d L at fixed amplitudes (lambda and the response amplitudes re-solved), for
// perturbations dL that keep the Hermitian pairing dL[k2][k1][Q] = conj(dL[k1][k2][Q])^T:
//   d alpha = sum grad[k1][k2][Q][p][q] dL[k1][k2][Q][p][q].
// The scaled arrays are Ls = L / sqrt(Nk) and Lcs[k1][k2][Q][p][q] = conj(L[k2][k1][Q][q][p]) / sqrt(Nk),
// so under the pairing dLs = dLcs = dL / sqrt(Nk) and the gradient is (Lsbar + Lcsbar) / sqrt(Nk).
void alpha_chol_grad(lrcc_ctx *c, int j, int X, int Y, const lrcc_solve_opts &o, double *out) {
    const int nk = c->nk, no = c->no, nv = c->nv, n = c->n, naux = c->naux;
    const i64 n1 = (i64)nk * no * nv, n2 = (i64)nk * nk * nk * no * no * nv * nv;
    hipStream_t st = c->own_stream;
    DevMem tmp;
    SolveCtx D;
    GradAdjoints GA = grad_adjoints(c, j, X, Y, o, tmp, D);
    const int ax = GA.ax, ay = GA.ay, nax = GA.nax;
    auto vec = [&](int R) { Vecs v; v.s = tmp.get((size_t)R * n1 * 16); v.d = tmp.get((size_t)R * n2 * 16); return v; };
    auto sub = [&](const Vecs &v, int r) { Vecs u; u.s = (char *)v.s + (size_t)r * n1 * 16; u.d = (char *)v.d + (size_t)r * n2 * 16; return u; };
    Vecs sol{c->sol1, c->sol2};
    auto tsol = [&](int sg, int a) { return sub(sol, (j * 2 + sg) * nax + a); };
    const Vecs &A = GA.A, &Z = GA.Z;
    State<double> &S = c->s64;
    const i64 nt1 = S.t1.count(), nt2 = S.t2.count();
    void *T1 = tmp.get(nt1 * 16), *T2 = tmp.get(nt2 * 16);
    HIPCHK(hipMemcpyAsync(T1, S.t1.p, nt1 * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(T2, S.t2.p, nt2 * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    HamBar B;
    hambar_alloc(c, B);
    DevMem wm;
    std::unique_ptr<Program> pv(build_param_vjp(c, B, wm)), sr(build_state_reverse(c, B, wm)),
        cr(build_class_reverse(c, B));
    Vecs u = vec(1);
    void *z2tmp = tmp.get(n2 * 16);
    Vecs lam{c->lam1, c->lam2};
    // Gamma(cu * uu, t; T at the current amplitudes) into the block cotangents
    auto gamma = [&](const Vecs &uu, double cu, const Vecs &t) {
        HIPCHK(scale_copy(u.s, uu.s, cu, 0.0, n1, st));
        HIPCHK(scale_copy(u.d, uu.d, cu, 0.0, n2, st));
        c->io_x1 = t.s; c->io_x2 = t.d; c->io_y1 = u.s; c->io_y2 = u.d; c->io_omega = nullptr;
        HIPCHK(pv->run(st));
    };
    // amplitudes T + e x (T2 in crystal normalisation: x2 / Nk)
    auto shift = [&](const Vecs *x, double e) {
        HIPCHK(hipMemcpyAsync(S.t1.p, T1, nt1 * 16, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(S.t2.p, T2, nt2 * 16, hipMemcpyDeviceToDevice, st));
        if (x) {
            HIPCHK(scale_copy(u.s, x->s, e, 0.0, n1, st));
            HIPCHK(add_inplace<double>(S.t1.p, u.s, nt1, st));
            HIPCHK(scale_copy(u.d, x->d, e / nk, 0.0, n2, st));
            HIPCHK(add_inplace<double>(S.t2.p, u.d, nt2, st));
        }
        run_precompute(c, false, st);
    };
    const size_t nl = (size_t)nk * nk * naux * n * n;
    std::vector<cd> G[2], ls(nl), lcs(nl);
    for (int sg = 0; sg < 2; ++sg) {
        // sg 0: g(w): aX = A[0] along t^X(-w), aY = A[2] along t^Y(w); sg 1: g(-w) likewise
        const Vecs tx = tsol(1 - sg, ax), ty = tsol(sg, ay);
        const Vecs aX = sub(A, sg == 0 ? 0 : 1), aY = sub(A, sg == 0 ? 2 : 3);
        const Vecs zz = sub(Z, sg);
        hambar_clear(B.classes, st);
        hambar_clear(B.blocks, st);
        // - <aY, dA tY> - <aX, dA tX> - <lambda, dA z> at T
        gamma(aY, -1.0, ty);
        gamma(aX, -1.0, tx);
        gamma(lam, -1.0, zz);
        HIPCHK(sr->run(st));
        // <lambda, dOmega''[tX, tY]> = d/de Gamma(lambda, tY; T + e tX): 4-point derivative, exact
        // for the cubic dependence of A on T
        const double h = step_for(D, tx);
        const int shifts[4] = {-2, -1, 1, 2};
        const double coef[4] = {1.0, -8.0, 8.0, -1.0};
        for (int k = 0; k < 4; ++k) {
            shift(&tx, shifts[k] * h);
            hambar_clear(B.blocks, st);
            gamma(lam, coef[k] / (12.0 * h), ty);
            HIPCHK(sr->run(st));
        }
        shift(nullptr, 0.0);
        // energy terms: dE''[tX, tY] = sum d<ij||ab> tX_ia tY_jb and <db, z> with
        // b = -(f_ia + <ij||ab> t_jb, <ij||ab> / Nk): -z_ia t_jb - z_ijab / (4 Nk)
        HIPCHK(outer_oovv(B.oovv.p, tx.s, ty.s, 1.0, nk, no, nv, st));
        HIPCHK(outer_oovv(B.oovv.p, zz.s, S.t1.p, -1.0, nk, no, nv, st));
        HIPCHK(scale_copy(z2tmp, zz.d, -0.25 / nk, 0.0, n2, st));
        HIPCHK(add_inplace<double>(B.oovv.p, z2tmp, n2, st));
        HIPCHK(cr->run(st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(ls.data(), B.Ls, nl * 16, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(lcs.data(), B.Lcs, nl * 16, hipMemcpyDeviceToHost));
        G[sg].resize(nl);
        const double r = 1.0 / std::sqrt((double)nk);
        for (size_t e = 0; e < nl; ++e) G[sg][e] = (ls[e] + lcs[e]) * r;
    }
    run_precompute(c, true, st);   // amplitudes restored: every block of both precisions
    // alpha = -1/(2 Nk) [g(w) + conj(g(-w))]; conj(dL[k1][k2][Q][p][q]) = dL[k2][k1][Q][q][p]
    std::vector<cd> g(nl);
    auto at = [&](int k1, int k2, int q, int p, int r) { return ((((size_t)k1 * nk + k2) * naux + q) * n + p) * n + r; };
    for (int k1 = 0; k1 < nk; ++k1)
        for (int k2 = 0; k2 < nk; ++k2)
            for (int q = 0; q < naux; ++q)
                for (int p = 0; p < n; ++p)
                    for (int r = 0; r < n; ++r)
                        g[at(k1, k2, q, p, r)] = -0.5 / nk * (G[0][at(k1, k2, q, p, r)] + std::conj(G[1][at(k2, k1, q, r, p)]));
    std::memcpy(out, g.data(), g.size() * 16);
}

// ---------------------------------------------------------------- EOM-CCSD excitation energies
// The poles of the linear response function are the eigenvalues of the CCSD
// Jacobian.  Davidson iteration on the device sigma (complex128, one vector per
// application) with the Hermitian inner product of the solver (doubles weighted
// 1/4), Rayleigh-Ritz on the projected matrix G = V^H A V (host, small_eig),
// residuals r = (A - theta) x, corrections from the dressed diagonal
// preconditioner at Re(theta), restarts from the current Ritz vectors.
void eom_roots(lrcc_ctx *c, int nroots, double tol, int max_iter, std::vector<cd> &omega, lrcc_solve_report &rep) {
    auto t0 = std::chrono::steady_clock::now();
    const int nk = c->nk, no = c->no, nv = c->nv;
    const i64 n1 = (i64)nk * no * nv, n2 = (i64)nk * nk * nk * no * no * nv * nv;
    if (!c->own_stream) HIPCHK(hipStreamCreate(&c->own_stream));
    hipStream_t st = c->own_stream;
    if (nroots < 1 || nroots > n1) throw LrccError(LRCC_E_ARG, "nroots must lie in 1..nk*nocc*nvir");
    const int nguess = (int)std::min<i64>(n1, std::max(2 * nroots, nroots + 4));
    const int mmax = std::max(nguess + 2 * nroots, std::min(80, 6 * nroots + 8));
    DevMem mem;
    Vecs Vb{mem.get((size_t)mmax * n1 * 16), mem.get((size_t)mmax * n2 * 16)};
    Vecs Wb{mem.get((size_t)mmax * n1 * 16), mem.get((size_t)mmax * n2 * 16)};
    Vecs Rb{mem.get((size_t)nroots * n1 * 16), mem.get((size_t)nroots * n2 * 16)};
    Vecs Tb{mem.get((size_t)mmax * n1 * 16), mem.get((size_t)mmax * n2 * 16)};   // restart scratch
    auto at = [&](const Vecs &b, int i) { Vecs u; u.s = (char *)b.s + (size_t)i * n1 * 16; u.d = (char *)b.d + (size_t)i * n2 * 16; return u; };
    SolveCtx S;
    S.c = c; S.R = 1; S.n1 = n1; S.n2 = n2; S.st = st;
    S.part = mem.get((size_t)dot_blocks(n2) * 16 * 2);
    S.dout = mem.get(32);
    S.alpha = mem.get(32);
    void *coef = mem.get((size_t)mmax * mmax * 16);
    double *dom = (double *)mem.get(8);
    Program *sig = sigma_program(c, LRCC_FP64, 1);
    int napply = 0;
    auto apply = [&](const Vecs &y, const Vecs &x) {
        c->io_x1 = x.s; c->io_x2 = x.d; c->io_y1 = y.s; c->io_y2 = y.d; c->io_omega = nullptr;
        HIPCHK(sig->run(st));
        ++napply;
    };
    int m = 0;
    std::vector<cd> G;   // m x m, row-major, G[i][j] = <V_i, W_j>
    auto grow = [&](int mnew) {
        std::vector<cd> H((size_t)mnew * mnew, 0.0);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) H[(size_t)i * mnew + j] = G[(size_t)i * m + j];
        G.swap(H);
    };
    // orthonormalise candidate u (in place) against V[0..m) twice; append it (and A u) if it survives
    auto add = [&](const Vecs &u) {
        double n0 = S.norm(u)[0];
        if (n0 == 0) return false;
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < m; ++i) {
                const cd h = S.dot(at(Vb, i), u)[0];
                S.axpby(u, at(Vb, i), std::vector<cd>(1, -h), 1.0);
            }
        const double nu = S.norm(u)[0];
        if (nu < 1e-8 * n0 || m >= mmax) return false;
        S.axpby(at(Vb, m), u, std::vector<cd>(1, cd(1.0 / nu, 0.0)), 0.0);
        apply(at(Wb, m), at(Vb, m));
        grow(m + 1);
        for (int i = 0; i <= m; ++i) {
            G[(size_t)i * (m + 1) + m] = S.dot(at(Vb, i), at(Wb, m))[0];
            if (i < m) G[(size_t)m * (m + 1) + i] = S.dot(at(Vb, m), at(Wb, i))[0];
        }
        ++m;
        return true;
    };
    // initial guesses: singles at the smallest dressed diagonal differences
    {
        std::vector<double> eo((size_t)nk * no), ev((size_t)nk * nv);
        HIPCHK(hipMemcpy(eo.data(), c->s64.d_o1, eo.size() * 8, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(ev.data(), c->s64.d_v1, ev.size() * 8, hipMemcpyDeviceToHost));
        std::vector<std::pair<double, i64>> cand;
        for (int k = 0; k < nk; ++k)
            for (int i = 0; i < no; ++i)
                for (int a = 0; a < nv; ++a)
                    cand.push_back({ev[(size_t)k * nv + a] - eo[(size_t)k * no + i], ((i64)k * no + i) * nv + a});
        std::stable_sort(cand.begin(), cand.end());
        Vecs u = at(Rb, 0);
        for (int g = 0; g < nguess && g < (int)cand.size(); ++g) {
            HIPCHK(hipMemsetAsync(u.s, 0, n1 * 16, st));
            HIPCHK(hipMemsetAsync(u.d, 0, n2 * 16, st));
            const double one[2] = {1.0, 0.0};
            HIPCHK(hipMemcpyAsync((char *)u.s + cand[g].second * 16, one, 16, hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            (void)add(u);
        }
    }
    rep = lrcc_solve_report{};
    std::vector<cd> theta(nroots);
    std::vector<double> res(nroots, 1e300);
    int it = 0;
    for (; it < max_iter; ++it) {
        std::vector<cd> w, Vs;
        if (!small_eig(m, G, w, Vs)) throw LrccError(LRCC_E_NOCONV, "subspace eigenproblem did not converge");
        std::vector<int> ord(m);
        for (int i = 0; i < m; ++i) ord[i] = i;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return w[a].real() < w[b].real(); });
        // residuals r_k = W s_k - theta_k V s_k
        std::vector<cd> cw((size_t)nroots * m), cv((size_t)nroots * m);
        for (int k = 0; k < nroots; ++k) {
            theta[k] = w[ord[k]];
            for (int i = 0; i < m; ++i) {
                cw[(size_t)k * m + i] = Vs[(size_t)i * m + ord[k]];
                cv[(size_t)k * m + i] = -theta[k] * Vs[(size_t)i * m + ord[k]];
            }
        }
        HIPCHK(hipMemcpy(coef, cw.data(), cw.size() * 16, hipMemcpyHostToDevice));
        HIPCHK(combine(Rb.s, Wb.s, coef, nroots, m, n1, 0.0, st));
        HIPCHK(combine(Rb.d, Wb.d, coef, nroots, m, n2, 0.0, st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(coef, cv.data(), cv.size() * 16, hipMemcpyHostToDevice));
        HIPCHK(combine(Rb.s, Vb.s, coef, nroots, m, n1, 1.0, st));
        HIPCHK(combine(Rb.d, Vb.d, coef, nroots, m, n2, 1.0, st));
        HIPCHK(hipStreamSynchronize(st));
        bool done = true;
        for (int k = 0; k < nroots; ++k) {
            res[k] = S.norm(at(Rb, k))[0];
            if (res[k] > tol) done = false;
        }
        if (verbose()) {
            std::fprintf(stderr, "[lrcc] eom iteration %d subspace %d:", it, m);
            for (int k = 0; k < nroots; ++k) std::fprintf(stderr, " %.10f(%.1e)", theta[k].real(), res[k]);
            std::fprintf(stderr, "\n");
        }
        if (done) break;
        // restart from the Ritz vectors when the new directions would not fit
        int nnew = 0;
        for (int k = 0; k < nroots; ++k) nnew += res[k] > tol;
        if (m + nnew > mmax) {
            const int p = std::min(m, 2 * nroots + 2);
            // orthonormal combinations of the p lowest Ritz vectors (coefficients in the orthonormal basis)
            std::vector<cd> C((size_t)p * m);
            int q = 0;
            for (int k = 0; k < m && q < p; ++k) {
                std::vector<cd> x(m);
                for (int i = 0; i < m; ++i) x[i] = Vs[(size_t)i * m + ord[k]];
                for (int pass = 0; pass < 2; ++pass)
                    for (int l = 0; l < q; ++l) {
                        cd h = 0;
                        for (int i = 0; i < m; ++i) h += std::conj(C[(size_t)l * m + i]) * x[i];
                        for (int i = 0; i < m; ++i) x[i] -= h * C[(size_t)l * m + i];
                    }
                double nx = 0;
                for (auto &e : x) nx += std::norm(e);
                nx = std::sqrt(nx);
                if (nx < 1e-8) continue;
                for (int i = 0; i < m; ++i) C[(size_t)q * m + i] = x[i] / nx;
                ++q;
            }
            HIPCHK(hipMemcpy(coef, C.data(), (size_t)q * m * 16, hipMemcpyHostToDevice));
            HIPCHK(combine(Tb.s, Vb.s, coef, q, m, n1, 0.0, st));
            HIPCHK(combine(Tb.d, Vb.d, coef, q, m, n2, 0.0, st));
            HIPCHK(hipMemcpyAsync(Vb.s, Tb.s, (size_t)q * n1 * 16, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(Vb.d, Tb.d, (size_t)q * n2 * 16, hipMemcpyDeviceToDevice, st));
            HIPCHK(combine(Tb.s, Wb.s, coef, q, m, n1, 0.0, st));
            HIPCHK(combine(Tb.d, Wb.d, coef, q, m, n2, 0.0, st));
            HIPCHK(hipMemcpyAsync(Wb.s, Tb.s, (size_t)q * n1 * 16, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(Wb.d, Tb.d, (size_t)q * n2 * 16, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            // G' = C^H G C
            std::vector<cd> GC((size_t)m * q, 0.0), Gn((size_t)q * q, 0.0);
            for (int i = 0; i < m; ++i)
                for (int b = 0; b < q; ++b)
                    for (int j = 0; j < m; ++j) GC[(size_t)i * q + b] += G[(size_t)i * m + j] * C[(size_t)b * m + j];
            for (int a = 0; a < q; ++a)
                for (int b = 0; b < q; ++b)
                    for (int i = 0; i < m; ++i) Gn[(size_t)a * q + b] += std::conj(C[(size_t)a * m + i]) * GC[(size_t)i * q + b];
            G.swap(Gn);
            m = q;
        }
        // corrections (D - Re theta)^-1 r for the unconverged roots
        for (int k = 0; k < nroots; ++k) {
            if (res[k] <= tol) continue;
            const double wr = theta[k].real();
            HIPCHK(hipMemcpy(dom, &wr, 8, hipMemcpyHostToDevice));
            Vecs u = at(Tb, 0);
            const State<double> &T = c->s64;
            HIPCHK(precond(u.s, u.d, at(Rb, k).s, at(Rb, k).d, (const double *)T.d_o1, (const double *)T.d_v1,
                           (const double *)T.d_o2, (const double *)T.d_v2, dom, c->km, 1, no, nv, st));
            HIPCHK(hipStreamSynchronize(st));
            (void)add(u);
        }
    }
    omega = theta;
    rep.converged = *std::max_element(res.begin(), res.end()) <= tol;
    rep.outer = it + 1;
    rep.sigma_fp64 = napply;
    rep.rhs_sigmas = napply;
    rep.max_rel_residual = *std::max_element(res.begin(), res.end());
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------- ground-state CCSD
// The CCSD residual is a quartic polynomial in T, so with A the Jacobian
//   Omega(T) = Omega(0) + int_0^1 A(sT) T ds
// and the integrand is cubic in s: the 2-point Gauss-Legendre rule on [0,1]
// reproduces it exactly.  Each residual costs two re-runs of the amplitude-
// dependent blocks and two single-RHS sigma applications.  Omega(0) =
// (f_ai, <ab||ij>).  Jacobi steps t <- t + Omega / D with the orbital-energy
// denominators of Eq. D and DIIS on the amplitude change (Sec. II.C).
void ccsd_residual(lrcc_ctx *c, SolveCtx &S, const Vecs &T, const Vecs &om0, const Vecs &out, const Vecs &tmp) {
    State<double> &St = c->s64;
    const i64 n1 = S.n1, n2 = S.n2;
    const double g = 0.5 / std::sqrt(3.0);
    const double nodes[2] = {0.5 - g, 0.5 + g};
    S.copy(out, om0);
    Program *sig = sigma_program(c, LRCC_FP64, 1, false);
    for (int q = 0; q < 2; ++q) {
        // state amplitudes = s T (T2 in crystal normalisation)
        HIPCHK(scale_copy(St.t1.p, T.s, nodes[q], 0.0, n1, S.st));
        HIPCHK(scale_copy(St.t2.p, T.d, nodes[q] / c->nk, 0.0, n2, S.st));
        run_precompute(c, false, S.st);
        c->io_x1 = T.s; c->io_x2 = T.d; c->io_y1 = tmp.s; c->io_y2 = tmp.d; c->io_omega = nullptr;
        HIPCHK(sig->run(S.st, nullptr));
        S.rhs_sig += 1;
        S.axpby(out, tmp, std::vector<cd>(1, cd(0.5, 0.0)), 1.0);
    }
}

void solve_ccsd(lrcc_ctx *c, double tol, int max_iter, int ndiis, lrcc_solve_report &rep, double &energy) {
    auto t0 = std::chrono::steady_clock::now();
    if (!c->s64.ready) build_state(c);
    if (!c->own_stream) HIPCHK(hipStreamCreate(&c->own_stream));
    hipStream_t st = c->own_stream;
    const int nk = c->nk, o = c->no, v = c->nv, n = c->n;
    SolveCtx S;
    S.c = c; S.R = 1; S.st = st; S.omega = nullptr;
    S.n1 = (i64)nk * o * v;
    S.n2 = (i64)nk * nk * nk * o * o * v * v;
    DevMem m;
    auto mk = [&]() { Vecs x; x.s = m.get(S.n1 * 16); x.d = m.get(S.n2 * 16); return x; };
    S.part = m.get((size_t)dot_blocks(S.n2) * 16);
    S.dout = m.get(16);
    S.alpha = m.get(16);
    Vecs om0 = mk(), T = mk(), res = mk(), tmp = mk(), step = mk();
    std::vector<Vecs> hist, errs;
    // Omega(0): singles f_ai (stored [k][i][a]), doubles <ab||ij> = conj(<ij||ab>) (per-cell: x Nk)
    HIPCHK(axis_slice<double>(c->fock, om0.s, 1, nk, n, 0, o, o, v, 1, st));
    HIPCHK(conj_scale(om0.d, c->g_oovv.p, (double)nk, S.n2, st));
    S.zero(T);
    double rn = 0;
    int it = 0;
    for (; it < max_iter; ++it) {
        ccsd_residual(c, S, T, om0, res, tmp);
        rn = std::sqrt(std::max(0.0, S.dot(res, res)[0].real()));
        if (verbose()) std::fprintf(stderr, "[lrcc] ccsd iteration %d |Omega| %.3e\n", it, rn);
        if (rn <= tol) break;
        // Jacobi: t_new = t + Omega / D = t - Omega / (e_a + e_b - e_i - e_j)
        HIPCHK(precond(step.s, step.d, res.s, res.d, (const double *)c->eps_o, (const double *)c->eps_v,
                       (const double *)c->eps_o, (const double *)c->eps_v, nullptr, c->km, 1, o, v, st));
        Vecs tn = mk();
        S.copy(tn, T);
        S.axpby(tn, step, std::vector<cd>(1, cd(-1.0, 0.0)), 1.0);
        Vecs e = mk();
        S.copy(e, tn);
        S.axpby(e, T, std::vector<cd>(1, cd(-1.0, 0.0)), 1.0);
        hist.push_back(tn);
        errs.push_back(e);
        if ((int)hist.size() > ndiis) { hist.erase(hist.begin()); errs.erase(errs.begin()); }
        const int k = (int)hist.size();
        if (k >= 2) {
            // DIIS: min |sum c_i e_i| with sum c_i = 1 (Hermitian error matrix)
            std::vector<cd> B((k + 1) * (k + 1), 0.0), rhs(k + 1, 0.0);
            for (int a = 0; a < k; ++a)
                for (int b = 0; b <= a; ++b) {
                    cd d = S.dot(errs[a], errs[b])[0];
                    B[a * (k + 1) + b] = d;
                    B[b * (k + 1) + a] = std::conj(d);
                }
            for (int a = 0; a < k; ++a) { B[a * (k + 1) + k] = -1.0; B[k * (k + 1) + a] = -1.0; }
            rhs[k] = -1.0;
            // Gaussian elimination with partial pivoting
            const int N = k + 1;
            std::vector<cd> A = B, x = rhs;
            for (int col = 0; col < N; ++col) {
                int piv = col;
                for (int r = col + 1; r < N; ++r) if (std::abs(A[r * N + col]) > std::abs(A[piv * N + col])) piv = r;
                for (int q = 0; q < N; ++q) std::swap(A[col * N + q], A[piv * N + q]);
                std::swap(x[col], x[piv]);
                if (std::abs(A[col * N + col]) < 1e-300) continue;
                for (int r = col + 1; r < N; ++r) {
                    cd f = A[r * N + col] / A[col * N + col];
                    for (int q = col; q < N; ++q) A[r * N + q] -= f * A[col * N + q];
                    x[r] -= f * x[col];
                }
            }
            for (int r = N - 1; r >= 0; --r) {
                cd acc = x[r];
                for (int q = r + 1; q < N; ++q) acc -= A[r * N + q] * x[q];
                x[r] = std::abs(A[r * N + r]) > 1e-300 ? acc / A[r * N + r] : 0.0;
            }
            S.zero(T);
            for (int a = 0; a < k; ++a) S.axpby(T, hist[a], std::vector<cd>(1, x[a]), 1.0);
        } else {
            S.copy(T, tn);
        }
    }
    // converged amplitudes into the state (crystal normalisation) and every derived block
    HIPCHK(scale_copy(c->s64.t1.p, T.s, 1.0, 0.0, S.n1, st));
    HIPCHK(scale_copy(c->s64.t2.p, T.d, 1.0 / nk, 0.0, S.n2, st));
    run_precompute(c, true, st);
    // energy per cell (Eq. ene): (1/Nk) [f_ia t_ia + 1/4 <ij||ab> tau_ijab] in supercell quantities
    {
        State<double> &Sd = c->s64;
        Vecs tau{Sd.t1.p, Sd.tau.p}, f{Sd.fov.p, c->g_oovv.p};
        cd e1, e2;
        HIPCHK(batched_dot(Sd.fov.p, Sd.t1.p, 1, S.n1, 1.0, S.part, S.dout, st, 0));
        HIPCHK(hipMemcpy(&e1, S.dout, 16, hipMemcpyDeviceToHost));
        HIPCHK(batched_dot(c->g_oovv.p, Sd.tau.p, 1, S.n2, 0.25, S.part, S.dout, st, 0));
        HIPCHK(hipMemcpy(&e2, S.dout, 16, hipMemcpyDeviceToHost));
        energy = (e1 + e2).real() / nk;
        (void)tau; (void)f;
    }
    c->amp = true;
    c->lam_valid = false;
    rep = lrcc_solve_report{};
    rep.converged = rn <= tol;
    rep.outer = it + 1;
    rep.sigma_fp64 = (int)S.rhs_sig;
    rep.rhs_sigmas = S.rhs_sig;
    rep.max_rel_residual = rn;
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Device copies of the Hamiltonian and the stored integral blocks (all but vvvv).
void setup_hamiltonian(lrcc_ctx *c, int nk, int nocc, int nvir, int naux, const double *fock, const double *chol,
                       const double *dip) {
    const int n = nocc + nvir;
    c->ham = c->amp = false;
    c->progs.clear();
    c->progmem.clear();
    c->pre64.reset();
    c->pre32.reset();
    for (int x = 0; x < 3; ++x) { c->prex[x].reset(); c->xs[x].mem.release(); c->xs[x].ready = false; }
    c->prog_xi.reset();
    c->prog_grad.reset();
    c->prog_epp.reset();
    c->amem.release();
    c->linU_T = c->linU_y = c->linW_T = c->linW_y = c->lin_tmp = nullptr;
    c->lin_T_ready = c->lin_on = false;
    c->solv.release();
    c->sol1 = c->sol2 = nullptr;
    c->sol_bytes = 0;
    c->nfreq = 0;
    c->nrhs_sol = 0;
    c->axes.clear();
    c->alpha.clear();
    c->last_omega.clear();
    // one-body density programs and their amplitude copies (sized by the old shape)
    c->dens.clear();
    c->densmem.clear();
    c->gmem.release();
    c->dT1 = KT{};
    c->dT2 = KT{};
    // staging and vector-Jacobian scratch (sized by the old shape)
    c->stage.release();
    c->stage_b1 = c->stage_b2 = c->stage_nrhs = 0;
    c->vjpmem.release();
    c->vjp_n1 = c->vjp_n2 = 0;
    c->guess.clear();
    ++c->gen;
    c->lam_valid = false;
    c->s64.ready = c->s32.ready = false;
    c->s64.mem.release();
    c->s32.mem.release();
    c->hmem.release();
    c->nk = nk; c->no = nocc; c->nv = nvir; c->naux = naux; c->n = n;
    if (!c->km_set) c->km = KMesh{nk, 1, 1};
    const i64 nL = (i64)nk * nk * naux * n * n;
    c->fock = c->hmem.get((size_t)nk * n * n * 16);
    if (!g_dry_run) HIPCHK(hipMemcpy(c->fock, fock, (size_t)nk * n * n * 16, hipMemcpyHostToDevice));
    c->dip = c->hmem.get((size_t)3 * nk * n * n * 16);
    if (!g_dry_run && dip) HIPCHK(hipMemcpy(c->dip, dip, (size_t)3 * nk * n * n * 16, hipMemcpyHostToDevice));
    c->eps_o = c->hmem.get((size_t)nk * nocc * 8);
    c->eps_v = c->hmem.get((size_t)nk * nvir * 8);
    if (!g_dry_run) {
        std::vector<double> eo((size_t)nk * nocc), ev((size_t)nk * nvir);
        for (int k = 0; k < nk; ++k)
            for (int p = 0; p < n; ++p) {
                const double d = fock[2 * (((size_t)k * n + p) * n + p)];
                if (p < nocc) eo[(size_t)k * nocc + p] = d; else ev[(size_t)k * nvir + p - nocc] = d;
            }
        HIPCHK(hipMemcpy(c->eps_o, eo.data(), eo.size() * 8, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->eps_v, ev.data(), ev.size() * 8, hipMemcpyHostToDevice));
    }
    void *Lraw = c->hmem.get(nL * 16);
    if (!g_dry_run) HIPCHK(hipMemcpy(Lraw, chol, nL * 16, hipMemcpyHostToDevice));
    c->Ls = c->hmem.get(nL * 16);
    c->Lcs = c->hmem.get(nL * 16);
    const double sc = 1.0 / std::sqrt((double)nk);
    if (!g_dry_run) {
        HIPCHK(chol_slice<double>(Lraw, c->Ls, nk, naux, n, 0, n, 0, n, sc, 0, nullptr));
        HIPCHK(chol_slice<double>(Lraw, c->Lcs, nk, naux, n, 0, n, 0, n, sc, 1, nullptr));
    }
    Program P;
    c->g_oooo = alloc_kt<double>(c, c->hmem, "oooo");
    c->g_ooov = alloc_kt<double>(c, c->hmem, "ooov");
    c->g_oovv = alloc_kt<double>(c, c->hmem, "oovv");
    c->g_ovov = alloc_kt<double>(c, c->hmem, "ovov");
    c->g_ovvo = alloc_kt<double>(c, c->hmem, "ovvo");
    c->g_ovvv = alloc_kt<double>(c, c->hmem, "ovvv");
    c->g_ovoo = alloc_kt<double>(c, c->hmem, "ovoo");
    for (KT *t : {&c->g_oooo, &c->g_ooov, &c->g_oovv, &c->g_ovov, &c->g_ovvo, &c->g_ovvv, &c->g_ovoo})
        build_eri(c, P, *t, 1.0);
    if (!g_dry_run) {
        HIPCHK(P.run(nullptr));
        HIPCHK(hipDeviceSynchronize());
    }
}

template <typename F>
lrcc_status guarded(lrcc_ctx *c, F &&f) {
    if (!c) return LRCC_E_ARG;
    try {
        HIPCHK(hipSetDevice(c->dev));
        f();
        c->err.clear();
        return LRCC_OK;
    } catch (LrccError &e) {
        c->err = e.what();
        return (lrcc_status)e.code;
    } catch (std::exception &e) {
        c->err = e.what();
        return LRCC_E_HIP;
    }
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

lrcc_status lrcc_create(int hip_device, lrcc_ctx **out) {
    if (!out) return LRCC_E_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        g_create_err = "no HIP device available";
        return LRCC_E_HIP;
    }
    if (hip_device < 0 || hip_device >= n) {
        g_create_err = "device index out of range";
        return LRCC_E_ARG;
    }
    if (hipSetDevice(hip_device) != hipSuccess) {
        g_create_err = "hipSetDevice failed";
        return LRCC_E_HIP;
    }
    auto *c = new lrcc_ctx();
    c->dev = hip_device;
    *out = c;
    return LRCC_OK;
}

void lrcc_destroy(lrcc_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->dev);
    (void)hipDeviceSynchronize();
    c->progs.clear();
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

const char *lrcc_last_error(const lrcc_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

}  // extern "C"

// Hermiticity of cnt complex [n][n] blocks (relative tolerance 1e-10) -> LRCC_E_ARG
static void check_hermitian(const double *m, int cnt, int n, const char *what) {
    double mx = 0, dev = 0;
    for (int b = 0; b < cnt; ++b)
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                const double *x = m + 2 * (((i64)b * n + p) * n + q), *y = m + 2 * (((i64)b * n + q) * n + p);
                dev = std::max(dev, std::max(std::fabs(x[0] - y[0]), std::fabs(x[1] + y[1])));
                mx = std::max(mx, std::max(std::fabs(x[0]), std::fabs(x[1])));
            }
    if (dev > 1e-10 * std::max(1.0, mx)) throw LrccError(LRCC_E_ARG, std::string(what) + " is not Hermitian");
}

extern "C" {

lrcc_status lrcc_set_kmesh(lrcc_ctx *c, int n0, int n1, int n2) {
    return guarded(c, [&] {
        if (n0 < 1 || n1 < 1 || n2 < 1 || (i64)n0 * n1 * n2 > 46340)
            throw LrccError(LRCC_E_ARG, "mesh extents must be positive (and n0 n1 n2 at most 46340)");
        c->km = KMesh{n0, n1, n2};
        c->km_set = true;
        c->ham = c->amp = false;
        c->nfreq = 0;
        c->lam_valid = false;
        c->guess.clear();
        ++c->gen;
    });
}

lrcc_status lrcc_set_hamiltonian(lrcc_ctx *c, int nk, int nocc, int nvir, int naux, const double *fock,
                                 const double *chol, const double *dip) {
    return guarded(c, [&] {
        if (nk < 1 || nocc < 1 || nvir < 1 || naux < 1 || !fock || !chol || !dip)
            throw LrccError(LRCC_E_ARG, "invalid sizes or null pointer");
        if (c->km_set && c->km.size() != nk)
            throw LrccError(LRCC_E_SHAPE, "nk differs from the number of points of the k mesh");
        const int n = nocc + nvir;
        check_hermitian(fock, nk, n, "fock");
        check_hermitian(dip, 3 * nk, n, "dip");
        // Hermitian pairing chol[k2][k1][Q] = conj(chol[k1][k2][Q])^T
        double mx = 0, dev = 0;
        for (int k1 = 0; k1 < nk; ++k1)
            for (int k2 = 0; k2 < nk; ++k2)
                for (int Q = 0; Q < naux; ++Q)
                    for (int p = 0; p < n; ++p)
                        for (int q = 0; q < n; ++q) {
                            const double *x = chol + 2 * ((((i64)(k1 * nk + k2) * naux + Q) * n + p) * n + q);
                            const double *y = chol + 2 * ((((i64)(k2 * nk + k1) * naux + Q) * n + q) * n + p);
                            dev = std::max(dev, std::max(std::fabs(x[0] - y[0]), std::fabs(x[1] + y[1])));
                            mx = std::max(mx, std::max(std::fabs(x[0]), std::fabs(x[1])));
                        }
        if (dev > 1e-10 * std::max(1.0, mx)) throw LrccError(LRCC_E_ARG, "chol violates the Hermitian pairing");
        setup_hamiltonian(c, nk, nocc, nvir, naux, fock, chol, dip);
        c->ham = true;
    });
}

lrcc_status lrcc_set_amplitudes(lrcc_ctx *c, const double *t1, const double *t2) {
    return guarded(c, [&] {
        if (!c->ham) throw LrccError(LRCC_E_STATE, "set_hamiltonian must be called first");
        if (!t1 || !t2) throw LrccError(LRCC_E_ARG, "null amplitude pointer");
        const int nk = c->nk, o = c->no, v = c->nv;
        // antisymmetry of t2 in (i,j) and (a,b) across k blocks
        double mx = 0, dev = 0;
        auto at = [&](int ki, int kj, int ka, int i, int j, int a, int b) {
            return t2 + 2 * ((((((i64)(ki * nk + kj) * nk + ka) * o + i) * o + j) * v + a) * v + b);
        };
        for (int ki = 0; ki < nk; ++ki)
            for (int kj = 0; kj < nk; ++kj)
                for (int ka = 0; ka < nk; ++ka) {
                    const int kb = c->km.comb(ki, kj, ka);
                    for (int i = 0; i < o; ++i)
                        for (int j = 0; j < o; ++j)
                            for (int a = 0; a < v; ++a)
                                for (int b = 0; b < v; ++b) {
                                    const double *x = at(ki, kj, ka, i, j, a, b);
                                    const double *y = at(kj, ki, ka, j, i, a, b);
                                    const double *z = at(ki, kj, kb, i, j, b, a);
                                    dev = std::max({dev, std::fabs(x[0] + y[0]), std::fabs(x[1] + y[1]),
                                                    std::fabs(x[0] + z[0]), std::fabs(x[1] + z[1])});
                                    mx = std::max({mx, std::fabs(x[0]), std::fabs(x[1])});
                                }
                }
        if (dev > 1e-10 * std::max(1.0, mx)) throw LrccError(LRCC_E_ARG, "t2 is not antisymmetric");
        c->amp = false;
        if (!c->s64.ready) build_state(c);
        upload_amplitudes(c, t1, t2);
        run_precompute(c, true);
        c->amp = true;
        c->lam_valid = false;
    });
}

lrcc_status lrcc_apply_sigma_dev(lrcc_ctx *c, int nrhs, const double *omega, const void *x1, const void *x2,
                                 void *y1, void *y2, int precision, void *stream) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nrhs < 1 || !x1 || !x2 || !y1 || !y2) throw LrccError(LRCC_E_ARG, "invalid nrhs or null pointer");
        if (precision != LRCC_FP64 && precision != LRCC_FP32) throw LrccError(LRCC_E_ARG, "unknown precision");
        Program *p = sigma_program(c, precision, nrhs);
        c->io_x1 = x1; c->io_x2 = x2; c->io_y1 = y1; c->io_y2 = y2; c->io_omega = omega;
        HIPCHK(run_sigma(c, p, (hipStream_t)stream));
    });
}

lrcc_status lrcc_apply_sigma_dev_noalloc(lrcc_ctx *c, int nrhs, const double *omega, const void *x1,
                                         const void *x2, void *y1, void *y2, int precision, void *stream) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nrhs < 1 || !x1 || !x2 || !y1 || !y2) throw LrccError(LRCC_E_ARG, "invalid nrhs or null pointer");
        if (precision != LRCC_FP64 && precision != LRCC_FP32) throw LrccError(LRCC_E_ARG, "unknown precision");
        hipStream_t st = (hipStream_t)stream;
        size_t cap = 0;
        void *base = noalloc_scratch(c->dev, &cap);
        // the previous call on this stream may still read the array the recording overwrites
        HIPCHK(hipStreamSynchronize(st));
        // record the sigma program with every device allocation taken from the static array
        std::unique_ptr<Program> p;
        DevMem wm;
        arena_begin(base, cap);
        try {
            p.reset(precision == LRCC_FP64 ? build_sigma<double>(c, c->s64, nrhs, wm)
                                           : build_sigma<float>(c, c->s32, nrhs, wm));
        } catch (...) {
            arena_end();
            throw;
        }
        arena_end();
        c->io_x1 = x1; c->io_x2 = x2; c->io_y1 = y1; c->io_y2 = y2; c->io_omega = omega;
        HIPCHK(p->run(st));
    });
}

lrcc_status lrcc_apply_sigma_adjoint_dev(lrcc_ctx *c, int nrhs, const double *omega, const void *x1, const void *x2,
                                         void *y1, void *y2, int precision, void *stream) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nrhs < 1 || !x1 || !x2 || !y1 || !y2) throw LrccError(LRCC_E_ARG, "invalid nrhs or null pointer");
        if (precision != LRCC_FP64 && precision != LRCC_FP32) throw LrccError(LRCC_E_ARG, "unknown precision");
        Program *p = sigma_program(c, precision, nrhs, true);
        c->io_x1 = x1; c->io_x2 = x2; c->io_y1 = y1; c->io_y2 = y2; c->io_omega = omega;
        HIPCHK(run_sigma(c, p, (hipStream_t)stream));
    });
}

lrcc_status lrcc_sigma_vjp_dev(lrcc_ctx *c, int nrhs, const double *omega, const void *g1, const void *g2,
                               void *gx1, void *gx2, int precision, void *stream) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nrhs < 1 || !g1 || !g2 || !gx1 || !gx2) throw LrccError(LRCC_E_ARG, "invalid nrhs or null pointer");
        if (precision != LRCC_FP64 && precision != LRCC_FP32) throw LrccError(LRCC_E_ARG, "unknown precision");
        const int nk = c->nk, o = c->no, v = c->nv;
        const i64 n1 = (i64)nrhs * nk * o * v, n2 = (i64)nrhs * nk * nk * nk * o * o * v * v;
        if (n1 > c->vjp_n1 || n2 > c->vjp_n2) {
            // each buffer must hold its own part: grow both when either is too small
            c->vjpmem.release();
            c->vjp_n1 = std::max(n1, c->vjp_n1);
            c->vjp_n2 = std::max(n2, c->vjp_n2);
            c->vj1 = c->vjpmem.get(c->vjp_n1 * 16); c->vj2 = c->vjpmem.get(c->vjp_n2 * 16);
            c->vw1 = c->vjpmem.get(c->vjp_n1 * 16); c->vw2 = c->vjpmem.get(c->vjp_n2 * 16);
        }
        hipStream_t st = (hipStream_t)stream;
        // z = (conj g1, P conj g2): the cotangent restricted to antisymmetric doubles, in the
        // pairing sum z1 y1 + 1/4 sum z2 y2 of the transpose product
        HIPCHK(conj_scale(c->vj1, g1, 1.0, n1, st));
        HIPCHK(antisym(g2, c->vj2, nrhs, c->km, o, v, 1.0, 1, st));
        Program *p = sigma_program(c, precision, nrhs, true);
        c->io_x1 = c->vj1; c->io_x2 = c->vj2; c->io_y1 = c->vw1; c->io_y2 = c->vw2; c->io_omega = omega;
        HIPCHK(run_sigma(c, p, st));
        // back to the Euclidean pairing over full arrays, projected on antisymmetric doubles
        HIPCHK(conj_scale(gx1, c->vw1, 1.0, n1, st));
        HIPCHK(antisym(c->vw2, gx2, nrhs, c->km, o, v, 1.0 / 16.0, 1, st));
    });
}

static lrcc_status apply_host(lrcc_ctx *c, int nrhs, const double *omega, const double *x1, const double *x2,
                              double *y1, double *y2, int precision, bool adjoint);

lrcc_status lrcc_apply_sigma_adjoint(lrcc_ctx *c, int nrhs, const double *omega, const double *x1,
                                     const double *x2, double *y1, double *y2, int precision) {
    return apply_host(c, nrhs, omega, x1, x2, y1, y2, precision, true);
}

lrcc_status lrcc_apply_sigma(lrcc_ctx *c, int nrhs, const double *omega, const double *x1, const double *x2,
                             double *y1, double *y2, int precision) {
    return apply_host(c, nrhs, omega, x1, x2, y1, y2, precision, false);
}

static lrcc_status apply_host(lrcc_ctx *c, int nrhs, const double *omega, const double *x1, const double *x2,
                              double *y1, double *y2, int precision, bool adjoint) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nrhs < 1 || !x1 || !x2 || !y1 || !y2) throw LrccError(LRCC_E_ARG, "invalid nrhs or null pointer");
        const int nk = c->nk, o = c->no, v = c->nv;
        const size_t b1 = (size_t)nrhs * nk * o * v * 16, b2 = (size_t)nrhs * nk * nk * nk * o * o * v * v * 16;
        if (b1 > c->stage_b1 || b2 > c->stage_b2 || (size_t)nrhs > c->stage_nrhs) {
            // each staging buffer must hold its own part: grow all when any is too small
            c->stage.release();
            c->stage_b1 = std::max(b1, c->stage_b1);
            c->stage_b2 = std::max(b2, c->stage_b2);
            c->stage_nrhs = std::max((size_t)nrhs, c->stage_nrhs);
            c->st_x1 = c->stage.get(c->stage_b1); c->st_y1 = c->stage.get(c->stage_b1);
            c->st_x2 = c->stage.get(c->stage_b2); c->st_y2 = c->stage.get(c->stage_b2);
            c->st_om = c->stage.get(c->stage_nrhs * 8);
        }
        HIPCHK(hipMemcpy(c->st_x1, x1, b1, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->st_x2, x2, b2, hipMemcpyHostToDevice));
        std::vector<double> om(nrhs, 0.0);
        if (omega) for (int r = 0; r < nrhs; ++r) om[r] = omega[r];
        HIPCHK(hipMemcpy(c->st_om, om.data(), nrhs * 8, hipMemcpyHostToDevice));
        lrcc_status s = adjoint ? lrcc_apply_sigma_adjoint_dev(c, nrhs, (const double *)c->st_om, c->st_x1,
                                                               c->st_x2, c->st_y1, c->st_y2, precision, nullptr)
                                : lrcc_apply_sigma_dev(c, nrhs, (const double *)c->st_om, c->st_x1, c->st_x2,
                                                       c->st_y1, c->st_y2, precision, nullptr);
        if (s != LRCC_OK) throw LrccError(s, c->err);
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(y1, c->st_y1, b1, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(y2, c->st_y2, b2, hipMemcpyDeviceToHost));
    });
}

void lrcc_solve_opts_default(lrcc_solve_opts *o) {
    if (o) default_opts(*o);
}

lrcc_status lrcc_solve_response_dev(lrcc_ctx *c, int nrhs, const double *omega, const void *b1, const void *b2,
                                    void *x1, void *x2, const lrcc_solve_opts *opts, lrcc_solve_report *report,
                                    void *stream) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nrhs < 1 || !b1 || !b2 || !x1 || !x2) throw LrccError(LRCC_E_ARG, "invalid nrhs or null pointer");
        lrcc_solve_opts o;
        default_opts(o);
        if (opts) o = *opts;
        if (o.precision != LRCC_FP64 && o.precision != LRCC_FP32) throw LrccError(LRCC_E_ARG, "unknown precision");
        if (!(o.tol > 0) || o.krylov < 0 || o.max_iter < 1) throw LrccError(LRCC_E_ARG, "bad solver options");
        lrcc_solve_report rep;
        Vecs b{const_cast<void *>(b1), const_cast<void *>(b2)}, x{x1, x2};
        hipStream_t st = (hipStream_t)stream;
        if (!st) {
            if (!c->own_stream) HIPCHK(hipStreamCreate(&c->own_stream));
            st = c->own_stream;
        }
        bool sing = false;
        solve_response(c, nrhs, omega, b, x, o, rep, st, false, false, &sing);
        if (report) *report = rep;
        if (!rep.converged) throw_unconverged("response solve", rep, sing);
    });
}

lrcc_status lrcc_solve_response(lrcc_ctx *c, int nrhs, const double *omega, const double *b1, const double *b2,
                                double *x1, double *x2, const lrcc_solve_opts *opts, lrcc_solve_report *report) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nrhs < 1 || !b1 || !b2 || !x1 || !x2) throw LrccError(LRCC_E_ARG, "invalid nrhs or null pointer");
        const int nk = c->nk, o = c->no, v = c->nv;
        const size_t s1 = (size_t)nrhs * nk * o * v * 16, s2 = (size_t)nrhs * nk * nk * nk * o * o * v * v * 16;
        DevMem m;
        void *db1 = m.get(s1), *db2 = m.get(s2), *dx1 = m.get(s1), *dx2 = m.get(s2), *dom = m.get(nrhs * 8);
        HIPCHK(hipMemcpy(db1, b1, s1, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(db2, b2, s2, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dx1, x1, s1, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dx2, x2, s2, hipMemcpyHostToDevice));
        std::vector<double> om(nrhs, 0.0);
        if (omega) for (int r = 0; r < nrhs; ++r) om[r] = omega[r];
        HIPCHK(hipMemcpy(dom, om.data(), nrhs * 8, hipMemcpyHostToDevice));
        lrcc_status st = lrcc_solve_response_dev(c, nrhs, (const double *)dom, db1, db2, dx1, dx2, opts, report, nullptr);
        const bool unconverged = st == LRCC_E_NOCONV || st == LRCC_E_SINGULAR;
        if (st != LRCC_OK && !unconverged) throw LrccError(st, c->err);
        HIPCHK(hipMemcpy(x1, dx1, s1, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(x2, dx2, s2, hipMemcpyDeviceToHost));
        if (unconverged) throw LrccError(st, c->err);
    });
}

lrcc_status lrcc_solve(lrcc_ctx *c, unsigned axis_mask, int nfreq, const double *omega, const lrcc_solve_opts *opts,
                       lrcc_solve_report *report) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nfreq < 1 || !omega || (axis_mask & ~7u)) throw LrccError(LRCC_E_ARG, "invalid frequencies or axis mask");
        lrcc_solve_opts o;
        default_opts(o);
        if (opts) o = *opts;
        if (o.precision != LRCC_FP64 && o.precision != LRCC_FP32) throw LrccError(LRCC_E_ARG, "unknown precision");
        if (!(o.tol > 0) || o.krylov < 0 || o.max_iter < 1) throw LrccError(LRCC_E_ARG, "bad solver options");
        for (int j = 0; j < nfreq; ++j)
            if (!std::isfinite(omega[j])) throw LrccError(LRCC_E_ARG, "frequencies must be finite");
        lrcc_solve_report rep{};
        c->nfreq = 0;
        try {
            solve_alpha(c, axis_mask, nfreq, omega, o, rep);
        } catch (LrccError &) {
            if (report) *report = rep;   // the report of the failing solve
            throw;
        }
        if (report) *report = rep;
    });
}

lrcc_status lrcc_alpha_velocity_gauge(lrcc_ctx *c, unsigned axis_mask, int nfreq, const double *omega,
                                      const double *mom, const lrcc_solve_opts *opts, double *alpha,
                                      lrcc_solve_report *report) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nfreq < 1 || !omega || !mom || !alpha || (axis_mask & ~7u))
            throw LrccError(LRCC_E_ARG, "invalid frequencies, axis mask or null pointer");
        for (int j = 0; j < nfreq; ++j)
            if (!(omega[j] != 0.0) || !std::isfinite(omega[j]))
                throw LrccError(LRCC_E_ARG, "velocity-gauge frequencies must be finite and non-zero");
        check_hermitian(mom, 3 * c->nk, c->n, "mom");
        lrcc_solve_opts o;
        default_opts(o);
        if (opts) o = *opts;
        if (o.precision != LRCC_FP64 && o.precision != LRCC_FP32) throw LrccError(LRCC_E_ARG, "unknown precision");
        lrcc_solve_report rep{};
        // the perturbation operators are read from the dipole buffer by the xi and eta
        // programs: swap the momentum matrices in for this solve, restore afterwards
        const size_t bytes = (size_t)3 * c->nk * c->n * c->n * 16;
        DevMem keep;
        void *saved = keep.get(bytes);
        HIPCHK(hipMemcpy(saved, c->dip, bytes, hipMemcpyDeviceToDevice));
        struct Restore {
            lrcc_ctx *c;
            void *saved;
            size_t bytes;
            ~Restore() {
                (void)hipMemcpy(c->dip, saved, bytes, hipMemcpyDeviceToDevice);
                c->nfreq = 0;   // the stored solutions are those of the momentum operator
            }
        } restore{c, saved, bytes};
        HIPCHK(hipMemcpy(c->dip, mom, bytes, hipMemcpyHostToDevice));
        std::vector<double> w(nfreq + 1, 0.0);
        for (int j = 0; j < nfreq; ++j) w[j + 1] = omega[j];
        c->nfreq = 0;
        solve_alpha(c, axis_mask, nfreq + 1, w.data(), o, rep);
        for (int j = 0; j < nfreq; ++j)
            for (int e = 0; e < 18; ++e)
                alpha[j * 18 + e] = (c->alpha[(size_t)(j + 1) * 18 + e] - c->alpha[e]) / (omega[j] * omega[j]);
        if (report) *report = rep;
    });
}

lrcc_status lrcc_solve_ccsd(lrcc_ctx *c, double tol, int max_iter, double *t1, double *t2, double *energy,
                            lrcc_solve_report *report) {
    return guarded(c, [&] {
        if (!c->ham) throw LrccError(LRCC_E_STATE, "set_hamiltonian must be called first");
        if (!(tol > 0) || max_iter < 1) throw LrccError(LRCC_E_ARG, "bad tolerance or iteration limit");
        lrcc_solve_report rep{};
        double e = 0;
        solve_ccsd(c, tol, max_iter, 8, rep, e);
        if (energy) *energy = e;
        if (report) *report = rep;
        const i64 n1 = (i64)c->nk * c->no * c->nv, n2 = (i64)c->nk * c->nk * c->nk * c->no * c->no * c->nv * c->nv;
        if (t1) HIPCHK(hipMemcpy(t1, c->s64.t1.p, n1 * 16, hipMemcpyDeviceToHost));
        if (t2) {
            HIPCHK(hipMemcpy(t2, c->s64.t2.p, n2 * 16, hipMemcpyDeviceToHost));
            for (i64 q = 0; q < 2 * n2; ++q) t2[q] *= c->nk;
        }
        if (!rep.converged) throw LrccError(LRCC_E_NOCONV, "CCSD did not converge: |Omega| = " + std::to_string(rep.max_rel_residual));
    });
}

lrcc_status lrcc_alpha_dipole_gradient(lrcc_ctx *c, int ifreq, int x, int y, const lrcc_solve_opts *opts,
                                       double *grad) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (!grad || x < 0 || x > 2 || y < 0 || y > 2) throw LrccError(LRCC_E_ARG, "invalid axis or null pointer");
        lrcc_solve_opts o;
        default_opts(o);
        if (opts) o = *opts;
        alpha_dip_grad(c, ifreq, x, y, o, grad);
    });
}

lrcc_status lrcc_alpha_chol_gradient(lrcc_ctx *c, int ifreq, int x, int y, const lrcc_solve_opts *opts,
                                     double *grad) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (!grad || x < 0 || x > 2 || y < 0 || y > 2) throw LrccError(LRCC_E_ARG, "invalid axis or null pointer");
        lrcc_solve_opts o;
        default_opts(o);
        if (opts) o = *opts;
        alpha_chol_grad(c, ifreq, x, y, o, grad);
    });
}

lrcc_status lrcc_alpha_fock_gradient(lrcc_ctx *c, int ifreq, int x, int y, const lrcc_solve_opts *opts,
                                    double *grad) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (!grad || x < 0 || x > 2 || y < 0 || y > 2) throw LrccError(LRCC_E_ARG, "invalid axis or null pointer");
        lrcc_solve_opts o;
        default_opts(o);
        if (opts) o = *opts;
        alpha_fock_grad(c, ifreq, x, y, o, grad);
    });
}

struct lrcc_group {
    std::vector<lrcc_ctx *> ctx;
    std::string err;
    // per (precision, nrhs and joined flag per chain): device tables of the joint ladder launch,
    // with the generations of the chains' contexts they were built from (the tables copy the
    // chains' buffer addresses and shapes, which a new Hamiltonian, mesh or state replaces)
    std::map<std::vector<int>, std::unique_ptr<DevMem>> tabmem;
    std::map<std::vector<int>, LadderGroup> tab;
    std::map<std::vector<int>, std::vector<unsigned long long>> tabgen;
    unsigned *counter = nullptr;
    DevMem mem;
    int nblocks = 0;
};

lrcc_status lrcc_group_create(lrcc_ctx *const *ctxs, int n, lrcc_group **out) {
    if (!out || !ctxs || n < 1) return LRCC_E_ARG;
    *out = nullptr;
    try {
        auto g = std::make_unique<lrcc_group>();
        for (int i = 0; i < n; ++i) {
            if (!ctxs[i]) return LRCC_E_ARG;
            if (ctxs[i]->dev != ctxs[0]->dev) return LRCC_E_ARG;
            g->ctx.push_back(ctxs[i]);
        }
        if (hipSetDevice(ctxs[0]->dev) != hipSuccess) return LRCC_E_HIP;
        g->counter = (unsigned *)g->mem.get(256);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctxs[0]->dev) != hipSuccess) return LRCC_E_HIP;
        g->nblocks = prop.multiProcessorCount;
        *out = g.release();
        return LRCC_OK;
    } catch (...) {
        return LRCC_E_OOM;
    }
}

void lrcc_group_destroy(lrcc_group *g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx[0]->dev);
    delete g;
}

const char *lrcc_group_last_error(const lrcc_group *g) { return g ? g->err.c_str() : "null group"; }

}  // extern "C"

template <typename T>
static void group_apply(lrcc_group *g, const int *nrhs, const double *const *omega, const void *const *x1,
                        const void *const *x2, void *const *y1, void *const *y2, int precision, hipStream_t st) {
    const int n = (int)g->ctx.size();
    std::vector<Program *> prog(n);
    std::vector<int> join;
    std::vector<int> key{precision};
    for (int i = 0; i < n; ++i) {
        lrcc_ctx *c = g->ctx[i];
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called on every chain");
        if (nrhs[i] < 1 || !x1[i] || !x2[i] || !y1[i] || !y2[i]) throw LrccError(LRCC_E_ARG, "invalid nrhs or null pointer");
        prog[i] = sigma_program(c, precision, nrhs[i]);
        const Program *p = prog[i];
        const bool j = p->ladder_args && p->ladder_args->packed == 2;
        if (j) join.push_back(i);
        key.push_back(nrhs[i]);
        key.push_back(j ? 1 : 0);
    }
    std::vector<unsigned long long> gens(n);
    for (int i = 0; i < n; ++i) gens[i] = g->ctx[i]->gen;
    auto io = [&](int i) {
        lrcc_ctx *c = g->ctx[i];
        c->io_x1 = x1[i]; c->io_x2 = x2[i]; c->io_y1 = y1[i]; c->io_y2 = y2[i]; c->io_omega = omega ? omega[i] : nullptr;
    };
    std::vector<bool> joined(n, false);
    for (int i : join) joined[i] = true;
    // everything before the ladder (whole programs for chains that do not join)
    for (int i = 0; i < n; ++i) {
        io(i);
        HIPCHK(prog[i]->run_range(st, 0, joined[i] ? prog[i]->ladder_op : prog[i]->ops.size()));
    }
    if (!join.empty()) {
        auto it = g->tab.find(key);
        if (it != g->tab.end() && g->tabgen[key] != gens) {
            // a chain's programs were rebuilt since this table was made: its addresses are stale
            g->tab.erase(it);
            g->tabmem.erase(key);
            g->tabgen.erase(key);
            it = g->tab.end();
        }
        if (it == g->tab.end()) {
            // ladders by decreasing cost per item
            std::vector<int> order = join;
            auto cost = [&](int i) {
                const LadderArgs &a = *prog[i]->ladder_args;
                return (double)a.nk * a.v * a.v * (256.0 + a.naux);
            };
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
            std::vector<LadderArgs> args;
            std::vector<long long> start{0}, tiles;
            for (int i : order) {
                const LadderArgs a = ladder_prepared(*prog[i]->ladder_args);
                long long blocks = 0;
                args.push_back(a);
                tiles.push_back(ladder_group_tiles<T>(a, &blocks));
                start.push_back(start.back() + tiles.back() * blocks);
            }
            auto mem = std::make_unique<DevMem>();
            LadderGroup lg{};
            lg.args = (const LadderArgs *)mem->get(args.size() * sizeof(LadderArgs));
            lg.start = (const long long *)mem->get(start.size() * sizeof(long long));
            lg.tiles = (const long long *)mem->get(tiles.size() * sizeof(long long));
            HIPCHK(hipMemcpy((void *)lg.args, args.data(), args.size() * sizeof(LadderArgs), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy((void *)lg.start, start.data(), start.size() * sizeof(long long), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy((void *)lg.tiles, tiles.data(), tiles.size() * sizeof(long long), hipMemcpyHostToDevice));
            lg.n = (int)args.size();
            lg.total = start.back();
            lg.counter = g->counter;
            g->tabmem[key] = std::move(mem);
            g->tabgen[key] = gens;
            it = g->tab.emplace(key, lg).first;
        }
        HIPCHK(launch_ladder_group<T>(it->second, g->nblocks, st));
        for (int i : join) {
            io(i);
            HIPCHK(prog[i]->run_range(st, prog[i]->ladder_op + 1, prog[i]->ops.size()));
        }
    }
}

extern "C" {

lrcc_status lrcc_group_apply_sigma_dev(lrcc_group *g, const int *nrhs, const double *const *omega,
                                       const void *const *x1, const void *const *x2, void *const *y1,
                                       void *const *y2, int precision, void *stream) {
    if (!g) return LRCC_E_ARG;
    try {
        if (!nrhs || !x1 || !x2 || !y1 || !y2) throw LrccError(LRCC_E_ARG, "null argument array");
        if (precision != LRCC_FP64 && precision != LRCC_FP32) throw LrccError(LRCC_E_ARG, "unknown precision");
        HIPCHK(hipSetDevice(g->ctx[0]->dev));
        if (precision == LRCC_FP64) group_apply<double>(g, nrhs, omega, x1, x2, y1, y2, precision, (hipStream_t)stream);
        else group_apply<float>(g, nrhs, omega, x1, x2, y1, y2, precision, (hipStream_t)stream);
        g->err.clear();
        return LRCC_OK;
    } catch (LrccError &e) {
        g->err = e.what();
        return (lrcc_status)e.code;
    } catch (std::exception &e) {
        g->err = e.what();
        return LRCC_E_ARG;
    }
}

lrcc_status lrcc_eom_roots(lrcc_ctx *c, int nroots, double tol, int max_iter, double *omega,
                           lrcc_solve_report *report) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (!omega) throw LrccError(LRCC_E_ARG, "null output");
        std::vector<cd> w;
        lrcc_solve_report rep{};
        eom_roots(c, nroots, tol > 0 ? tol : 1e-8, max_iter > 0 ? max_iter : 200, w, rep);
        std::memcpy(omega, w.data(), w.size() * 16);
        if (report) *report = rep;
        if (!rep.converged) throw LrccError(LRCC_E_NOCONV, "Davidson iteration did not converge");
    });
}

lrcc_status lrcc_alpha_lambda_bar(lrcc_ctx *c, int nfreq, const lrcc_solve_opts *opts, double *alpha,
                                  lrcc_solve_report *report) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (!alpha) throw LrccError(LRCC_E_ARG, "null output");
        if (nfreq != c->nfreq) throw LrccError(LRCC_E_ARG, "nfreq does not match the last solve");
        lrcc_solve_opts o;
        default_opts(o);
        if (opts) o = *opts;
        lrcc_solve_report rep{};
        alpha_lambda_bar(c, o, alpha, rep);
        if (report) *report = rep;
    });
}

lrcc_status lrcc_get_alpha(const lrcc_ctx *cc, int nfreq, double *alpha) {
    lrcc_ctx *c = const_cast<lrcc_ctx *>(cc);   // only the error text is written
    return guarded(c, [&] {
        if (!alpha) throw LrccError(LRCC_E_ARG, "null output");
        if (c->nfreq == 0 || nfreq != c->nfreq) throw LrccError(LRCC_E_STATE, "no polarizability for that many frequencies");
        std::memcpy(alpha, c->alpha.data(), c->alpha.size() * 8);
    });
}

lrcc_status lrcc_get_solution(const lrcc_ctx *cc, int axis, int ifreq, int sign, double *x1, double *x2) {
    lrcc_ctx *c = const_cast<lrcc_ctx *>(cc);   // only the error text is written
    return guarded(c, [&] {
        if (!x1 || !x2 || (sign != 1 && sign != -1)) throw LrccError(LRCC_E_ARG, "bad argument");
        if (c->nfreq == 0 || ifreq < 0 || ifreq >= c->nfreq) throw LrccError(LRCC_E_STATE, "no solution stored");
        int a = -1;
        for (size_t q = 0; q < c->axes.size(); ++q) if (c->axes[q] == axis) a = (int)q;
        if (a < 0) throw LrccError(LRCC_E_ARG, "axis was not solved");
        const int nax = (int)c->axes.size();
        const int r = (ifreq * 2 + (sign > 0 ? 0 : 1)) * nax + a;
        const i64 n1 = (i64)c->nk * c->no * c->nv, n2 = (i64)c->nk * c->nk * c->nk * c->no * c->no * c->nv * c->nv;
        HIPCHK(hipMemcpy(x1, (char *)c->sol1 + (size_t)r * n1 * 16, n1 * 16, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(x2, (char *)c->sol2 + (size_t)r * n2 * 16, n2 * 16, hipMemcpyDeviceToHost));
    });
}

lrcc_status lrcc_set_guess(lrcc_ctx *c, int axis, int ifreq, int sign, const double *x1, const double *x2) {
    return guarded(c, [&] {
        if (!x1 || !x2 || axis < 0 || axis > 2 || ifreq < 0 || (sign != 1 && sign != -1))
            throw LrccError(LRCC_E_ARG, "bad axis, frequency index, sign or null pointer");
        if (!c->ham) throw LrccError(LRCC_E_STATE, "set_hamiltonian must be called first");
        const i64 n1 = (i64)c->nk * c->no * c->nv, n2 = (i64)c->nk * c->nk * c->nk * c->no * c->no * c->nv * c->nv;
        for (const double *x : {x1, x2}) {
            const i64 cnt = 2 * (x == x1 ? n1 : n2);
            for (i64 q = 0; q < cnt; ++q)
                if (!std::isfinite(x[q])) throw LrccError(LRCC_E_ARG, "guess holds a non-finite value");
        }
        auto m = std::make_unique<DevMem>();
        char *d = (char *)m->get((size_t)(n1 + n2) * 16);
        HIPCHK(hipMemcpy(d, x1, (size_t)n1 * 16, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d + (size_t)n1 * 16, x2, (size_t)n2 * 16, hipMemcpyHostToDevice));
        c->guess[{axis, ifreq, sign}] = std::move(m);
    });
}

lrcc_status lrcc_get_lambda(lrcc_ctx *c, double *l1, double *l2) {
    return guarded(c, [&] {
        if (!l1 || !l2) throw LrccError(LRCC_E_ARG, "null output");
        if (!c->lam_valid) throw LrccError(LRCC_E_STATE, "lambda not solved yet (call lrcc_solve)");
        const i64 n1 = (i64)c->nk * c->no * c->nv, n2 = (i64)c->nk * c->nk * c->nk * c->no * c->no * c->nv * c->nv;
        HIPCHK(hipMemcpy(l1, c->lam1, n1 * 16, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(l2, c->lam2, n2 * 16, hipMemcpyDeviceToHost));
    });
}

lrcc_status lrcc_set_ladder_mode(lrcc_ctx *c, int mode) {
    return guarded(c, [&] {
        if (mode < 0 || mode > 3) throw LrccError(LRCC_E_ARG, "ladder mode must be 0, 1, 2 or 3");
        if (c->s64.ready) throw LrccError(LRCC_E_STATE, "the ladder mode is fixed once amplitudes are set");
        c->ladder_mode = mode;
    });
}

lrcc_status lrcc_set_autotune(lrcc_ctx *c, int enable) {
    return guarded(c, [&] { c->autotune = enable != 0; });
}

lrcc_status lrcc_set_graphs(lrcc_ctx *c, int enable) {
    return guarded(c, [&] {
        c->use_graphs = enable != 0;
        if (!c->use_graphs)
            for (auto &p : c->progs) p.second->drop_graphs();
    });
}

lrcc_status lrcc_set_profiling(lrcc_ctx *c, int enable) {
    return guarded(c, [&] { c->prof.on = enable != 0; });
}

lrcc_status lrcc_read_profile(lrcc_ctx *c, double *ms, long long *count) {
    return guarded(c, [&] {
        if (!ms || !count) throw LrccError(LRCC_E_ARG, "null output");
        c->prof.read(ms, count);
    });
}

lrcc_status lrcc_sigma_flops(lrcc_ctx *c, int nrhs, int precision, double *executed) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (!executed || nrhs < 1) throw LrccError(LRCC_E_ARG, "bad argument");
        *executed = (double)sigma_program(c, precision, nrhs)->flops;
    });
}

lrcc_status lrcc_ladder_flops(lrcc_ctx *c, int nrhs, int precision, double *executed) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (!executed || nrhs < 1) throw LrccError(LRCC_E_ARG, "bad argument");
        Program *P = sigma_program(c, precision, nrhs);
        // the rebuild-in-LDS ladder: count for the kernel variant in use (the autotuner may
        // have replaced the one the program was recorded with)
        *executed = P->ladder_args ? ladder_executed_flops(*P->ladder_args, precision == LRCC_FP64)
                                   : (double)P->tag_flops[TAG_LADDER];
    });
}

lrcc_status lrcc_ladder_path(lrcc_ctx *c, int nrhs, int precision, int *path) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (!path || nrhs < 1) throw LrccError(LRCC_E_ARG, "bad argument");
        *path = sigma_program(c, precision, nrhs)->ladder_path;
    });
}

lrcc_status lrcc_ladder_mfma_flops(lrcc_ctx *c, int nrhs, int precision, double *mfma) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (!mfma || nrhs < 1) throw LrccError(LRCC_E_ARG, "bad argument");
        Program *P = sigma_program(c, precision, nrhs);
        const bool fp64 = precision == LRCC_FP64;
        *mfma = P->ladder_args ? ladder_mfma_flops(*P->ladder_args, fp64) : P->tag_mfma_flops(TAG_LADDER);
    });
}

lrcc_status lrcc_plan_check(int nk, int nocc, int nvir, int naux, int nrhs, char *msg, int msglen) {
    return lrcc_plan_check_mesh(nk, 1, 1, nocc, nvir, naux, nrhs, msg, msglen);
}

lrcc_status lrcc_plan_check_mesh(int n0, int n1, int n2, int nocc, int nvir, int naux, int nrhs, char *msg,
                                 int msglen) {
    if (msg && msglen > 0) msg[0] = 0;
    if (n0 < 1 || n1 < 1 || n2 < 1 || (i64)n0 * n1 * n2 > 46340 || nocc < 1 || nvir < 1 || naux < 1 || nrhs < 1)
        return LRCC_E_ARG;
    const int nk = n0 * n1 * n2;
    lrcc_status st = LRCC_OK;
    g_dry_run = true;
    try {
        lrcc_ctx c;
        c.km = KMesh{n0, n1, n2};
        c.km_set = true;
        setup_hamiltonian(&c, nk, nocc, nvir, naux, nullptr, nullptr, nullptr);
        c.ham = true;
        build_state(&c);
        c.amp = true;
        (void)sigma_program(&c, LRCC_FP64, nrhs);
        (void)sigma_program(&c, LRCC_FP32, nrhs);
        (void)sigma_program(&c, LRCC_FP64, nrhs, true);
        (void)sigma_program(&c, LRCC_FP32, nrhs, true);
        (void)sigma_program(&c, LRCC_FP64, 1, true);
        (void)sigma_program(&c, LRCC_FP64, 1, true, kLeanSigma);
        (void)sigma_program(&c, LRCC_FP64, 1, false, kLeanSigma);
        (void)sigma_program(&c, LRCC_FP64, 1, true, kRTermSigma);
        ensure_alpha_programs(&c);
        for (int x = 0; x < 3; ++x) (void)sigma_program(&c, LRCC_FP64, 1, true, 1 + x);
        (void)dens_program(&c, 1);
        (void)dens_program(&c, 4);
        // the class-at-a-time ladder (mode 3) records other launches
        c.ladder_mode = 3;
        c.progs.clear();
        c.progmem.clear();
        for (int adj = 0; adj < 2; ++adj) {
            (void)sigma_program(&c, LRCC_FP64, nrhs, adj != 0);
            (void)sigma_program(&c, LRCC_FP32, nrhs, adj != 0);
            (void)sigma_program(&c, LRCC_FP64, 1, adj != 0);
            (void)sigma_program(&c, LRCC_FP64, 1, adj != 0, kLeanSigma);
            if (adj) (void)sigma_program(&c, LRCC_FP64, 1, true, kRTermSigma);
        }
    } catch (LrccError &e) {
        st = (lrcc_status)e.code;
        if (msg && msglen > 0) snprintf(msg, msglen, "%s", e.what());
    } catch (std::exception &e) {
        st = LRCC_E_ARG;
        if (msg && msglen > 0) snprintf(msg, msglen, "%s", e.what());
    }
    g_dry_run = false;
    return st;
}

lrcc_status lrcc_sizes(const lrcc_ctx *c, long long *n1, long long *n2) {
    if (!c || !n1 || !n2) return LRCC_E_ARG;
    if (!c->ham) return LRCC_E_STATE;
    *n1 = (long long)c->nk * c->no * c->nv;
    *n2 = (long long)c->nk * c->nk * c->nk * c->no * c->no * c->nv * c->nv;
    return LRCC_OK;
}

}  // extern "C"
