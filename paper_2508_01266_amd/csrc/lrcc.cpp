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
#include <complex>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/lrcc.h"
#include "common.hpp"
#include "elem.hpp"
#include "plan.hpp"

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
            for (void *p : ptrs) (void)hipFree(p);
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
    KT Fae, Fmi, Fme, Fbe, Fmj, Wp, Wbar, Q, R, S, U, Yp, H, G2;
    void *La = nullptr, *Lb = nullptr;
    bool ready = false;
};

}  // namespace

struct lrcc_ctx {
    int dev = 0;
    std::string err;
    int nk = 0, no = 0, nv = 0, naux = 0, n = 0;
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
    size_t stage_bytes = 0;
    void *st_x1 = nullptr, *st_x2 = nullptr, *st_y1 = nullptr, *st_y2 = nullptr, *st_om = nullptr;
    Profiler prof;
};

static std::string g_create_err;

namespace {

KT make_kt(lrcc_ctx *c, const char *cls, void *p, int nR = 0, std::initializer_list<int> sg = {1, 1, -1, -1}) {
    KT t;
    t.p = p;
    t.cls = cls;
    t.nR = nR;
    t.nk = c->nk;
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
                    const int k3 = ((k0 + k1 - k2) % nk + nk) % nk;
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
void precompute(lrcc_ctx *c, const double *t1h, const double *t2h) {
    const int nk = c->nk, o = c->no, v = c->nv, n = c->n, naux = c->naux;
    State<double> &S = c->s64;
    S.mem.release();
    c->s32.mem.release();
    S.ready = c->s32.ready = false;
    c->progs.clear();
    c->progmem.clear();
    DevMem &m = S.mem;
    Program P;

    S.t1 = alloc_kt<double>(c, m, "ov");
    S.t2 = alloc_kt<double>(c, m, "oovv");
    // paper -> crystal normalisation of T2
    if (!g_dry_run) {
        HIPCHK(hipMemcpy(S.t1.p, t1h, S.t1.count() * 16, hipMemcpyHostToDevice));
        std::vector<double> tmp(S.t2.count() * 2);
        std::memcpy(tmp.data(), t2h, tmp.size() * sizeof(double));
        for (auto &x : tmp) x /= nk;
        HIPCHK(hipMemcpy(S.t2.p, tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice));
    }
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
        P.ops.push_back([=](hipStream_t s) { return tau_like<double>(t1p, t2p, t1p, tau, nk, 1, o, v, 0.5, 0, s); });
        P.ops.push_back([=](hipStream_t s) { return tau_like<double>(t1p, t2p, t1p, ttp, nk, 1, o, v, 0.25, 0, s); });
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
    contract<double>(P, S.Wbar, "mbej", t2, "jnfb", oovv, "mnef", -1.0);
    KT ytmp = alloc_kt<double>(c, m, "oovo");
    contract<double>(P, ytmp, "mnej", t1, "jf", oovv, "mnef", 1.0, false);
    contract<double>(P, S.Wbar, "mbej", t1, "nb", ytmp, "mnej", -1.0);
    // Q_ijam = sum_ef tau_ijef <am||ef>
    S.Q = alloc_kt<double>(c, m, "oovo");
    contract<double>(P, S.Q, "ijam", tau, "ijef", ovvv, "maef", -1.0, false);
    // R_iabf = sum_me t_imae <mb||ef>   (k_i + k_f = k_a + k_b)
    S.R = alloc_kt<double>(c, m, "ovvv", 0, {1, -1, -1, 1});
    contract<double>(P, S.R, "iabf", t2, "imae", ovvv, "mbef", 1.0, false);
    // S_ijan = sum_me t_imae <mn||ej>
    S.S = alloc_kt<double>(c, m, "oovo");
    contract<double>(P, S.S, "ijan", t2, "imae", ooov, "mnje", -1.0, false);
    // U_ianf = sum_me t_imae <mn||ef>   (k_i + k_f = k_a + k_n)
    S.U = alloc_kt<double>(c, m, "ovov", 0, {1, -1, -1, 1});
    contract<double>(P, S.U, "ianf", t2, "imae", oovv, "mnef", 1.0, false);
    // Yp_ijan = sum_f t_jf U_ianf
    S.Yp = alloc_kt<double>(c, m, "oovo");
    contract<double>(P, S.Yp, "ijan", t1, "jf", S.U, "ianf", 1.0, false);
    // H_abej = 1/2 <ab||ej> - sum_m t_ma <mb||ej>
    S.H = alloc_kt<double>(c, m, "vvvo");
    build_eri(c, P, S.H, 0.5);
    contract<double>(P, S.H, "abej", t1, "ma", ovvo, "mbej", -1.0);
    // G2_ijbm = sum_e t_ie <mb||ej>
    S.G2 = alloc_kt<double>(c, m, "oovo");
    contract<double>(P, S.G2, "ijbm", t1, "ie", ovvo, "mbej", 1.0, false);
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
    if (!g_dry_run) {
        HIPCHK(P.run(nullptr));
        HIPCHK(hipDeviceSynchronize());
    }
    S.ready = true;

    // single-precision copies of everything the sigma reads
    State<float> &F = c->s32;
    Program P2;
    auto cv = [&](KT &d, const KT &s) { convert_kt<float>(P2, F, d, s, c); };
    cv(F.fov, S.fov); cv(F.t1, S.t1); cv(F.t2, S.t2); cv(F.tau, S.tau);
    cv(F.g_oovv, S.g_oovv); cv(F.g_ooov, S.g_ooov); cv(F.g_ovov, S.g_ovov); cv(F.g_ovvv, S.g_ovvv);
    cv(F.g_ovoo, S.g_ovoo);
    cv(F.Fae, S.Fae); cv(F.Fmi, S.Fmi); cv(F.Fme, S.Fme); cv(F.Fbe, S.Fbe); cv(F.Fmj, S.Fmj);
    cv(F.Wp, S.Wp); cv(F.Wbar, S.Wbar); cv(F.Q, S.Q); cv(F.R, S.R); cv(F.S, S.S); cv(F.U, S.U);
    cv(F.Yp, S.Yp); cv(F.H, S.H); cv(F.G2, S.G2);
    F.La = F.mem.get(lvv * 8);
    F.Lb = F.mem.get(lvv * 8);
    {
        void *a = S.La, *b = S.Lb, *fa = F.La, *fb = F.Lb;
        P2.ops.push_back([=](hipStream_t s) { return convert_f64_f32(a, fa, lvv, s); });
        P2.ops.push_back([=](hipStream_t s) { return convert_f64_f32(b, fb, lvv, s); });
    }
    if (!g_dry_run) {
        HIPCHK(P2.run(nullptr));
        HIPCHK(hipDeviceSynchronize());
    }
    F.ready = true;
}

// ---------------------------------------------------------------- sigma program
template <typename T>
Program *build_sigma(lrcc_ctx *c, State<T> &S, int R, DevMem &wm, int prec) {
    const int nk = c->nk, o = c->no, v = c->nv, naux = c->naux;
    auto P = new Program();
    auto A = [&](const char *cls) { return alloc_kt<T>(c, wm, cls, R); };
    KT x1 = A("ov"), x2 = A("oovv"), dtau = A("oovv"), Z = A("oovv"), s1 = A("ov");
    KT dFae = A("vv"), dFmi = A("oo"), dFme = A("ov"), dFbe = A("vv"), dFmj = A("oo");
    KT Zmn = A("oooo"), Vx = A("oooo"), Yx = A("oovo");
    const i64 nb3 = (i64)nk * nk * nk;
    // caller layout -> internal (paper -> crystal normalisation for doubles)
    P->ops.push_back([=](hipStream_t s) { return rhs_to_block<double, T>(c->io_x1, x1.p, R, nk, (i64)o * v, 1.0, s); });
    P->ops.push_back([=](hipStream_t s) {
        return rhs_to_block<double, T>(c->io_x2, x2.p, R, nb3, (i64)o * o * v * v, 1.0 / nk, s);
    });
    {
        void *t1p = S.t1.p;
        P->ops.push_back([=](hipStream_t s) { return tau_like<T>(x1.p, x2.p, t1p, dtau.p, nk, R, o, v, 1.0, 1, s); });
    }
    const KT &t1 = S.t1, &t2 = S.t2;
    // X-dependent one-body intermediates (derivatives of F_ae, F_mi, F_me)
    contract<T>(*P, dFae, "Rae", x1, "Rma", S.fov, "me", -0.5, false);
    contract<T>(*P, dFae, "Rae", x1, "Rmf", S.g_ovvv, "mafe", 1.0);
    contract<T>(*P, dFae, "Rae", x2, "Rmnaf", S.g_oovv, "mnef", -0.25);
    contract<T>(*P, dFae, "Rae", dtau, "Rmnaf", S.g_oovv, "mnef", -0.25);
    contract<T>(*P, dFmi, "Rmi", x1, "Rie", S.fov, "me", 0.5, false);
    contract<T>(*P, dFmi, "Rmi", x1, "Rne", S.g_ooov, "mnie", 1.0);
    contract<T>(*P, dFmi, "Rmi", x2, "Rinef", S.g_oovv, "mnef", 0.25);
    contract<T>(*P, dFmi, "Rmi", dtau, "Rinef", S.g_oovv, "mnef", 0.25);
    contract<T>(*P, dFme, "Rme", x1, "Rnf", S.g_oovv, "mnef", 1.0, false);
    // singles (Eq. tx1 operator part)
    contract<T>(*P, s1, "Ria", x1, "Rie", S.Fae, "ae", 1.0, false);
    contract<T>(*P, s1, "Ria", t1, "ie", dFae, "Rae", 1.0);
    contract<T>(*P, s1, "Ria", x1, "Rma", S.Fmi, "mi", -1.0);
    contract<T>(*P, s1, "Ria", t1, "ma", dFmi, "Rmi", -1.0);
    contract<T>(*P, s1, "Ria", x2, "Rimae", S.Fme, "me", 1.0);
    contract<T>(*P, s1, "Ria", t2, "imae", dFme, "Rme", 1.0);
    contract<T>(*P, s1, "Ria", x1, "Rnf", S.g_ovov, "naif", -1.0);
    contract<T>(*P, s1, "Ria", x2, "Rimef", S.g_ovvv, "maef", -0.5);
    contract<T>(*P, s1, "Ria", x2, "Rmnae", S.g_ooov, "nmie", 0.5);
    // dressed one-body derivatives entering the doubles
    kt_copy<T>(*P, dFbe, dFae);
    contract<T>(*P, dFbe, "Rbe", x1, "Rmb", S.Fme, "me", -0.5);
    contract<T>(*P, dFbe, "Rbe", t1, "mb", dFme, "Rme", -0.5);
    kt_copy<T>(*P, dFmj, dFmi);
    contract<T>(*P, dFmj, "Rmj", x1, "Rje", S.Fme, "me", 0.5);
    contract<T>(*P, dFmj, "Rmj", t1, "je", dFme, "Rme", 0.5);
    // doubles: Z collects every term; sigma2 = P(ij)P(ab) Z.  Terms antisymmetric in
    // both pairs enter with 1/4, terms antisymmetric in one pair with 1/2.
    contract<T>(*P, Z, "Rijab", x2, "Rijae", S.Fbe, "be", 0.5, false);
    contract<T>(*P, Z, "Rijab", t2, "ijae", dFbe, "Rbe", 0.5);
    contract<T>(*P, Z, "Rijab", x2, "Rimab", S.Fmj, "mj", -0.5);
    contract<T>(*P, Z, "Rijab", t2, "imab", dFmj, "Rmj", -0.5);
    {
        LadderArgs la{};
        la.Y = dtau.p;
        la.La = S.La;
        la.Lb = S.Lb;
        la.Z = Z.p;
        la.nk = nk;
        la.nrhs = R;
        la.o = o;
        la.v = v;
        la.naux = naux;
        la.alpha = 0.25;
        P->ops.push_back([=](hipStream_t s) { return launch_ladder<T>(la, s); });
        P->tag_last(TAG_LADDER);
        P->flops += (i64)ladder_executed_flops(la);
    }
    contract<T>(*P, Zmn, "Rijmn", dtau, "Rijef", S.g_oovv, "mnef", 1.0, false);
    contract<T>(*P, Z, "Rijab", Zmn, "Rijmn", t2, "mnab", 1.0 / 16);
    contract<T>(*P, Z, "Rijab", S.Wp, "mnij", dtau, "Rmnab", 1.0 / 8);
    contract<T>(*P, Vx, "Rijmn", x1, "Rje", S.g_ooov, "mnie", 1.0, false);
    contract<T>(*P, Vx, "Rjimn", x1, "Rje", S.g_ooov, "mnie", -1.0);
    contract<T>(*P, Z, "Rijab", Vx, "Rijmn", S.tau, "mnab", 1.0 / 8);
    contract<T>(*P, Z, "Rijab", S.Q, "ijam", x1, "Rmb", -0.25);
    // ring terms (P(ij)P(ab))
    contract<T>(*P, Z, "Rijab", x2, "Rimae", S.Wbar, "mbej", 1.0);
    contract<T>(*P, Z, "Rijab", S.R, "iabf", x1, "Rjf", 1.0);
    contract<T>(*P, Z, "Rijab", S.S, "ijan", x1, "Rnb", -1.0);
    contract<T>(*P, Yx, "Rijan", x1, "Rjf", S.U, "ianf", 1.0, false);
    contract<T>(*P, Z, "Rijab", Yx, "Rijan", t1, "nb", -1.0);
    contract<T>(*P, Z, "Rijab", S.Yp, "ijan", x1, "Rnb", -1.0);
    contract<T>(*P, Z, "Rijab", x1, "Rie", S.H, "abej", 1.0);
    contract<T>(*P, Z, "Rijab", S.G2, "ijbm", x1, "Rma", -1.0);
    contract<T>(*P, Z, "Rijab", S.g_ovoo, "mbij", x1, "Rma", -0.5);
    // outputs in the caller layout: y = (A - omega) x, paper normalisation
    P->ops.push_back([=](hipStream_t s) { return s1_out<T>(s1.p, c->io_x1, c->io_y1, c->io_omega, nk, R, o, v, s); });
    P->ops.push_back([=](hipStream_t s) {
        return pp_out<T>(Z.p, c->io_x2, c->io_y2, c->io_omega, nk, R, o, v, (double)nk, s);
    });
    (void)prec;
    return P;
}

Program *sigma_program(lrcc_ctx *c, int prec, int R) {
    auto key = std::make_pair(prec, R);
    auto it = c->progs.find(key);
    if (it != c->progs.end()) return it->second.get();
    auto mem = std::make_unique<DevMem>();
    Program *p = prec == LRCC_FP64 ? build_sigma<double>(c, c->s64, R, *mem, prec)
                                   : build_sigma<float>(c, c->s32, R, *mem, prec);
    c->progs[key].reset(p);
    c->progmem[key] = std::move(mem);
    return p;
}


// Device copies of the Hamiltonian and the stored integral blocks (all but vvvv).
void setup_hamiltonian(lrcc_ctx *c, int nk, int nocc, int nvir, int naux, const double *fock, const double *chol) {
    const int n = nocc + nvir;
    c->ham = c->amp = false;
    c->progs.clear();
    c->progmem.clear();
    c->s64.mem.release();
    c->s32.mem.release();
    c->hmem.release();
    c->nk = nk; c->no = nocc; c->nv = nvir; c->naux = naux; c->n = n;
    const i64 nL = (i64)nk * nk * naux * n * n;
    c->fock = c->hmem.get((size_t)nk * n * n * 16);
    if (!g_dry_run) HIPCHK(hipMemcpy(c->fock, fock, (size_t)nk * n * n * 16, hipMemcpyHostToDevice));
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
    delete c;
}

const char *lrcc_last_error(const lrcc_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

lrcc_status lrcc_set_hamiltonian(lrcc_ctx *c, int nk, int nocc, int nvir, int naux, const double *fock,
                                 const double *chol, const double *dip) {
    return guarded(c, [&] {
        if (nk < 1 || nocc < 1 || nvir < 1 || naux < 1 || !fock || !chol || !dip)
            throw LrccError(LRCC_E_ARG, "invalid sizes or null pointer");
        const int n = nocc + nvir;
        // Hermiticity of fock and dip
        auto herm = [&](const double *m, int cnt, const char *what) {
            double mx = 0, dev = 0;
            for (int b = 0; b < cnt; ++b)
                for (int p = 0; p < n; ++p)
                    for (int q = 0; q < n; ++q) {
                        const double *x = m + 2 * (((i64)b * n + p) * n + q), *y = m + 2 * (((i64)b * n + q) * n + p);
                        dev = std::max(dev, std::max(std::fabs(x[0] - y[0]), std::fabs(x[1] + y[1])));
                        mx = std::max(mx, std::max(std::fabs(x[0]), std::fabs(x[1])));
                    }
            if (dev > 1e-10 * std::max(1.0, mx)) throw LrccError(LRCC_E_ARG, std::string(what) + " is not Hermitian");
        };
        herm(fock, nk, "fock");
        herm(dip, 3 * nk, "dip");
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
        setup_hamiltonian(c, nk, nocc, nvir, naux, fock, chol);
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
                    const int kb = ((ki + kj - ka) % nk + nk) % nk;
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
        precompute(c, t1, t2);
        c->amp = true;
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
        HIPCHK(p->run((hipStream_t)stream, &c->prof));
    });
}

lrcc_status lrcc_apply_sigma(lrcc_ctx *c, int nrhs, const double *omega, const double *x1, const double *x2,
                             double *y1, double *y2, int precision) {
    return guarded(c, [&] {
        if (!c->amp) throw LrccError(LRCC_E_STATE, "set_amplitudes must be called first");
        if (nrhs < 1 || !x1 || !x2 || !y1 || !y2) throw LrccError(LRCC_E_ARG, "invalid nrhs or null pointer");
        const int nk = c->nk, o = c->no, v = c->nv;
        const size_t b1 = (size_t)nrhs * nk * o * v * 16, b2 = (size_t)nrhs * nk * nk * nk * o * o * v * v * 16;
        const size_t need = 2 * b1 + 2 * b2 + (size_t)nrhs * 8;
        if (need > c->stage_bytes) {
            c->stage.release();
            c->st_x1 = c->stage.get(b1); c->st_y1 = c->stage.get(b1);
            c->st_x2 = c->stage.get(b2); c->st_y2 = c->stage.get(b2);
            c->st_om = c->stage.get((size_t)nrhs * 8);
            c->stage_bytes = need;
        }
        HIPCHK(hipMemcpy(c->st_x1, x1, b1, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->st_x2, x2, b2, hipMemcpyHostToDevice));
        std::vector<double> om(nrhs, 0.0);
        if (omega) for (int r = 0; r < nrhs; ++r) om[r] = omega[r];
        HIPCHK(hipMemcpy(c->st_om, om.data(), nrhs * 8, hipMemcpyHostToDevice));
        lrcc_status s = lrcc_apply_sigma_dev(c, nrhs, (const double *)c->st_om, c->st_x1, c->st_x2, c->st_y1,
                                             c->st_y2, precision, nullptr);
        if (s != LRCC_OK) throw LrccError(s, c->err);
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(y1, c->st_y1, b1, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(y2, c->st_y2, b2, hipMemcpyDeviceToHost));
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

lrcc_status lrcc_plan_check(int nk, int nocc, int nvir, int naux, int nrhs, char *msg, int msglen) {
    if (msg && msglen > 0) msg[0] = 0;
    if (nk < 1 || nocc < 1 || nvir < 1 || naux < 1 || nrhs < 1) return LRCC_E_ARG;
    lrcc_status st = LRCC_OK;
    g_dry_run = true;
    try {
        lrcc_ctx c;
        setup_hamiltonian(&c, nk, nocc, nvir, naux, nullptr, nullptr);
        c.ham = true;
        precompute(&c, nullptr, nullptr);
        c.amp = true;
        (void)sigma_program(&c, LRCC_FP64, nrhs);
        (void)sigma_program(&c, LRCC_FP32, nrhs);
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
