// Small dense complex eigenproblems (host).  Standard dense algorithms: Householder
// reduction to upper Hessenberg form, single-shift complex QR iteration with
// Wilkinson shifts and deflation (Givens rotations), eigenvectors of the triangular
// Schur factor by back substitution, transformed back with the Schur vectors.
#include "eig.hpp"

#include <algorithm>
#include <cmath>

namespace lrcc {

typedef std::complex<double> cd;

bool small_eig(int n, std::vector<cd> A, std::vector<cd> &w, std::vector<cd> &V) {
    auto a = [&](int i, int j) -> cd & { return A[(size_t)i * n + j]; };
    std::vector<cd> Q((size_t)n * n, 0.0);
    auto q = [&](int i, int j) -> cd & { return Q[(size_t)i * n + j]; };
    for (int i = 0; i < n; ++i) q(i, i) = 1.0;
    // Householder reduction: A <- H A H, Q <- Q H
    for (int k = 0; k + 2 < n; ++k) {
        double nx = 0;
        for (int i = k + 1; i < n; ++i) nx += std::norm(a(i, k));
        nx = std::sqrt(nx);
        if (nx == 0) continue;
        std::vector<cd> v(n, 0.0);
        const cd x0 = a(k + 1, k);
        const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
        for (int i = k + 1; i < n; ++i) v[i] = a(i, k);
        v[k + 1] += ph * nx;
        double vn = 0;
        for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
        if (vn == 0) continue;
        // A <- (I - 2 v v^H / vn) A
        for (int j = 0; j < n; ++j) {
            cd s = 0;
            for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * a(i, j);
            s *= 2.0 / vn;
            for (int i = k + 1; i < n; ++i) a(i, j) -= v[i] * s;
        }
        // A <- A (I - 2 v v^H / vn), Q likewise
        for (int i = 0; i < n; ++i) {
            cd s = 0, t = 0;
            for (int j = k + 1; j < n; ++j) { s += a(i, j) * v[j]; t += q(i, j) * v[j]; }
            s *= 2.0 / vn;
            t *= 2.0 / vn;
            for (int j = k + 1; j < n; ++j) { a(i, j) -= s * std::conj(v[j]); q(i, j) -= t * std::conj(v[j]); }
        }
        for (int i = k + 2; i < n; ++i) a(i, k) = 0.0;
    }
    // shifted QR on the active window [0, hi]
    const double eps = 1e-15;
    int hi = n - 1, iter = 0;
    while (hi > 0) {
        if (++iter > 100 * n) return false;
        int lo = hi;
        while (lo > 0) {
            const double s = std::abs(a(lo - 1, lo - 1)) + std::abs(a(lo, lo));
            if (std::abs(a(lo, lo - 1)) <= eps * std::max(s, 1e-300)) { a(lo, lo - 1) = 0.0; break; }
            --lo;
        }
        if (lo == hi) { --hi; iter = 0; continue; }
        // Wilkinson shift from the trailing 2x2 block
        const cd p = a(hi - 1, hi - 1), r = a(hi - 1, hi), s2 = a(hi, hi - 1), t = a(hi, hi);
        const cd tr = p + t, det = p * t - r * s2;
        const cd disc = std::sqrt(tr * tr / 4.0 - det);
        cd mu1 = tr / 2.0 + disc, mu2 = tr / 2.0 - disc;
        cd mu = std::abs(mu1 - t) < std::abs(mu2 - t) ? mu1 : mu2;
        if (iter % 11 == 10) mu = t + std::abs(a(hi, hi - 1));   // exceptional shift
        // QR step on rows/cols lo..hi of (A - mu I) via Givens rotations, applied to the full matrix
        std::vector<cd> cs(hi - lo), sn(hi - lo);
        for (int i = lo; i <= hi; ++i) a(i, i) -= mu;
        for (int k = lo; k < hi; ++k) {
            const cd x = a(k, k), y = a(k + 1, k);
            const double den = std::sqrt(std::norm(x) + std::norm(y));
            const cd c = den > 0 ? x / den : cd(1.0), sg = den > 0 ? y / den : cd(0.0);
            cs[k - lo] = c;
            sn[k - lo] = sg;
            // rows k, k+1:  [c^H s^H; -s c] applied from the left
            for (int j = k; j < n; ++j) {
                const cd u = a(k, j), v = a(k + 1, j);
                a(k, j) = std::conj(c) * u + std::conj(sg) * v;
                a(k + 1, j) = -sg * u + c * v;
            }
        }
        for (int k = lo; k < hi; ++k) {
            const cd c = cs[k - lo], sg = sn[k - lo];
            // columns k, k+1 from the right with the adjoint rotation
            for (int i = 0; i <= std::min(hi, k + 1); ++i) {
                const cd u = a(i, k), v = a(i, k + 1);
                a(i, k) = u * c + v * sg;
                a(i, k + 1) = -u * std::conj(sg) + v * std::conj(c);
            }
            for (int i = 0; i < n; ++i) {
                const cd u = q(i, k), v = q(i, k + 1);
                q(i, k) = u * c + v * sg;
                q(i, k + 1) = -u * std::conj(sg) + v * std::conj(c);
            }
        }
        for (int i = lo; i <= hi; ++i) a(i, i) += mu;
    }
    // eigenvectors of the upper-triangular Schur factor, then back to the original basis
    w.assign(n, 0.0);
    V.assign((size_t)n * n, 0.0);
    double tn = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) tn = std::max(tn, std::abs(a(i, j)));
    const double small = std::max(tn, 1e-300) * 1e-14;
    for (int k = 0; k < n; ++k) {
        w[k] = a(k, k);
        std::vector<cd> y(n, 0.0);
        y[k] = 1.0;
        for (int i = k - 1; i >= 0; --i) {
            cd s = 0;
            for (int j = i + 1; j <= k; ++j) s += a(i, j) * y[j];
            cd d = a(i, i) - a(k, k);
            if (std::abs(d) < small) d = small;
            y[i] = -s / d;
        }
        double nv = 0;
        std::vector<cd> x(n, 0.0);
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j <= k; ++j) x[i] += q(i, j) * y[j];
            nv += std::norm(x[i]);
        }
        nv = std::sqrt(nv);
        for (int i = 0; i < n; ++i) V[(size_t)i * n + k] = x[i] / nv;
    }
    return true;
}

}  // namespace lrcc
