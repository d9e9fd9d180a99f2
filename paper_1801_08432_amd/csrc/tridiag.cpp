// Symmetric tridiagonal eigenproblem in float64 on the host: the eigenvalues
// of the Lanczos matrix of alphas and betas (Ch. 7, "Standard Lanczos
// algorithm"; the paper hands this step to a double-precision LAPACK solver).
//
// Implicit QL iteration with Wilkinson-type shifts (the textbook method for a
// tridiagonal matrix: chase a bulge with Givens rotations from the bottom of
// the unreduced block up, deflate when an off-diagonal becomes negligible),
// accumulating the rotations into the eigenvector matrix.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

#include "fotci_internal.h"

namespace fotci {

void tridiag_eig(int n, std::vector<double> &d, std::vector<double> e, std::vector<double> &z) {
    z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
    if (n <= 1) return;
    e.resize(n, 0.0);
    e[n - 1] = 0.0;
    const double eps = std::numeric_limits<double>::epsilon();
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            // find the first negligible off-diagonal at or below l
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 100) fail(FOTCI_ENOTCONV, "tridiagonal QL did not converge");
            // shift from the leading 2x2 block of the unreduced part
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool underflow = false;
            for (; i >= l; --i) {
                double f = s * e[i];
                double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    underflow = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int k = 0; k < n; ++k) {
                    double *zk = &z[(size_t)k * n];
                    f = zk[i + 1];
                    zk[i + 1] = s * zk[i] + c * f;
                    zk[i] = c * zk[i] - s * f;
                }
            }
            if (underflow) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    // ascending order
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    std::vector<double> d2(n), z2((size_t)n * n);
    for (int k = 0; k < n; ++k) {
        d2[k] = d[idx[k]];
        for (int i = 0; i < n; ++i) z2[(size_t)i * n + k] = z[(size_t)i * n + idx[k]];
    }
    d.swap(d2);
    z.swap(z2);
}

// Dense symmetric eigenproblem (host, float64) by cyclic Jacobi rotations:
// each rotation zeroes one off-diagonal pair (p, q) with the angle chosen from
// t = tan(theta) as the smaller root of t^2 + 2 t cot(2 theta) - 1 = 0, and is
// accumulated into the eigenvector matrix; sweeps repeat until the
// off-diagonal part is negligible against the matrix norm. Used for the
// projected matrix of thick-restart Lanczos, which after a restart is a
// diagonal block with an arrow column and a tridiagonal tail.
void sym_eig(int n, std::vector<double> a, std::vector<double> &d, std::vector<double> &z) {
    z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
    auto A = [&](int i, int j) -> double & { return a[(size_t)i * n + j]; };
    double norm = 0.0;
    for (double v : a) norm += v * v;
    norm = std::sqrt(norm);
    const double eps = std::numeric_limits<double>::epsilon();
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A(p, q) * A(p, q);
        if (std::sqrt(2.0 * off) <= eps * norm || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A(p, q);
                if (apq == 0.0) continue;
                const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {   // columns p, q
                    const double akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * akq;
                    A(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // rows p, q
                    const double apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * aqk;
                    A(q, k) = s * apk + c * aqk;
                }
                A(p, q) = A(q, p) = 0.0;
                for (int k = 0; k < n; ++k) {
                    const double zkp = z[(size_t)k * n + p], zkq = z[(size_t)k * n + q];
                    z[(size_t)k * n + p] = c * zkp - s * zkq;
                    z[(size_t)k * n + q] = s * zkp + c * zkq;
                }
            }
    }
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return A(x, x) < A(y, y); });
    d.resize(n);
    std::vector<double> z2((size_t)n * n);
    for (int k = 0; k < n; ++k) {
        d[k] = A(idx[k], idx[k]);
        for (int i = 0; i < n; ++i) z2[(size_t)i * n + k] = z[(size_t)i * n + idx[k]];
    }
    z.swap(z2);
}

}  // namespace fotci
