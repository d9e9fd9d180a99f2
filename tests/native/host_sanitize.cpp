// Host-side setup code of libfotci under AddressSanitizer and
// UndefinedBehaviorSanitizer: the basis and jump builders (Ch. 2,
// "Representation of the basis" and "Representation of the Hamiltonian"), the
// J-coupled decoupling (App. A, eq. hamdef) and the host eigensolvers, linked
// without any device code and checked against closed forms:
//   - basis dimensions printed in the paper (Table al27, 20Ne, 28Si, 48Cr)
//     and the 5p5n 20-state dimension 18,600,516;
//   - one-body jumps per SD n (N_s - n + 1), two-body jump totals;
//   - the decoupled j = 1/2, J = 0 pair element equals V_0;
//   - tridiagonal QL on the 1-D Laplacian (eigenvalues 2 - 2 cos(k pi/(n+1)))
//     and Jacobi on a random symmetric matrix (A z = lambda z);
//   - invalid inputs fail with FOTCI_EINVAL and leak nothing.
// Build and run: tests/test_host_sanitizers.py.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "fotci_internal.h"

namespace fotci {
struct Thrown {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg) { throw Thrown{code, msg}; }
void set_error(const std::string &) {}
}  // namespace fotci

extern "C" int fotci_build_basis_impl(int32_t, const int32_t *, const int32_t *, int32_t, int32_t, int32_t, int32_t,
                                      fotci_basis **);
extern "C" int fotci_build_jumps_impl(const fotci_basis *, fotci_jumps **);
extern "C" int fotci_decouple_tbme_impl(int32_t, const int32_t *, const int32_t *, int32_t, const fotci_tbme *,
                                        int32_t, const fotci_tbme *, int32_t, const fotci_tbme *, double *, double *,
                                        double *);

static int n_fail = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, #c); \
            ++n_fail;                                                        \
        }                                                                    \
    } while (0)

static fotci_basis *basis(std::vector<int32_t> tj, int Z, int N, int two_M, std::vector<int32_t> par = {}) {
    if (par.empty()) par.assign(tj.size(), 1);
    fotci_basis *b = nullptr;
    fotci_build_basis_impl((int32_t)tj.size(), tj.data(), par.data(), Z, N, two_M, 1, &b);
    return b;
}

static int64_t count_two_body(const fotci_jumps *j, int kind) { return (int64_t)j->rec[kind].size(); }

int main() {
    using namespace fotci;
    // dimensions (Table al27 total; 20Ne, 28Si, 48Cr shapes; the 5p5n workload)
    struct D {
        std::vector<int32_t> tj;
        int Z, N, M;
        int64_t dim;
    } dims[] = {{{1, 3, 5}, 5, 6, 1, 80115},   {{1, 3, 5}, 2, 2, 0, 640},        {{1, 3, 5}, 6, 6, 0, 93710},
                {{1, 3, 5, 7}, 4, 4, 0, 1963461}, {{1, 3, 5, 7}, 5, 5, 0, 18600516}, {{1, 3, 5}, 0, 0, 0, 1}};
    for (const D &d : dims) {
        fotci_basis *b = basis(d.tj, d.Z, d.N, d.M);
        CHECK(b && b->dim == d.dim);
        delete b;
    }
    // jumps: one-body n (N_s - n + 1) per SD (all SDs kept at M = 0), two-body totals
    {
        fotci_basis *b = basis({1, 3, 5, 7}, 4, 4, 0);
        fotci_jumps *j = nullptr;
        fotci_build_jumps_impl(b, &j);
        CHECK(j != nullptr);
        const int64_t nsd = (int64_t)b->p.sd.size();
        CHECK(nsd == 4845);
        CHECK(count_two_body(j, FOTCI_JUMP_P1) == nsd * 4 * (20 - 4 + 1));
        CHECK(count_two_body(j, FOTCI_JUMP_N1) == nsd * 4 * (20 - 4 + 1));
        CHECK(count_two_body(j, FOTCI_JUMP_PP2) == 497790);
        CHECK(count_two_body(j, FOTCI_JUMP_NN2) == 497790);
        delete j;
        delete b;
    }
    {
        fotci_basis *b = basis({1, 3, 5}, 3, 1, 2, {1, -1, 1});   // mixed parity, odd particle numbers
        CHECK(b != nullptr);
        fotci_jumps *j = nullptr;
        fotci_build_jumps_impl(b, &j);
        CHECK(j != nullptr);
        delete j;
        delete b;
    }
    // decoupling: one j = 1/2 pair with J = 0 gives V[(-1/2, 1/2), (-1/2, 1/2)] = V_0
    {
        const int32_t tj[1] = {1}, par[1] = {1};
        fotci_tbme e{0, 0, 0, 0, 0, -2.5};
        double vpp[1] = {0}, vpn[16] = {0};
        fotci_decouple_tbme_impl(1, tj, par, 1, &e, 0, nullptr, 0, nullptr, vpp, nullptr, vpn);
        CHECK(std::fabs(vpp[0] - (-2.5)) < 1e-14);
    }
    // a random J-coupled pn list on the 12-state space: the output is exactly symmetric
    {
        const int32_t tj[3] = {1, 3, 5}, par[3] = {1, 1, 1};
        std::mt19937_64 rng(7);
        std::normal_distribution<double> nd;
        std::vector<fotci_tbme> pn;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d) {
                        if (a * 3 + b > c * 3 + d) continue;
                        const int lo = std::max(std::abs(tj[a] - tj[b]), std::abs(tj[c] - tj[d]));
                        const int hi = std::min(tj[a] + tj[b], tj[c] + tj[d]);
                        for (int J = lo; J <= hi; J += 2) pn.push_back({a, b, c, d, J, nd(rng)});
                    }
        std::vector<double> v(144 * 144);
        fotci_decouple_tbme_impl(3, tj, par, 0, nullptr, 0, nullptr, (int32_t)pn.size(), pn.data(), nullptr, nullptr,
                                 v.data());
        for (int r = 0; r < 144; ++r)
            for (int c = 0; c < 144; ++c) CHECK(v[r * 144 + c] == v[c * 144 + r]);
    }
    // host eigensolvers
    {
        const int n = 50;
        std::vector<double> d(n, 2.0), e(n - 1, -1.0), z;
        tridiag_eig(n, d, e, z);
        for (int k = 0; k < n; ++k) CHECK(std::fabs(d[k] - (2.0 - 2.0 * std::cos((k + 1) * M_PI / (n + 1)))) < 1e-12);
        std::mt19937_64 rng(11);
        std::normal_distribution<double> nd;
        const int m = 40;
        std::vector<double> a(m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j <= i; ++j) a[i * m + j] = a[j * m + i] = nd(rng);
        std::vector<double> w, zz;
        sym_eig(m, a, w, zz);
        for (int k = 0; k < m; ++k) {
            double r = 0.0;
            for (int i = 0; i < m; ++i) {
                double s = 0.0;
                for (int j = 0; j < m; ++j) s += a[i * m + j] * zz[j * m + k];
                r = std::max(r, std::fabs(s - w[k] * zz[i * m + k]));
            }
            CHECK(r < 1e-11);
        }
    }
    // invalid inputs fail cleanly
    {
        int code = 0;
        const int32_t tj[2] = {1, 3}, par[2] = {1, 1};
        fotci_basis *b = nullptr;
        try {
            fotci_build_basis_impl(2, tj, par, 2, 1, 0, 1, &b);   // 2M parity does not match Z + N
        } catch (const Thrown &t) {
            code = t.code;
        }
        CHECK(code == FOTCI_EINVAL && b == nullptr);
        code = 0;
        const int32_t bad[1] = {2};
        try {
            fotci_build_basis_impl(1, bad, par, 1, 1, 0, 1, &b);   // even 2j
        } catch (const Thrown &t) {
            code = t.code;
        }
        CHECK(code == FOTCI_EINVAL && b == nullptr);
        code = 0;
        fotci_tbme odd{0, 0, 0, 0, 1, 1.0};   // J = 1/2 is outside the coupling of two j = 1/2
        double v[1];
        try {
            const int32_t one[1] = {1};
            fotci_decouple_tbme_impl(1, one, par, 1, &odd, 0, nullptr, 0, nullptr, v, nullptr, nullptr);
        } catch (const Thrown &t) {
            code = t.code;
        }
        CHECK(code == FOTCI_EINVAL);
    }
    std::printf("host sanitizer checks: %d failed\n", n_fail);
    return n_fail == 0 ? 0 : 1;
}
