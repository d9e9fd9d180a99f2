// J-coupled two-body matrix elements to the m-scheme arrays the Hamiltonian
// takes (App. A, "The Hamiltonian and other operators in second
// quantization", eq. hamdef: V_J(ab,cd) is the matrix element between
// normalised two-body states of good J, and the pair creation operator
// couples a+ b+ with Clebsch-Gordan coefficients).
//
// For two like particles with m-states al < be of orbits a <= b (orbits in
// input order, 2m ascending inside an orbit, so al < be holds whenever a < b)
// the normalised pair state has amplitude zeta_ab (j_a m_al j_b m_be | J M)
// on a+_al a+_be |0>, zeta_ab = sqrt(2) for a == b and 1 otherwise; hence
//   V[(al be),(ga de)] = sum_J zeta_ab zeta_cd V_J(ab,cd) CG(al be; J M) CG(ga de; J M).
// A proton-neutron pair is a product state of distinguishable particles and
// carries no zeta. The host work is the "time to decouple" of Ch. 8.
#include <cmath>
#include <cstring>
#include <vector>

#include "fotci_internal.h"

namespace fotci {
namespace {

// Racah's closed form for (j1 m1, j2 m2 | J M), arguments doubled.
struct Factorials {
    double f[171];
    Factorials() {
        f[0] = 1.0;
        for (int i = 1; i <= 170; ++i) f[i] = f[i - 1] * i;
    }
};

double clebsch_gordan(int tj1, int tm1, int tj2, int tm2, int tJ, int tM) {
    static const Factorials table;   // initialised once, thread-safe
    const double *fact = table.f;
    if (tm1 + tm2 != tM) return 0.0;
    if (tJ < std::abs(tj1 - tj2) || tJ > tj1 + tj2 || ((tj1 + tj2 + tJ) & 1)) return 0.0;
    if (std::abs(tm1) > tj1 || std::abs(tm2) > tj2 || std::abs(tM) > tJ) return 0.0;
    if (((tj1 + tm1) & 1) || ((tj2 + tm2) & 1) || ((tJ + tM) & 1)) return 0.0;
    const int a = (tJ + tj1 - tj2) / 2, b = (tJ - tj1 + tj2) / 2, c = (tj1 + tj2 - tJ) / 2;
    const int d = (tj1 + tj2 + tJ) / 2 + 1;
    const double pre = (tJ + 1) * fact[a] * fact[b] * fact[c] / fact[d] * fact[(tJ + tM) / 2] * fact[(tJ - tM) / 2] *
                       fact[(tj1 - tm1) / 2] * fact[(tj1 + tm1) / 2] * fact[(tj2 - tm2) / 2] * fact[(tj2 + tm2) / 2];
    double s = 0.0;
    for (int k = 0; k <= c; ++k) {
        const int e[6] = {k, c - k, (tj1 - tm1) / 2 - k, (tj2 + tm2) / 2 - k, (tJ - tj2 + tm1) / 2 + k,
                          (tJ - tj1 - tm2) / 2 + k};
        bool ok = true;
        double den = 1.0;
        for (int x : e) {
            if (x < 0) {
                ok = false;
                break;
            }
            den *= fact[x];
        }
        if (ok) s += ((k & 1) ? -1.0 : 1.0) / den;
    }
    return s * std::sqrt(pre);
}

struct Orbits {
    int n = 0, ns = 0;
    std::vector<int> two_j, par, first;   // first m-state of each orbit
};

void check_element(const Orbits &o, const fotci_tbme &t, bool like) {
    const int idx[4] = {t.a, t.b, t.c, t.d};
    for (int i : idx)
        if (i < 0 || i >= o.n) fail(FOTCI_EINVAL, "orbit index out of range");
    if (!std::isfinite(t.v)) fail(FOTCI_EINVAL, "matrix element not finite");
    if (like && (t.a > t.b || t.c > t.d)) fail(FOTCI_EINVAL, "like-particle pairs need a <= b and c <= d");
    auto in_range = [&](int x, int y) {
        return t.two_J >= std::abs(o.two_j[x] - o.two_j[y]) && t.two_J <= o.two_j[x] + o.two_j[y] &&
               ((o.two_j[x] + o.two_j[y] + t.two_J) & 1) == 0;
    };
    if (!in_range(t.a, t.b) || !in_range(t.c, t.d)) fail(FOTCI_EINVAL, "2J outside the coupling range of a pair");
    if (o.par[t.a] * o.par[t.b] != o.par[t.c] * o.par[t.d]) fail(FOTCI_EINVAL, "matrix element changes parity");
    if (like && t.v != 0.0 && ((t.a == t.b) || (t.c == t.d)) && ((t.two_J / 2) & 1))
        fail(FOTCI_EINVAL, "odd J for two like particles in one orbit");
}

// Accumulate one element into the full matrix m (row-major, n x n), with the
// mirror when the orbit pairs differ; rows/columns are pair indices (like
// particles) or al * ns + be (proton-neutron).
void add_element(const Orbits &o, const fotci_tbme &t, bool like, std::vector<double> &m, int n) {
    const double za = (like && t.a == t.b) ? std::sqrt(2.0) : 1.0;
    const double zc = (like && t.c == t.d) ? std::sqrt(2.0) : 1.0;
    const bool mirror = !(t.a == t.c && t.b == t.d);
    struct P {
        int idx;      // pair index (like particles) or al * ns + be
        int two_m;    // 2M of the pair
        int ma, mb;   // 2m of its two states
    };
    auto pairs = [&](int a, int b) {
        std::vector<P> out;
        for (int i = 0; i < o.two_j[a] + 1; ++i)
            for (int k = 0; k < o.two_j[b] + 1; ++k) {
                const int al = o.first[a] + i, be = o.first[b] + k;
                if (like && al >= be) continue;
                const int ma = -o.two_j[a] + 2 * i, mb = -o.two_j[b] + 2 * k;
                out.push_back({like ? pair_index(al, be, o.ns) : al * o.ns + be, ma + mb, ma, mb});
            }
        return out;
    };
    const std::vector<P> bra = pairs(t.a, t.b), ket = pairs(t.c, t.d);
    for (const P &p : bra) {
        const double x = za * clebsch_gordan(o.two_j[t.a], p.ma, o.two_j[t.b], p.mb, t.two_J, p.two_m);
        if (x == 0.0) continue;
        for (const P &q : ket) {
            if (q.two_m != p.two_m) continue;
            const double z = zc * clebsch_gordan(o.two_j[t.c], q.ma, o.two_j[t.d], q.mb, t.two_J, q.two_m);
            if (z == 0.0) continue;
            const double v = x * t.v * z;
            m[(size_t)p.idx * n + q.idx] += v;
            if (mirror) m[(size_t)q.idx * n + p.idx] += v;
        }
    }
}

// copy the upper triangle to the lower one: exactly symmetric output
void symmetrise(std::vector<double> &m, int n) {
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < r; ++c) m[(size_t)r * n + c] = m[(size_t)c * n + r];
}

}  // namespace
}  // namespace fotci

using namespace fotci;

extern "C" int fotci_decouple_tbme_impl(int32_t n_orbits, const int32_t *two_j, const int32_t *parity, int32_t n_pp,
                                        const fotci_tbme *pp, int32_t n_nn, const fotci_tbme *nn, int32_t n_pn,
                                        const fotci_tbme *pn, double *v_pp, double *v_nn, double *v_pn) {
    if (n_orbits < 1 || !two_j) fail(FOTCI_EINVAL, "no orbits");
    if ((n_pp > 0 && !pp) || (n_nn > 0 && !nn) || (n_pn > 0 && !pn) || n_pp < 0 || n_nn < 0 || n_pn < 0)
        fail(FOTCI_EINVAL, "bad element list");
    Orbits o;
    o.n = n_orbits;
    for (int i = 0; i < n_orbits; ++i) {
        if (two_j[i] < 1 || (two_j[i] & 1) == 0) fail(FOTCI_EINVAL, "2j must be a positive odd integer");
        const int p = parity ? parity[i] : 1;
        if (p != 1 && p != -1) fail(FOTCI_EINVAL, "parity must be +1 or -1");
        o.two_j.push_back(two_j[i]);
        o.par.push_back(p);
        o.first.push_back(o.ns);
        o.ns += two_j[i] + 1;
    }
    if (o.ns > 32) fail(FOTCI_EINVAL, "more than 32 m-states");
    for (int i = 0; i < n_pp; ++i) check_element(o, pp[i], true);
    for (int i = 0; i < n_nn; ++i) check_element(o, nn[i], true);
    for (int i = 0; i < n_pn; ++i) check_element(o, pn[i], false);
    const int npairs = o.ns * (o.ns - 1) / 2, n2 = o.ns * o.ns;
    struct Job {
        const fotci_tbme *e;
        int n;
        double *out;
        bool like;
        int dim;
    } jobs[3] = {{pp, n_pp, v_pp, true, npairs}, {nn, n_nn, v_nn, true, npairs}, {pn, n_pn, v_pn, false, n2}};
    for (const Job &jb : jobs) {
        if (!jb.out) continue;
        std::vector<double> m((size_t)jb.dim * jb.dim, 0.0);
        for (int i = 0; i < jb.n; ++i) add_element(o, jb.e[i], jb.like, m, jb.dim);
        symmetrise(m, jb.dim);
        std::memcpy(jb.out, m.data(), m.size() * sizeof(double));
    }
    return FOTCI_OK;
}
