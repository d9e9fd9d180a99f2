// Host setup: the factorised M-scheme basis and the one-species jump lists.
//
// Basis: Ch. 2 "Use of quantum numbers: factorization of the basis" and Ch. 6
// "Writing out the basis" -- proton SDs x neutron SDs in sectors of fixed
// (2M, parity); every proton SD of a sector pairs with every neutron SD of the
// conjugate sector; index = pstart(ip) + nstart(jn), neutrons innermost.
// Jumps: Ch. 2 "Representation of the Hamiltonian" -- the action of a
// one-species operator string on that species' SDs, stored once and reused
// for every spectator SD of the other species.
#include <algorithm>
#include <cstring>
#include <map>

#include "fotci_internal.h"

namespace fotci {

namespace {

inline int sign_below(uint32_t m, int i) { return (__builtin_popcount(m & ((1u << i) - 1u)) & 1) ? -1 : 1; }

// p+_a p_c |m>: 0 if it vanishes, else the sign; *out = result mask.
inline int one_body_action(uint32_t m, int a, int c, uint32_t *out) {
    if (!((m >> c) & 1u)) return 0;
    int s = sign_below(m, c);
    m &= ~(1u << c);
    if ((m >> a) & 1u) return 0;
    s *= sign_below(m, a);
    *out = m | (1u << a);
    return s;
}

// p+_a p+_b p_d p_c |m>, operators applied rightmost first: p_c, p_d, p+_b, p+_a
inline int two_body_action(uint32_t m, int a, int b, int c, int d, uint32_t *out) {
    if (!((m >> c) & 1u)) return 0;
    int s = sign_below(m, c);
    m &= ~(1u << c);
    if (!((m >> d) & 1u)) return 0;
    s *= sign_below(m, d);
    m &= ~(1u << d);
    if ((m >> b) & 1u) return 0;
    s *= sign_below(m, b);
    m |= 1u << b;
    if ((m >> a) & 1u) return 0;
    s *= sign_below(m, a);
    *out = m | (1u << a);
    return s;
}

void sd_qn(uint32_t m, const std::vector<MState> &ms, int *two_m, int *par) {
    int tm = 0, p = 1;
    for (size_t i = 0; i < ms.size(); ++i)
        if ((m >> i) & 1u) {
            tm += ms[i].two_m;
            p *= ms[i].parity;
        }
    *two_m = tm;
    *par = p;
}

bool sector_less(std::pair<int, int> a, std::pair<int, int> b) {
    if (a.first != b.first) return a.first < b.first;
    return (a.second == 1 ? 0 : 1) < (b.second == 1 ? 0 : 1);
}

// All n-bit masks of ns bits grouped by (2M, parity), each group ascending.
std::map<std::pair<int, int>, std::vector<uint32_t>> enumerate_species(const std::vector<MState> &ms, int n) {
    std::map<std::pair<int, int>, std::vector<uint32_t>> g;
    const int ns = (int)ms.size();
    if (n == 0) {
        g[{0, 1}].push_back(0u);
        return g;
    }
    uint64_t m = (1ull << n) - 1ull;
    const uint64_t lim = 1ull << ns;
    while (m < lim) {
        int tm, p;
        sd_qn((uint32_t)m, ms, &tm, &p);
        g[{tm, p}].push_back((uint32_t)m);
        // next mask with the same popcount (ascending)
        uint64_t c = m & (~m + 1ull);
        uint64_t r = m + c;
        m = (((r ^ m) >> 2) / c) | r;
    }
    return g;
}

}  // namespace

int pair_index(int a, int b, int ns) { return a * ns - a * (a + 1) / 2 + (b - a - 1); }

int32_t SpeciesBasis::find(uint32_t mask, const std::vector<MState> &ms) const {
    int tm, p;
    sd_qn(mask, ms, &tm, &p);
    for (size_t s = 0; s < sectors.size(); ++s) {
        if (sectors[s].two_m != tm || sectors[s].parity != p) continue;
        auto b = sd.begin() + sectors[s].first;
        auto e = b + sectors[s].count;
        auto it = std::lower_bound(b, e, mask);
        if (it != e && *it == mask) return (int32_t)(it - sd.begin());
        return -1;
    }
    return -1;
}

}  // namespace fotci

using namespace fotci;

extern "C" int fotci_build_basis_impl(int32_t n_orbits, const int32_t *two_j, const int32_t *parity, int32_t Z,
                                      int32_t N, int32_t two_M, int32_t parity_total, fotci_basis **out) {
    if (!out) fail(FOTCI_EINVAL, "out is NULL");
    if (n_orbits <= 0 || !two_j || !parity) fail(FOTCI_EINVAL, "no orbits given");
    if (parity_total != 1 && parity_total != -1) fail(FOTCI_EINVAL, "parity_total must be +1 or -1");
    auto *b = new fotci_basis();
    try {
        int ns = 0;
        for (int o = 0; o < n_orbits; ++o) {
            if (two_j[o] <= 0 || (two_j[o] & 1) == 0) fail(FOTCI_EINVAL, "2j must be odd and positive");
            if (parity[o] != 1 && parity[o] != -1) fail(FOTCI_EINVAL, "orbit parity must be +1 or -1");
            for (int tm = -two_j[o]; tm <= two_j[o]; tm += 2) b->ms.push_back({o, two_j[o], tm, parity[o]});
            ns += two_j[o] + 1;
            if (ns > 32) fail(FOTCI_EINVAL, "more than 32 m-states per species");
        }
        if (Z < 0 || N < 0 || Z > ns || N > ns) fail(FOTCI_EINVAL, "particle number out of range");
        if (((two_M % 2) + 2) % 2 != (Z + N) % 2) fail(FOTCI_EINVAL, "parity of 2M does not match Z+N");
        b->n_orbits = n_orbits;
        b->two_M = two_M;
        b->parity = parity_total;
        b->p.n = Z;
        b->n.n = N;
        auto gp = enumerate_species(b->ms, Z);
        auto gn = enumerate_species(b->ms, N);
        std::vector<std::pair<int, int>> pkeys;
        for (auto &kv : gp) pkeys.push_back(kv.first);
        std::sort(pkeys.begin(), pkeys.end(), sector_less);
        std::vector<std::pair<std::pair<int, int>, std::pair<int, int>>> kept;
        for (auto k : pkeys) {
            std::pair<int, int> conj{two_M - k.first, parity_total * k.second};
            if (gn.count(conj)) kept.push_back({k, conj});
        }
        if (kept.empty()) fail(FOTCI_EINVAL, "empty basis");
        std::vector<std::pair<int, int>> nkeys;
        for (auto &kc : kept) nkeys.push_back(kc.second);
        std::sort(nkeys.begin(), nkeys.end(), sector_less);
        std::map<std::pair<int, int>, int> nsec_of;
        for (auto k : nkeys) {
            auto &v = gn[k];
            nsec_of[k] = (int)b->n.sectors.size();
            b->n.sectors.push_back({k.first, k.second, (int)b->n.sd.size(), (int)v.size()});
            for (size_t r = 0; r < v.size(); ++r) {
                b->n.sd.push_back(v[r]);
                b->n.sd_sector.push_back((int32_t)b->n.sectors.size() - 1);
                b->n.sd_local.push_back((int32_t)r);
                b->nstart.push_back((int64_t)r);
            }
        }
        int64_t off = 0;
        for (auto &kc : kept) {
            auto &v = gp[kc.first];
            int ps = (int)b->p.sectors.size();
            b->p.sectors.push_back({kc.first.first, kc.first.second, (int)b->p.sd.size(), (int)v.size()});
            int nsec = nsec_of[kc.second];
            const auto &nsx = b->n.sectors[nsec];
            BasisSector bs{kc.first.first, kc.first.second, ps, nsec, (int)b->p.sd.size(), (int)v.size(),
                           nsx.first, nsx.count, off};
            b->sectors.push_back(bs);
            for (size_t r = 0; r < v.size(); ++r) {
                b->p.sd.push_back(v[r]);
                b->p.sd_sector.push_back(ps);
                b->p.sd_local.push_back((int32_t)r);
                b->p_basis_sector.push_back((int32_t)b->sectors.size() - 1);
                b->pstart.push_back(off + (int64_t)r * nsx.count);
            }
            off += (int64_t)v.size() * nsx.count;
        }
        b->dim = off;
        if (b->p.sd.size() > (size_t)INT32_MAX / 2 || b->n.sd.size() > (size_t)INT32_MAX / 2)
            fail(FOTCI_EINVAL, "too many Slater determinants");
    } catch (...) {
        delete b;
        throw;
    }
    *out = b;
    return FOTCI_OK;
}

extern "C" int fotci_build_jumps_impl(const fotci_basis *b, fotci_jumps **out) {
    if (!b || !out) fail(FOTCI_EINVAL, "NULL argument");
    auto *j = new fotci_jumps();
    j->b = b;
    const auto &ms = b->ms;
    const int ns = (int)ms.size();
    j->ns = ns;
    j->npairs = ns * (ns - 1) / 2;
    const int npairs = j->npairs;
    // pairs and the rows allowed for each column pair
    std::vector<int> pa(npairs), pb(npairs);
    for (int a = 0; a < ns; ++a)
        for (int c = a + 1; c < ns; ++c) {
            int r = pair_index(a, c, ns);
            pa[r] = a;
            pb[r] = c;
        }
    std::vector<std::vector<int>> allowed(npairs);
    for (int col = 0; col < npairs; ++col)
        for (int row = 0; row < npairs; ++row)
            if (ms[pa[row]].two_m + ms[pb[row]].two_m == ms[pa[col]].two_m + ms[pb[col]].two_m &&
                ms[pa[row]].parity * ms[pb[row]].parity == ms[pa[col]].parity * ms[pb[col]].parity)
                allowed[col].push_back(row);

    for (int sp = 0; sp < 2; ++sp) {
        const SpeciesBasis &S = sp == 0 ? b->p : b->n;
        auto &two = j->rec[sp == 0 ? FOTCI_JUMP_PP2 : FOTCI_JUMP_NN2];
        auto &one = j->rec[sp == 0 ? FOTCI_JUMP_P1 : FOTCI_JUMP_N1];
        int occ[32];
        for (int32_t src = 0; src < (int32_t)S.sd.size(); ++src) {
            uint32_t m = S.sd[src];
            int no = 0;
            for (int i = 0; i < ns; ++i)
                if ((m >> i) & 1u) occ[no++] = i;
            const int sec = S.sd_sector[src];
            const auto &sx = S.sectors[sec];
            for (int i1 = 0; i1 < no; ++i1)
                for (int i2 = i1 + 1; i2 < no; ++i2) {
                    int c = occ[i1], d = occ[i2];
                    int col = pair_index(c, d, ns);
                    for (int row : allowed[col]) {
                        uint32_t res;
                        int s = two_body_action(m, pa[row], pb[row], c, d, &res);
                        if (!s) continue;
                        // same species sector: binary search inside it
                        auto bgn = S.sd.begin() + sx.first, end = bgn + sx.count;
                        auto it = std::lower_bound(bgn, end, res);
                        if (it == end || *it != res) fail(FOTCI_EINVAL, "internal: two-body jump left its sector");
                        two.push_back({src, (int32_t)(it - S.sd.begin()), (int32_t)(row * npairs + col), (int8_t)s});
                    }
                }
            for (int i1 = 0; i1 < no; ++i1) {
                int c = occ[i1];
                for (int a = 0; a < ns; ++a) {
                    uint32_t res;
                    int s = one_body_action(m, a, c, &res);
                    if (!s) continue;
                    int32_t dst = S.find(res, ms);
                    if (dst < 0) continue;
                    one.push_back({src, dst, (int32_t)(a * ns + c), (int8_t)s});
                }
            }
        }
        auto canon = [](const JumpRec &x, const JumpRec &y) {
            if (x.dst != y.dst) return x.dst < y.dst;
            if (x.src != y.src) return x.src < y.src;
            return x.label < y.label;
        };
        std::sort(two.begin(), two.end(), canon);
        std::sort(one.begin(), one.end(), canon);
    }
    // one-body operator classes
    OpClasses &cl = j->cls;
    std::map<std::pair<int, int>, int> key2q;
    std::vector<std::pair<int, int>> keys;
    for (int a = 0; a < ns; ++a)
        for (int c = 0; c < ns; ++c) {
            std::pair<int, int> k{ms[a].two_m - ms[c].two_m, ms[a].parity * ms[c].parity};
            if (!key2q.count(k)) {
                key2q[k] = 0;
                keys.push_back(k);
            }
        }
    std::sort(keys.begin(), keys.end(), [](std::pair<int, int> x, std::pair<int, int> y) {
        if (x.first != y.first) return x.first < y.first;
        return x.second > y.second;
    });
    cl.nq = (int)keys.size();
    for (int q = 0; q < cl.nq; ++q) {
        key2q[keys[q]] = q;
        cl.delta.push_back(keys[q].first);
        cl.rho.push_back(keys[q].second);
    }
    cl.ops.assign(cl.nq, {});
    cl.class_of.assign(ns * ns, -1);
    cl.local_of.assign(ns * ns, -1);
    for (int a = 0; a < ns; ++a)
        for (int c = 0; c < ns; ++c) {
            int q = key2q[{ms[a].two_m - ms[c].two_m, ms[a].parity * ms[c].parity}];
            int lab = a * ns + c;
            cl.class_of[lab] = q;
            cl.local_of[lab] = (int)cl.ops[q].size();
            cl.ops[q].push_back(lab);
        }
    for (int q = 0; q < cl.nq; ++q) {
        auto it = key2q.find({-keys[q].first, keys[q].second});
        if (it == key2q.end()) fail(FOTCI_EINVAL, "internal: operator class without conjugate");
        cl.conj.push_back(it->second);
    }
    *out = j;
    return FOTCI_OK;
}
