// Invariants of the pn gather lists that the pn kernel relies on, checked on
// the host tables libfotci builds (no device needed):
//   - every neutron one-body jump into a destination sector appears exactly
//     once in the list of its (sector, class, source tile), with the R element
//     (source column in the tile, label), destination column and phase it
//     implies;
//   - each list is a whole number of 64-entry rounds; in every lane, a
//     destination's entries form chunks of consecutive rounds ending in the
//     flush bit, and only padding (the null code) follows a lane's last chunk;
//   - two chunks of one destination never flush in the same pair of rounds
//     (the kernel reads the output row for both rounds of a pair before
//     writing either).
// The same for the lists of the float32 one-vector kernel, one per (sector,
// class, pair of source tiles, destination-column parity), whose R element
// also names the tile of the pair, and whose destinations all have the
// list's parity (the wave that owns those columns of the shared row).
// Usage: pack_check Z N (20-state space 2j = 1,3,5,7, 2M = Z + N mod 2).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "fotci_internal.h"

int main(int argc, char **argv) {
    const int32_t tj[4] = {1, 3, 5, 7}, par[4] = {1, 1, 1, 1};
    const int Z = argc > 1 ? atoi(argv[1]) : 3, N = argc > 2 ? atoi(argv[2]) : 3;
    fotci_basis *b = nullptr;
    fotci_jumps *j = nullptr;
    fotci_ham *h = nullptr;
    if (fotci_build_basis(4, tj, par, Z, N, (Z + N) % 2, 1, &b) || fotci_build_jumps(b, &j)) {
        printf("setup failed: %s\n", fotci_last_error());
        return 2;
    }
    const int ns = 20, np = ns * (ns - 1) / 2;
    std::vector<double> ep(4, 0.5), en(4, -0.3), vpp((size_t)np * np, 0.0), vnn((size_t)np * np, 0.0),
        vpn((size_t)ns * ns * ns * ns, 0.0);
    if (fotci_set_interaction(j, ep.data(), en.data(), vpp.data(), vnn.data(), vpn.data(), &h)) {
        printf("interaction failed: %s\n", fotci_last_error());
        return 2;
    }
    const auto &t = h->tt;
    const auto &cl = j->cls;
    const int S = (int)b->sectors.size(), nq = cl.nq, nch = std::max(t.n_t16, 1), n2 = std::max(t.n_s2, 1);
    std::vector<int> nsec_to_bsec(b->n.sectors.size(), -1);
    for (int s = 0; s < S; ++s) nsec_to_bsec[b->sectors[s].n_sector] = s;
    long bad = 0, entries = 0, slots = 0;
    // pairs = false: per-tile lists; true: the tile-pair, destination-parity lists
    for (const bool pairs : {false, true}) {
        const int rbits = pairs ? fotci::kPn2RBits : fotci::kPnRBits;
        const int dbits = pairs ? fotci::kPn2DstBits : fotci::kPnDstBits;
        const uint32_t null_code = (uint32_t)t.max_nn << rbits;
        const uint32_t kElem = (1u << rbits) - 1u, kDst = (1u << dbits) - 1u;
        const uint32_t n_elem = (uint32_t)((pairs ? 2 : 1) * fotci::kPnTile * fotci::kPnRStride);
        const auto &ptr = pairs ? t.pn2_ptr : t.pn_ptr;
        const auto &codes = pairs ? t.pn2_code : t.pn_code;
        if (ptr.size() != (size_t)S * nq * (pairs ? 2 * n2 : nch) + 1) ++bad;
        // expected entries per slot from the jump records
        std::map<int64_t, std::multiset<uint32_t>> want;
        for (const auto &r : j->rec[FOTCI_JUMP_N1]) {
            const int s = nsec_to_bsec[b->n.sd_sector[r.dst]];
            if (s < 0) continue;
            const int sl = b->n.sd_local[r.src], dl = b->n.sd_local[r.dst], tile = sl / fotci::kPnTile;
            const int64_t sq = (int64_t)s * nq + cl.class_of[r.label];
            const int64_t slot = pairs ? (sq * n2 + tile / 2) * 2 + (dl & 1) : sq * nch + tile;
            const uint32_t elem = (uint32_t)((pairs ? (tile & 1) * fotci::kPnTile * fotci::kPnRStride : 0) +
                                             (sl % fotci::kPnTile) * fotci::kPnRStride + cl.local_of[r.label]);
            want[slot].insert((r.phase < 0 ? 0x80000000u : 0u) | ((uint32_t)dl << rbits) | elem);
        }
        long ent_here = 0;
        for (size_t sl = 0; sl + 1 < ptr.size(); ++sl) {
            const int e0 = ptr[sl], e1 = ptr[sl + 1];
            if ((e1 - e0) % 64) ++bad;
            const int nr = (e1 - e0) / 64;
            slots += e1 - e0;
            std::multiset<uint32_t> got;
            std::map<uint32_t, std::set<int>> flush_pairs;
            for (int l = 0; l < 64; ++l) {
                bool open = false, ended = false;
                uint32_t cur = 0;
                for (int r = 0; r < nr; ++r) {
                    const uint32_t c = codes[e0 + 64 * r + l];
                    if (c == null_code) {
                        if (open) ++bad;   // a chunk must end in a flush
                        ended = true;
                        continue;
                    }
                    if (ended) ++bad;   // a real entry after padding
                    ++ent_here;
                    got.insert(c & ~fotci::kPnFlush);
                    const uint32_t dst = (c >> rbits) & kDst;
                    if ((c & kElem) >= n_elem) ++bad;
                    if (pairs && (dst & 1) != (sl & 1)) ++bad;   // the list's parity
                    if (open && dst != cur) ++bad;   // chunks are consecutive per destination
                    open = true;
                    cur = dst;
                    if (c & fotci::kPnFlush) {
                        if (!flush_pairs[dst].insert(r / 2).second) ++bad;
                        open = false;
                    }
                }
                if (open) ++bad;
            }
            auto it = want.find((int64_t)sl);
            const std::multiset<uint32_t> empty;
            if (got != (it == want.end() ? empty : it->second)) ++bad;
        }
        long want_n = 0;
        for (const auto &kv : want) want_n += (long)kv.second.size();
        if (want_n != ent_here) ++bad;
        entries += ent_here;
    }
    printf("Z=%d N=%d: %ld slots, %ld entries, %ld violations\n", Z, N, slots, entries, bad);
    return bad == 0 ? 0 : 1;
}
