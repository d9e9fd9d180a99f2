// Host side of the Hamiltonian: validation of the interaction, the device
// table layout (jumps grouped for destination-ordered gathers, pn matrix
// elements blocked by one-body operator class) and the upload into the
// caller's workspace.
//
// Matrix-element reconstruction follows Ch. 2 "Representation of the
// Hamiltonian": a pp (nn) matrix element is the sum, over the proton
// (neutron) two-body jumps between the same pair of SDs, of phase x V[label];
// a pn matrix element is phase_p x phase_n x V_pn for a pair of one-body
// jumps whose Jz changes cancel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "fotci_internal.h"

namespace fotci {

void hip_check(int err, const char *what) {
    if (err != hipSuccess) fail(FOTCI_EHIP, std::string(what) + ": " + hipGetErrorString((hipError_t)err));
}

void build_species_tables(const fotci_jumps *j, int sp, HostSpeciesTables &t) {
    const fotci_basis *b = j->b;
    const SpeciesBasis &S = sp == 0 ? b->p : b->n;
    const int n_sd = (int)S.sd.size();
    t.masks = S.sd;
    const auto &two = j->rec[sp == 0 ? FOTCI_JUMP_PP2 : FOTCI_JUMP_NN2];
    t.code2.resize(two.size());
    t.off_rowptr.assign(n_sd + 1, 0);
    t.off_col.clear();
    t.off_j0.clear();
    t.off_j1.clear();
    t.diag_j0.assign(n_sd, 0);
    t.diag_j1.assign(n_sd, 0);
    for (size_t k = 0; k < two.size(); ++k) t.code2[k] = two[k].label * 2 + (two[k].phase < 0 ? 1 : 0);
    size_t k = 0;
    while (k < two.size()) {
        size_t e = k;
        while (e < two.size() && two[e].dst == two[k].dst && two[e].src == two[k].src) ++e;
        const int dst = two[k].dst, src = two[k].src;
        if (src == dst) {
            t.diag_j0[dst] = (int32_t)k;
            t.diag_j1[dst] = (int32_t)e;
        } else {
            t.off_col.push_back(src);
            t.off_j0.push_back((int32_t)k);
            t.off_j1.push_back((int32_t)e);
            t.off_rowptr[dst + 1]++;
        }
        k = e;
    }
    for (int i = 0; i < n_sd; ++i) t.off_rowptr[i + 1] += t.off_rowptr[i];
    // one-body: by (dst, class, src, local op), the jumps with src == dst
    // (number operators of the occupied orbits) first in their class
    const OpClasses &cl = j->cls;
    const int nq = cl.nq;
    const auto &one = j->rec[sp == 0 ? FOTCI_JUMP_P1 : FOTCI_JUMP_N1];
    std::vector<JumpRec> ob(one.begin(), one.end());
    std::stable_sort(ob.begin(), ob.end(), [&](const JumpRec &x, const JumpRec &y) {
        if (x.dst != y.dst) return x.dst < y.dst;
        int qx = cl.class_of[x.label], qy = cl.class_of[y.label];
        if (qx != qy) return qx < qy;
        const bool dx = x.src == x.dst, dy = y.src == y.dst;
        if (dx != dy) return dx;
        if (x.src != y.src) return x.src < y.src;
        return cl.local_of[x.label] < cl.local_of[y.label];
    });
    t.ob_ptr.assign((size_t)n_sd * nq + 1, 0);
    t.ob_src.resize(ob.size());
    t.ob_code.resize(ob.size());
    for (size_t i = 0; i < ob.size(); ++i) {
        t.ob_ptr[(size_t)ob[i].dst * nq + cl.class_of[ob[i].label] + 1]++;
        t.ob_src[i] = ob[i].src;
        t.ob_code[i] = cl.local_of[ob[i].label] * 2 + (ob[i].phase < 0 ? 1 : 0);
    }
    for (size_t i = 0; i < (size_t)n_sd * nq; ++i) t.ob_ptr[i + 1] += t.ob_ptr[i];
}

// Extra tables of the tiled kernels: ELL layouts of the merged pp and nn
// entries per sector, the workgroup tiles, the neutron one-body jumps
// regrouped by source chunk for the pn gather, and the pn workgroup order
// (rows of the largest sectors first, so the longest workgroups start early).
void build_tiled_tables(fotci_ham *h) {
    const fotci_basis *b = h->j->b;
    const OpClasses &cl = h->j->cls;
    const int nq = cl.nq;
    const int S = (int)b->sectors.size();
    HostTiled &t = h->tt;
    constexpr int kTL = kPnTile;   // source tile of the pn kernel
    bool ok = true;
    for (int q = 0; q < nq; ++q)
        if (cl.ops[q].size() > 64) ok = false;
    t.max_nn = t.max_np = 0;
    for (const auto &s : b->sectors) {
        t.max_nn = std::max(t.max_nn, s.nn);
        t.max_np = std::max(t.max_np, s.np);
    }
    // LDS tiles hold up to 64 KiB of float64 (8 rows / columns of the largest sector)
    if ((int64_t)t.max_nn * 8 > 65536 || (int64_t)t.max_np * 8 > 65536 || t.max_nn >= (1 << 18)) ok = false;
    // the pn kernel keeps one output row and the contraction operand in LDS
    t.ok = ok;
    t.p_ob_base.resize(h->tp.ob_src.size());
    for (size_t k = 0; k < h->tp.ob_src.size(); ++k) t.p_ob_base[k] = b->pstart[h->tp.ob_src[k]];
    // per (row, class): the proton jumps that leave the row's SD unchanged,
    // which lead its list; the pn kernels contract them as one
    t.pn_ndiag.assign(h->tp.ob_ptr.size() - 1, 0);
    for (size_t rq = 0; rq + 1 < h->tp.ob_ptr.size(); ++rq) {
        const int ip = (int)(rq / (size_t)nq), a0 = h->tp.ob_ptr[rq], a1 = h->tp.ob_ptr[rq + 1];
        int nd = 0;
        while (a0 + nd < a1 && h->tp.ob_src[a0 + nd] == ip) ++nd;
        for (int k = a0 + nd; k < a1; ++k)
            if (h->tp.ob_src[k] == ip) ok = false;   // not at the front: the merge would be wrong
        t.pn_ndiag[rq] = (int8_t)std::min(nd, 127);
        if (nd > 127) ok = false;
    }
    // ELL tables
    auto ell = [&](const HostSpeciesTables &ts, const SpeciesBasis &sb, bool neutron, std::vector<int64_t> &base,
                   std::vector<int32_t> &E, std::vector<int32_t> &src, std::vector<int32_t> &ent) {
        base.assign(S, 0);
        E.assign(S, 0);
        src.clear();
        ent.clear();
        for (int s = 0; s < S; ++s) {
            const auto &bs = b->sectors[s];
            const int first = neutron ? bs.n_first : bs.p_first;
            const int n = neutron ? bs.nn : bs.np;
            int e = 0;
            for (int i = 0; i < n; ++i) e = std::max(e, ts.off_rowptr[first + i + 1] - ts.off_rowptr[first + i]);
            E[s] = e;
            base[s] = (int64_t)src.size();
            src.resize(src.size() + (size_t)e * n, 0);
            ent.resize(ent.size() + (size_t)e * n, -1);
            for (int i = 0; i < n; ++i)
                for (int k = ts.off_rowptr[first + i], r = 0; k < ts.off_rowptr[first + i + 1]; ++k, ++r) {
                    src[base[s] + (int64_t)r * n + i] = sb.sd_local[ts.off_col[k]];
                    ent[base[s] + (int64_t)r * n + i] = k;
                }
        }
    };
    ell(h->tn, b->n, true, t.nn_ell_base, t.nn_ell_E, t.nn_ell_src, t.nn_ell_ent);
    ell(h->tp, b->p, false, t.pp_ell_base, t.pp_ell_E, t.pp_ell_src, t.pp_ell_ent);
    // workgroup tiles: 8 rows (nn kernel) / 8 columns (pp kernel) per tile
    t.rt_sec.clear();
    t.rt_r0.clear();
    t.ct_sec.clear();
    t.ct_c0.clear();
    for (int s = 0; s < S; ++s) {
        for (int r = 0; r < b->sectors[s].np; r += 8) {
            t.rt_sec.push_back(s);
            t.rt_r0.push_back(r);
        }
        for (int c = 0; c < b->sectors[s].nn; c += 8) {
            t.ct_sec.push_back(s);
            t.ct_c0.push_back(c);
        }
    }
    // pn gather lists: neutron one-body jumps into the columns of each
    // destination sector, grouped by (neutron class, kPnTile-column source tile)
    t.n_t16 = (t.max_nn + kTL - 1) / kTL;
    const int nch = std::max(t.n_t16, 1);
    int kpmax = 1;
    for (size_t i = 0; i + 1 < h->tp.ob_ptr.size(); ++i) kpmax = std::max(kpmax, h->tp.ob_ptr[i + 1] - h->tp.ob_ptr[i]);
    t.kp_pad = (kpmax + 3) & ~3;
    // up to 32 proton jumps per class in the pn kernel; x addressed with 32-bit byte offsets
    // destination columns (and one padding column) in kPnDstBits bits of a gather code
    static_assert(kPnTile * kPnRStride <= (1 << kPnRBits), "R element must fit its code field");
    if (kpmax > 32 || b->dim * 8 >= ((int64_t)1 << 31) || t.max_nn >= (1 << kPnDstBits) - 1) ok = false;
    std::vector<int32_t> nsec_to_bsec(b->n.sectors.size(), -1);
    for (int s = 0; s < S; ++s) nsec_to_bsec[b->sectors[s].n_sector] = s;
    const auto &rec = h->j->rec[FOTCI_JUMP_N1];
    // Gather lists of the neutron one-body jumps, one list per slot (slot_of),
    // each entry's code from code_of (sign, destination column << rbits, R
    // element); see below for how a list is packed.
    auto build_lists = [&](int64_t nslots, auto slot_of, auto code_of, int rbits, std::vector<int32_t> &ptr,
                           std::vector<uint32_t> &codes) {
        // group the jumps by slot, ordered inside a slot by (source, label)
        std::vector<int64_t> cnt((size_t)nslots + 1, 0);
        for (const auto &r : rec) cnt[slot_of(r) + 1]++;
        for (size_t i = 0; i + 1 < cnt.size(); ++i) cnt[i + 1] += cnt[i];
        std::vector<size_t> order(rec.size());
        {
            std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
            std::vector<size_t> by_src(rec.size());
            for (size_t i = 0; i < rec.size(); ++i) by_src[i] = i;
            std::stable_sort(by_src.begin(), by_src.end(), [&](size_t x, size_t y) {
                if (rec[x].src != rec[y].src) return rec[x].src < rec[y].src;
                return rec[x].label < rec[y].label;
            });
            for (size_t i : by_src) order[fill[slot_of(rec[i])]++] = i;
        }
        // Pack each slot into rounds of 64 lanes. A destination column's entries
        // go to one lane in consecutive rounds (a chunk); the chunk's last entry
        // carries the flush bit, so the kernel sums the chunk in a register and
        // touches the output row once for it. The kernel works through rounds in
        // pairs, reading the output row for both rounds before writing either,
        // so two chunks of one destination must flush in different pairs; apart
        // from that a destination may be split over several lanes, which keeps
        // the rounds near ceil(entries / 64) even when one column receives many
        // entries. Destinations are placed most entries first, each chunk in the
        // lane with the most free rounds, for the smallest round count that
        // succeeds; unused slots get the null code (R element 0, the spare
        // column, no flush).
        const uint32_t null_code = (uint32_t)t.max_nn << rbits;
        ptr.assign(cnt.size(), 0);
        codes.clear();
        std::vector<std::pair<uint32_t, std::vector<uint32_t>>> bydst;
        std::vector<std::vector<uint32_t>> lanes(64);
        std::vector<int> lane_order(64);
        std::vector<char> used_pairs;
        auto pack = [&](int nr) -> bool {
            for (auto &l : lanes) l.clear();
            if ((int)used_pairs.size() < (nr + 1) / 2) used_pairs.resize((nr + 1) / 2);
            for (auto &dl : bydst) {
                const auto &e = dl.second;
                size_t done = 0;
                std::fill(used_pairs.begin(), used_pairs.begin() + (nr + 1) / 2, 0);   // pairs where a chunk flushes
                while (done < e.size()) {
                    // a chunk in lane l: as many entries as fit whose flush falls in a pair not yet used
                    auto try_lane = [&](int l) -> bool {
                        const int at = (int)lanes[l].size();
                        int size = std::min<int>((int)(e.size() - done), nr - at);
                        while (size > 0 && used_pairs[(at + size - 1) / 2]) --size;
                        if (size <= 0) return false;
                        used_pairs[(at + size - 1) / 2] = 1;
                        for (int i = 0; i < size; ++i) lanes[l].push_back(e[done + i] | (i + 1 == size ? kPnFlush : 0u));
                        done += (size_t)size;
                        return true;
                    };
                    // the emptiest lane first; the others by free rounds only if it cannot take a chunk
                    int best = 0;
                    for (int l = 1; l < 64; ++l)
                        if (lanes[l].size() < lanes[best].size()) best = l;
                    bool placed = try_lane(best);
                    if (!placed) {
                        for (int l = 0; l < 64; ++l) lane_order[l] = l;
                        std::stable_sort(lane_order.begin(), lane_order.end(),
                                         [&](int x, int y) { return lanes[x].size() < lanes[y].size(); });
                        for (int l : lane_order)
                            if (l != best && try_lane(l)) {
                                placed = true;
                                break;
                            }
                    }
                    if (!placed) return false;
                }
            }
            return true;
    };
        for (size_t sl = 0; sl + 1 < cnt.size(); ++sl) {
            ptr[sl] = (int32_t)codes.size();
            if (cnt[sl] == cnt[sl + 1]) continue;
            bydst.clear();
            std::map<uint32_t, size_t> where;
            for (int64_t k = cnt[sl]; k < cnt[sl + 1]; ++k) {
                const auto &r = rec[order[k]];
                const uint32_t dcol = (uint32_t)b->n.sd_local[r.dst];
                const uint32_t code = code_of(r);
                auto it = where.find(dcol);
                if (it == where.end()) {
                    where[dcol] = bydst.size();
                    bydst.push_back({dcol, {code}});
                } else {
                    bydst[it->second].second.push_back(code);
                }
            }
            std::stable_sort(bydst.begin(), bydst.end(), [](const auto &x, const auto &y) {
                if (x.second.size() != y.second.size()) return x.second.size() > y.second.size();
                return x.first < y.first;
            });
            const int64_t n = cnt[sl + 1] - cnt[sl];
            int nr = (int)std::max<int64_t>(1, (n + 63) / 64);
            while (!pack(nr)) ++nr;
            for (int rr = 0; rr < nr; ++rr)
                for (int l = 0; l < 64; ++l) codes.push_back(rr < (int)lanes[l].size() ? lanes[l][rr] : null_code);
        }
        ptr[cnt.size() - 1] = (int32_t)codes.size();
    };
    // one list per (sector, class, source tile) for the float64, block and
    // adjoint kernels
    auto slot = [&](const JumpRec &r) -> int64_t {
        const int s = nsec_to_bsec[b->n.sd_sector[r.dst]];
        const int qn = cl.class_of[r.label];
        const int ch = b->n.sd_local[r.src] / kTL;
        return ((int64_t)s * nq + qn) * nch + ch;
    };
    auto code1 = [&](const JumpRec &r) -> uint32_t {
        const uint32_t so = (uint32_t)(b->n.sd_local[r.src] % kTL);
        const uint32_t B = (uint32_t)cl.local_of[r.label];
        return (r.phase < 0 ? 0x80000000u : 0u) | ((uint32_t)b->n.sd_local[r.dst] << kPnRBits) |
               (so * (uint32_t)kPnRStride + B);
    };
    build_lists((int64_t)S * nq * nch, slot, code1, kPnRBits, t.pn_ptr, t.pn_code);
    // the float32 one-vector kernel: a step is a pair of source tiles (one
    // per wave), and each list holds the step's jumps into the destination
    // columns of one parity, which one wave owns in the shared output row;
    // the R element names the tile of the pair
    t.n_s2 = (nch + 1) / 2;
    auto slot2 = [&](const JumpRec &r) -> int64_t {
        const int s = nsec_to_bsec[b->n.sd_sector[r.dst]];
        const int qn = cl.class_of[r.label];
        const int ch = b->n.sd_local[r.src] / kTL;
        return (((int64_t)s * nq + qn) * t.n_s2 + ch / 2) * 2 + (b->n.sd_local[r.dst] & 1);
    };
    auto code2 = [&](const JumpRec &r) -> uint32_t {
        const int sl = b->n.sd_local[r.src];
        const uint32_t B = (uint32_t)cl.local_of[r.label];
        return (r.phase < 0 ? 0x80000000u : 0u) | ((uint32_t)b->n.sd_local[r.dst] << kPn2RBits) |
               ((uint32_t)((sl / kTL) & 1) * (uint32_t)(kPnTile * kPnRStride) + (uint32_t)(sl % kTL) * kPnRStride + B);
    };
    build_lists((int64_t)S * nq * t.n_s2 * 2, slot2, code2, kPn2RBits, t.pn2_ptr, t.pn2_code);
    // the pn kernel reads the codes through a buffer resource with 32-bit byte offsets
    if ((int64_t)t.pn_code.size() * 4 > INT32_MAX || (int64_t)t.pn2_code.size() * 4 > INT32_MAX) ok = false;
    if (t.max_nn + 1 + 128 > (1 << kPn2DstBits)) ok = false;
    t.ok = ok;
    const int npsd = (int)b->p.sd.size();
    t.order.resize(npsd);
    for (int i = 0; i < npsd; ++i) t.order[i] = i;
    std::stable_sort(t.order.begin(), t.order.end(), [&](int x, int y) {
        return b->sectors[b->p_basis_sector[x]].nn > b->sectors[b->p_basis_sector[y]].nn;
    });
}

void block_pn(fotci_ham *h) {
    const OpClasses &cl = h->j->cls;
    const int ns = h->j->ns;
    const size_t ns2 = (size_t)ns * ns;
    h->vq_off.assign(cl.nq, 0);
    h->vq_nb.assign(cl.nq, 0);
    size_t tot = 0;
    for (int q = 0; q < cl.nq; ++q) {
        h->vq_off[q] = (int32_t)tot;
        h->vq_nb[q] = (int32_t)cl.ops[cl.conj[q]].size();
        tot += cl.ops[q].size() * cl.ops[cl.conj[q]].size();
    }
    h->vq.assign(tot, 0.0);
    for (int q = 0; q < cl.nq; ++q) {
        const auto &A = cl.ops[q];
        const auto &B = cl.ops[cl.conj[q]];
        for (size_t ia = 0; ia < A.size(); ++ia) {
            const int a = A[ia] / ns, c = A[ia] % ns;
            for (size_t ib = 0; ib < B.size(); ++ib) {
                const int bb = B[ib] / ns, d = B[ib] % ns;
                h->vq[h->vq_off[q] + ia * B.size() + ib] = h->v_pn[((size_t)a * ns + bb) * ns2 + (size_t)c * ns + d];
            }
        }
    }
}

void fill_species_values(fotci_ham *h) {
    const fotci_basis *b = h->j->b;
    for (int sp = 0; sp < 2; ++sp) {
        HostSpeciesTables &t = sp == 0 ? h->tp : h->tn;
        const auto &spe = sp == 0 ? h->spe_p : h->spe_n;
        t.eps.resize(b->ms.size());
        for (size_t i = 0; i < b->ms.size(); ++i) t.eps[i] = spe[b->ms[i].orbit];
        t.v2 = sp == 0 ? h->v_pp : h->v_nn;
    }
    block_pn(h);
}

namespace {

void validate(const fotci_jumps *j, const double *spe_p, const double *spe_n, const double *v_pp,
              const double *v_nn, const double *v_pn) {
    if (!spe_p || !spe_n || !v_pp || !v_nn || !v_pn) fail(FOTCI_EINVAL, "interaction array is NULL");
    const auto &ms = j->b->ms;
    const int ns = j->ns, np = j->npairs;
    std::vector<int> pa(np), pb(np);
    for (int a = 0; a < ns; ++a)
        for (int c = a + 1; c < ns; ++c) {
            pa[pair_index(a, c, ns)] = a;
            pb[pair_index(a, c, ns)] = c;
        }
    for (int o = 0; o < j->b->n_orbits; ++o)
        if (!std::isfinite(spe_p[o]) || !std::isfinite(spe_n[o])) fail(FOTCI_EINVAL, "non-finite energy");
    for (const double *v : {v_pp, v_nn}) {
        for (int r = 0; r < np; ++r)
            for (int c = 0; c < np; ++c) {
                const double x = v[(size_t)r * np + c];
                if (!std::isfinite(x)) fail(FOTCI_EINVAL, "non-finite two-body matrix element");
                if (x != v[(size_t)c * np + r]) fail(FOTCI_EINVAL, "two-body matrix not symmetric");
                const bool ok = ms[pa[r]].two_m + ms[pb[r]].two_m == ms[pa[c]].two_m + ms[pb[c]].two_m &&
                                ms[pa[r]].parity * ms[pb[r]].parity == ms[pa[c]].parity * ms[pb[c]].parity;
                if (!ok && x != 0.0) fail(FOTCI_EINVAL, "two-body matrix element violates Jz or parity");
            }
    }
    const size_t n2 = (size_t)ns * ns;
    for (size_t r = 0; r < n2; ++r)
        for (size_t c = 0; c < n2; ++c) {
            const double x = v_pn[r * n2 + c];
            if (!std::isfinite(x)) fail(FOTCI_EINVAL, "non-finite pn matrix element");
            if (x != v_pn[c * n2 + r]) fail(FOTCI_EINVAL, "pn matrix not symmetric");
            const int a = (int)(r / ns), bb = (int)(r % ns), cc = (int)(c / ns), d = (int)(c % ns);
            const bool ok = ms[a].two_m + ms[bb].two_m == ms[cc].two_m + ms[d].two_m &&
                            ms[a].parity * ms[bb].parity == ms[cc].parity * ms[d].parity;
            if (!ok && x != 0.0) fail(FOTCI_EINVAL, "pn matrix element violates Jz or parity");
        }
}

void copy_values(fotci_ham *h, const double *spe_p, const double *spe_n, const double *v_pp, const double *v_nn,
                 const double *v_pn) {
    const int no = h->j->b->n_orbits, np = h->j->npairs, ns = h->j->ns;
    h->spe_p.assign(spe_p, spe_p + no);
    h->spe_n.assign(spe_n, spe_n + no);
    h->v_pp.assign(v_pp, v_pp + (size_t)np * np);
    h->v_nn.assign(v_nn, v_nn + (size_t)np * np);
    h->v_pn.assign(v_pn, v_pn + (size_t)ns * ns * ns * ns);
}

struct Item {
    const void *host;
    size_t bytes;
    void **dev;
};

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Device-table items in upload order; pointers in h->dev are set from ws.
std::vector<Item> items(fotci_ham *h) {
    const fotci_basis *b = h->j->b;
    DevHam &d = h->dev;
    std::vector<Item> it;
    HostCommonTables &c = h->tc;
    c.p_sector.assign(b->p_basis_sector.begin(), b->p_basis_sector.end());
    c.n_local.assign(b->n.sd_local.begin(), b->n.sd_local.end());
    c.sec_nn.clear();
    c.sec_nfirst.clear();
    c.sec_pfirst.clear();
    c.sec_np.clear();
    c.sec_off.clear();
    for (const auto &s : b->sectors) {
        c.sec_nn.push_back(s.nn);
        c.sec_nfirst.push_back(s.n_first);
        c.sec_pfirst.push_back(s.p_first);
        c.sec_np.push_back(s.np);
        c.sec_off.push_back(s.offset);
    }
    c.conjq.assign(h->j->cls.conj.begin(), h->j->cls.conj.end());
    c.ms_orbit.clear();
    for (const auto &m : b->ms) c.ms_orbit.push_back(m.orbit);
    c.n_bsector.assign(b->n.sd.size(), -1);
    for (size_t s = 0; s < b->sectors.size(); ++s)
        for (int r = 0; r < b->sectors[s].nn; ++r) c.n_bsector[b->sectors[s].n_first + r] = (int32_t)s;
    c.cls_off.assign(1, 0);
    c.cls_ops.clear();
    for (const auto &ops : h->j->cls.ops) {
        for (int lab : ops) c.cls_ops.push_back(lab);
        c.cls_off.push_back((int32_t)c.cls_ops.size());
    }
    auto add = [&](const void *p, size_t bytes, void *devfield) { it.push_back({p, bytes, (void **)devfield}); };
    add(c.p_sector.data(), c.p_sector.size() * 4, &d.p_sector);
    add(b->pstart.data(), b->pstart.size() * 8, &d.p_pstart);
    add(c.n_local.data(), c.n_local.size() * 4, &d.n_local);
    add(c.sec_nn.data(), c.sec_nn.size() * 4, &d.sec_nn);
    add(c.sec_nfirst.data(), c.sec_nfirst.size() * 4, &d.sec_nfirst);
    add(c.sec_pfirst.data(), c.sec_pfirst.size() * 4, &d.sec_pfirst);
    add(c.sec_np.data(), c.sec_np.size() * 4, &d.sec_np);
    add(c.sec_off.data(), c.sec_off.size() * 8, &d.sec_off);
    add(c.conjq.data(), c.conjq.size() * 4, &d.conjq);
    add(c.ms_orbit.data(), c.ms_orbit.size() * 4, &d.ms_orbit);
    add(c.n_bsector.data(), c.n_bsector.size() * 4, &d.n_bsector);
    add(c.cls_off.data(), c.cls_off.size() * 4, &d.cls_off);
    add(c.cls_ops.data(), c.cls_ops.size() * 4, &d.cls_ops);
    add(h->vq_off.data(), h->vq_off.size() * 4, &d.vq_off);
    add(h->vq_nb.data(), h->vq_nb.size() * 4, &d.vq_nb);
    add(h->vq.data(), h->vq.size() * 8, &d.vq64);
    add(nullptr, h->vq.size() * 4, &d.vq32);
    add(nullptr, h->tn.masks.size() * 8, &d.scratch_ncol);
    HostTiled &tt = h->tt;
    DevTiled &dt = h->dev_tiled;
    dt.ok = tt.ok ? 1 : 0;
    dt.pn_priv = h->pn_priv;
    dt.nn_ell_len = (int64_t)tt.nn_ell_src.size();
    dt.pp_ell_len = (int64_t)tt.pp_ell_src.size();
    dt.n_rtiles = (int32_t)tt.rt_sec.size();
    dt.n_ctiles = (int32_t)tt.ct_sec.size();
    dt.rt_rows = 8;
    dt.ct_cols = 8;
    dt.n_t16 = std::max(tt.n_t16, 1);
    dt.n_pn_code = (int64_t)tt.pn_code.size();
    dt.pn_null = (uint32_t)tt.max_nn << kPnRBits;
    dt.n_pn2_code = (int64_t)tt.pn2_code.size();
    dt.pn2_null = (uint32_t)tt.max_nn << kPn2RBits;
    dt.n_s2 = std::max(tt.n_s2, 1);
    dt.kp_pad = tt.kp_pad;
    dt.max_nn = tt.max_nn;
    dt.max_np = tt.max_np;
    add(tt.order.data(), tt.order.size() * 4, &dt.order);
    add(tt.p_ob_base.data(), tt.p_ob_base.size() * 8, &dt.p_ob_base);
    add(tt.nn_ell_base.data(), tt.nn_ell_base.size() * 8, &dt.nn_ell_base);
    add(tt.nn_ell_E.data(), tt.nn_ell_E.size() * 4, &dt.nn_ell_E);
    add(tt.nn_ell_src.data(), tt.nn_ell_src.size() * 4, &dt.nn_ell_src);
    add(tt.nn_ell_ent.data(), tt.nn_ell_ent.size() * 4, &dt.nn_ell_ent);
    add(nullptr, tt.nn_ell_src.size() * sizeof(EllE64), &dt.nn_ell_e64);
    add(nullptr, tt.nn_ell_src.size() * sizeof(EllE32), &dt.nn_ell_e32);
    add(tt.pp_ell_base.data(), tt.pp_ell_base.size() * 8, &dt.pp_ell_base);
    add(tt.pp_ell_E.data(), tt.pp_ell_E.size() * 4, &dt.pp_ell_E);
    add(tt.pp_ell_src.data(), tt.pp_ell_src.size() * 4, &dt.pp_ell_src);
    add(tt.pp_ell_ent.data(), tt.pp_ell_ent.size() * 4, &dt.pp_ell_ent);
    add(nullptr, tt.pp_ell_src.size() * sizeof(EllE64), &dt.pp_ell_e64);
    add(nullptr, tt.pp_ell_src.size() * sizeof(EllE32), &dt.pp_ell_e32);
    add(tt.rt_sec.data(), tt.rt_sec.size() * 4, &dt.rt_sec);
    add(tt.rt_r0.data(), tt.rt_r0.size() * 4, &dt.rt_r0);
    add(tt.ct_sec.data(), tt.ct_sec.size() * 4, &dt.ct_sec);
    add(tt.ct_c0.data(), tt.ct_c0.size() * 4, &dt.ct_c0);
    add(tt.pn_ptr.data(), tt.pn_ptr.size() * 4, &dt.pn_ptr);
    add(tt.pn_code.data(), tt.pn_code.size() * 4, &dt.pn_code);
    add(tt.pn2_ptr.data(), tt.pn2_ptr.size() * 4, &dt.pn2_ptr);
    add(tt.pn_ndiag.data(), tt.pn_ndiag.size(), &dt.pn_ndiag);
    add(tt.pn2_code.data(), tt.pn2_code.size() * 4, &dt.pn2_code);
    for (int sp = 0; sp < 2; ++sp) {
        HostSpeciesTables &t = sp == 0 ? h->tp : h->tn;
        DevSpecies &ds = sp == 0 ? d.p : d.n;
        add(t.masks.data(), t.masks.size() * 4, &ds.masks);
        add(t.code2.data(), t.code2.size() * 4, &ds.code2);
        add(t.off_rowptr.data(), t.off_rowptr.size() * 4, &ds.off_rowptr);
        add(t.off_col.data(), t.off_col.size() * 4, &ds.off_col);
        add(t.off_j0.data(), t.off_j0.size() * 4, &ds.off_j0);
        add(t.off_j1.data(), t.off_j1.size() * 4, &ds.off_j1);
        add(t.diag_j0.data(), t.diag_j0.size() * 4, &ds.diag_j0);
        add(t.diag_j1.data(), t.diag_j1.size() * 4, &ds.diag_j1);
        add(t.ob_ptr.data(), t.ob_ptr.size() * 4, &ds.ob_ptr);
        add(t.ob_src.data(), t.ob_src.size() * 4, &ds.ob_src);
        add(t.ob_code.data(), t.ob_code.size() * 4, &ds.ob_code);
        add(t.eps.data(), t.eps.size() * 8, &ds.eps);
        add(t.v2.data(), t.v2.size() * 8, &ds.v2);
        add(nullptr, t.off_col.size() * 8, &ds.off_val64);
        add(nullptr, t.off_col.size() * 4, &ds.off_val32);
        add(nullptr, t.masks.size() * 8, &ds.d64);
        add(nullptr, t.masks.size() * 4, &ds.d32);
    }
    return it;
}

void fill_dev_scalars(fotci_ham *h) {
    const fotci_basis *b = h->j->b;
    DevHam &d = h->dev;
    d.ns = h->j->ns;
    d.npairs = h->j->npairs;
    d.nq = h->j->cls.nq;
    d.n_sectors = (int32_t)b->sectors.size();
    d.n_vq = (int32_t)h->vq.size();
    d.dim = b->dim;
    d.p.n_sd = (int32_t)h->tp.masks.size();
    d.p.n_off = (int32_t)h->tp.off_col.size();
    d.n.n_sd = (int32_t)h->tn.masks.size();
    d.n.n_off = (int32_t)h->tn.off_col.size();
}

}  // namespace

}  // namespace fotci

using namespace fotci;

extern "C" int fotci_set_interaction_impl(const fotci_jumps *j, const double *spe_p, const double *spe_n,
                                          const double *v_pp, const double *v_nn, const double *v_pn,
                                          fotci_ham **out) {
    if (!j || !out) fail(FOTCI_EINVAL, "NULL argument");
    validate(j, spe_p, spe_n, v_pp, v_nn, v_pn);
    auto *h = new fotci_ham();
    try {
        h->j = j;
        copy_values(h, spe_p, spe_n, v_pp, v_nn, v_pn);
        build_species_tables(j, 0, h->tp);
        build_species_tables(j, 1, h->tn);
        build_tiled_tables(h);
        fill_species_values(h);
        fill_dev_scalars(h);
        int64_t off = 0;
        for (auto &x : items(h)) off = align256(off) + (int64_t)x.bytes;
        h->layout_total = align256(off);
    } catch (...) {
        delete h;
        throw;
    }
    *out = h;
    return FOTCI_OK;
}

extern "C" int64_t fotci_ham_workspace_bytes_impl(const fotci_ham *h) {
    if (!h) fail(FOTCI_EINVAL, "NULL handle");
    return h->layout_total;
}

extern "C" int fotci_ham_upload_impl(fotci_ham *h, void *ws, int64_t bytes, void *stream) {
    if (!h || !ws) fail(FOTCI_EINVAL, "NULL argument");
    if (((uintptr_t)ws & 255u) != 0) fail(FOTCI_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < h->layout_total) fail(FOTCI_ENOMEM, "workspace smaller than fotci_ham_workspace_bytes");
    hipStream_t st = (hipStream_t)stream;
    int64_t off = 0;
    for (auto &x : items(h)) {
        off = align256(off);
        *x.dev = (char *)ws + off;
        if (x.host && x.bytes) hip_check(hipMemcpyAsync(*x.dev, x.host, x.bytes, hipMemcpyHostToDevice, st), "upload");
        off += (int64_t)x.bytes;
    }
    h->ws = ws;
    h->ws_bytes = bytes;
    launch_materialize(h, stream);
    hip_check(hipStreamSynchronize(st), "upload sync");
    h->uploaded = true;
    return FOTCI_OK;
}

extern "C" int fotci_ham_set_values_impl(fotci_ham *h, const double *spe_p, const double *spe_n, const double *v_pp,
                                         const double *v_nn, const double *v_pn, void *stream) {
    if (!h) fail(FOTCI_EINVAL, "NULL handle");
    validate(h->j, spe_p, spe_n, v_pp, v_nn, v_pn);
    copy_values(h, spe_p, spe_n, v_pp, v_nn, v_pn);
    fill_species_values(h);
    if (h->uploaded) {
        hipStream_t st = (hipStream_t)stream;
        hip_check(hipMemcpyAsync((void *)h->dev.vq64, h->vq.data(), h->vq.size() * 8, hipMemcpyHostToDevice, st),
                  "upload");
        for (int sp = 0; sp < 2; ++sp) {
            HostSpeciesTables &t = sp == 0 ? h->tp : h->tn;
            DevSpecies &ds = sp == 0 ? h->dev.p : h->dev.n;
            hip_check(hipMemcpyAsync((void *)ds.eps, t.eps.data(), t.eps.size() * 8, hipMemcpyHostToDevice, st),
                      "upload");
            hip_check(hipMemcpyAsync((void *)ds.v2, t.v2.data(), t.v2.size() * 8, hipMemcpyHostToDevice, st),
                      "upload");
        }
        launch_materialize(h, stream);
        hip_check(hipStreamSynchronize(st), "upload sync");
    }
    return FOTCI_OK;
}

extern "C" int fotci_ham_op_counts_impl(const fotci_ham *h, int64_t *ops_pp, int64_t *ops_nn, int64_t *ops_pn,
                                        int64_t *ops_diag) {
    if (!h) fail(FOTCI_EINVAL, "NULL handle");
    const fotci_basis *b = h->j->b;
    const int nq = h->j->cls.nq;
    int64_t pp = 0, nn = 0, pn = 0;
    for (const auto &s : b->sectors) {
        for (int ip = s.p_first; ip < s.p_first + s.np; ++ip)
            pp += (int64_t)(h->tp.off_rowptr[ip + 1] - h->tp.off_rowptr[ip]) * s.nn;
        for (int jn = s.n_first; jn < s.n_first + s.nn; ++jn)
            nn += (int64_t)(h->tn.off_rowptr[jn + 1] - h->tn.off_rowptr[jn]) * s.np;
        for (int q = 0; q < nq; ++q) {
            const int qn = h->j->cls.conj[q];
            int64_t cp = 0, cn = 0;
            for (int ip = s.p_first; ip < s.p_first + s.np; ++ip)
                cp += h->tp.ob_ptr[(size_t)ip * nq + q + 1] - h->tp.ob_ptr[(size_t)ip * nq + q];
            for (int jn = s.n_first; jn < s.n_first + s.nn; ++jn)
                cn += h->tn.ob_ptr[(size_t)jn * nq + qn + 1] - h->tn.ob_ptr[(size_t)jn * nq + qn];
            pn += cp * cn;
        }
    }
    if (ops_pp) *ops_pp = pp;
    if (ops_nn) *ops_nn = nn;
    if (ops_pn) *ops_pn = pn;
    if (ops_diag) *ops_diag = b->dim;
    return FOTCI_OK;
}

// Work of the pn kernel in one apply_H, from the same tables and in the same
// order the kernel visits them: per destination row and operator class with
// proton jumps, every source tile whose gather list is not empty (the
// per-tile lists), or every existing tile of a tile pair whose two lists are
// not both empty (the float32 one-vector kernel with its shared output row).
extern "C" int fotci_ham_pn_work_impl(const fotci_ham *h, int32_t mode, int64_t *tile_visits, int64_t *mfma_instr,
                                      int64_t *gather_slots) {
    if (!h || (mode != FOTCI_MODE_F32 && mode != FOTCI_MODE_F64)) fail(FOTCI_EINVAL, "bad argument");
    const HostTiled &t = h->tt;
    if (!t.ok) fail(FOTCI_ESTATE, "the tiled kernels are not available for this basis");
    const fotci_basis *b = h->j->b;
    const int nq = h->j->cls.nq;
    const int ntl = std::max(t.n_t16, 1), ns2 = std::max(t.n_s2, 1);
    const auto &tc = h->tc;
    // the launch's choice of kernel for float32 vectors
    const bool pairs = mode == FOTCI_MODE_F32 && h->pn_priv && pn_split_row_fits(t.max_nn);
    int64_t visits = 0, mfma = 0, slots = 0;
    for (int ip = 0; ip < (int)b->p.sd.size(); ++ip) {
        const int s = tc.p_sector[ip];
        for (int q = 0; q < nq; ++q) {
            const int a0 = h->tp.ob_ptr[(size_t)ip * nq + q], a1 = h->tp.ob_ptr[(size_t)ip * nq + q + 1];
            if (a0 == a1) continue;
            const int qn = h->j->cls.conj[q];
            const int nbt = (h->vq_nb[q] + 15) / 16;
            const int nd = t.pn_ndiag[(size_t)ip * nq + q];
            const int kst = (a1 - a0 - (nd > 1 ? nd - 1 : 0) + 3) / 4;
            const int nns = tc.sec_nn[tc.p_sector[h->tp.ob_src[a0]]];
            const int ntiles = (nns + kPnTile - 1) / kPnTile;
            if (pairs) {
                const int64_t base = ((int64_t)s * nq + qn) * ns2 * 2;
                for (int st = 0; st < (ntiles + 1) / 2; ++st) {
                    const int64_t ne = t.pn2_ptr[base + 2 * st + 2] - t.pn2_ptr[base + 2 * st];
                    if (ne == 0) continue;
                    const int nt = std::min(2, ntiles - 2 * st);
                    visits += nt;
                    mfma += (int64_t)nt * (kPnTile / 16) * nbt * kst;
                    slots += ne;
                }
            } else {
                const int64_t base = ((int64_t)s * nq + qn) * ntl;
                for (int tt = 0; tt < ntiles; ++tt) {
                    const int64_t ne = t.pn_ptr[base + tt + 1] - t.pn_ptr[base + tt];
                    if (ne == 0) continue;
                    visits += 1;
                    mfma += (int64_t)(kPnTile / 16) * nbt * kst;
                    slots += ne;
                }
            }
        }
    }
    if (tile_visits) *tile_visits = visits;
    if (mfma_instr) *mfma_instr = mfma;
    if (gather_slots) *gather_slots = slots;
    return FOTCI_OK;
}

extern "C" int fotci_ham_set_pn_private_rows_impl(fotci_ham *h, int32_t enable) {
    if (!h || (enable != 0 && enable != 1)) fail(FOTCI_EINVAL, "bad argument");
    h->pn_priv = enable;
    h->dev_tiled.pn_priv = enable;
    return FOTCI_OK;
}
