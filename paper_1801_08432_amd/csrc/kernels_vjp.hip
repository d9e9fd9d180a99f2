// Adjoint of y = H(V) x for a scalar loss L = <g, y> (float64).
//
//   dL/dx = H g, since H is real symmetric;
//   dL/dV[label] = <g| O_label |x>: the label-wise transition density of the
//   operator string that V[label] multiplies (the m-scheme analogue of the
//   paper's two-body densities, Ch. 5 "Two-body densities": a density is what
//   <g|H|x> becomes when every interaction element but one is zero and that
//   one is 1).
// Each density is a sum over the same jumps apply_H uses:
//   pp: phase * <g row dst, x row src> per proton two-body jump;
//   nn: phase * <g column dst, x column src> per neutron two-body jump;
//   pn: phase_p phase_n g[ip',jn'] x[ip,jn] per pair of one-body jumps;
//   spe: <g, n_orbit x> from the row/column dots of the diagonal.
// Label bins receive float64 atomic adds (several jumps share a label).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "tiled_common.h"

namespace fotci {

namespace {


__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// block-wide sum returned to every thread
__device__ __forceinline__ double block_sum_all(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kT / 64; ++w) t += lds[w];
    return t;
}

__global__ __launch_bounds__(kT) void k_zero(double *p, int n) {
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Proton side, one block per destination proton SD ip: the diagonal row dot
// (proton single-particle energies and diagonal two-body labels), the
// per-element products for the neutron diagonal (column sums, atomically),
// and, with with_off, row dots against every source row of its off-diagonal
// two-body entries (used when the tiled tables are not available;
// k_vjp_sddmm<false> otherwise).
__global__ __launch_bounds__(kT) void k_vjp_proton(DevHam P, const double *__restrict__ x,
                                                   const double *__restrict__ g, double *d_spe_p,
                                                   double *d_v_pp, double *dcol_n, int with_off) {
    __shared__ double lds[kT / 64];
    const int ip = blockIdx.x;
    const int s = P.p_sector[ip];
    const int nn = P.sec_nn[s], nf = P.sec_nfirst[s];
    const int64_t base = P.p_pstart[ip];
    // diagonal row dot
    double acc = 0.0;
    for (int c = threadIdx.x; c < nn; c += kT) {
        const double gx = g[base + c] * x[base + c];
        acc += gx;
        if (dcol_n) atomicAdd(&dcol_n[nf + c], gx);
    }
    const double dd = block_sum_all(acc, lds);
    if (threadIdx.x == 0) {
        if (d_spe_p) {
            const uint32_t m = P.p.masks[ip];
            for (int b = 0; b < P.ns; ++b)
                if ((m >> b) & 1u) atomicAdd(&d_spe_p[P.ms_orbit[b]], dd);
        }
        if (d_v_pp)
            for (int j = P.p.diag_j0[ip]; j < P.p.diag_j1[ip]; ++j) {
                const int code = P.p.code2[j];
                atomicAdd(&d_v_pp[code >> 1], (code & 1) ? -dd : dd);
            }
    }
    if (!d_v_pp || !with_off) return;
    for (int k = P.p.off_rowptr[ip]; k < P.p.off_rowptr[ip + 1]; ++k) {
        const int64_t sb = P.p_pstart[P.p.off_col[k]];
        double a = 0.0;
        for (int c = threadIdx.x; c < nn; c += kT) a += g[base + c] * x[sb + c];
        const double dot = block_sum_all(a, lds);
        if (threadIdx.x == 0)
            for (int j = P.p.off_j0[k]; j < P.p.off_j1[k]; ++j) {
                const int code = P.p.code2[j];
                atomicAdd(&d_v_pp[code >> 1], (code & 1) ? -dot : dot);
            }
    }
}

// Neutron side, one block per destination neutron SD jn: the diagonal (the
// column sums of g o x) and, with with_off, the off-diagonal entries as column
// dots over the proton rows of its basis sector (used when the tiled tables
// are not available; k_vjp_nn_sddmm otherwise).
__global__ __launch_bounds__(kT) void k_vjp_neutron(DevHam P, const double *__restrict__ x,
                                                    const double *__restrict__ g, const double *dcol_n,
                                                    double *d_spe_n, double *d_v_nn, int with_off) {
    __shared__ double lds[kT / 64];
    const int jn = blockIdx.x;
    const int s = P.n_bsector[jn];
    if (s < 0) return;
    const int np = P.sec_np[s], nn = P.sec_nn[s];
    const int64_t off = P.sec_off[s];
    const int cd = P.n_local[jn];
    if (threadIdx.x == 0) {
        const double dd = dcol_n[jn];
        if (d_spe_n) {
            const uint32_t m = P.n.masks[jn];
            for (int b = 0; b < P.ns; ++b)
                if ((m >> b) & 1u) atomicAdd(&d_spe_n[P.ms_orbit[b]], dd);
        }
        if (d_v_nn)
            for (int j = P.n.diag_j0[jn]; j < P.n.diag_j1[jn]; ++j) {
                const int code = P.n.code2[j];
                atomicAdd(&d_v_nn[code >> 1], (code & 1) ? -dd : dd);
            }
    }
    if (!d_v_nn || !with_off) return;
    for (int k = P.n.off_rowptr[jn]; k < P.n.off_rowptr[jn + 1]; ++k) {
        const int cs = P.n_local[P.n.off_col[k]];
        double a = 0.0;
        for (int r = threadIdx.x; r < np; r += kT) a += g[off + (int64_t)r * nn + cd] * x[off + (int64_t)r * nn + cs];
        const double dot = block_sum_all(a, lds);
        if (threadIdx.x == 0)
            for (int j = P.n.off_j0[k]; j < P.n.off_j1[k]; ++j) {
                const int code = P.n.code2[j];
                atomicAdd(&d_v_nn[code >> 1], (code & 1) ? -dot : dot);
            }
    }
}

// pn, one block per (destination proton SD ip', operator class q): bins
// (A, B) of V^q accumulate phase_p phase_n g[ip',jn'] x[ip,jn] in LDS, then
// go to the full (N_s^2)^2 layout of V_pn with global atomics.
constexpr int kMaxBins = 4096;
__global__ __launch_bounds__(kT) void k_vjp_pn(DevHam P, const double *__restrict__ x,
                                               const double *__restrict__ g, double *d_v_pn) {
    __shared__ double bins[kMaxBins];
    const int nq = P.nq;
    const int ip = blockIdx.x / nq;
    const int q = blockIdx.x % nq;
    const int a0 = P.p.ob_ptr[(int64_t)ip * nq + q], a1 = P.p.ob_ptr[(int64_t)ip * nq + q + 1];
    if (a0 == a1) return;
    const int qn = P.conjq[q];
    const int na = P.cls_off[q + 1] - P.cls_off[q];
    const int nb = P.vq_nb[q];
    for (int i = threadIdx.x; i < na * nb; i += kT) bins[i] = 0.0;
    __syncthreads();
    const int s = P.p_sector[ip];
    const int nn = P.sec_nn[s], nf = P.sec_nfirst[s];
    const int64_t base = P.p_pstart[ip];
    for (int ka = a0; ka < a1; ++ka) {
        const int ca = P.p.ob_code[ka];
        const int A = ca >> 1;
        const double sa = (ca & 1) ? -1.0 : 1.0;
        const int64_t sbase = P.p_pstart[P.p.ob_src[ka]];
        for (int c = threadIdx.x; c < nn; c += kT) {
            const int jn = nf + c;
            const double gv = sa * g[base + c];
            const int b0 = P.n.ob_ptr[(int64_t)jn * nq + qn], b1 = P.n.ob_ptr[(int64_t)jn * nq + qn + 1];
            for (int kb = b0; kb < b1; ++kb) {
                const int cb = P.n.ob_code[kb];
                const double v = gv * x[sbase + P.n_local[P.n.ob_src[kb]]];
                atomicAdd(&bins[A * nb + (cb >> 1)], (cb & 1) ? -v : v);
            }
        }
    }
    __syncthreads();
    const int ns = P.ns;
    const int64_t ns2 = (int64_t)ns * ns;
    for (int i = threadIdx.x; i < na * nb; i += kT) {
        const double v = bins[i];
        if (v == 0.0) continue;
        const int la = P.cls_ops[P.cls_off[q] + i / nb];
        const int lb = P.cls_ops[P.cls_off[qn] + i % nb];
        const int a = la / ns, c = la % ns, b = lb / ns, d = lb % ns;
        atomicAdd(&d_v_pn[((int64_t)a * ns + b) * ns2 + (int64_t)c * ns + d], v);
    }
}

// Two-body densities of one species as a sampled product. In a basis sector
// (the row-major np x nn blocks G and X of g and x):
//   neutrons (NEUT): the entry from column cs to column cd needs
//     D[cd, cs] = sum_r g[r, cd] x[r, cs], D = G^T X;
//   protons: the entry from row rs to row rd needs
//     D[rd, rs] = sum_c g[rd, c] x[rs, c], D = G X^T;
// sampled on the pattern of the species' two-body jumps, and
// d_v[label] += phase D for every jump of the entry. One wave per 32 x 32
// tile of D that holds an entry: the sum runs on the matrix cores (16x16x4
// float64), the tile goes to LDS, and the wave samples it at the ELL entries
// (the tables of the tiled apply) of its 32 destination columns or rows.
constexpr int kSd = 32;

template <bool NEUT>
__global__ __launch_bounds__(64) void k_vjp_sddmm(DevHam P, DevTiled TT, const double *__restrict__ x,
                                                  const double *__restrict__ g, double *d_v) {
    __shared__ double Dt[kSd][kSd + 1];
    int b = blockIdx.x, s = 0;
    for (; s < P.n_sectors; ++s) {
        const int m = NEUT ? P.sec_nn[s] : P.sec_np[s];
        const int nb = (m + kSd - 1) / kSd;
        if (b < nb * nb) break;
        b -= nb * nb;
    }
    if (s >= P.n_sectors) return;   // uniform
    const int np = P.sec_np[s], nn = P.sec_nn[s];
    const int m = NEUT ? nn : np;   // D is m x m
    const int K = NEUT ? np : nn;   // summed index
    const int nbk = (m + kSd - 1) / kSd;
    const int d0 = kSd * (b / nbk), s0 = kSd * (b % nbk);
    const int64_t off = P.sec_off[s];
    const int E = NEUT ? TT.nn_ell_E[s] : TT.pp_ell_E[s];
    const int64_t eb = NEUT ? TT.nn_ell_base[s] : TT.pp_ell_base[s];
    const int32_t *esrc = NEUT ? TT.nn_ell_src : TT.pp_ell_src;
    const int32_t *eent = NEUT ? TT.nn_ell_ent : TT.pp_ell_ent;
    const DevSpecies &sp = NEUT ? P.n : P.p;
    const int lane = threadIdx.x;
    // skip tiles that no entry samples
    bool hit = false;
    for (int i = lane; i < kSd * E; i += 64) {
        const int dd = d0 + (i & (kSd - 1));
        if (dd >= m) continue;
        const int64_t k = eb + (int64_t)(i / kSd) * m + dd;
        if (eent[k] >= 0 && esrc[k] >= s0 && esrc[k] < s0 + kSd) hit = true;
    }
    if (__ballot(hit) == 0) return;   // uniform
    doublex4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Mma<double>::zero();
    // lane: summed index k0 + lane / 16 of each step of 4, tile index 16 i + lane % 16
    const int cl = lane & 15;
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int kk = k0 + (lane >> 4);
        double a[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int dd = d0 + 16 * i + cl, ss = s0 + 16 * i + cl;
            const bool ok = kk < K;
            if (NEUT) {   // G^T[dd][kk] = g[kk, dd], X[kk][ss] = x[kk, ss]
                a[i] = ok && dd < m ? g[off + (int64_t)kk * nn + dd] : 0.0;
                bv[i] = ok && ss < m ? x[off + (int64_t)kk * nn + ss] : 0.0;
            } else {      // G[dd][kk] = g[dd, kk], X^T[kk][ss] = x[ss, kk]
                a[i] = ok && dd < m ? g[off + (int64_t)dd * nn + kk] : 0.0;
                bv[i] = ok && ss < m ? x[off + (int64_t)ss * nn + kk] : 0.0;
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = Mma<double>::mma(a[i], bv[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) Dt[16 * i + Mma<double>::row(lane, q)][16 * j + cl] = acc[i][j][q];
    __syncthreads();
    for (int i = lane; i < kSd * E; i += 64) {
        const int c = i & (kSd - 1), dd = d0 + c;
        if (dd >= m) continue;
        const int64_t k = eb + (int64_t)(i / kSd) * m + dd;
        const int ent = eent[k];
        const int src = esrc[k];
        if (ent < 0 || src < s0 || src >= s0 + kSd) continue;
        const double dv = Dt[c][src - s0];
        for (int j = sp.off_j0[ent]; j < sp.off_j1[ent]; ++j) {
            const int code = sp.code2[j];
            atomicAdd(&d_v[code >> 1], (code & 1) ? -dv : dv);
        }
    }
}

// pn densities on the matrix cores: the transpose of the pn part of apply_H.
// For a destination row ip' and class q with proton jumps k (source rows
// ip_k, labels A_k, phases) and the neutron jumps of the conjugate class
// grouped by 32-column source tile t:
//   dV^q[A_k, B] += phase_k sum_t sum_so x[ip_k, 32t + so] G_t[so, B],
//   G_t[so, B] = phase_l g[ip', dst_l] for the neutron jump l with source
//   column 32t + so and label B (at most one: the source and the label fix
//   the destination), 0 otherwise.
// A wave scatters G_t for its tiles into its LDS tile -- the layout of the
// forward kernel's R tile, so the gather codes address it unchanged; padding
// codes are skipped -- contracts it with the x rows on the matrix cores
// (M = proton jumps, N = labels B, K = source columns), then clears the
// entries it wrote. Each wave adds its sums to dV_pn with float64 atomics.
constexpr int kVjpThreads = 64 * kPnWaves;

// The loads of one tile (its x operands and the first kPnRounds rounds of
// gather codes), issued a tile ahead of its use as in the forward kernel.
template <int KB>
struct VjpTile {
    double xa[KB][kPnTile / 4];
    uint32_t cr[kPnRounds];
    int e0, e1;
};

// Tile j of the wave (t = wid + W*j); past the last tile it is marked empty.
template <int KB>
__device__ __forceinline__ void vjp_fetch(VjpTile<KB> &b, int j, int wid, int ntiles, const int32_t *__restrict__ pnp,
                                          const unsigned *voff, __amdgpu_buffer_rsrc_t xr,
                                          __amdgpu_buffer_rsrc_t cres, int lane) {
    const int t = wid + kPnWaves * j;
    const int tc = min(t, ntiles - 1);
    b.e0 = pnp[tc];
    b.e1 = t < ntiles ? pnp[tc + 1] : b.e0;
    const unsigned toff = (unsigned)(kPnTile * tc) * 8u;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int ks = 0; ks < kPnTile / 4; ++ks) b.xa[kb][ks] = buffer_load<double>(xr, voff[kb] + toff + 32u * ks, 0);
#pragma unroll
    for (int i = 0; i < kPnRounds; ++i) b.cr[i] = buffer_load_u32(cres, (unsigned)(b.e0 + lane + 64 * i) * 4u);
}

// Scatter G_t (value) or clear it (value == false) for the tile's codes;
// rounds past the prefetched ones are loaded here.
__device__ __forceinline__ void vjp_scatter(const uint32_t (&cr)[kPnRounds], int e0, int ne, bool value,
                                            __amdgpu_buffer_rsrc_t cres, uint32_t null_code,
                                            const double *__restrict__ gl, double *__restrict__ Gt, int lane) {
    constexpr uint32_t kElem = (1u << kPnRBits) - 1u, kDst = (1u << kPnDstBits) - 1u;
    auto one = [&](uint32_t c) {
        if (c == null_code) return;
        Gt[c & kElem] = value ? signed_by(gl[(c >> kPnRBits) & kDst], c) : 0.0;
    };
#pragma unroll
    for (int i = 0; i < kPnRounds; ++i)
        if (64 * i < ne) one(cr[i]);
    for (int i = 64 * kPnRounds; i < ne; i += 64) one(buffer_load_u32(cres, (unsigned)(e0 + i + lane) * 4u));
}

template <int KB, int NBT>
__device__ __forceinline__ void vjp_work(const VjpTile<KB> &b, doublex4 (&acc)[KB][NBT], __amdgpu_buffer_rsrc_t cres,
                                         uint32_t null_code, const double *__restrict__ gl, double *__restrict__ Gt,
                                         int lane) {
    if (b.e0 == b.e1) return;   // uniform: no neutron jump leaves this tile
    const int ne = b.e1 - b.e0;
    vjp_scatter(b.cr, b.e0, ne, true, cres, null_code, gl, Gt, lane);
    // a wave's LDS operations complete in issue order: the reads below see
    // the scatter above, and the clearing below follows the reads
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int ks = 0; ks < kPnTile / 4; ++ks) {
        const double *Gr = Gt + (4 * ks + (lane >> 4)) * kPnRStride + (lane & 15);
#pragma unroll
        for (int bt = 0; bt < NBT; ++bt) {
            const double v = Gr[16 * bt];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) acc[kb][bt] = Mma<double>::mma(b.xa[kb][ks], v, acc[kb][bt]);
        }
    }
    __builtin_amdgcn_wave_barrier();
    vjp_scatter(b.cr, b.e0, ne, false, cres, null_code, gl, Gt, lane);
    __builtin_amdgcn_wave_barrier();
}

template <int KB, int NBT>
__device__ __forceinline__ void vjp_pn_class(const DevHam &P, const DevTiled &TT, int a0, int kp, int nB, int q,
                                             int qn, const int32_t *__restrict__ pnp, int ntiles,
                                             __amdgpu_buffer_rsrc_t xr, __amdgpu_buffer_rsrc_t cres,
                                             const double *__restrict__ gl, double *__restrict__ Gt, int wid,
                                             int lane, double *d_v_pn) {
    if (wid >= ntiles) return;
    doublex4 acc[KB][NBT];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int bt = 0; bt < NBT; ++bt) acc[kb][bt] = Mma<double>::zero();
    // A operand: lane holds x[ip_k, column] for k = 16 kb + lane % 16 and the
    // column lane / 16 of each 4-column step; rows past kp read zero
    unsigned voff[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int k = 16 * kb + (lane & 15);
        voff[kb] = k < kp ? (unsigned)(TT.p_ob_base[a0 + k] + (lane >> 4)) * 8u : kOutOfRange;
    }
    const uint32_t null_code = TT.pn_null;
    VjpTile<KB> A, B;
    vjp_fetch<KB>(A, 0, wid, ntiles, pnp, voff, xr, cres, lane);
    for (int j = 0;; j += 2) {
        vjp_fetch<KB>(B, j + 1, wid, ntiles, pnp, voff, xr, cres, lane);
        vjp_work<KB, NBT>(A, acc, cres, null_code, gl, Gt, lane);
        if (wid + kPnWaves * (j + 1) >= ntiles) break;
        vjp_fetch<KB>(A, j + 2, wid, ntiles, pnp, voff, xr, cres, lane);
        vjp_work<KB, NBT>(B, acc, cres, null_code, gl, Gt, lane);
        if (wid + kPnWaves * (j + 2) >= ntiles) break;
    }
    const int ns = P.ns;
    const int64_t ns2 = (int64_t)ns * ns;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int bt = 0; bt < NBT; ++bt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 16 * kb + Mma<double>::row(lane, r), Bl = 16 * bt + (lane & 15);
                if (k >= kp || Bl >= nB) continue;
                const int ck = P.p.ob_code[a0 + k];
                const double v = (ck & 1) ? -acc[kb][bt][r] : acc[kb][bt][r];
                if (v == 0.0) continue;
                const int la = P.cls_ops[P.cls_off[q] + (ck >> 1)];
                const int lb = P.cls_ops[P.cls_off[qn] + Bl];
                const int a = la / ns, c = la % ns, b = lb / ns, d = lb % ns;
                atomicAdd(&d_v_pn[((int64_t)a * ns + b) * ns2 + (int64_t)c * ns + d], v);
            }
}

template <int KB>
__device__ __forceinline__ void vjp_pn_nbt(int nbt, const DevHam &P, const DevTiled &TT, int a0, int kp, int nB,
                                           int q, int qn, const int32_t *pnp, int ntiles, __amdgpu_buffer_rsrc_t xr,
                                           __amdgpu_buffer_rsrc_t cres, const double *gl, double *Gt, int wid,
                                           int lane, double *d_v_pn) {
    switch (nbt) {
        case 1: vjp_pn_class<KB, 1>(P, TT, a0, kp, nB, q, qn, pnp, ntiles, xr, cres, gl, Gt, wid, lane, d_v_pn); break;
        case 2: vjp_pn_class<KB, 2>(P, TT, a0, kp, nB, q, qn, pnp, ntiles, xr, cres, gl, Gt, wid, lane, d_v_pn); break;
        case 3: vjp_pn_class<KB, 3>(P, TT, a0, kp, nB, q, qn, pnp, ntiles, xr, cres, gl, Gt, wid, lane, d_v_pn); break;
        default: vjp_pn_class<KB, 4>(P, TT, a0, kp, nB, q, qn, pnp, ntiles, xr, cres, gl, Gt, wid, lane, d_v_pn); break;
    }
}

// One workgroup per destination proton row: the row of g is staged in LDS
// once, then every operator class with proton jumps into the row.
__global__ __launch_bounds__(kVjpThreads) void k_vjp_pn_mfma(DevHam P, DevTiled TT, const double *__restrict__ x,
                                                             const double *__restrict__ g, double *d_v_pn) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int gstride = (TT.max_nn + 2) & ~1;                  // keeps the tiles 16-byte aligned
    double *gl = reinterpret_cast<double *>(smem_raw);          // [max_nn] row of g
    double *Gall = gl + gstride;                                // [waves][kPnTile * kPnRStride]
    const int ip = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s = P.p_sector[ip];
    const int nn = P.sec_nn[s];
    const int64_t base = P.p_pstart[ip];
    for (int c = tid; c < nn; c += kVjpThreads) gl[c] = g[base + c];
    for (int i = tid; i < kPnWaves * kPnTile * kPnRStride; i += kVjpThreads) Gall[i] = 0.0;
    __syncthreads();
    double *Gt = Gall + wid * kPnTile * kPnRStride;
    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc((void *)x, (short)0, (int)(P.dim * (int64_t)sizeof(double)), kBufFlags);
    const __amdgpu_buffer_rsrc_t cres =
        __builtin_amdgcn_make_buffer_rsrc((void *)TT.pn_code, (short)0, (int)(TT.n_pn_code * 4), kBufFlags);
    const int nq = P.nq, ntl = TT.n_t16;
    for (int q = 0; q < nq; ++q) {
        const int a0 = P.p.ob_ptr[(int64_t)ip * nq + q], a1 = P.p.ob_ptr[(int64_t)ip * nq + q + 1];
        if (a0 == a1) continue;   // uniform across the workgroup
        const int qn = P.conjq[q];
        const int nB = P.vq_nb[q];
        const int nns = P.sec_nn[P.p_sector[P.p.ob_src[a0]]];
        const int ntiles = (nns + kPnTile - 1) / kPnTile;
        const int32_t *pnp = TT.pn_ptr + ((int64_t)s * nq + qn) * ntl;
        const int kp = a1 - a0, nbt = (nB + 15) >> 4;
        if (kp > 16)
            vjp_pn_nbt<2>(nbt, P, TT, a0, kp, nB, q, qn, pnp, ntiles, xr, cres, gl, Gt, wid, lane, d_v_pn);
        else
            vjp_pn_nbt<1>(nbt, P, TT, a0, kp, nB, q, qn, pnp, ntiles, xr, cres, gl, Gt, wid, lane, d_v_pn);
    }
}

// One-body transition densities (Ch. 5, "One-body density matrices", before J
// coupling): rho[a*ns + c] = <g| c+_a c_c |x>. Between vectors of one basis
// only the operator class with no change of m and parity (q0) contributes,
// so source and destination SDs share a basis sector: proton densities are
// row dots g[row ip'] . x[row ip] per jump, neutron densities column dots.
__global__ __launch_bounds__(kT) void k_obd_proton(DevHam P, int q0, const double *__restrict__ x,
                                                   const double *__restrict__ g, double *rho) {
    __shared__ double lds[kT / 64];
    const int ip = blockIdx.x;
    const int nq = P.nq;
    const int a0 = P.p.ob_ptr[(int64_t)ip * nq + q0], a1 = P.p.ob_ptr[(int64_t)ip * nq + q0 + 1];
    if (a0 == a1) return;
    const int nn = P.sec_nn[P.p_sector[ip]];
    const int64_t base = P.p_pstart[ip];
    const int32_t *ops = P.cls_ops + P.cls_off[q0];
    for (int k = a0; k < a1; ++k) {
        const int64_t sb = P.p_pstart[P.p.ob_src[k]];
        double a = 0.0;
        for (int c = threadIdx.x; c < nn; c += kT) a += g[base + c] * x[sb + c];
        const double dot = block_sum_all(a, lds);
        if (threadIdx.x == 0) {
            const int code = P.p.ob_code[k];
            atomicAdd(&rho[ops[code >> 1]], (code & 1) ? -dot : dot);
        }
    }
}

// Neutron side: thread = destination neutron SD jn' (a column of its basis
// sector), block row = a chunk of kObdRows proton rows. Each thread keeps one
// float64 accumulator per jump into its column (kObdJumps at a time) and
// walks the rows: g[r, col] is read coalesced across the threads, the x
// values it pairs with lie in the same row.
constexpr int kObdRows = 64;
constexpr int kObdJumps = 16;

__global__ __launch_bounds__(kT) void k_obd_neutron(DevHam P, int q0, const double *__restrict__ x,
                                                    const double *__restrict__ g, double *rho) {
    const int jn = blockIdx.x * kT + threadIdx.x;
    if (jn >= P.n.n_sd) return;
    const int s = P.n_bsector[jn];
    if (s < 0) return;
    const int np = P.sec_np[s], nn = P.sec_nn[s];
    const int r0 = blockIdx.y * kObdRows, r1 = min(np, r0 + kObdRows);
    if (r0 >= r1) return;
    const int nq = P.nq;
    const int a0 = P.n.ob_ptr[(int64_t)jn * nq + q0], a1 = P.n.ob_ptr[(int64_t)jn * nq + q0 + 1];
    const int64_t off = P.sec_off[s];
    const int cd = P.n_local[jn];
    const int32_t *ops = P.cls_ops + P.cls_off[q0];
    for (int k0 = a0; k0 < a1; k0 += kObdJumps) {
        const int kc = min(kObdJumps, a1 - k0);
        int cs[kObdJumps];
        double acc[kObdJumps];
#pragma unroll
        for (int k = 0; k < kObdJumps; ++k) {
            cs[k] = k < kc ? P.n_local[P.n.ob_src[k0 + k]] : cd;
            acc[k] = 0.0;
        }
        for (int r = r0; r < r1; ++r) {
            const int64_t row = off + (int64_t)r * nn;
            const double gv = g[row + cd];
#pragma unroll
            for (int k = 0; k < kObdJumps; ++k) acc[k] += gv * x[row + cs[k]];
        }
        for (int k = 0; k < kc; ++k) {
            const int code = P.n.ob_code[k0 + k];
            atomicAdd(&rho[ops[code >> 1]], (code & 1) ? -acc[k] : acc[k]);
        }
    }
}

}  // namespace

void launch_one_body_density(const DevHam &d, const std::vector<int32_t> &h_sec_np, int q0, const double *g,
                             const double *x, double *rho_p, double *rho_n, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int n2 = d.ns * d.ns;
    if (rho_p) {
        hipLaunchKernelGGL(k_zero, dim3((n2 + kT - 1) / kT), dim3(kT), 0, st, rho_p, n2);
        hipLaunchKernelGGL(k_obd_proton, dim3(d.p.n_sd), dim3(kT), 0, st, d, q0, x, g, rho_p);
    }
    if (rho_n) {
        hipLaunchKernelGGL(k_zero, dim3((n2 + kT - 1) / kT), dim3(kT), 0, st, rho_n, n2);
        int max_np = 1;
        for (int v : h_sec_np) max_np = std::max(max_np, v);
        const dim3 grid((d.n.n_sd + kT - 1) / kT, (max_np + kObdRows - 1) / kObdRows);
        hipLaunchKernelGGL(k_obd_neutron, grid, dim3(kT), 0, st, d, q0, x, g, rho_n);
    }
    hip_check(hipGetLastError(), "one-body density launch");
}

// Column-sum scratch of fotci_apply_H_vjp_static: one array per GPU (each
// device holds its own copy of a __device__ variable), shared by every call on
// that GPU and kept until the process ends. In host code `scratch` names a
// host-side stand-in; its device address comes from hipGetSymbolAddress, once
// per device, and only that address is handed to kernels.
static __device__ __align__(256) double scratch[kStaticNcolMax];

double *static_ncol_scratch() {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    int dev = -1;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) fail(FOTCI_EINVAL, "device ordinal out of range for the static scratch");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        ptr[dev] = (double *)p;
    }
    return ptr[dev];
}

void launch_vjp(const DevHam &d, const fotci_ham *h, const double *x, const double *g, double *dx, double *d_spe_p,
                double *d_spe_n, double *d_v_pp, double *d_v_nn, double *d_v_pn, void *stream, double *ncol) {
    hipStream_t st = (hipStream_t)stream;
    if (dx) launch_apply(h, FOTCI_MODE_F64, g, dx, stream);
    const DevTiled &tt = h->dev_tiled;
    // off-diagonal pp / nn densities as sampled products when the tiled tables exist
    auto sddmm_tiles = [&](bool neut) {
        int64_t tiles = 0;
        for (size_t si = 0; si < h->tc.sec_nn.size(); ++si) {
            const int64_t mb = ((neut ? h->tc.sec_nn[si] : h->tc.sec_np[si]) + kSd - 1) / kSd;
            tiles += mb * mb;
        }
        return tiles;
    };
    const bool sd_p = d_v_pp && tt.ok, sd_n = d_v_nn && tt.ok;
    double *dcol = nullptr;
    const bool need_n = d_spe_n || d_v_nn;
    if (need_n) {
        // column sums of g o x per neutron SD: in the Hamiltonian's workspace,
        // or in the caller-chosen buffer (the static scratch)
        dcol = ncol ? ncol : d.scratch_ncol;
        hipLaunchKernelGGL(k_zero, dim3((d.n.n_sd + kT - 1) / kT), dim3(kT), 0, st, dcol, d.n.n_sd);
    }
    if (d_spe_p || d_v_pp || need_n)
        hipLaunchKernelGGL(k_vjp_proton, dim3(d.p.n_sd), dim3(kT), 0, st, d, x, g, d_spe_p, d_v_pp, dcol,
                           sd_p ? 0 : 1);
    if (need_n) hipLaunchKernelGGL(k_vjp_neutron, dim3(d.n.n_sd), dim3(kT), 0, st, d, x, g, (const double *)dcol,
                                   d_spe_n, d_v_nn, sd_n ? 0 : 1);
    if (sd_p) {
        const int64_t tiles = sddmm_tiles(false);
        if (tiles > 0) hipLaunchKernelGGL(k_vjp_sddmm<false>, dim3((unsigned)tiles), dim3(64), 0, st, d, tt, x, g, d_v_pp);
    }
    if (sd_n) {
        const int64_t tiles = sddmm_tiles(true);
        if (tiles > 0) hipLaunchKernelGGL(k_vjp_sddmm<true>, dim3((unsigned)tiles), dim3(64), 0, st, d, tt, x, g, d_v_nn);
    }
    if (d_v_pn) {
        const DevTiled &t = tt;
        const size_t lds = ((size_t)((t.max_nn + 2) & ~1) + (size_t)kPnWaves * kPnTile * kPnRStride) * sizeof(double);
        if (t.ok && lds <= 65536) {
            hipLaunchKernelGGL(k_vjp_pn_mfma, dim3(d.p.n_sd), dim3(kVjpThreads), lds, st, d, t, x, g, d_v_pn);
        } else {
            for (int q = 0; q < d.nq; ++q)
                if ((int64_t)h->j->cls.ops[q].size() * h->vq_nb[q] > kMaxBins)
                    fail(FOTCI_EINVAL, "pn operator class too large for the adjoint kernel");
            hipLaunchKernelGGL(k_vjp_pn, dim3(d.p.n_sd * d.nq), dim3(kT), 0, st, d, x, g, d_v_pn);
        }
    }
    hip_check(hipGetLastError(), "vjp launch");
}

}  // namespace fotci
