// Tiled apply_H for gfx950: three kernels, each reading x through LDS.
//
// A sector block of x is the dense matrix X_s (np_s x nn_s, neutron index
// contiguous), and (Ch. 2, "Representation of the Hamiltonian")
//   Y_s = (d_p + d_n) o X_s + X_s H_nn^{s T} + H_pp^s X_s
//       + sum_{A,B} V_AB P_A X_{s-Delta} N_B^T .
//
// k_nn_diag  one workgroup per tile of 8 proton rows of a sector: the rows
//            are staged in LDS (interleaved so a column's rows are adjacent)
//            and every output column walks its neutron entries once for all
//            rows of the tile (ELL layout: coalesced across columns).
//            Writes y.
// k_pp       one workgroup per tile of 8 neutron columns of a sector: the
//            whole column slab of X_s is staged in LDS and every output row
//            walks its proton entries (ELL across rows). Adds to y.
// k_pn       one workgroup per destination proton row ip' and every operator
//            class q (Jz change Delta of the proton one-body operator; the
//            neutron one is opposite):
//              R[B, jn] = sum_k (phase_k V^q[A_k, B]) x[ip_k, jn]
//            over the K_p proton one-body jumps (ip_k -> ip', label A_k) is a
//            dense contraction on the matrix cores (M = neutron labels B, N =
//            source neutron columns jn, K = proton jumps); each wave takes
//            32-column source tiles, keeps its R tile in LDS, and the neutron
//            one-body jumps whose source lies in the tile (pre-grouped by
//            tile, read coalesced) add phase_l R[B_l, jn_l] into the
//            workgroup's output row held in LDS. Within a tile every
//            destination column belongs to one lane, which sums its entries
//            in a register and adds them to the row with one LDS atomic.
//            This is the proton-first grouping of sum_{A,B} V_AB P_A X N_B^T:
//            the contraction over B is dense, so the matrix cores execute
//            about 6.5 times the useful multiply-adds of the pn part. Adds to
//            y. With a vector stride NB the same kernel serves the pn part of
//            the block apply, one vector per workgroup. Float64.
// k_pn2      the float32 pn kernel: as k_pn, but the two waves of a
//            workgroup work through pairs of source tiles in step, each
//            owning the destination columns of one parity, and update the row
//            with plain LDS reads and writes; six workgroups fit a CU.
#include <hip/hip_runtime.h>

#include "tiled_common.h"

namespace fotci {

namespace {

__global__ __launch_bounds__(kT) void k_ell_values(const int32_t *__restrict__ src, const int32_t *__restrict__ ent,
                                                   const double *__restrict__ off, EllE64 *__restrict__ e64,
                                                   EllE32 *__restrict__ e32, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const int e = ent[i];
    const double v = e >= 0 ? off[e] : 0.0;
    const uint64_t bits = __double_as_longlong(v);
    e64[i] = EllE64{src[i], (uint32_t)bits, (uint32_t)(bits >> 32)};
    e32[i] = EllE32{src[i], (float)v};
}

// ------------------------------------------------------------ diagonal + nn
// RT rows are staged per pass (RT * max_nn * sizeof(T) <= kLdsTile).
template <typename T, int RT>
__global__ __launch_bounds__(kTS) void k_nn_diag(DevHam P, DevTiled TT, const T *__restrict__ x, T *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *Xl = reinterpret_cast<T *>(smem_raw);   // Xl[c * RT + r]
    const int tid = threadIdx.x;
    const int s = TT.rt_sec[blockIdx.x], r0t = TT.rt_r0[blockIdx.x];
    const int np = P.sec_np[s], nn = P.sec_nn[s], nf = P.sec_nfirst[s], pf = P.sec_pfirst[s];
    const int64_t off = P.sec_off[s];
    const int E = TT.nn_ell_E[s];
    const int64_t eb = TT.nn_ell_base[s];
    const auto *ev = TabT<T>::nn_ell(TT);
    const T *dpa = TabT<T>::diag(P.p);
    const T *dn = TabT<T>::diag(P.n);
    const int rend = min(r0t + kTile, np);
    for (int r0 = r0t; r0 < rend; r0 += RT) {
        const int nr = min(RT, rend - r0);
        const T *xs = x + off + (int64_t)r0 * nn;
        __syncthreads();
#pragma unroll 4
        for (int idx = tid; idx < RT * nn; idx += kTS) {
            const int r = idx / nn, c = idx - r * nn;
            // rows past the tile's end load row nr-1 and store zero: no branch around the load
            const T v = xs[(int64_t)min(r, nr - 1) * nn + c];
            Xl[c * RT + (r ^ slab_swz<T, RT>(c))] = r < nr ? v : T(0);
        }
        T dp[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) dp[r] = r < nr ? dpa[pf + r0 + r] : T(0);
        __syncthreads();
        for (int c = tid; c < nn; c += kTS) {
            T acc[RT];
            const T dnc = dn[nf + c];
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = (dp[r] + dnc) * Xl[c * RT + (r ^ slab_swz<T, RT>(c))];
#pragma unroll 8
            for (int e = 0; e < E; ++e) {
                const auto ent = ell_load(ev, eb + (int64_t)e * nn + c);
                const int src = ent.src;
                const T v = ent.v;
                const T *xr = Xl + src * RT;
                const int sw = slab_swz<T, RT>(src);
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r] += v * xr[r ^ sw];
            }
#pragma unroll
            for (int r = 0; r < RT; ++r)
                if (r < nr) y[off + (int64_t)(r0 + r) * nn + c] = acc[r];
        }
    }
}

// ---------------------------------------------------------------------- pp
// CT columns are staged per pass (max_np * CT * sizeof(T) <= kLdsTile).
// STAGED (float32, np <= kPpRows * kTS): each thread keeps the sums of its rows
// in registers, the slab is then overwritten with them, and y is updated in a
// second pass in which consecutive threads cover a row's CT columns (the
// row-per-thread update touches 64 rows per wave instruction: 0.347 against
// 0.268 ms at pf 5p5n). Float64 keeps the row-per-thread update (twice the
// registers per row; the staged form ran at 1.87 against 0.68 ms).
constexpr int kPpRows = 4;   // rows per thread of the staged pp update
template <typename T, int CT, bool STAGED>
__global__ __launch_bounds__(kTS) void k_pp(DevHam P, DevTiled TT, const T *__restrict__ x, T *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *Xl = reinterpret_cast<T *>(smem_raw);   // Xl[r * CT + c]
    const int tid = threadIdx.x;
    const int tile = pp_tile_of<kPpRunLines * pp_line_group<T, 1>()>(blockIdx.x);
    if (tile >= TT.n_ctiles) return;
    const int s = TT.ct_sec[tile], c0t = TT.ct_c0[tile];
    const int np = P.sec_np[s], nn = P.sec_nn[s];
    const int64_t off = P.sec_off[s];
    const int E = TT.pp_ell_E[s];
    if (E == 0) return;
    const int64_t eb = TT.pp_ell_base[s];
    const auto *ev = TabT<T>::pp_ell(TT);
    const int cend = min(c0t + kTile, nn);
    // one row's ELL walk into acc
    auto walk = [&](int r, T (&acc)[CT]) {
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] = 0;
#pragma unroll 8
        for (int e = 0; e < E; ++e) {
            const auto ent = ell_load(ev, eb + (int64_t)e * np + r);
            const int src = ent.src;
            const T v = ent.v;
            const T *xr = Xl + src * CT;
            const int sw = slab_swz<T, CT>(src);
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[c] += v * xr[c ^ sw];
        }
    };
    for (int c0 = c0t; c0 < cend; c0 += CT) {
        const int nc = min(CT, cend - c0);
        __syncthreads();
#pragma unroll 4
        for (int idx = tid; idx < np * CT; idx += kTS) {
            const int r = idx / CT, c = idx - r * CT;
            const T v = x[off + (int64_t)r * nn + c0 + min(c, nc - 1)];   // unconditional load
            Xl[r * CT + (c ^ slab_swz<T, CT>(r))] = c < nc ? v : T(0);
        }
        __syncthreads();
        if constexpr (STAGED) {
            T acc[kPpRows][CT];
#pragma unroll
            for (int i = 0; i < kPpRows; ++i)
                if (tid + i * kTS < np) walk(tid + i * kTS, acc[i]);
            __syncthreads();   // every read of the slab is done
#pragma unroll
            for (int i = 0; i < kPpRows; ++i) {
                const int r = tid + i * kTS;
                if (r < np)
#pragma unroll
                    for (int c = 0; c < CT; ++c) Xl[r * CT + c] = acc[i][c];
            }
            __syncthreads();
            for (int idx = tid; idx < np * CT; idx += kTS) {
                const int r = idx / CT, c = idx - r * CT;
                if (c < nc) y[off + (int64_t)r * nn + c0 + c] += Xl[idx];
            }
        } else {
            for (int r = tid; r < np; r += kTS) {
                T acc[CT];
                walk(r, acc);
                T *yr = y + off + (int64_t)r * nn + c0;
#pragma unroll
                for (int c = 0; c < CT; ++c)
                    if (c < nc) yr[c] += acc[c];
            }
        }
    }
}

// ---------------------------------------------------------------------- pn
// Waves work independently on kPnTile-column source tiles: each contracts its
// tile on the matrix cores (16 columns per instruction) into a wave-private
// R in LDS and gathers the neutron jumps whose source lies in the tile into
// its output row. x is read with buffer loads: each lane's offset is fixed
// for the whole class and the tile's column offset is added to it; padding
// lanes point past the end of x and read zero.

// The loads of one source tile: KST x values per lane for each 16-column
// block and the first kPnRounds rounds of gather codes. Their number is fixed
// and no lane skips them (buffer loads past a range return 0), so the compiler can count them and let the
// next tile's loads stay in flight while the current tile is worked on.
template <typename T, int KST>
struct PnTile {
    T xv[kPnHalves][KST];
    uint32_t cr[kPnRounds];
    int e0, e1;
};

// Tile j of the wave (t = wid + W*j); past the last tile it reloads that tile
// and is marked empty.
template <typename T, int KST, int NB>
__device__ __forceinline__ void pn_fetch(PnTile<T, KST> &b, int j, int wid, int ntiles, PnBounds &pb,
                                         const unsigned *voff, unsigned goff, __amdgpu_buffer_rsrc_t xr,
                                         const int32_t *__restrict__ pnp, __amdgpu_buffer_rsrc_t cres, int lane) {
    if (j > 0 && (j & 63) == 0) pn_bounds(pb, j, wid, ntiles, pnp, lane);   // uniform, every 64 tiles
    const int tt = wid + kPnWaves * j;
    const int tc = min(tt, ntiles - 1);
    b.e0 = __builtin_amdgcn_readlane(pb.b0, j & 63);
    b.e1 = tt < ntiles ? __builtin_amdgcn_readlane(pb.b1, j & 63) : b.e0;
    // the whole offset goes into the range-checked vector offset, so the
    // ragged last tile of the last row reads zero past the end of x
    const unsigned toff = (unsigned)(kPnTile * tc) * (unsigned)(NB * sizeof(T)) + goff;
#pragma unroll
    for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
        for (int ks = 0; ks < KST; ++ks)
            b.xv[h][ks] = buffer_load<T>(xr, voff[ks] + toff + (unsigned)(16 * h * NB * sizeof(T)), 0);
#pragma unroll
    for (int i = 0; i < kPnRounds; ++i) b.cr[i] = buffer_load_u32(cres, (unsigned)(b.e0 + lane + 64 * i) * 4u);
}

// Contraction and gather of one fetched tile; cv holds the class's C operand.
// yl is the workgroup's shared output row, updated with one LDS atomic per
// chunk.
template <typename T, int NBT, int KST>
__device__ __forceinline__ void pn_work(const PnTile<T, KST> &b, const T (&cv)[NBT][KST],
                                        __amdgpu_buffer_rsrc_t cres, int lane, T *__restrict__ R,
                                        T *__restrict__ yl) {
    typedef typename Mma<T>::acc_t acc_t;
    if (b.e0 == b.e1) return;   // uniform: no neutron jump leaves this tile
    acc_t acc[kPnHalves][NBT];
#pragma unroll
    for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
        for (int bt = 0; bt < NBT; ++bt) acc[h][bt] = Mma<T>::zero();
#pragma unroll
    for (int ks = 0; ks < KST; ++ks)
#pragma unroll
        for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
            for (int bt = 0; bt < NBT; ++bt) acc[h][bt] = Mma<T>::mma(cv[bt][ks], b.xv[h][ks], acc[h][bt]);
#pragma unroll
    for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
        for (int bt = 0; bt < NBT; ++bt) Lds<T>::store(R, lane, h, bt, acc[h][bt]);
    // a wave's LDS operations complete in issue order: the gather below
    // sees the stores above without a workgroup barrier
    __builtin_amdgcn_wave_barrier();
    // The list of a tile is a whole number of 64-entry rounds, so rounds are
    // skipped per wave, not per lane.
    const int ne = b.e1 - b.e0;
    // shared row: the lane sums its chunk in a register and adds it with
    // one LDS atomic at the chunk's flagged last entry
    constexpr uint32_t kElem = (1u << kPnRBits) - 1u, kDst = (1u << kPnDstBits) - 1u;
    T run = 0;
#pragma unroll
    for (int i = 0; i < kPnRounds; ++i)
        if (64 * i < ne) {
            const uint32_t c = b.cr[i];
            run += signed_by(R[c & kElem], c);
            if (c & kPnFlush) {
                atomicAdd(&yl[(c >> kPnRBits) & kDst], run);
                run = 0;
            }
        }
    for (int i = 64 * kPnRounds; i < ne; i += 64) {
        const uint32_t c = buffer_load_u32(cres, (unsigned)(b.e0 + i + lane) * 4u);
        run += signed_by(R[c & kElem], c);
        if (c & kPnFlush) {
            atomicAdd(&yl[(c >> kPnRBits) & kDst], run);
            run = 0;
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// One wave's tiles of one class, specialised on the number of 16-row tiles
// of neutron labels (NBT) and of 4-jump k-steps (KST) so the inner loop has
// no runtime guards around the matrix-core instructions. Two register sets
// alternate: the loads of the wave's next tile are issued before the current
// tile's contraction and gather.
// The class's operands are read by each lane from the (cache-resident)
// tables: lane (col_l, kq) holds C[B = 16 bt + col_l][k = 4 ks + kq] =
// phase_k V^q[A_k, B] for the matrix cores and the byte offset of its x
// element in source row k; no workgroup barrier separates the classes.
template <typename T, int NBT, int KST, int NB>
__device__ __forceinline__ void pn_tiles(const PnClass &pc, const T *__restrict__ V, unsigned goff,
                                         __amdgpu_buffer_rsrc_t xr,
                                         const int32_t *__restrict__ pnp, __amdgpu_buffer_rsrc_t cres, int ntiles,
                                         int wid, int lane, T *__restrict__ R, T *__restrict__ yl) {
    if (wid >= ntiles) return;
    unsigned voff[KST];
    T cv[NBT][KST];   // the class's C operand stays in registers for all tiles
    pn_operand<T, NBT, KST, NB>(pc, V, cv, voff, lane);
    PnBounds pb;
    pn_bounds(pb, 0, wid, ntiles, pnp, lane);
    constexpr int W = kPnWaves;
    if constexpr (sizeof(T) == 4) {
        // three register sets in rotation: tiles j+1 and j+2 are in flight while tile j is worked on
        PnTile<T, KST> A, B, C;
        pn_fetch<T, KST, NB>(A, 0, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
        pn_fetch<T, KST, NB>(B, 1, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
        for (int j = 0;; j += 3) {
            pn_fetch<T, KST, NB>(C, j + 2, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
            pn_work<T, NBT, KST>(A, cv, cres, lane, R, yl);
            if (wid + W * (j + 1) >= ntiles) break;
            pn_fetch<T, KST, NB>(A, j + 3, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
            pn_work<T, NBT, KST>(B, cv, cres, lane, R, yl);
            if (wid + W * (j + 2) >= ntiles) break;
            pn_fetch<T, KST, NB>(B, j + 4, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
            pn_work<T, NBT, KST>(C, cv, cres, lane, R, yl);
            if (wid + W * (j + 3) >= ntiles) break;
        }
    } else {
        // double: two register sets (the operands are twice as wide)
        PnTile<T, KST> A, B;
        pn_fetch<T, KST, NB>(A, 0, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
        for (int j = 0;; j += 2) {
            pn_fetch<T, KST, NB>(B, j + 1, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
            pn_work<T, NBT, KST>(A, cv, cres, lane, R, yl);
            if (wid + W * (j + 1) >= ntiles) break;
            pn_fetch<T, KST, NB>(A, j + 2, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
            pn_work<T, NBT, KST>(B, cv, cres, lane, R, yl);
            if (wid + W * (j + 2) >= ntiles) break;
        }
    }
}

template <typename T, int NBT, int NB>
__device__ __forceinline__ void pn_tiles_k(int ksteps, const PnClass &pc, const T *V, unsigned goff,
                                           __amdgpu_buffer_rsrc_t xr,
                                           const int32_t *pnp, __amdgpu_buffer_rsrc_t pnc, int ntiles, int wid,
                                           int lane, T *R, T *yl) {
    switch (ksteps) {
        case 1: pn_tiles<T, NBT, 1, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl); break;
        case 2: pn_tiles<T, NBT, 2, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl); break;
        case 3: pn_tiles<T, NBT, 3, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl); break;
        case 4: pn_tiles<T, NBT, 4, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl); break;
        case 5: pn_tiles<T, NBT, 5, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl); break;
        case 6: pn_tiles<T, NBT, 6, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl); break;
        case 7: pn_tiles<T, NBT, 7, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl); break;
        default: pn_tiles<T, NBT, 8, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl); break;
    }
}

// The waves of a workgroup accumulate into one shared output row (max_nn + 1
// in dynamic LDS) with LDS atomics. NB: x and y hold a block of NB vectors stored row-wise
// (element i of vector v at i * NB + v) and a workgroup handles one vector
// g0 of one destination row; NB == 1 is the one-vector apply. For NB > 1 the
// grid is 1-D and the NB workgroups of a row are consecutive slots of one XCD
// (workgroups are dealt to the 8 XCDs in turn), so the strided loads of the
// block's vectors share that XCD's L2.
template <typename T, int NB>
__global__ __launch_bounds__(kPnThreads) void k_pn(DevHam P, DevTiled TT, const T *__restrict__ x,
                                                   T *__restrict__ y) {
    __shared__ __align__(16) T Rw[kPnWaves][kPnTile * kPnRStride];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *yl = reinterpret_cast<T *>(smem_raw);   // output row [max_nn + 1]

    int slot = blockIdx.x, g0 = 0;
    if constexpr (NB > 1) {
        const int xcd = blockIdx.x & 7, s8 = blockIdx.x >> 3;
        slot = (s8 / NB) * 8 + xcd;
        g0 = s8 % NB;
        if (slot >= P.p.n_sd) return;   // uniform: the grid is padded to a multiple of 8 rows
    }
    const int ip = TT.order[slot];
    const unsigned goff = (unsigned)g0 * (unsigned)sizeof(T);
    const int tid = threadIdx.x;
    // the wave index is uniform across the wave: keep it (and the tile loop) scalar
    const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s = P.p_sector[ip];
    const int nn = P.sec_nn[s];
    const int64_t base = P.p_pstart[ip];
    const int nq = P.nq;
    const int ntl = TT.n_t16;
    const T *vq = TabT<T>::vq(P);
    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc((void *)x, (short)0, (int)(P.dim * (int64_t)(NB * sizeof(T))), kBufFlags);
    const __amdgpu_buffer_rsrc_t cres =
        __builtin_amdgcn_make_buffer_rsrc((void *)TT.pn_code, (short)0, (int)(TT.n_pn_code * 4), kBufFlags);
    T *R = Rw[wid];
    for (int c = tid; c < nn; c += kPnThreads) yl[c] = 0;
    __syncthreads();
    bool any = false;
    PnClass pc;
    pc.ob_code = P.p.ob_code;
    pc.ob_base = TT.p_ob_base;
    for (int q = 0; q < nq; ++q) {
        const int a0 = P.p.ob_ptr[(int64_t)ip * nq + q], a1 = P.p.ob_ptr[(int64_t)ip * nq + q + 1];
        if (a0 == a1) continue;   // uniform across the workgroup
        any = true;
        const int qn = P.conjq[q];
        const int nB = P.vq_nb[q];
        const int nbt = (nB + 15) >> 4;
        const T *V = vq + P.vq_off[q];
        const int nns = P.sec_nn[P.p_sector[P.p.ob_src[a0]]];
        const int64_t pslot = ((int64_t)s * nq + qn) * ntl;
        pc.a0 = a0;
        pc.nd = TT.pn_ndiag[(int64_t)ip * nq + q];
        pc.kp = a1 - a0 - (pc.nd > 1 ? pc.nd - 1 : 0);
        pc.nB = nB;
        const int ksteps = (pc.kp + 3) >> 2;
        const int ntiles = (nns + kPnTile - 1) / kPnTile;
        const int32_t *pnp = TT.pn_ptr + pslot;
        switch (nbt) {
            case 1: pn_tiles_k<T, 1, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, R, yl); break;
            case 2: pn_tiles_k<T, 2, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, R, yl); break;
            case 3: pn_tiles_k<T, 3, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, R, yl); break;
            default: pn_tiles_k<T, 4, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, R, yl); break;
        }
    }
    if (!any) return;
    __syncthreads();
    for (int c = tid; c < nn; c += kPnThreads) y[(base + c) * NB + g0] += yl[c];
}

// ------------------------------------------------------ pn, one shared row
// One vector. The two waves of a workgroup share one output row, wave
// w owning the destination columns of parity w. Source tiles go in pairs
// (steps): wave w contracts tile 2j + w into its R tile, the workgroup
// synchronises, each wave gathers the step's jumps into its own columns from
// both R tiles, and a second barrier keeps the R tiles until both gathers are
// done. One output row per workgroup instead of one per wave: six workgroups
// (12 waves) fit a CU's LDS instead of five.
static_assert(kPnWaves == 2, "the shared-row pn kernel splits the destination columns by parity");

struct Pn2Bounds {
    int e0, e1;   // this wave's list of the step; bit 31 of e0: the step has jumps (either list)
};

// bounds of steps j0 + lane (past the last step: empty)
__device__ __forceinline__ void pn2_bounds(Pn2Bounds &pb, int j0, int nsteps, const int32_t *__restrict__ pnp,
                                           int wid, int lane) {
    const int st = j0 + lane;
    const int sc = min(st, nsteps - 1);
    const int lo = pnp[2 * sc], mid = pnp[2 * sc + 1], hi = pnp[2 * sc + 2];
    const bool any = st < nsteps && lo != hi;
    pb.e0 = (wid == 0 ? lo : mid) | (any ? (int)0x80000000u : 0);
    pb.e1 = wid == 0 ? mid : hi;
}

template <typename T, int KST>
struct Pn2Tile {
    T xv[kPnHalves][KST];
    uint32_t cr[kPnRounds];
    int e0, e1;    // this wave's list
    bool any;      // the step has jumps (uniform across the workgroup)
    bool mine;     // this wave's tile exists
};

template <typename T, int KST, int NB>
__device__ __forceinline__ void pn2_fetch(Pn2Tile<T, KST> &b, int j, int wid, int ntiles, int nsteps, Pn2Bounds &pb,
                                          const unsigned *voff, unsigned goff, __amdgpu_buffer_rsrc_t xr,
                                          const int32_t *__restrict__ pnp, __amdgpu_buffer_rsrc_t cres, int lane) {
    if (j > 0 && (j & 63) == 0) pn2_bounds(pb, j, nsteps, pnp, wid, lane);   // uniform, every 64 steps
    const int e0 = __builtin_amdgcn_readlane(pb.e0, j & 63);
    b.any = e0 < 0;
    b.e0 = e0 & 0x7fffffff;
    b.e1 = __builtin_amdgcn_readlane(pb.e1, j & 63);
    const int tt = 2 * j + wid;
    b.mine = tt < ntiles;
    const int tc = min(tt, ntiles - 1);
    const unsigned toff = (unsigned)(kPnTile * tc) * (unsigned)(NB * sizeof(T)) + goff;
#pragma unroll
    for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
        for (int ks = 0; ks < KST; ++ks)
            b.xv[h][ks] = buffer_load<T>(xr, voff[ks] + toff + (unsigned)(16 * h * NB * sizeof(T)), 0);
#pragma unroll
    for (int i = 0; i < kPnRounds; ++i) b.cr[i] = buffer_load_u32(cres, (unsigned)(b.e0 + lane + 64 * i) * 4u);
}

template <typename T, int NBT, int KST>
__device__ __forceinline__ void pn2_work(const Pn2Tile<T, KST> &b, const T (&cv)[NBT][KST],
                                         __amdgpu_buffer_rsrc_t cres, uint32_t null_code, int own, int wid,
                                         int lane, T *__restrict__ Rw, T *__restrict__ yl) {
    typedef typename Mma<T>::acc_t acc_t;
    if (!b.any) return;   // uniform across the workgroup
    if (b.mine) {
        acc_t acc[kPnHalves][NBT];
#pragma unroll
        for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
            for (int bt = 0; bt < NBT; ++bt) acc[h][bt] = Mma<T>::zero();
#pragma unroll
        for (int ks = 0; ks < KST; ++ks)
#pragma unroll
            for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
                for (int bt = 0; bt < NBT; ++bt) acc[h][bt] = Mma<T>::mma(cv[bt][ks], b.xv[h][ks], acc[h][bt]);
        T *R = Rw + wid * (kPnTile * kPnRStride);
#pragma unroll
        for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
            for (int bt = 0; bt < NBT; ++bt) Lds<T>::store(R, lane, h, bt, acc[h][bt]);
    }
    __syncthreads();
    // the lane-owned chunk gather: a chunk of one destination's entries sits
    // in consecutive rounds of one lane, which sums it and updates the row at
    // the chunk's flagged last entry; two chunks of one destination never
    // flush in one pair of rounds, so both rounds' row reads go out before
    // either write, and a round without a flush reads and writes the lane's
    // own scratch word past the row. Both R tiles, this wave's columns.
    constexpr uint32_t kElem = (1u << kPn2RBits) - 1u, kDst = (1u << kPn2DstBits) - 1u;
    const int ne = b.e1 - b.e0;
    const uint32_t ow = (uint32_t)own;
    T run = 0;
#pragma unroll
    for (int i = 0; i < kPnRounds; i += 2) {
        if (64 * i < ne) {
            const uint32_t c0 = b.cr[i];
            const uint32_t c1 = 64 * (i + 1) < ne ? b.cr[i + 1] : null_code;
            const T v0 = signed_by(Rw[c0 & kElem], c0);
            const T v1 = signed_by(Rw[c1 & kElem], c1);
            const uint32_t a0 = (c0 & kPnFlush) ? (c0 >> kPn2RBits) & kDst : ow;
            const uint32_t a1 = (c1 & kPnFlush) ? (c1 >> kPn2RBits) & kDst : ow;
            const T s0 = run + v0;
            const T r1 = (c0 & kPnFlush) ? T(0) : s0;
            const T s1 = r1 + v1;
            run = (c1 & kPnFlush) ? T(0) : s1;
            const T y0 = yl[a0];
            const T y1 = yl[a1];
            yl[a0] = y0 + s0;
            yl[a1] = y1 + s1;
        }
    }
    for (int i = 64 * kPnRounds; i < ne; i += 64) {
        const uint32_t c = buffer_load_u32(cres, (unsigned)(b.e0 + i + lane) * 4u);
        run += signed_by(Rw[c & kElem], c);
        if (c & kPnFlush) {
            yl[(c >> kPn2RBits) & kDst] += run;
            run = 0;
        }
    }
    // the R tiles are overwritten by the next step's contraction
    __syncthreads();
}

template <typename T, int NBT, int KST, int NB>
__device__ __forceinline__ void pn2_tiles(const PnClass &pc, const T *__restrict__ V, unsigned goff,
                                          __amdgpu_buffer_rsrc_t xr,
                                          const int32_t *__restrict__ pnp, __amdgpu_buffer_rsrc_t cres, int ntiles,
                                          int wid, int lane, T *__restrict__ Rw, T *__restrict__ yl) {
    const int nsteps = (ntiles + 1) >> 1;
    unsigned voff[KST];
    T cv[NBT][KST];
    pn_operand<T, NBT, KST, NB>(pc, V, cv, voff, lane);
    const int own = pc.spare + 64 * wid + lane;
    Pn2Bounds pb;
    pn2_bounds(pb, 0, nsteps, pnp, wid, lane);
    // three register sets in rotation: tiles j + 1 and j + 2 are in flight
    // while tile j is worked on
    Pn2Tile<T, KST> A, B, C;
    pn2_fetch<T, KST, NB>(A, 0, wid, ntiles, nsteps, pb, voff, goff, xr, pnp, cres, lane);
    pn2_fetch<T, KST, NB>(B, 1, wid, ntiles, nsteps, pb, voff, goff, xr, pnp, cres, lane);
    for (int j = 0;; j += 3) {
        pn2_fetch<T, KST, NB>(C, j + 2, wid, ntiles, nsteps, pb, voff, goff, xr, pnp, cres, lane);
        pn2_work<T, NBT, KST>(A, cv, cres, pc.null_code, own, wid, lane, Rw, yl);
        if (j + 1 >= nsteps) break;
        pn2_fetch<T, KST, NB>(A, j + 3, wid, ntiles, nsteps, pb, voff, goff, xr, pnp, cres, lane);
        pn2_work<T, NBT, KST>(B, cv, cres, pc.null_code, own, wid, lane, Rw, yl);
        if (j + 2 >= nsteps) break;
        pn2_fetch<T, KST, NB>(B, j + 4, wid, ntiles, nsteps, pb, voff, goff, xr, pnp, cres, lane);
        pn2_work<T, NBT, KST>(C, cv, cres, pc.null_code, own, wid, lane, Rw, yl);
        if (j + 3 >= nsteps) break;
    }
}

template <typename T, int NBT, int NB>
__device__ __forceinline__ void pn2_tiles_k(int ksteps, const PnClass &pc, const T *V, unsigned goff,
                                            __amdgpu_buffer_rsrc_t xr,
                                            const int32_t *pnp, __amdgpu_buffer_rsrc_t cres, int ntiles, int wid,
                                            int lane, T *Rw, T *yl) {
    switch (ksteps) {
        case 1: pn2_tiles<T, NBT, 1, NB>(pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
        case 2: pn2_tiles<T, NBT, 2, NB>(pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
        case 3: pn2_tiles<T, NBT, 3, NB>(pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
        case 4: pn2_tiles<T, NBT, 4, NB>(pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
        case 5: pn2_tiles<T, NBT, 5, NB>(pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
        case 6: pn2_tiles<T, NBT, 6, NB>(pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
        case 7: pn2_tiles<T, NBT, 7, NB>(pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
        default: pn2_tiles<T, NBT, 8, NB>(pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
    }
}

// Three waves per SIMD (six workgroups per CU, which the LDS allows). Used
// for float32; in float64 the two R tiles and the barriers made it slower
// (8.19 against 6.87 ms at pf 5p5n) than the shared row with atomics.
template <typename T, int NB>
__global__ __launch_bounds__(kPnThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_pn2(
    DevHam P, DevTiled TT, const T *__restrict__ x, T *__restrict__ y) {
    __shared__ __align__(16) T Rw[kPnWaves * kPnTile * kPnRStride];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *yl = reinterpret_cast<T *>(smem_raw);   // [max_nn + 1 + 64 * kPnWaves]
    // blocks of NB vectors stored row-wise: one vector g0 per workgroup, the
    // NB workgroups of a row consecutive slots of one XCD (as in k_pn)
    int slot = blockIdx.x, g0 = 0;
    if constexpr (NB > 1) {
        const int xcd = blockIdx.x & 7, s8 = blockIdx.x >> 3;
        slot = (s8 / NB) * 8 + xcd;
        g0 = s8 % NB;
        if (slot >= P.p.n_sd) return;   // uniform: the grid is padded to a multiple of 8 rows
    }
    const int ip = TT.order[slot];
    const unsigned goff = (unsigned)g0 * (unsigned)sizeof(T);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s = P.p_sector[ip];
    const int nn = P.sec_nn[s];
    const int64_t base = P.p_pstart[ip];
    const int nq = P.nq;
    const int ns2 = TT.n_s2;
    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc((void *)x, (short)0, (int)(P.dim * (int64_t)(NB * sizeof(T))), kBufFlags);
    const __amdgpu_buffer_rsrc_t cres =
        __builtin_amdgcn_make_buffer_rsrc((void *)TT.pn2_code, (short)0, (int)(TT.n_pn2_code * 4), kBufFlags);
    for (int c = tid; c < nn; c += kPnThreads) yl[c] = 0;
    __syncthreads();
    bool any = false;
    PnClass pc;
    pc.ob_code = P.p.ob_code;
    pc.ob_base = TT.p_ob_base;
    pc.null_code = TT.pn2_null;
    pc.spare = TT.max_nn + 1;
    for (int q = 0; q < nq; ++q) {
        const int a0 = P.p.ob_ptr[(int64_t)ip * nq + q], a1 = P.p.ob_ptr[(int64_t)ip * nq + q + 1];
        if (a0 == a1) continue;   // uniform across the workgroup
        any = true;
        const int qn = P.conjq[q];
        const int nB = P.vq_nb[q];
        const int nbt = (nB + 15) >> 4;
        const T *V = TabT<T>::vq(P) + P.vq_off[q];
        const int nns = P.sec_nn[P.p_sector[P.p.ob_src[a0]]];
        pc.a0 = a0;
        pc.nd = TT.pn_ndiag[(int64_t)ip * nq + q];
        pc.kp = a1 - a0 - (pc.nd > 1 ? pc.nd - 1 : 0);
        pc.nB = nB;
        const int ksteps = (pc.kp + 3) >> 2;
        const int ntiles = (nns + kPnTile - 1) / kPnTile;
        const int32_t *pnp = TT.pn2_ptr + ((int64_t)s * nq + qn) * ns2 * 2;
        switch (nbt) {
            case 1: pn2_tiles_k<T, 1, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
            case 2: pn2_tiles_k<T, 2, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
            case 3: pn2_tiles_k<T, 3, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
            default: pn2_tiles_k<T, 4, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, Rw, yl); break;
        }
    }
    if (!any) return;
    __syncthreads();
    for (int c = tid; c < nn; c += kPnThreads) y[(base + c) * NB + g0] += yl[c];
}

// float: the row split by column parity between the two waves (k_pn2) when
// it fits; otherwise, and for double, both waves add to the row with LDS
// atomics (k_pn; LDS float atomics are far slower than a read and a write)
template <typename T, int NB>
void launch_pn_nb(const DevHam &d, const DevTiled &t, const T *x, T *y, hipStream_t st) {
    const dim3 grid = NB == 1 ? dim3(d.p.n_sd) : dim3((unsigned)((d.p.n_sd + 7) / 8 * 8 * NB));
    bool priv = false;
    if constexpr (sizeof(T) == 4) {
        priv = t.pn_priv && pn_split_row_fits(t.max_nn);
        if (priv)
            hipLaunchKernelGGL((k_pn2<T, NB>), grid, dim3(kPnThreads),
                               (size_t)(t.max_nn + 1 + 64 * kPnWaves) * sizeof(T), st, d, t, x, y);
    }
    if (!priv)
        hipLaunchKernelGGL((k_pn<T, NB>), grid, dim3(kPnThreads), (size_t)(t.max_nn + 1) * sizeof(T), st, d, t,
                           x, y);
}

template <typename T>
void launch_all(const DevHam &d, const DevTiled &t, const T *x, T *y, hipStream_t st, void **ev) {
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[0], st), "event");
    const int rt = pick_tile(t.max_nn, sizeof(T));
    const size_t lds_nn = (size_t)rt * t.max_nn * sizeof(T);
    switch (rt) {
        case 8: hipLaunchKernelGGL((k_nn_diag<T, 8>), dim3(t.n_rtiles), dim3(kTS), lds_nn, st, d, t, x, y); break;
        case 4: hipLaunchKernelGGL((k_nn_diag<T, 4>), dim3(t.n_rtiles), dim3(kTS), lds_nn, st, d, t, x, y); break;
        case 2: hipLaunchKernelGGL((k_nn_diag<T, 2>), dim3(t.n_rtiles), dim3(kTS), lds_nn, st, d, t, x, y); break;
        default: hipLaunchKernelGGL((k_nn_diag<T, 1>), dim3(t.n_rtiles), dim3(kTS), lds_nn, st, d, t, x, y); break;
    }
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[1], st), "event");
    const int ct = pick_tile(t.max_np, sizeof(T));
    const size_t lds_pp = (size_t)ct * t.max_np * sizeof(T);
    const dim3 gpp(pp_grid(t.n_ctiles, kPpRunLines * pp_line_group<T, 1>()));
    if (sizeof(T) == 4 && t.max_np <= kPpRows * kTS) {
        switch (ct) {
            case 8: hipLaunchKernelGGL((k_pp<T, 8, true>), gpp, dim3(kTS), lds_pp, st, d, t, x, y); break;
            case 4: hipLaunchKernelGGL((k_pp<T, 4, true>), gpp, dim3(kTS), lds_pp, st, d, t, x, y); break;
            case 2: hipLaunchKernelGGL((k_pp<T, 2, true>), gpp, dim3(kTS), lds_pp, st, d, t, x, y); break;
            default: hipLaunchKernelGGL((k_pp<T, 1, true>), gpp, dim3(kTS), lds_pp, st, d, t, x, y); break;
        }
    } else {
        switch (ct) {
            case 8: hipLaunchKernelGGL((k_pp<T, 8, false>), gpp, dim3(kTS), lds_pp, st, d, t, x, y); break;
            case 4: hipLaunchKernelGGL((k_pp<T, 4, false>), gpp, dim3(kTS), lds_pp, st, d, t, x, y); break;
            case 2: hipLaunchKernelGGL((k_pp<T, 2, false>), gpp, dim3(kTS), lds_pp, st, d, t, x, y); break;
            default: hipLaunchKernelGGL((k_pp<T, 1, false>), gpp, dim3(kTS), lds_pp, st, d, t, x, y); break;
        }
    }
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[2], st), "event");
    launch_pn_nb<T, 1>(d, t, x, y, st);
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[3], st), "event");
}

}  // namespace

void launch_materialize_tiled(const DevHam &d, const DevTiled &t, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (t.nn_ell_len > 0)
        hipLaunchKernelGGL(k_ell_values, dim3((unsigned)((t.nn_ell_len + kT - 1) / kT)), dim3(kT), 0, st,
                           t.nn_ell_src, t.nn_ell_ent, (const double *)d.n.off_val64, t.nn_ell_e64, t.nn_ell_e32,
                           t.nn_ell_len);
    if (t.pp_ell_len > 0)
        hipLaunchKernelGGL(k_ell_values, dim3((unsigned)((t.pp_ell_len + kT - 1) / kT)), dim3(kT), 0, st,
                           t.pp_ell_src, t.pp_ell_ent, (const double *)d.p.off_val64, t.pp_ell_e64, t.pp_ell_e32,
                           t.pp_ell_len);
    hip_check(hipGetLastError(), "materialize launch");
}

void launch_pn_block(const DevHam &d, const DevTiled &t, int mode, int nb, const void *x, void *y, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (mode == FOTCI_MODE_F64) {
        const double *xd = (const double *)x;
        double *yd = (double *)y;
        switch (nb) {
            case 2: launch_pn_nb<double, 2>(d, t, xd, yd, st); break;
            case 4: launch_pn_nb<double, 4>(d, t, xd, yd, st); break;
            default: launch_pn_nb<double, 8>(d, t, xd, yd, st); break;
        }
    } else {
        const float *xf = (const float *)x;
        float *yf = (float *)y;
        switch (nb) {
            case 2: launch_pn_nb<float, 2>(d, t, xf, yf, st); break;
            case 4: launch_pn_nb<float, 4>(d, t, xf, yf, st); break;
            default: launch_pn_nb<float, 8>(d, t, xf, yf, st); break;
        }
    }
}

void launch_apply_tiled(const DevHam &d, const DevTiled &t, int mode, const void *x, void *y, void *stream,
                        void **events) {
    hipStream_t st = (hipStream_t)stream;
    if (d.p.n_sd == 0) return;
    if (!t.ok) fail(FOTCI_EINVAL, "basis too large for the tiled kernels (use FOTCI_MODE_F64_PLAIN)");
    if (mode == FOTCI_MODE_F64)
        launch_all<double>(d, t, (const double *)x, (double *)y, st, events);
    else
        launch_all<float>(d, t, (const float *)x, (float *)y, st, events);
    hip_check(hipGetLastError(), "apply launch");
}

}  // namespace fotci
