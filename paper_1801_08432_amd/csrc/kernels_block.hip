// Block apply_H: Y = H X for a block of NB vectors stored row-wise, vector
// index fastest (X[i * NB + v]), so that every matrix element and index that
// a kernel fetches serves NB multiply-adds (Ch. "Block Lanczos": the block is
// kept as the transpose of the column-wise block for locality, and the loop
// over the vectors of the block is the innermost one).
//
// The kernels are the tiled one-vector kernels with the vector index added as
// the innermost dimension of every tile, reading the same tables:
// k_nn_diag_blk  RT proton rows x NB vectors of a sector staged in LDS per
//                pass (RT * NB <= 8: the slab and the accumulators are the size
//                of the one-vector kernel's); each ELL entry of an output
//                column serves RT * NB multiply-adds. Writes Y.
// k_pp_blk       CT neutron columns x NB vectors staged per pass (CT * NB <= 8);
//                each ELL entry of an output row serves CT * NB. Adds to Y.
// k_pn_blk       one workgroup per (destination proton row, group of VC
//                vectors), VC * sizeof(T) = 16 bytes: every lane loads the VC
//                values of one source element with one 16-byte load, each
//                class's matrix-core operand and each gather code serve the VC
//                vectors, and each vector has its own output row in LDS.
//                Adds to Y.
// Per vector the arithmetic is the one-vector kernels' in the same order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tiled_common.h"

namespace fotci {

namespace {

// NB consecutive elements: one row of a block, moved as a unit.
template <typename T, int NB>
struct alignas(NB * sizeof(T) < 16 ? NB * sizeof(T) : 16) Row {
    T v[NB];
};

template <typename T, int NB>
__device__ __forceinline__ Row<T, NB> row_zero() {
    Row<T, NB> r;
#pragma unroll
    for (int v = 0; v < NB; ++v) r.v[v] = T(0);
    return r;
}

// ------------------------------------------------------------ diagonal + nn
template <typename T, int RT, int NB>
__global__ __launch_bounds__(kT) void k_nn_diag_blk(DevHam P, DevTiled TT, const T *__restrict__ x,
                                                    T *__restrict__ y) {
    typedef Row<T, NB> RowT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    RowT *Xl = reinterpret_cast<RowT *>(smem_raw);   // Xl[c * RT + r]
    const RowT *xb = reinterpret_cast<const RowT *>(x);
    RowT *yb = reinterpret_cast<RowT *>(y);
    const int tid = threadIdx.x;
    const int s = TT.rt_sec[blockIdx.x], r0t = TT.rt_r0[blockIdx.x];
    const int np = P.sec_np[s], nn = P.sec_nn[s], nf = P.sec_nfirst[s], pf = P.sec_pfirst[s];
    const int64_t off = P.sec_off[s];
    const int E = TT.nn_ell_E[s];
    const int64_t eb = TT.nn_ell_base[s];
    const T *ev = TabT<T>::nn_ell(TT);
    const T *dpa = TabT<T>::diag(P.p);
    const T *dn = TabT<T>::diag(P.n);
    const int rend = min(r0t + kTile, np);
    for (int r0 = r0t; r0 < rend; r0 += RT) {
        const int nr = min(RT, rend - r0);
        const RowT *xs = xb + off + (int64_t)r0 * nn;
        __syncthreads();
#pragma unroll 4
        for (int idx = tid; idx < RT * nn; idx += kT) {
            const int r = idx / nn, c = idx - r * nn;
            // rows past the tile's end load row nr-1 and store zero: no branch around the load
            const RowT v = xs[(int64_t)min(r, nr - 1) * nn + c];
            Xl[c * RT + r] = r < nr ? v : row_zero<T, NB>();
        }
        T dp[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) dp[r] = r < nr ? dpa[pf + r0 + r] : T(0);
        __syncthreads();
        for (int c = tid; c < nn; c += kT) {
            T acc[RT][NB];
            const T dnc = dn[nf + c];
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const RowT xr = Xl[c * RT + r];
#pragma unroll
                for (int v = 0; v < NB; ++v) acc[r][v] = (dp[r] + dnc) * xr.v[v];
            }
#pragma unroll 4
            for (int e = 0; e < E; ++e) {
                const int64_t k = eb + (int64_t)e * nn + c;
                const int src = TT.nn_ell_src[k];
                const T val = ev[k];
                const RowT *xr = Xl + src * RT;
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    const RowT t = xr[r];
#pragma unroll
                    for (int v = 0; v < NB; ++v) acc[r][v] += val * t.v[v];
                }
            }
#pragma unroll
            for (int r = 0; r < RT; ++r)
                if (r < nr) {
                    RowT o;
#pragma unroll
                    for (int v = 0; v < NB; ++v) o.v[v] = acc[r][v];
                    yb[off + (int64_t)(r0 + r) * nn + c] = o;
                }
        }
    }
}

// ---------------------------------------------------------------------- pp
template <typename T, int CT, int NB>
__global__ __launch_bounds__(kT) void k_pp_blk(DevHam P, DevTiled TT, const T *__restrict__ x, T *__restrict__ y) {
    typedef Row<T, NB> RowT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    RowT *Xl = reinterpret_cast<RowT *>(smem_raw);   // Xl[r * CT + c]
    const RowT *xb = reinterpret_cast<const RowT *>(x);
    RowT *yb = reinterpret_cast<RowT *>(y);
    const int tid = threadIdx.x;
    const int s = TT.ct_sec[blockIdx.x], c0t = TT.ct_c0[blockIdx.x];
    const int np = P.sec_np[s], nn = P.sec_nn[s];
    const int64_t off = P.sec_off[s];
    const int E = TT.pp_ell_E[s];
    if (E == 0) return;
    const int64_t eb = TT.pp_ell_base[s];
    const T *ev = TabT<T>::pp_ell(TT);
    const int cend = min(c0t + kTile, nn);
    for (int c0 = c0t; c0 < cend; c0 += CT) {
        const int nc = min(CT, cend - c0);
        __syncthreads();
#pragma unroll 4
        for (int idx = tid; idx < np * CT; idx += kT) {
            const int r = idx / CT, c = idx - r * CT;
            const RowT v = xb[off + (int64_t)r * nn + c0 + min(c, nc - 1)];   // unconditional load
            Xl[idx] = c < nc ? v : row_zero<T, NB>();
        }
        __syncthreads();
        for (int r = tid; r < np; r += kT) {
            T acc[CT][NB];
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int v = 0; v < NB; ++v) acc[c][v] = 0;
#pragma unroll 4
            for (int e = 0; e < E; ++e) {
                const int64_t k = eb + (int64_t)e * np + r;
                const int src = TT.pp_ell_src[k];
                const T val = ev[k];
                const RowT *xr = Xl + src * CT;
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const RowT t = xr[c];
#pragma unroll
                    for (int v = 0; v < NB; ++v) acc[c][v] += val * t.v[v];
                }
            }
            RowT *yr = yb + off + (int64_t)r * nn + c0;
#pragma unroll
            for (int c = 0; c < CT; ++c)
                if (c < nc) {
                    RowT o = yr[c];
#pragma unroll
                    for (int v = 0; v < NB; ++v) o.v[v] += acc[c][v];
                    yr[c] = o;
                }
        }
    }
}

// ---------------------------------------------------------------------- pn
// Vectors handled by one workgroup: one 16-byte load per lane and element.
template <typename T, int NB>
constexpr int pn_group() {
    return (int)(16 / sizeof(T)) < NB ? (int)(16 / sizeof(T)) : NB;
}

// VC consecutive values at byte offset off of x (all of it in the
// range-checked vector offset, so reads past the end of x return zero).
template <typename T, int VC>
__device__ __forceinline__ Row<T, VC> load_x(__amdgpu_buffer_rsrc_t r, unsigned off) {
    constexpr int bytes = VC * (int)sizeof(T);
    static_assert(bytes == 4 || bytes == 8 || bytes == 16, "one load per element group");
    if constexpr (bytes == 4)
        return __builtin_bit_cast(Row<T, VC>, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    else if constexpr (bytes == 8)
        return __builtin_bit_cast(Row<T, VC>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    else
        return __builtin_bit_cast(Row<T, VC>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}

// The loads of one source tile for the workgroup's VC vectors, and the first
// kPnRounds rounds of its gather codes (a fixed number of loads, as in the
// one-vector kernel, so the next tile's loads stay in flight).
template <typename T, int KST, int VC>
struct PnTileB {
    Row<T, VC> xv[kPnHalves][KST];
    uint32_t cr[kPnRounds];
    int e0, e1;
};

// Tile j of the wave (t = wid + W*j); past the last tile it reloads that tile
// and is marked empty. voff: the lane's element offset of its source row in
// x, in bytes; the tile's column offset is added to it.
template <typename T, int KST, int VC, int NB>
__device__ __forceinline__ void pnb_fetch(PnTileB<T, KST, VC> &b, int j, int wid, int ntiles, PnBounds &pb,
                                          const unsigned *voff, unsigned goff, __amdgpu_buffer_rsrc_t xr,
                                          const int32_t *__restrict__ pnp, __amdgpu_buffer_rsrc_t cres, int lane) {
    if (j > 0 && (j & 63) == 0) pn_bounds(pb, j, wid, ntiles, pnp, lane);   // uniform, every 64 tiles
    const int tt = wid + kPnWaves * j;
    const int tc = min(tt, ntiles - 1);
    b.e0 = __builtin_amdgcn_readlane(pb.b0, j & 63);
    b.e1 = tt < ntiles ? __builtin_amdgcn_readlane(pb.b1, j & 63) : b.e0;
    const unsigned toff = (unsigned)(kPnTile * tc) * (unsigned)(NB * sizeof(T)) + goff;
#pragma unroll
    for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
        for (int ks = 0; ks < KST; ++ks)
            b.xv[h][ks] = load_x<T, VC>(xr, voff[ks] + toff + (unsigned)(16 * h * NB * sizeof(T)));
#pragma unroll
    for (int i = 0; i < kPnRounds; ++i) b.cr[i] = buffer_load_u32(cres, (unsigned)(b.e0 + lane + 64 * i) * 4u);
}

// Contraction and gather of one fetched tile for each of the VC vectors in
// turn; yl: the wave's (PRIV) or the workgroup's output rows, vector v at
// yl + v * ystride. The R tile is reused from one vector to the next: a
// wave's LDS operations complete in issue order.
template <typename T, bool PRIV, int NBT, int KST, int VC>
__device__ __forceinline__ void pnb_work(const PnTileB<T, KST, VC> &b, const T (&cv)[NBT][KST],
                                         __amdgpu_buffer_rsrc_t cres, uint32_t null_code, int lane,
                                         T *__restrict__ R, T *__restrict__ yl, int ystride) {
    typedef typename Mma<T>::acc_t acc_t;
    if (b.e0 == b.e1) return;   // uniform: no neutron jump leaves this tile
    const int ne = b.e1 - b.e0;
#pragma unroll
    for (int v = 0; v < VC; ++v) {
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
                for (int bt = 0; bt < NBT; ++bt) acc[h][bt] = Mma<T>::mma(cv[bt][ks], b.xv[h][ks].v[v], acc[h][bt]);
#pragma unroll
        for (int h = 0; h < kPnHalves; ++h)
#pragma unroll
            for (int bt = 0; bt < NBT; ++bt) Lds<T>::store(R, lane, h, bt, acc[h][bt]);
        __builtin_amdgcn_wave_barrier();
        T *ylv = yl + v * ystride;
#pragma unroll
        for (int i = 0; i < kPnRounds; ++i)
            if (64 * i < ne) pn_add<T, PRIV>(ylv, R, b.cr[i], null_code);
        for (int i = 64 * kPnRounds; i < ne; i += 64)
            pn_add<T, PRIV>(ylv, R, buffer_load_u32(cres, (unsigned)(b.e0 + i + lane) * 4u), null_code);
        __builtin_amdgcn_wave_barrier();
    }
}

template <typename T, bool PRIV, int NBT, int KST, int NB>
__device__ __forceinline__ void pnb_tiles(const PnClass &pc, const T *__restrict__ V, unsigned goff,
                                          __amdgpu_buffer_rsrc_t xr, const int32_t *__restrict__ pnp,
                                          __amdgpu_buffer_rsrc_t cres, int ntiles, int wid, int lane,
                                          T *__restrict__ R, T *__restrict__ yl, int ystride) {
    constexpr int VC = pn_group<T, NB>();
    if (wid >= ntiles) return;
    const int col_l = lane & 15, kq = lane >> 4;
    unsigned voff[KST];
    T cv[NBT][KST];
#pragma unroll
    for (int ks = 0; ks < KST; ++ks) {
        const int k = 4 * ks + kq;
        const bool ok = k < pc.kp;
        const int code = ok ? pc.ob_code[pc.a0 + k] : 0;
        voff[ks] = ok ? (unsigned)(pc.ob_base[pc.a0 + k] + col_l) * (unsigned)(NB * sizeof(T)) : kOutOfRange;
#pragma unroll
        for (int bt = 0; bt < NBT; ++bt) {
            const int B = 16 * bt + col_l;
            const T v = ok && B < pc.nB ? V[(code >> 1) * pc.nB + B] : (T)0;
            cv[bt][ks] = (code & 1) ? -v : v;
        }
    }
    PnBounds pb;
    pn_bounds(pb, 0, wid, ntiles, pnp, lane);
    constexpr int W = kPnWaves;
    PnTileB<T, KST, VC> A, B;
    pnb_fetch<T, KST, VC, NB>(A, 0, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
    for (int j = 0;; j += 2) {
        pnb_fetch<T, KST, VC, NB>(B, j + 1, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
        pnb_work<T, PRIV, NBT, KST, VC>(A, cv, cres, pc.null_code, lane, R, yl, ystride);
        if (wid + W * (j + 1) >= ntiles) break;
        pnb_fetch<T, KST, VC, NB>(A, j + 2, wid, ntiles, pb, voff, goff, xr, pnp, cres, lane);
        pnb_work<T, PRIV, NBT, KST, VC>(B, cv, cres, pc.null_code, lane, R, yl, ystride);
        if (wid + W * (j + 2) >= ntiles) break;
    }
}

template <typename T, bool PRIV, int NBT, int NB>
__device__ __forceinline__ void pnb_tiles_k(int ksteps, const PnClass &pc, const T *V, unsigned goff,
                                            __amdgpu_buffer_rsrc_t xr, const int32_t *pnp,
                                            __amdgpu_buffer_rsrc_t pnc, int ntiles, int wid, int lane, T *R, T *yl,
                                            int ys) {
    switch (ksteps) {
        case 1: pnb_tiles<T, PRIV, NBT, 1, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl, ys); break;
        case 2: pnb_tiles<T, PRIV, NBT, 2, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl, ys); break;
        case 3: pnb_tiles<T, PRIV, NBT, 3, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl, ys); break;
        case 4: pnb_tiles<T, PRIV, NBT, 4, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl, ys); break;
        case 5: pnb_tiles<T, PRIV, NBT, 5, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl, ys); break;
        case 6: pnb_tiles<T, PRIV, NBT, 6, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl, ys); break;
        case 7: pnb_tiles<T, PRIV, NBT, 7, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl, ys); break;
        default: pnb_tiles<T, PRIV, NBT, 8, NB>(pc, V, goff, xr, pnp, pnc, ntiles, wid, lane, R, yl, ys); break;
    }
}

// blockIdx.x: destination proton row (largest rows first); blockIdx.y: the
// group of VC vectors. PRIV: each wave accumulates into its own VC output
// rows (summed at the end); otherwise VC shared rows with LDS atomics.
template <typename T, bool PRIV, int NB>
__global__ __launch_bounds__(kPnThreads) void k_pn_blk(DevHam P, DevTiled TT, const T *__restrict__ x,
                                                       T *__restrict__ y) {
    constexpr int VC = pn_group<T, NB>();
    __shared__ __align__(16) T Rw[kPnWaves][kPnTile * kPnRStride];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *yall = reinterpret_cast<T *>(smem_raw);   // [waves (PRIV)][VC][ystride]

    const int ip = TT.order[blockIdx.x];
    const int g0 = VC * (int)blockIdx.y;   // first vector of the group
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s = P.p_sector[ip];
    const int nn = P.sec_nn[s];
    const int64_t base = P.p_pstart[ip];
    const int nq = P.nq;
    const int ntl = TT.n_t16;
    const T *vq = TabT<T>::vq(P);
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)x, (short)0, (int)(P.dim * (int64_t)(NB * sizeof(T))), kBufFlags);
    const __amdgpu_buffer_rsrc_t cres =
        __builtin_amdgcn_make_buffer_rsrc((void *)TT.pn_code, (short)0, (int)(TT.n_pn_code * 4), kBufFlags);
    T *R = Rw[wid];
    const int ystride = TT.max_nn + 1;   // one padding column per row
    T *yl = PRIV ? yall + wid * VC * ystride : yall;
    constexpr int nrows = (PRIV ? kPnWaves : 1) * VC;
    for (int w = 0; w < nrows; ++w)
        for (int c = tid; c < nn; c += kPnThreads) yall[w * ystride + c] = 0;
    __syncthreads();
    const unsigned goff = (unsigned)(g0 * sizeof(T));
    bool any = false;
    PnClass pc;
    pc.ob_code = P.p.ob_code;
    pc.ob_base = TT.p_ob_base;
    pc.null_code = TT.pn_null;
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
        pc.kp = a1 - a0;
        pc.nB = nB;
        const int ksteps = (pc.kp + 3) >> 2;
        const int ntiles = (nns + kPnTile - 1) / kPnTile;
        const int32_t *pnp = TT.pn_ptr + pslot;
        switch (nbt) {
            case 1: pnb_tiles_k<T, PRIV, 1, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, R, yl, ystride); break;
            case 2: pnb_tiles_k<T, PRIV, 2, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, R, yl, ystride); break;
            case 3: pnb_tiles_k<T, PRIV, 3, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, R, yl, ystride); break;
            default: pnb_tiles_k<T, PRIV, 4, NB>(ksteps, pc, V, goff, xr, pnp, cres, ntiles, wid, lane, R, yl, ystride); break;
        }
    }
    if (!any) return;
    __syncthreads();
    for (int c = tid; c < nn; c += kPnThreads) {
        Row<T, VC> o = *reinterpret_cast<const Row<T, VC> *>(y + (base + c) * NB + g0);
#pragma unroll
        for (int v = 0; v < VC; ++v) {
            T sum = yall[v * ystride + c];
            if (PRIV)
#pragma unroll
                for (int w = 1; w < kPnWaves; ++w) sum += yall[(w * VC + v) * ystride + c];
            o.v[v] += sum;
        }
        *reinterpret_cast<Row<T, VC> *>(y + (base + c) * NB + g0) = o;
    }
}

constexpr size_t kLdsMax = 163840;   // LDS per workgroup on gfx950

// The staged tile of the nn and pp kernels: rt rows (columns) with
// rt * NB <= kTile, so only these instances exist.
template <typename T, int NB>
void launch_nn_blk(int rt, const DevHam &d, const DevTiled &t, const T *x, T *y, size_t lds, hipStream_t st) {
    if constexpr (4 * NB <= kTile) {
        if (rt == 4) {
            hipLaunchKernelGGL((k_nn_diag_blk<T, 4, NB>), dim3(t.n_rtiles), dim3(kT), lds, st, d, t, x, y);
            return;
        }
    }
    if constexpr (2 * NB <= kTile) {
        if (rt == 2) {
            hipLaunchKernelGGL((k_nn_diag_blk<T, 2, NB>), dim3(t.n_rtiles), dim3(kT), lds, st, d, t, x, y);
            return;
        }
    }
    hipLaunchKernelGGL((k_nn_diag_blk<T, 1, NB>), dim3(t.n_rtiles), dim3(kT), lds, st, d, t, x, y);
}

template <typename T, int NB>
void launch_pp_blk(int ct, const DevHam &d, const DevTiled &t, const T *x, T *y, size_t lds, hipStream_t st) {
    if constexpr (4 * NB <= kTile) {
        if (ct == 4) {
            hipLaunchKernelGGL((k_pp_blk<T, 4, NB>), dim3(t.n_ctiles), dim3(kT), lds, st, d, t, x, y);
            return;
        }
    }
    if constexpr (2 * NB <= kTile) {
        if (ct == 2) {
            hipLaunchKernelGGL((k_pp_blk<T, 2, NB>), dim3(t.n_ctiles), dim3(kT), lds, st, d, t, x, y);
            return;
        }
    }
    hipLaunchKernelGGL((k_pp_blk<T, 1, NB>), dim3(t.n_ctiles), dim3(kT), lds, st, d, t, x, y);
}

template <typename T, int NB>
void launch_block(const DevHam &d, const DevTiled &t, const T *x, T *y, hipStream_t st, void **ev) {
    constexpr int VC = pn_group<T, NB>();
    const size_t row = (size_t)NB * sizeof(T);
    // nn: rt rows per pass, pp: ct columns per pass, rt * NB and ct * NB <= kTile
    const int rt = std::min(pick_tile(t.max_nn, (int)row), kTile / NB);
    const int ct = std::min(pick_tile(t.max_np, (int)row), kTile / NB);
    const size_t lds_nn = (size_t)rt * t.max_nn * row;
    const size_t lds_pp = (size_t)ct * t.max_np * row;
    const size_t lds_r = (size_t)kPnWaves * kPnTile * kPnRStride * sizeof(T);
    const size_t lds_shared = (size_t)VC * (t.max_nn + 1) * sizeof(T);
    const size_t lds_priv = (size_t)kPnWaves * lds_shared;
    bool priv = false;
    if constexpr (sizeof(T) == 4) priv = t.pn_priv && lds_r + lds_priv <= kLdsMax;
    if (lds_nn > kLdsMax || lds_pp > kLdsMax || lds_r + lds_shared > kLdsMax)
        fail(FOTCI_EINVAL, "sectors too large for the block kernels' LDS tiles");
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[0], st), "event");
    launch_nn_blk<T, NB>(rt, d, t, x, y, lds_nn, st);
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[1], st), "event");
    launch_pp_blk<T, NB>(ct, d, t, x, y, lds_pp, st);
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[2], st), "event");
    const dim3 grid(d.p.n_sd, NB / VC);
    if constexpr (sizeof(T) == 4) {
        if (priv) hipLaunchKernelGGL((k_pn_blk<T, true, NB>), grid, dim3(kPnThreads), lds_priv, st, d, t, x, y);
    }
    if (!priv) hipLaunchKernelGGL((k_pn_blk<T, false, NB>), grid, dim3(kPnThreads), lds_shared, st, d, t, x, y);
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[3], st), "event");
}

template <typename T>
void launch_block_nb(const DevHam &d, const DevTiled &t, int nb, const T *x, T *y, hipStream_t st, void **ev) {
    switch (nb) {
        case 2: launch_block<T, 2>(d, t, x, y, st, ev); break;
        case 4: launch_block<T, 4>(d, t, x, y, st, ev); break;
        case 8: launch_block<T, 8>(d, t, x, y, st, ev); break;
        default: fail(FOTCI_EINVAL, "n_block must be 1, 2, 4 or 8");
    }
}

}  // namespace

void launch_apply_block(const DevHam &d, const DevTiled &t, int mode, int nb, const void *x, void *y, void *stream,
                        void **events) {
    hipStream_t st = (hipStream_t)stream;
    if (mode != FOTCI_MODE_F64 && mode != FOTCI_MODE_F32)
        fail(FOTCI_EINVAL, "block apply_H needs a tiled mode (FOTCI_MODE_F64 or FOTCI_MODE_F32)");
    if (nb != 2 && nb != 4 && nb != 8) fail(FOTCI_EINVAL, "n_block must be 1, 2, 4 or 8");
    if ((((uintptr_t)x) | ((uintptr_t)y)) & 15u) fail(FOTCI_EINVAL, "block vectors must be 16-byte aligned");
    if (d.p.n_sd == 0) return;
    if (!t.ok) fail(FOTCI_EINVAL, "basis too large for the tiled kernels");
    const int64_t es = mode == FOTCI_MODE_F64 ? 8 : 4;
    // the pn kernel addresses x with 32-bit byte offsets, padding lanes at kOutOfRange
    if (d.dim * nb * es > (int64_t)kOutOfRange) fail(FOTCI_EINVAL, "block too large for 32-bit buffer offsets");
    if (mode == FOTCI_MODE_F64)
        launch_block_nb<double>(d, t, nb, (const double *)x, (double *)y, st, events);
    else
        launch_block_nb<float>(d, t, nb, (const float *)x, (float *)y, st, events);
    hip_check(hipGetLastError(), "block apply launch");
}

}  // namespace fotci
