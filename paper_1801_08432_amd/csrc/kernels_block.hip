// Block apply_H: Y = H X for a block of NB vectors stored row-wise, vector
// index fastest (X[i * NB + v]), so that every matrix element and index that
// a kernel fetches serves NB multiply-adds (Ch. "Block Lanczos": the block is
// kept as the transpose of the column-wise block for locality, and the loop
// over the vectors of the block is the innermost one).
//
// The nn and pp kernels are the tiled one-vector kernels with the vector
// index added as the innermost dimension of every staged tile, reading the
// same tables:
// k_nn_diag_blk  RT proton rows x NB vectors of a sector staged in LDS per
//                pass (RT * NB <= 8: the slab and the accumulators are the size
//                of the one-vector kernel's); each ELL entry of an output
//                column serves RT * NB multiply-adds. Writes Y.
// k_pp_blk       CT neutron columns x NB vectors staged per pass (CT * NB <= 8);
//                each ELL entry of an output row serves CT * NB. Adds to Y.
// The pn part is the one-vector pn kernel with a vector stride, one vector
// per workgroup (launch_pn_block): grouping vectors in a workgroup multiplies
// its LDS output rows and cuts occupancy, which costs more than the shared
// class operands and gather codes save.
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
__global__ __launch_bounds__(kTS) void k_nn_diag_blk(DevHam P, DevTiled TT, const T *__restrict__ x,
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
    const auto *ev = TabT<T>::nn_ell(TT);
    const T *dpa = TabT<T>::diag(P.p);
    const T *dn = TabT<T>::diag(P.n);
    const int rend = min(r0t + kTile, np);
    for (int r0 = r0t; r0 < rend; r0 += RT) {
        const int nr = min(RT, rend - r0);
        const RowT *xs = xb + off + (int64_t)r0 * nn;
        __syncthreads();
#pragma unroll 4
        for (int idx = tid; idx < RT * nn; idx += kTS) {
            const int r = idx / nn, c = idx - r * nn;
            // rows past the tile's end load row nr-1 and store zero: no branch around the load
            const RowT v = xs[(int64_t)min(r, nr - 1) * nn + c];
            Xl[c * RT + r] = r < nr ? v : row_zero<T, NB>();
        }
        T dp[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) dp[r] = r < nr ? dpa[pf + r0 + r] : T(0);
        __syncthreads();
        for (int c = tid; c < nn; c += kTS) {
            T acc[RT][NB];
            const T dnc = dn[nf + c];
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const RowT xr = Xl[c * RT + r];
#pragma unroll
                for (int v = 0; v < NB; ++v) acc[r][v] = (dp[r] + dnc) * xr.v[v];
            }
#pragma unroll 8
            for (int e = 0; e < E; ++e) {
                const auto ent = ell_load(ev, eb + (int64_t)e * nn + c);
                const int src = ent.src;
                const T val = ent.v;
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
__global__ __launch_bounds__(kTS) void k_pp_blk(DevHam P, DevTiled TT, const T *__restrict__ x, T *__restrict__ y) {
    typedef Row<T, NB> RowT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    RowT *Xl = reinterpret_cast<RowT *>(smem_raw);   // Xl[r * CT + c]
    const RowT *xb = reinterpret_cast<const RowT *>(x);
    RowT *yb = reinterpret_cast<RowT *>(y);
    const int tid = threadIdx.x;
    const int tile = pp_tile_of<pp_line_group<T, NB>()>(blockIdx.x);
    if (tile >= TT.n_ctiles) return;
    const int s = TT.ct_sec[tile], c0t = TT.ct_c0[tile];
    const int np = P.sec_np[s], nn = P.sec_nn[s];
    const int64_t off = P.sec_off[s];
    const int E = TT.pp_ell_E[s];
    if (E == 0) return;
    const int64_t eb = TT.pp_ell_base[s];
    const auto *ev = TabT<T>::pp_ell(TT);
    const int cend = min(c0t + kTile, nn);
    for (int c0 = c0t; c0 < cend; c0 += CT) {
        const int nc = min(CT, cend - c0);
        __syncthreads();
#pragma unroll 4
        for (int idx = tid; idx < np * CT; idx += kTS) {
            const int r = idx / CT, c = idx - r * CT;
            const RowT v = xb[off + (int64_t)r * nn + c0 + min(c, nc - 1)];   // unconditional load
            Xl[idx] = c < nc ? v : row_zero<T, NB>();
        }
        __syncthreads();
        for (int r = tid; r < np; r += kTS) {
            T acc[CT][NB];
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int v = 0; v < NB; ++v) acc[c][v] = 0;
#pragma unroll 8
            for (int e = 0; e < E; ++e) {
                const auto ent = ell_load(ev, eb + (int64_t)e * np + r);
                const int src = ent.src;
                const T val = ent.v;
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

constexpr size_t kLdsMax = 163840;   // LDS per workgroup on gfx950

// The staged tile of the nn and pp kernels: rt rows (columns) with
// rt * NB <= kTile, so only these instances exist.
template <typename T, int NB>
void launch_nn_blk(int rt, const DevHam &d, const DevTiled &t, const T *x, T *y, size_t lds, hipStream_t st) {
    if constexpr (4 * NB <= kTile) {
        if (rt == 4) {
            hipLaunchKernelGGL((k_nn_diag_blk<T, 4, NB>), dim3(t.n_rtiles), dim3(kTS), lds, st, d, t, x, y);
            return;
        }
    }
    if constexpr (2 * NB <= kTile) {
        if (rt == 2) {
            hipLaunchKernelGGL((k_nn_diag_blk<T, 2, NB>), dim3(t.n_rtiles), dim3(kTS), lds, st, d, t, x, y);
            return;
        }
    }
    hipLaunchKernelGGL((k_nn_diag_blk<T, 1, NB>), dim3(t.n_rtiles), dim3(kTS), lds, st, d, t, x, y);
}

template <typename T, int NB>
void launch_pp_blk(int ct, const DevHam &d, const DevTiled &t, const T *x, T *y, size_t lds, hipStream_t st) {
    const dim3 grid(pp_grid(t.n_ctiles, pp_line_group<T, NB>()));
    if constexpr (4 * NB <= kTile) {
        if (ct == 4) {
            hipLaunchKernelGGL((k_pp_blk<T, 4, NB>), grid, dim3(kTS), lds, st, d, t, x, y);
            return;
        }
    }
    if constexpr (2 * NB <= kTile) {
        if (ct == 2) {
            hipLaunchKernelGGL((k_pp_blk<T, 2, NB>), grid, dim3(kTS), lds, st, d, t, x, y);
            return;
        }
    }
    hipLaunchKernelGGL((k_pp_blk<T, 1, NB>), grid, dim3(kTS), lds, st, d, t, x, y);
}

template <typename T, int NB>
void launch_block(const DevHam &d, const DevTiled &t, const T *x, T *y, hipStream_t st, void **ev) {
    const size_t row = (size_t)NB * sizeof(T);
    // nn: rt rows per pass, pp: ct columns per pass, rt * NB and ct * NB <= kTile
    const int rt = std::min(pick_tile(t.max_nn, (int)row), kTile / NB);
    const int ct = std::min(pick_tile(t.max_np, (int)row), kTile / NB);
    const size_t lds_nn = (size_t)rt * t.max_nn * row;
    const size_t lds_pp = (size_t)ct * t.max_np * row;
    const size_t lds_pn = (size_t)kPnWaves * kPnTile * kPnRStride * sizeof(T) + (size_t)(t.max_nn + 1) * sizeof(T);
    if (lds_nn > kLdsMax || lds_pp > kLdsMax || lds_pn > kLdsMax)
        fail(FOTCI_EINVAL, "sectors too large for the block kernels' LDS tiles");
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[0], st), "event");
    launch_nn_blk<T, NB>(rt, d, t, x, y, lds_nn, st);
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[1], st), "event");
    launch_pp_blk<T, NB>(ct, d, t, x, y, lds_pp, st);
    if (ev) hip_check(hipEventRecord((hipEvent_t)ev[2], st), "event");
    launch_pn_block(d, t, sizeof(T) == 8 ? FOTCI_MODE_F64 : FOTCI_MODE_F32, NB, x, y, st);
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
