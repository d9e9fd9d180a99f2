// Device helpers shared by the tiled apply_H kernels (one vector, and blocks
// of vectors stored element-major): tile sizes, matrix-core wrappers, buffer
// loads, the per-wave R tile layout of the pn contraction and the gather-list
// bookkeeping. Included by the .hip files only.
#pragma once

#include <hip/hip_runtime.h>

#include "fotci_internal.h"

namespace fotci {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;      // threads per workgroup (4 waves)
// Threads of the nn and pp workgroups (one vector and blocks): 8 waves share
// a staged slab (three slabs of 53 KB fit a CU, so 24 waves), which hides the
// ELL loads' latency better than 4 waves (f32 nn 0.253 -> 0.205 ms, pp 0.285
// -> 0.249 ms at pf 5p5n; blocks of 4: nn 0.99 -> 0.89 ms, pp 1.33 -> 1.29 ms)
// or 16 (0.220 / 0.270 ms).
constexpr int kTS = 512;
constexpr int kTile = 8;     // rows (nn kernel) / columns (pp kernel) per tile
// Bytes of LDS for a staged tile: at most half of a CU's 160 KiB, so that two
// workgroups share a CU (a 106 KiB float64 slab left one per CU, 4 waves,
// and ran the nn kernel at 0.79 ms against 0.58 ms with half the rows).
constexpr int kLdsTile = 81920;

template <typename T>
struct Mma;
template <>
struct Mma<float> {
    typedef floatx4 acc_t;
    static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // output row of accumulator element r held by `lane` (column = lane % 16)
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Mma<double> {
    typedef doublex4 acc_t;
    static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // the float64 variant interleaves rows: element r of `lane` is row lane/16 + 4r
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <typename T>
struct TabT;
template <>
struct TabT<double> {
    static __device__ __forceinline__ const double *diag(const DevSpecies &s) { return s.d64; }
    static __device__ __forceinline__ const double *vq(const DevHam &h) { return h.vq64; }
    static __device__ __forceinline__ const EllE64 *nn_ell(const DevTiled &t) { return t.nn_ell_e64; }
    static __device__ __forceinline__ const EllE64 *pp_ell(const DevTiled &t) { return t.pp_ell_e64; }
};
template <>
struct TabT<float> {
    static __device__ __forceinline__ const float *diag(const DevSpecies &s) { return s.d32; }
    static __device__ __forceinline__ const float *vq(const DevHam &h) { return h.vq32; }
    static __device__ __forceinline__ const EllE32 *nn_ell(const DevTiled &t) { return t.nn_ell_e32; }
    static __device__ __forceinline__ const EllE32 *pp_ell(const DevTiled &t) { return t.pp_ell_e32; }
};

// One ELL entry of the nn / pp kernels as one vector load.
struct EllVal32 {
    int src;
    float v;
};
struct EllVal64 {
    int src;
    double v;
};
__device__ __forceinline__ EllVal32 ell_load(const EllE32 *__restrict__ e, int64_t k) {
    const uint2 q = *reinterpret_cast<const uint2 *>(e + k);
    return EllVal32{(int)q.x, __uint_as_float(q.y)};
}
__device__ __forceinline__ EllVal64 ell_load(const EllE64 *__restrict__ e, int64_t k) {
    const uint3 q = *reinterpret_cast<const uint3 *>(e + k);
    return EllVal64{(int)q.x, __hiloint2double((int)q.z, (int)q.y)};
}

constexpr int kPnThreads = 64 * kPnWaves;
constexpr int kPnHalves = kPnTile / 16;   // 16-column matrix-core blocks per tile
constexpr unsigned kBufFlags = 0x00020000u;   // raw buffer, 32-bit data format
constexpr unsigned kOutOfRange = 0x7ff00000u;  // byte offset beyond any x

template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double buffer_load<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// flip the sign of v when bit 31 of code is set
__device__ __forceinline__ float signed_by(float v, uint32_t code) {
    return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) ^ (code & 0x80000000u));
}
__device__ __forceinline__ double signed_by(double v, uint32_t code) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) ^ ((uint64_t)(code & 0x80000000u) << 32));
}


// LDS layout of the per-wave tile R[B][col] (B < 64 neutron labels, col <
// kPnTile source columns): column-major with column stride kPnRStride = 68
// elements. float: a lane's four accumulator rows (4 consecutive B) leave in
// one 16-byte store, and 8 lanes of a store cover all 32 banks. double: the
// accumulator rows of a lane are 4 apart and leave in four stores. h selects
// the 16-column block of the tile.
template <typename T>
struct Lds;
template <>
struct Lds<float> {
    static __device__ __forceinline__ void store(float *R, int lane, int h, int bt, const floatx4 &acc) {
        *(floatx4 *)(R + ((lane & 15) + 16 * h) * kPnRStride + 16 * bt + 4 * (lane >> 4)) = acc;
    }
};
template <>
struct Lds<double> {
    static __device__ __forceinline__ void store(double *R, int lane, int h, int bt, const doublex4 &acc) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            R[((lane & 15) + 16 * h) * kPnRStride + 16 * bt + Mma<double>::row(lane, r)] = acc[r];
    }
};

__device__ __forceinline__ uint32_t buffer_load_u32(__amdgpu_buffer_rsrc_t r, unsigned voff) {
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, 0);
}

constexpr int kPnRounds = 8;   // gather rounds of a tile loaded with the tile's x values

// Gather-list ranges of the wave's tiles t = wid + W*(j0 + lane), one tile
// per lane (ends past the last tile clamp to it), read once per 64 tiles so
// that the tile loop picks them with readlane and issues no dependent load.
struct PnBounds {
    int b0, b1;
};

__device__ __forceinline__ void pn_bounds(PnBounds &pb, int j0, int wid, int ntiles, const int32_t *__restrict__ pnp,
                                          int lane) {
    const int tt = wid + kPnWaves * (j0 + lane);
    pb.b0 = pnp[min(tt, ntiles)];
    pb.b1 = pnp[min(tt + 1, ntiles)];
}

// Operands of one operator class for a destination row.
struct PnClass {
    const int32_t *ob_code;   // proton one-body jumps into the row for this class: (local op << 1) | sign
    const int64_t *ob_base;   // their source rows' offsets in x
    int a0, kp, nB;           // kp: contracted jumps, the leading nd >= 2 unchanged-SD jumps counted once
    int nd;                   // jumps at the front of the list that leave the row's SD unchanged
    uint32_t null_code;       // padding entry of the tile-pair gather lists (k_pn2)
    int spare;                // first per-lane scratch word past the output row (k_pn2)
};

// A lane's slice of the class operand C[B][k] = phase_k V^q[A_k, B] (lane
// (col_l, kq) holds B = 16 bt + col_l, k = 4 ks + kq) and the byte offsets of
// its x elements in source row k. The nd >= 2 jumps that leave the row's SD
// unchanged (its occupied orbits' number operators, all from the row itself)
// are one operand row, k = 0, holding the sum of their V rows: x of the row
// is contracted once instead of nd times. Slot k >= 1 is then jump k + nd - 1.
template <typename T, int NBT, int KST, int NB>
__device__ __forceinline__ void pn_operand(const PnClass &pc, const T *__restrict__ V, T (&cv)[NBT][KST],
                                           unsigned (&voff)[KST], int lane) {
    const int col_l = lane & 15, kq = lane >> 4;
    const int shift = pc.nd > 1 ? pc.nd - 1 : 0;
#pragma unroll
    for (int ks = 0; ks < KST; ++ks) {
        const int k = 4 * ks + kq;
        const bool ok = k < pc.kp;
        const int kk = k == 0 ? 0 : k + shift;
        const int code = ok ? pc.ob_code[pc.a0 + kk] : 0;
        voff[ks] = ok ? (unsigned)(pc.ob_base[pc.a0 + kk] + col_l) * (unsigned)(NB * sizeof(T)) : kOutOfRange;
#pragma unroll
        for (int bt = 0; bt < NBT; ++bt) {
            const int B = 16 * bt + col_l;
            const bool live = ok && B < pc.nB;
            T v = live ? V[(code >> 1) * pc.nB + B] : (T)0;
            v = (code & 1) ? -v : v;
            if (ks == 0 && k == 0 && live)
                for (int d = 1; d <= shift; ++d) {
                    const int cd = pc.ob_code[pc.a0 + d];
                    const T vd = V[(cd >> 1) * pc.nB + B];
                    v += (cd & 1) ? -vd : vd;
                }
            cv[bt][ks] = v;
        }
    }
}

// Workgroups are dealt to the 8 XCDs in turn (slot b runs on XCD b % 8). A
// column tile of the pp kernels reads and updates kTile columns (times NB
// vectors) of each row of its sector, so G consecutive tiles share the
// 128-byte lines of x and y; pp_tile_of gives each run of G tiles to one XCD,
// whose L2 then serves every line to all of them instead of each XCD fetching
// it. The grid is padded to a multiple of 8 * G; slots past the last tile
// return. The one-vector pp kernel hands out runs of kPpRunLines lines' worth
// of tiles (4 measured faster than 1, 2, 8 or 16).
constexpr int kPpRunLines = 4;
template <typename T, int NB>
constexpr int pp_line_group() {
    return kTile * NB * (int)sizeof(T) >= 128 ? 1 : 128 / (kTile * NB * (int)sizeof(T));
}
template <int G>
__device__ __forceinline__ int pp_tile_of(int b) {
    const int xcd = b & 7, s8 = b >> 3;
    return (s8 / G) * (8 * G) + xcd * G + s8 % G;
}
inline unsigned pp_grid(int n_tiles, int g) { return (unsigned)((n_tiles + 8 * g - 1) / (8 * g) * (8 * g)); }

// Largest tile (8, 4, 2 or 1 rows or columns) whose staged slab of max_len
// elements of elem bytes each fits kLdsTile.
// A staged line of 32 bytes (8 float or 4 double) is read as two 16-byte
// halves; swapping the halves of every other run of 8 lines spreads the
// lanes' random lines over all 16 LDS bank groups instead of the 8 even or
// odd ones. Returns the element XOR mask for `line`.
template <typename T, int L>
__device__ __forceinline__ int slab_swz(int line) {
    if constexpr (L * sizeof(T) == 32) return ((line >> 3) & 1) * (L / 2);
    else return 0;
}

inline int pick_tile(int max_len, int elem) {
    int t = kTile;
    while (t > 1 && (int64_t)t * max_len * elem > kLdsTile) t >>= 1;
    return t;
}

}  // namespace
}  // namespace fotci
