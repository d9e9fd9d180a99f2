// Lanczos with full reorthogonalisation on the device (Ch. 7, "Standard
// Lanczos algorithm"), with float64 reductions for every inner product.
//
// Per iteration i: (1) y = H v_i; (2) alpha_i = <v_i, y>; (3)-(4)
// w = y - alpha_i v_i - beta_{i-1} v_{i-1}; reorthogonalisation against every
// stored vector by classical Gram-Schmidt, twice (alpha is taken before the
// reorthogonalisation, the ordering the chapter recommends); (5) beta_i =
// ||w||; (6) v_{i+1} = w / beta_i. Lanczos vectors are stored in the mode's
// precision (float64 or float32); w, alpha, beta and the coefficients are
// float64. The tridiagonal eigenproblem is solved on the host in float64; the
// Ritz vectors are formed on the device with float64 accumulation and, with
// refinement, their float64 Rayleigh quotients are the returned eigenvalues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "fotci_internal.h"

namespace fotci {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
// Lanczos steps issued between two reads of alpha and beta by the host
constexpr int kLazySteps = 16;
constexpr int kRowsPerThread = 8;
constexpr int kChunk = kThreads * kRowsPerThread;   // rows per block in the tall-skinny kernels
constexpr int kMaxIter = 4096;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide float64 sum; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kWaves; ++w) t += lds[w];
    __syncthreads();
    return t;
}

template <typename TA, typename TB>
__global__ __launch_bounds__(kThreads) void k_dot_partial(const TA *__restrict__ a, const TB *__restrict__ b,
                                                          int64_t n, double *__restrict__ partial) {
    __shared__ double lds[kWaves];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        acc += (double)a[i] * (double)b[i];
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// out[0] = sum(partial[0..nb)) (sqrt if take_sqrt); deterministic order.
__global__ __launch_bounds__(kThreads) void k_finish(const double *__restrict__ partial, int nb, double *out,
                                                     int take_sqrt) {
    __shared__ double lds[kWaves];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += kThreads) acc += partial[i];
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(acc) : acc;
}

// w = y - alpha v_i - beta v_{i-1} (beta term skipped when vprev is null)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_three_term(const T *__restrict__ y, const T *__restrict__ vi,
                                                         const T *__restrict__ vprev, const double *alpha,
                                                         const double *beta, double *__restrict__ w, int64_t n) {
    const double a = *alpha;
    const double b = vprev ? *beta : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double t = (double)y[i] - a * (double)vi[i];
        if (vprev) t -= b * (double)vprev[i];
        w[i] = t;
    }
}

// Tall-skinny kernels over the stored basis V (k vectors of n rows, leading
// dimension ld, a multiple of 64 elements so every vector starts 256-byte
// aligned). A block owns kChunk consecutive rows; each thread owns
// kRowsPerThread of them, read as 16-byte vectors so that one load
// instruction of a wave covers 1 KiB of contiguous rows. Loops over the basis
// vectors are unrolled by kJU, so each thread has the loads of kJU vectors in
// flight at once. The last block of the rows takes a guarded scalar path.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};

constexpr int kJU = 4;

template <typename T>
__device__ __forceinline__ int64_t row_of(int64_t r0, int q, int e) {
    constexpr int NV = Vec16<T>::n;
    return r0 + (int64_t)q * kThreads * NV + (int64_t)threadIdx.x * NV + e;
}

// Rows of basis vector `v` owned by this thread, widened to float64 (0 past n).
// A pass reads each stored basis element once, so the 16-byte loads are
// nontemporal: the stream does not displace the vectors read again (w), and
// the pass runs ~6% faster than with ordinary loads.
template <typename T, bool FULL>
__device__ __forceinline__ void load_rows(const T *__restrict__ v, int64_t r0, int64_t n, double (&out)[kRowsPerThread]) {
    typedef T NTV __attribute__((ext_vector_type(Vec16<T>::n)));
    constexpr int NV = Vec16<T>::n;
    constexpr int NL = kRowsPerThread / NV;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        if (FULL) {
            const NTV t = __builtin_nontemporal_load((const NTV *)(v + row_of<T>(r0, q, 0)));
            const T *tp = (const T *)&t;
#pragma unroll
            for (int e = 0; e < NV; ++e) out[q * NV + e] = (double)tp[e];
        } else {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const int64_t r = row_of<T>(r0, q, e);
                out[q * NV + e] = r < n ? (double)v[r] : 0.0;
            }
        }
    }
}

// The same rows (the mapping of basis type T) of the float64 vector w.
template <typename T, bool FULL>
__device__ __forceinline__ void load_w(const double *__restrict__ w, int64_t r0, int64_t n,
                                       double (&out)[kRowsPerThread]) {
    constexpr int NV = Vec16<T>::n;
    constexpr int NL = kRowsPerThread / NV;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        if (FULL) {
#pragma unroll
            for (int e = 0; e < NV; e += 2) {
                const double2 t = *(const double2 *)(w + row_of<T>(r0, q, e));
                out[q * NV + e] = t.x;
                out[q * NV + e + 1] = t.y;
            }
        } else {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const int64_t r = row_of<T>(r0, q, e);
                out[q * NV + e] = r < n ? w[r] : 0.0;
            }
        }
    }
}

// partial[j*nb + block] = sum over the block's rows of V_j[r] * w[r], j < k.
// Each wave reduces with shuffles; the waves' sums meet in LDS once per 256
// basis vectors.
template <typename T, bool FULL>
__device__ __forceinline__ void multidot_body(const T *__restrict__ V, int64_t ld, int k, const double *__restrict__ w,
                                              int64_t n, double *__restrict__ partial, double *__restrict__ sq_partial,
                                              double (*lds)[256]) {
    const int64_t r0 = (int64_t)blockIdx.x * kChunk;
    const int nb = gridDim.x;
    double wr[kRowsPerThread];
    load_w<T, FULL>(w, r0, n, wr);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (sq_partial) {   // ||w||^2 of the block's rows (before this pass)
        double sq = 0.0;
#pragma unroll
        for (int e = 0; e < kRowsPerThread; ++e) sq += wr[e] * wr[e];
        sq = block_sum(sq, &lds[0][0]);
        if (threadIdx.x == 0) sq_partial[blockIdx.x] = sq;
    }
    for (int j0 = 0; j0 < k; j0 += 256) {
        const int jn = min(256, k - j0);
        for (int jj = 0; jj < jn; jj += kJU) {
            double acc[kJU];
            double vr[kJU][kRowsPerThread];
#pragma unroll
            for (int u = 0; u < kJU; ++u)   // past the last vector: reload it, the sum is not stored
                load_rows<T, FULL>(V + (int64_t)min(j0 + jj + u, k - 1) * ld, r0, n, vr[u]);
#pragma unroll
            for (int u = 0; u < kJU; ++u) {
                acc[u] = 0.0;
#pragma unroll
                for (int e = 0; e < kRowsPerThread; ++e) acc[u] += vr[u][e] * wr[e];
            }
#pragma unroll
            for (int u = 0; u < kJU; ++u) {
                const double t = wave_sum(acc[u]);
                if (lane == 0 && jj + u < jn) lds[wid][jj + u] = t;
            }
        }
        __syncthreads();
        for (int jj = threadIdx.x; jj < jn; jj += kThreads) {
            double t = 0.0;
            for (int q = 0; q < kWaves; ++q) t += lds[q][jj];
            partial[(int64_t)(j0 + jj) * nb + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_multidot(const T *__restrict__ V, int64_t ld, int k,
                                                       const double *__restrict__ w, int64_t n,
                                                       double *__restrict__ partial, double *__restrict__ sq_partial) {
    __shared__ double lds[kWaves][256];
    if ((int64_t)(blockIdx.x + 1) * kChunk <= n)
        multidot_body<T, true>(V, ld, k, w, n, partial, sq_partial, lds);
    else
        multidot_body<T, false>(V, ld, k, w, n, partial, sq_partial, lds);
}

// c[j] = sum_b partial[j*nb + b]; one block per j.
__global__ __launch_bounds__(kThreads) void k_reduce_rows(const double *__restrict__ partial, int nb,
                                                          double *__restrict__ c) {
    __shared__ double lds[kWaves];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) acc += partial[(int64_t)j * nb + b];
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) c[j] = acc;
}

// w[r] -= sum_j c[j] V_j[r]; with sq_partial, also the block's sum of the
// updated w[r]^2 (the norm that follows the last pass).
template <typename T, bool FULL>
__device__ __forceinline__ void subtract_body(const T *__restrict__ V, int64_t ld, int k, const double *cs,
                                              double *__restrict__ w, int64_t n, double *__restrict__ sq_partial,
                                              double *lds) {
    const int64_t r0 = (int64_t)blockIdx.x * kChunk;
    double acc[kRowsPerThread];
#pragma unroll
    for (int e = 0; e < kRowsPerThread; ++e) acc[e] = 0.0;
    int j = 0;
    for (; j + kJU <= k; j += kJU) {
        double vr[kJU][kRowsPerThread];
#pragma unroll
        for (int u = 0; u < kJU; ++u) load_rows<T, FULL>(V + (int64_t)(j + u) * ld, r0, n, vr[u]);
#pragma unroll
        for (int u = 0; u < kJU; ++u) {
            const double cj = cs[j + u];
#pragma unroll
            for (int e = 0; e < kRowsPerThread; ++e) acc[e] += cj * vr[u][e];
        }
    }
    for (; j < k; ++j) {
        double vr[kRowsPerThread];
        load_rows<T, FULL>(V + (int64_t)j * ld, r0, n, vr);
        const double cj = cs[j];
#pragma unroll
        for (int e = 0; e < kRowsPerThread; ++e) acc[e] += cj * vr[e];
    }
    double wr[kRowsPerThread];
    load_w<T, FULL>(w, r0, n, wr);
    double sq = 0.0;
    constexpr int NV = Vec16<T>::n;
    constexpr int NL = kRowsPerThread / NV;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const int64_t r = row_of<T>(r0, q, e);
            const double t = wr[q * NV + e] - acc[q * NV + e];
            if (FULL || r < n) {
                w[r] = t;
                sq += t * t;
            }
        }
    }
    if (sq_partial) {
        sq = block_sum(sq, lds);
        if (threadIdx.x == 0) sq_partial[blockIdx.x] = sq;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_subtract(const T *__restrict__ V, int64_t ld, int k,
                                                       const double *__restrict__ c, double *__restrict__ w,
                                                       int64_t n, double *__restrict__ sq_partial) {
    extern __shared__ double cs[];   // k coefficients, then kWaves reduction slots
    for (int j = threadIdx.x; j < k; j += kThreads) cs[j] = c[j];
    __syncthreads();
    if ((int64_t)(blockIdx.x + 1) * kChunk <= n)
        subtract_body<T, true>(V, ld, k, cs, w, n, sq_partial, cs + k);
    else
        subtract_body<T, false>(V, ld, k, cs, w, n, sq_partial, cs + k);
}

// out = (T)(in * scale) with scale = 1 / *denom
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale_store(const double *__restrict__ in, const double *denom,
                                                          T *__restrict__ out, int64_t n) {
    const double s = 1.0 / *denom;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        out[i] = (T)(in[i] * s);
}

// Y_j[r] = sum_l V_l[r] S[l*s_ld + j0 + j] for j < nk <= 16 (float64
// accumulation), stored as TO with row stride y_ld: the Ritz vectors, and the
// new leading basis vectors at a thick restart.
template <typename T, typename TO>
__global__ __launch_bounds__(kThreads) void k_ritz(const T *__restrict__ V, int64_t ld, int k,
                                                   const double *__restrict__ S, int s_ld, int j0, int nk,
                                                   TO *__restrict__ Y, int64_t y_ld, int64_t n) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    double acc[16];
    for (int j = 0; j < nk; ++j) acc[j] = 0.0;
    for (int l = 0; l < k; ++l) {
        const double v = (double)V[(int64_t)l * ld + r];
        for (int j = 0; j < nk; ++j) acc[j] += v * S[l * s_ld + j0 + j];
    }
    for (int j = 0; j < nk; ++j) Y[(int64_t)j * y_ld + r] = (TO)acc[j];
}

// r = hy - theta y; partial sums of r^2
__global__ __launch_bounds__(kThreads) void k_resid_partial(const double *__restrict__ hy,
                                                            const double *__restrict__ y, const double *theta,
                                                            int64_t n, double *__restrict__ partial) {
    __shared__ double lds[kWaves];
    const double t = *theta;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const double r = hy[i] - t * y[i];
        acc += r * r;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// ------------------------------------------------------------ block Lanczos
// Blocks of NB vectors are stored row-wise, as the block apply_H takes them:
// row i of block j at V[j * ldb + i * NB + v] with ldb = ld * NB. A workgroup
// owns kThreads * brows rows; thread t owns rows r0 + q * kThreads + t
// (q < brows), so one load instruction of a wave reads 64 consecutive rows.
// brows shrinks as the NB x NB float64 accumulators grow (no spills).
constexpr int brows_of(int nb) { return nb <= 2 ? 8 : (nb == 4 ? 4 : 2); }
template <int NB>
constexpr int brows() {
    return brows_of(NB);
}
template <int NB>
constexpr int bchunk() {
    return kThreads * brows<NB>();
}
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Row i of a row-wise block, widened to float64 (zero for i >= n). NT: a
// stored basis block, read once per pass with nontemporal loads (as load_rows).
template <typename T, int NB, bool NT>
__device__ __forceinline__ void load_brow(const T *__restrict__ base, int64_t i, int64_t n, double (&out)[NB]) {
    if (i < n) {
        const T *p = base + i * NB;
        if constexpr (NB * sizeof(T) >= 16) {
            constexpr int NV = 16 / (int)sizeof(T);
            typedef T NTV __attribute__((ext_vector_type(16 / sizeof(T))));
#pragma unroll
            for (int q = 0; q < NB / NV; ++q) {
                const NTV t = NT ? __builtin_nontemporal_load((const NTV *)(p + q * NV)) : *(const NTV *)(p + q * NV);
                const T *tp = (const T *)&t;
#pragma unroll
                for (int e = 0; e < NV; ++e) out[q * NV + e] = (double)tp[e];
            }
        } else {
#pragma unroll
            for (int v = 0; v < NB; ++v) out[v] = (double)(NT ? __builtin_nontemporal_load(p + v) : p[v]);
        }
    } else {
#pragma unroll
        for (int v = 0; v < NB; ++v) out[v] = 0.0;
    }
}

// Sums each of the NQ values of every lane over the wave (NQ a power of two
// up to 64): each step exchanges half of the values a lane still holds with
// the lane `o` apart and keeps the other half, so the values are spread over
// the lanes with log2(NQ) steps and NQ - 1 exchanges; plain exchanges finish
// the sums. Lane l returns the total of value l >> (6 - log2 NQ).
template <int NQ, int ST>
__device__ __forceinline__ void spread_step(double (&a)[NQ], int lane) {
    if constexpr ((NQ >> ST) > 1) {
        constexpr int half = (NQ >> ST) / 2, o = 32 >> ST;
        const bool hi = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const double keep = hi ? a[i + half] : a[i];
            const double give = hi ? a[i] : a[i + half];
            a[i] = keep + __shfl_xor(give, o, 64);
        }
        spread_step<NQ, ST + 1>(a, lane);
    }
}

template <int NQ>
__device__ __forceinline__ double wave_sum_spread(double (&a)[NQ]) {
    constexpr int LOG = ilog2(NQ);
    spread_step<NQ, 0>(a, threadIdx.x & 63);
    double v = a[0];
#pragma unroll
    for (int o = 32 >> LOG; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// partial[(j*NB*NB + v*NB + u) * nb + block] = sum over the block's rows of
// V_j[i, v] W[i, u] for j < k: the workgroup's share of V_j^T W.
template <typename TV, int NB>
__global__ __launch_bounds__(kThreads) void k_bmultidot(const TV *__restrict__ V, int64_t ldb, int k,
                                                        const double *__restrict__ W, int64_t n,
                                                        double *__restrict__ partial) {
    constexpr int NQ = NB * NB, RPT = brows<NB>(), LOG = ilog2(NQ);
    __shared__ double lds[2][kWaves][NQ];
    const int64_t r0 = (int64_t)blockIdx.x * bchunk<NB>() + threadIdx.x;
    const int nb = gridDim.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double wr[RPT][NB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) load_brow<double, NB, false>(W, r0 + (int64_t)q * kThreads, n, wr[q]);
    for (int j = 0; j < k; ++j) {
        const TV *Vj = V + (int64_t)j * ldb;
        double acc[NQ];
#pragma unroll
        for (int e = 0; e < NQ; ++e) acc[e] = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            double vr[NB];
            load_brow<TV, NB, true>(Vj, r0 + (int64_t)q * kThreads, n, vr);
#pragma unroll
            for (int v = 0; v < NB; ++v)
#pragma unroll
                for (int u = 0; u < NB; ++u) acc[v * NB + u] += vr[v] * wr[q][u];
        }
        const double t = wave_sum_spread<NQ>(acc);
        // double-buffered: the readers of j - 1 passed this barrier's
        // predecessor before anyone writes the same buffer at j + 1
        if ((lane & ((64 >> LOG) - 1)) == 0) lds[j & 1][wid][lane >> (6 - LOG)] = t;
        __syncthreads();
        if (threadIdx.x < NQ) {
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) sum += lds[j & 1][w][threadIdx.x];
            partial[((int64_t)j * NQ + threadIdx.x) * nb + blockIdx.x] = sum;
        }
    }
}

// W[i, u] -= sum_{j < k} sum_v V_j[i, v] C[(j*NB + v)*NB + u].
template <typename TV, int NB>
__global__ __launch_bounds__(kThreads) void k_bsubtract(const TV *__restrict__ V, int64_t ldb, int k,
                                                        const double *__restrict__ C, double *__restrict__ W,
                                                        int64_t n) {
    constexpr int RPT = brows<NB>();
    const int64_t r0 = (int64_t)blockIdx.x * bchunk<NB>() + threadIdx.x;
    double acc[RPT][NB];
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[q][u] = 0.0;
    for (int j = 0; j < k; ++j) {
        const TV *Vj = V + (int64_t)j * ldb;
        const double *Cj = C + (int64_t)j * NB * NB;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            double vr[NB];
            load_brow<TV, NB, true>(Vj, r0 + (int64_t)q * kThreads, n, vr);
#pragma unroll
            for (int v = 0; v < NB; ++v)
#pragma unroll
                for (int u = 0; u < NB; ++u) acc[q][u] += vr[v] * Cj[v * NB + u];
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int64_t i = r0 + (int64_t)q * kThreads;
        if (i < n) {
            double *wp = W + i * NB;
#pragma unroll
            for (int u = 0; u < NB; ++u) wp[u] -= acc[q][u];
        }
    }
}

// out[i, u] = sum_v W[i, v] M[v*NB + u] (float64 sums, stored as TO); out may
// be W itself (each thread reads its row whole before writing it).
template <typename TO, int NB>
__global__ __launch_bounds__(kThreads) void k_bmix(const double *W, const double *__restrict__ M, TO *out,
                                                   int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double w[NB];
        load_brow<double, NB, false>(W, i, n, w);
        TO *op = out + i * NB;
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            double t = 0.0;
#pragma unroll
            for (int v = 0; v < NB; ++v) t += w[v] * M[v * NB + u];
            op[u] = (TO)t;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_widen(const T *__restrict__ a, double *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        b[i] = (double)a[i];
}

// Y_c[i] = sum_{j < k} sum_v V_j[i, v] S[(j*NB + v)*s_ld + c0 + c] for c < nc
// <= 16 (float64 sums): Ritz vectors from a row-wise block basis, stored one
// after another (row stride n).
template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void k_britz(const T *__restrict__ V, int64_t ldb, int k,
                                                    const double *__restrict__ S, int s_ld, int c0, int nc,
                                                    double *__restrict__ Y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    double acc[16];
    for (int c = 0; c < nc; ++c) acc[c] = 0.0;
    for (int j = 0; j < k; ++j) {
        double vr[NB];
        load_brow<T, NB, true>(V + (int64_t)j * ldb, i, n, vr);
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            const double *Sr = S + (int64_t)(j * NB + v) * s_ld + c0;
            for (int c = 0; c < nc; ++c) acc[c] += vr[v] * Sr[c];
        }
    }
    for (int c = 0; c < nc; ++c) Y[(int64_t)c * n + i] = acc[c];
}

int stream_blocks(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}
int chunk_blocks(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }

int64_t a256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Workspace of both drivers: nvec Lanczos vectors and nscr scratch vectors
// in the storage precision (leading dimension ld), then float64 work vectors
// and small arrays.
struct Layout {
    int64_t ld;   // basis leading dimension (elements): dim rounded up to 64
    int64_t basis, scratch, y, w, partial, sq, scal, coef, S, ritz, hy, hist, total;   // hist 0: none
};

Layout make_layout(int64_t dim, int es, int nvec, int nscr, int ncoef, int s_cols, int n_keep) {
    Layout L{};
    L.ld = (dim + 63) & ~(int64_t)63;
    int64_t off = 0;
    L.basis = off;
    off = a256(off + (int64_t)nvec * L.ld * es);
    L.scratch = off;
    off = a256(off + (int64_t)nscr * L.ld * es);
    L.y = off;
    off = a256(off + dim * es);
    L.w = off;
    off = a256(off + dim * 8);
    const int64_t nb = std::max<int64_t>(chunk_blocks(dim), 2048);
    L.partial = off;
    off = a256(off + (int64_t)std::max(ncoef, 1) * nb * 8);
    L.sq = off;
    off = a256(off + nb * 8);
    L.scal = off;
    off = a256(off + 64 * 8);
    L.coef = off;
    off = a256(off + (int64_t)ncoef * 8);
    L.S = off;
    off = a256(off + (int64_t)ncoef * s_cols * 8);
    L.ritz = off;
    off = a256(off + (int64_t)n_keep * dim * 8);
    L.hy = off;
    off = a256(off + dim * 8);
    L.hist = off;
    off = a256(off + (int64_t)std::max(ncoef, 1) * 16);
    L.total = off;
    return L;
}

int elem_size(int mode) { return (mode == FOTCI_MODE_F64 || mode == FOTCI_MODE_F64_PLAIN) ? 8 : 4; }

Layout standard_layout(const fotci_ham *h, const fotci_lanczos_opts *o) {
    return make_layout(h->j->b->dim, elem_size(o->mode), o->n_iter, 0, o->n_iter, o->n_keep, o->n_keep);
}

// Thick restart: n_basis + 1 vectors, n_thick scratch vectors.
Layout trlan_layout(const fotci_ham *h, const fotci_trlan_opts *o) {
    return make_layout(h->j->b->dim, elem_size(o->mode), o->n_basis + 1, o->n_thick, o->n_basis + 1,
                       std::max(o->n_thick, o->n_keep), o->n_keep);
}

// Block Lanczos: n_iter + 1 row-wise blocks, the block H V_n (mode precision)
// and its float64 copy W, partial sums of the block kernels, coefficients
// (Gram-Schmidt for every block, three-term, mixing and overlap matrices).
Layout block_layout(const fotci_ham *h, const fotci_block_lanczos_opts *o) {
    const int64_t dim = h->j->b->dim;
    const int nb = o->n_block, es = elem_size(o->mode);
    const int nblk = o->n_iter + 1, nq = nb * nb;
    const int64_t chunk = (int64_t)kThreads * brows_of(nb);   // bchunk<NB>()
    const int64_t nbc = std::max<int64_t>((dim + chunk - 1) / chunk, 2048);
    Layout L{};
    L.ld = (dim + 63) & ~(int64_t)63;
    int64_t off = 0;
    L.basis = off;
    off = a256(off + (int64_t)nblk * L.ld * nb * es);
    L.scratch = off;
    L.y = off;
    off = a256(off + dim * nb * es);
    L.w = off;
    off = a256(off + dim * nb * 8);
    L.partial = off;
    off = a256(off + (int64_t)nblk * nq * nbc * 8);
    L.sq = off;
    off = a256(off + nbc * 8);
    L.scal = off;
    off = a256(off + 64 * 8);
    L.coef = off;
    off = a256(off + (int64_t)(nblk + 4) * nq * 8);
    L.S = off;
    off = a256(off + (int64_t)o->n_iter * nb * o->n_keep * 8);
    L.ritz = off;
    off = a256(off + (int64_t)o->n_keep * dim * 8);
    L.hy = off;
    off = a256(off + dim * 8);
    L.total = off;
    return L;
}

// Device state and the steps shared by the standard and thick-restart drivers.
template <typename T>
struct Lz {
    const fotci_ham *h;
    hipStream_t st;
    int64_t dim, ld;
    int sb, cb, mode, hi_mode;
    T *basis, *scratch, *y;
    double *w, *partial, *sq, *scal, *coef, *Sd, *ritz, *hy;   // scal: [0] alpha [1] beta [2] norm [3] theta
                                                              // [4] resid [5] norm before reorthogonalisation
    double *hist;   // alpha_i, beta_i of the steps not yet read by the host (null in the block driver)
    int reorth;
    int second_passes = 0;

    Lz(const fotci_ham *h_, const Layout &L, int mode_, int reorth_, char *work, double *evecs, hipStream_t st_)
        : h(h_), st(st_), dim(h_->j->b->dim), ld(L.ld), sb(stream_blocks(dim)), cb(chunk_blocks(dim)),
          mode(mode_), hi_mode(mode_ == FOTCI_MODE_F64_PLAIN ? FOTCI_MODE_F64_PLAIN : FOTCI_MODE_F64),
          reorth(reorth_) {
        basis = (T *)(work + L.basis);
        scratch = (T *)(work + L.scratch);
        y = (T *)(work + L.y);
        w = (double *)(work + L.w);
        partial = (double *)(work + L.partial);
        sq = (double *)(work + L.sq);
        scal = (double *)(work + L.scal);
        coef = (double *)(work + L.coef);
        Sd = (double *)(work + L.S);
        ritz = evecs ? evecs : (double *)(work + L.ritz);
        hy = (double *)(work + L.hy);
        hist = L.hist ? (double *)(work + L.hist) : nullptr;
    }

    T *vec(int i) const { return basis + (int64_t)i * ld; }

    template <typename A, typename B>
    void dot_into(const A *a, const B *b, double *out, int take_sqrt) {
        hipLaunchKernelGGL((k_dot_partial<A, B>), dim3(sb), dim3(kThreads), 0, st, a, b, dim, partial);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, st, (const double *)partial, sb, out, take_sqrt);
    }

    // v_0 = pivot / ||pivot||
    void start(const double *pivot) {
        dot_into(pivot, pivot, scal + 2, 1);
        hipLaunchKernelGGL(k_scale_store<T>, dim3(sb), dim3(kThreads), 0, st, pivot, (const double *)(scal + 2),
                           basis, dim);
    }

    // One Lanczos step on v_i (Ch. 7, "Standard Lanczos algorithm"): y = H v_i,
    // alpha = <v_i, y>, w = y - alpha v_i - (beta v_{i-1} when three_term; the
    // arrow terms sum_mu s_mu v_mu, mu < n_arrow, after a thick restart), then
    // classical Gram-Schmidt twice against v_0..v_i and beta = ||w||.
    // Returns alpha and beta on the host.
    void step(int i, bool three_term, const std::vector<double> &arrow, double &alpha, double &beta) {
        issue(i, three_term, arrow);
        double ab[2];
        hip_check(hipMemcpyAsync(ab, scal, 16, hipMemcpyDeviceToHost, st), "lanczos copy");
        hip_check(hipStreamSynchronize(st), "lanczos sync");
        alpha = ab[0];
        beta = ab[1];
    }

    // The step without the round trip: alpha_i and beta_i also go to hist[2i],
    // hist[2i + 1], which the host reads for several steps at once (collect).
    // The next vector is w / beta computed on the device, so the host only has
    // to look at beta to stop at an invariant subspace, which it can do late:
    // steps after a breakdown work on garbage that is then discarded.
    void step_async(int i, bool three_term, const std::vector<double> &arrow) {
        issue(i, three_term, arrow);
        hip_check(hipMemcpyAsync(hist + 2 * i, scal, 16, hipMemcpyDeviceToDevice, st), "lanczos copy");
    }

    // alpha, beta of steps i0 <= i < i1 (issued with step_async) to the host
    void collect(int i0, int i1, std::vector<double> &ab) {
        ab.resize((size_t)2 * (i1 - i0));
        hip_check(hipMemcpyAsync(ab.data(), hist + 2 * i0, (size_t)16 * (i1 - i0), hipMemcpyDeviceToHost, st),
                  "lanczos copy");
        hip_check(hipStreamSynchronize(st), "lanczos sync");
    }

    void issue(int i, bool three_term, const std::vector<double> &arrow) {
        T *vi = vec(i);
        launch_apply(h, mode, vi, y, st);
        dot_into((const T *)vi, (const T *)y, scal + 0, 0);
        hipLaunchKernelGGL(k_three_term<T>, dim3(sb), dim3(kThreads), 0, st, (const T *)y, (const T *)vi,
                           (const T *)(three_term && i > 0 ? vi - ld : nullptr), (const double *)(scal + 0),
                           (const double *)(scal + 1), w, dim);
        if (!arrow.empty()) {
            const int na = (int)arrow.size();
            hip_check(hipMemcpyAsync(coef, arrow.data(), (size_t)na * 8, hipMemcpyHostToDevice, st), "arrow copy");
            hipLaunchKernelGGL(k_subtract<T>, dim3(cb), dim3(kThreads), (size_t)(na + kWaves) * 8, st,
                               (const T *)basis, ld, na, (const double *)coef, w, dim, (double *)nullptr);
        }
        // pass 1 (with DGKS also ||w|| before it); the subtract leaves ||w||^2 block sums in partial
        auto pass = [&](bool norm_before) {
            hipLaunchKernelGGL(k_multidot<T>, dim3(cb), dim3(kThreads), 0, st, (const T *)basis, ld, i + 1,
                               (const double *)w, dim, partial, norm_before ? sq : (double *)nullptr);
            hipLaunchKernelGGL(k_reduce_rows, dim3(i + 1), dim3(kThreads), 0, st, (const double *)partial, cb, coef);
            hipLaunchKernelGGL(k_subtract<T>, dim3(cb), dim3(kThreads), (size_t)(i + 1 + kWaves) * 8, st,
                               (const T *)basis, ld, i + 1, (const double *)coef, w, dim, partial);
            hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, st, (const double *)partial, cb, scal + 1, 1);
        };
        const bool dgks = reorth == FOTCI_REORTH_DGKS;
        pass(dgks);
        bool second = true;
        if (dgks) {
            hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, st, (const double *)sq, cb, scal + 5, 1);
            double nn[2];
            hip_check(hipMemcpyAsync(nn, scal + 1, 8, hipMemcpyDeviceToHost, st), "lanczos copy");
            hip_check(hipMemcpyAsync(nn + 1, scal + 5, 8, hipMemcpyDeviceToHost, st), "lanczos copy");
            hip_check(hipStreamSynchronize(st), "lanczos sync");
            second = nn[0] < 0.7071067811865476 * nn[1];
        }
        if (second) {
            pass(false);
            ++second_passes;
        }
        hip_check(hipGetLastError(), "lanczos launch");
    }

    // v_{i+1} = w / beta (beta in scal[1] from the last step)
    void store_next(int i) {
        hipLaunchKernelGGL(k_scale_store<T>, dim3(sb), dim3(kThreads), 0, st, (const double *)w,
                           (const double *)(scal + 1), vec(i + 1), dim);
    }

    // out_j = sum_{l<m} v_l Z[l, j0 + j] for j < nk, in chunks of 16 columns;
    // Z: host m x zc row-major.
    template <typename TO>
    void combine(int m, const std::vector<double> &Z, int zc, int nk, TO *out, int64_t out_ld) {
        hip_check(hipMemcpyAsync(Sd, Z.data(), (size_t)m * zc * 8, hipMemcpyHostToDevice, st), "coefficient copy");
        for (int j0 = 0; j0 < nk; j0 += 16) {
            const int nc = std::min(16, nk - j0);
            hipLaunchKernelGGL((k_ritz<T, TO>), dim3((int)((dim + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                               (const T *)basis, ld, m, (const double *)Sd, zc, j0, nc, out + (int64_t)j0 * out_ld,
                               out_ld, dim);
        }
        hip_check(hipGetLastError(), "combine launch");
    }

    // Ritz vectors of the lowest nk eigenpairs (theta ascending, columns of z,
    // m x m row-major) in float64, normalised; with refine, theta becomes the
    // float64 Rayleigh quotient; resid = ||H y - theta y||.
    void ritz_pairs(int m, const std::vector<double> &theta, const std::vector<double> &z, int nk, bool refine,
                    double *evals, double *resid) {
        std::vector<double> S((size_t)m * nk);
        for (int l = 0; l < m; ++l)
            for (int j = 0; j < nk; ++j) S[(size_t)l * nk + j] = z[(size_t)l * m + j];
        combine<double>(m, S, nk, nk, ritz, dim);
        finish_ritz(theta, nk, refine, evals, resid);
    }

    // The nk Ritz vectors in ritz (float64, one after another): normalised;
    // theta[j] replaced by the float64 Rayleigh quotient when refining;
    // resid[j] = ||H y - theta y||.
    void finish_ritz(const std::vector<double> &theta, int nk, bool refine, double *evals, double *resid) {
        for (int j = 0; j < nk; ++j) {
            double *yj = ritz + (int64_t)j * dim;
            dot_into((const double *)yj, (const double *)yj, scal + 2, 1);
            hipLaunchKernelGGL(k_scale_store<double>, dim3(sb), dim3(kThreads), 0, st, (const double *)yj,
                               (const double *)(scal + 2), yj, dim);
            launch_apply(h, hi_mode, yj, hy, st);
            if (refine) {
                dot_into((const double *)yj, (const double *)hy, scal + 3, 0);
            } else {
                hip_check(hipMemcpyAsync(scal + 3, &theta[j], 8, hipMemcpyHostToDevice, st), "theta copy");
            }
            hipLaunchKernelGGL(k_resid_partial, dim3(sb), dim3(kThreads), 0, st, (const double *)hy,
                               (const double *)yj, (const double *)(scal + 3), dim, partial);
            hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, st, (const double *)partial, sb, scal + 4, 1);
            double tr[2];
            hip_check(hipMemcpyAsync(tr, scal + 3, 16, hipMemcpyDeviceToHost, st), "ritz copy");
            hip_check(hipStreamSynchronize(st), "ritz sync");
            evals[j] = tr[0];
            resid[j] = tr[1];
        }
        hip_check(hipGetLastError(), "ritz launch");
    }
};

template <typename T>
void run(const fotci_ham *h, const fotci_lanczos_opts *o, const double *pivot, char *work, double *evals,
         double *resid, double *evecs, double *alpha_out, double *beta_out, hipStream_t st) {
    Lz<T> z(h, standard_layout(h, o), o->mode, o->reorth, work, evecs, st);
    z.start(pivot);
    std::vector<double> al, be, ab;
    const std::vector<double> none;
    double tnorm = 0.0;
    int k = 0;
    // false once the recurrence ends (last iteration or an invariant subspace)
    auto accept = [&](int i, double a, double b) -> bool {
        al.push_back(a);
        be.push_back(b);
        k = i + 1;
        tnorm = std::max(tnorm, std::fabs(a) + b + (i > 0 ? be[i - 1] : 0.0));
        return i < o->n_iter - 1 && b > 1e-12 * tnorm;
    };
    // the DGKS test needs the host inside every step; otherwise alpha and
    // beta are read every kLazySteps steps
    const bool lazy = o->reorth != FOTCI_REORTH_DGKS;
    int collected = 0;
    for (int i = 0; i < o->n_iter; ++i) {
        bool go = true;
        if (lazy) {
            z.step_async(i, true, none);
            if (i == o->n_iter - 1 || (i + 1) % kLazySteps == 0) {
                z.collect(collected, i + 1, ab);
                for (int j = collected; j <= i && go; ++j)
                    go = accept(j, ab[2 * (j - collected)], ab[2 * (j - collected) + 1]);
                collected = i + 1;
            }
        } else {
            double a, b;
            z.step(i, true, none, a, b);
            go = accept(i, a, b);
        }
        if (!go) break;
        z.store_next(i);
    }
    if (alpha_out)
        for (int i = 0; i < o->n_iter; ++i) alpha_out[i] = i < k ? al[i] : 0.0;
    if (beta_out)
        for (int i = 0; i < o->n_iter; ++i) beta_out[i] = i < (int)be.size() ? be[i] : 0.0;
    if (k < o->n_keep) fail(FOTCI_ENOTCONV, "Krylov space smaller than n_keep");
    std::vector<double> d(al.begin(), al.begin() + k), e(k > 1 ? k - 1 : 0), zz;
    for (int i = 0; i + 1 < k; ++i) e[i] = be[i];
    tridiag_eig(k, d, e, zz);
    z.ritz_pairs(k, d, zz, o->n_keep, o->refine != 0, evals, resid);
}

// Thick-restart Lanczos (Ch. 7, "Thick-restart Lanczos"). Each cycle extends
// the basis to n_basis + 1 vectors; the projected matrix T of the first
// n_basis vectors is diagonalised on the host; if the lowest n_keep Ritz
// pairs are not converged by the recurrence's estimate
// (|beta_last L[last, mu]| <= tol max(1, |E_mu|)),
// the n_thick lowest Ritz vectors become v_0..v_{nt-1}, the last Lanczos
// vector becomes v_nt, and T restarts as diag(E_mu) with the arrow column
// s_mu = beta_last L[last, mu] coupling them to v_nt. The first step after a
// restart subtracts the arrow terms instead of the three-term recurrence.
template <typename T>
void run_trlan(const fotci_ham *h, const fotci_trlan_opts *o, const double *pivot, char *work, double *evals,
               double *resid, double *evecs, int32_t *stats, hipStream_t st) {
    const Layout L = trlan_layout(h, o);
    Lz<T> z(h, L, o->mode, o->reorth, work, evecs, st);
    const int kb = o->n_basis, nt = o->n_thick;
    z.start(pivot);
    std::vector<double> Tm((size_t)(kb + 1) * (kb + 1), 0.0);
    auto TT = [&](int i, int j) -> double & { return Tm[(size_t)i * (kb + 1) + j]; };
    std::vector<double> arrow, ab;
    const bool lazy = o->reorth != FOTCI_REORTH_DGKS;   // as in the standard driver
    int j0 = 0, restarts = 0, applies = 0, converged = 0;
    double tnorm = 0.0;
    std::vector<double> theta, Z;
    int m = 0;
    for (;;) {
        m = kb;
        bool breakdown = false;
        // false at an invariant subspace: the Ritz pairs so far are exact
        auto accept = [&](int i, double a, double b) -> bool {
            TT(i, i) = a;
            TT(i, i + 1) = TT(i + 1, i) = b;
            double row = std::fabs(a) + b;
            for (int j = 0; j < i; ++j) row += std::fabs(TT(i, j));
            tnorm = std::max(tnorm, row);
            if (b > 1e-12 * tnorm) return true;
            m = i + 1;
            breakdown = true;
            return false;
        };
        int collected = j0;
        for (int i = j0; i < kb; ++i) {
            bool go = true;
            ++applies;
            if (lazy) {
                z.step_async(i, i > j0 || j0 == 0, i == j0 ? arrow : std::vector<double>());
                if (i == kb - 1 || (i + 1 - j0) % kLazySteps == 0) {
                    z.collect(collected, i + 1, ab);
                    for (int j = collected; j <= i && go; ++j)
                        go = accept(j, ab[2 * (j - collected)], ab[2 * (j - collected) + 1]);
                    collected = i + 1;
                }
            } else {
                double a, b;
                z.step(i, i > j0 || j0 == 0, i == j0 ? arrow : std::vector<double>(), a, b);
                go = accept(i, a, b);
            }
            if (!go) break;
            z.store_next(i);
        }
        std::vector<double> A((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) A[(size_t)i * m + j] = TT(i, j);
        sym_eig(m, A, theta, Z);
        const double blast = TT(m - 1, m);
        converged = 1;
        for (int mu = 0; mu < std::min(o->n_keep, m); ++mu)
            if (!(std::fabs(blast * Z[(size_t)(m - 1) * m + mu]) <= o->tol * std::max(1.0, std::fabs(theta[mu]))))
                converged = 0;
        if (breakdown) converged = m >= o->n_keep ? 1 : 0;
        if (converged || breakdown || restarts >= o->max_restarts) break;
        // restart: v'_mu = sum_i v_i Z[i, mu] for mu < nt (float64 sums, stored in the
        // basis precision), then v_m -> v_nt
        std::vector<double> Zt((size_t)m * nt);
        for (int i = 0; i < m; ++i)
            for (int mu = 0; mu < nt; ++mu) Zt[(size_t)i * nt + mu] = Z[(size_t)i * m + mu];
        z.template combine<T>(m, Zt, nt, nt, z.scratch, z.ld);
        hip_check(hipMemcpyAsync(z.basis, z.scratch, (size_t)nt * z.ld * sizeof(T), hipMemcpyDeviceToDevice, st),
                  "restart copy");
        hip_check(hipMemcpyAsync(z.vec(nt), z.vec(m), (size_t)z.dim * sizeof(T), hipMemcpyDeviceToDevice, st),
                  "restart copy");
        std::fill(Tm.begin(), Tm.end(), 0.0);
        arrow.assign(nt, 0.0);
        for (int mu = 0; mu < nt; ++mu) {
            TT(mu, mu) = theta[mu];
            arrow[mu] = blast * Z[(size_t)(m - 1) * m + mu];
            TT(mu, nt) = TT(nt, mu) = arrow[mu];
        }
        j0 = nt;
        ++restarts;
    }
    if (m < o->n_keep) fail(FOTCI_ENOTCONV, "Krylov space smaller than n_keep");
    z.ritz_pairs(m, theta, Z, o->n_keep, o->refine != 0, evals, resid);
    // The recurrence's estimate stops the cycles; the reported flag is the
    // true residual of the returned float64 Ritz vectors (H applied in
    // float64). With float32 storage these cannot fall far below
    // ~1e-7 ||H|| whatever the estimate says.
    for (int mu = 0; mu < o->n_keep; ++mu)
        if (!(resid[mu] <= o->tol * std::max(1.0, std::fabs(evals[mu])))) converged = 0;
    if (stats) {
        stats[0] = restarts;
        stats[1] = applies;
        stats[2] = converged;
    }
}

// Block Lanczos (Ch. "Block Lanczos"): H V_n = V_{n-1} B_{n-1}^T + V_n A_n +
// V_{n+1} B_n. Per block iteration: W = H V_n (block apply_H, widened to
// float64); A_n = V_n^T W, taken first as alpha is in the one-vector driver;
// W -= V_n A_n + V_{n-1} B_{n-1}^T; classical Gram-Schmidt against blocks
// 0..n, twice. The overlap O = W^T W = U Lambda U^T of the residual block
// gives B_n = Lambda^{1/2} U^T and V_{n+1} = W U Lambda^{-1/2}; the
// factorisation is repeated once on the new block (whose overlap is the
// identity to rounding) and B_n is the product of the two factors. Nearly
// dependent columns are replaced by new vectors (next_block); the iteration
// stops when the whole block is dependent on the basis. The block-tridiagonal
// T is diagonalised on the host.
template <typename T, int NB>
struct BlockRun {
    static constexpr int NQ = NB * NB;
    Lz<T> &z;
    hipStream_t st;
    int64_t dim, ldb;
    int gb, sbn;
    double *cg, *c3, *cm, *co;   // coefficient slots, see block_layout

    BlockRun(Lz<T> &z_, int n_iter)
        : z(z_), st(z_.st), dim(z_.dim), ldb(z_.ld * NB), gb((int)((z_.dim + bchunk<NB>() - 1) / bchunk<NB>())),
          sbn(stream_blocks(z_.dim)) {
        cg = z.coef;
        c3 = cg + (int64_t)(n_iter + 1) * NQ;
        cm = c3 + 2 * NQ;
        co = cm + NQ;
    }

    T *blk(int j) const { return z.basis + (int64_t)j * ldb; }

    // out[k*NQ] = V_j^T W for blocks 0..k-1 of V
    template <typename TV>
    void multidot(const TV *V, int64_t ld_v, int k, double *out) {
        hipLaunchKernelGGL((k_bmultidot<TV, NB>), dim3(gb), dim3(kThreads), 0, st, V, ld_v, k, (const double *)z.w,
                           dim, z.partial);
        hipLaunchKernelGGL(k_reduce_rows, dim3(k * NQ), dim3(kThreads), 0, st, (const double *)z.partial, gb, out);
    }

    // W -= sum_{j < k} V_{j0+j} C_j
    void subtract(int j0, int k, const double *C) {
        hipLaunchKernelGGL((k_bsubtract<T, NB>), dim3(gb), dim3(kThreads), 0, st, (const T *)blk(j0), ldb, k, C,
                           z.w, dim);
    }

    void to_host(double *host, const double *dev, int n) {
        hip_check(hipMemcpyAsync(host, dev, (size_t)n * 8, hipMemcpyDeviceToHost, st), "block copy");
    }
    void to_dev(double *dev, const double *host, int n) {
        hip_check(hipMemcpyAsync(dev, host, (size_t)n * 8, hipMemcpyHostToDevice, st), "block copy");
    }

    // O = W^T W on the host, exactly symmetric
    void overlap(std::vector<double> &O) {
        multidot<double>(z.w, 0, 1, co);
        O.assign(NQ, 0.0);
        to_host(O.data(), co, NQ);
        hip_check(hipStreamSynchronize(st), "block sync");
        for (int a = 0; a < NB; ++a)
            for (int b = 0; b < a; ++b) O[a * NB + b] = O[b * NB + a] = 0.5 * (O[a * NB + b] + O[b * NB + a]);
    }

    // O = U Lambda U^T: M = U Lambda^{-1/2}, B = Lambda^{1/2} U^T
    static void factor(const std::vector<double> &O, std::vector<double> &M, std::vector<double> &B, double &lmin,
                       double &lmax) {
        std::vector<double> lam, U;
        sym_eig(NB, O, lam, U);
        lmin = lam[0];
        lmax = lam[NB - 1];
        M.assign(NQ, 0.0);
        B.assign(NQ, 0.0);
        for (int v = 0; v < NB; ++v)
            for (int u = 0; u < NB; ++u) M[v * NB + u] = lam[u] > 0.0 ? U[v * NB + u] / std::sqrt(lam[u]) : 0.0;
        for (int a = 0; a < NB; ++a)
            for (int b = 0; b < NB; ++b) B[a * NB + b] = std::sqrt(std::max(lam[a], 0.0)) * U[b * NB + a];
    }

    // W (float64, unit-norm columns after the first mixing) -> block dst,
    // second factorisation; B = B2 * B1. False if an overlap eigenvalue is
    // <= floor.
    bool finish_block(int dst, const std::vector<double> &B1, double floor, std::vector<double> &B) {
        std::vector<double> O, M2, B2;
        double lmin, lmax;
        overlap(O);   // synchronises: earlier mixing has read cm
        factor(O, M2, B2, lmin, lmax);
        if (!(lmin > floor)) return false;
        to_dev(cm, M2.data(), NQ);
        hipLaunchKernelGGL((k_bmix<T, NB>), dim3(sbn), dim3(kThreads), 0, st, (const double *)z.w,
                           (const double *)cm, blk(dst), dim);
        B.assign(NQ, 0.0);
        for (int a = 0; a < NB; ++a)
            for (int c = 0; c < NB; ++c) {
                double t = 0.0;
                for (int b = 0; b < NB; ++b) t += B2[a * NB + b] * B1[b * NB + c];
                B[a * NB + c] = t;
            }
        hip_check(hipGetLastError(), "block launch");
        return true;
    }

    void mix_in_place(const std::vector<double> &M) {
        to_dev(cm, M.data(), NQ);
        hipLaunchKernelGGL((k_bmix<double, NB>), dim3(sbn), dim3(kThreads), 0, st, (const double *)z.w,
                           (const double *)cm, z.w, dim);
    }

    // The pivot block (in W) -> V_0; false if its columns are dependent.
    bool first_block() {
        std::vector<double> O, M1, B1, B;
        double lmin, lmax;
        overlap(O);
        factor(O, M1, B1, lmin, lmax);
        if (!(lmin > 1e-24 * lmax)) return false;
        mix_in_place(M1);
        return finish_block(0, B1, 0.0, B);
    }

    // The residual block W -> V_dst with W ~= V_dst B. A column whose overlap
    // eigenvalue has sqrt(lambda) <= 1e-7 ||T|| (the resolution of a Gram
    // matrix is about sqrt(eps) of the block's norm) is replaced by the basis
    // vector e_k, k = ((fills * NB + u) * 2654435761) mod dim, with a zero row
    // of B; after a replacement, or when a kept column has sqrt(lambda) <
    // 1e-4 ||T||, the block is orthogonalised against blocks 0..dst-1 again
    // (twice) before the second factorisation. False when every column is
    // dependent or the refreshed block has an overlap eigenvalue <= 1e-12.
    bool next_block(double tnorm, int dst, int &fills, std::vector<double> &B) {
        std::vector<double> O, lam, U;
        overlap(O);
        sym_eig(NB, O, lam, U);
        std::vector<double> M1(NQ, 0.0), B1(NQ, 0.0);
        int nbad = 0;
        double weakest = INFINITY;
        for (int u = 0; u < NB; ++u) {
            const double root = std::sqrt(std::max(lam[u], 0.0));
            if (root <= 1e-7 * tnorm) {
                ++nbad;
                continue;
            }
            weakest = std::min(weakest, root);
            for (int v = 0; v < NB; ++v) {
                M1[v * NB + u] = U[v * NB + u] / root;
                B1[u * NB + v] = root * U[v * NB + u];
            }
        }
        if (nbad == NB) return false;
        mix_in_place(M1);
        if (nbad > 0) {
            static const double one = 1.0;
            for (int u = 0; u < NB; ++u) {
                if (std::sqrt(std::max(lam[u], 0.0)) > 1e-7 * tnorm) continue;
                const uint64_t k = ((uint64_t)(fills * NB + u) * 2654435761ull) % (uint64_t)dim;
                hip_check(hipMemcpyAsync(z.w + k * NB + u, &one, 8, hipMemcpyHostToDevice, st), "restart vector");
            }
            ++fills;
        }
        if (nbad > 0 || weakest < 1e-4 * tnorm)
            for (int pass = 0; pass < 2; ++pass) {
                multidot<T>(blk(0), ldb, dst, cg);
                subtract(0, dst, cg);
            }
        return finish_block(dst, B1, 1e-12, B);
    }
};

double frob(const std::vector<double> &a) {
    double s = 0.0;
    for (double x : a) s += x * x;
    return std::sqrt(s);
}

template <typename T, int NB>
void run_block(const fotci_ham *h, const fotci_block_lanczos_opts *o, const double *pivot, char *work,
               double *evals, double *resid, double *evecs, int32_t *n_done, hipStream_t st) {
    constexpr int NQ = NB * NB;
    Lz<T> z(h, block_layout(h, o), o->mode, FOTCI_REORTH_CGS2, work, evecs, st);
    BlockRun<T, NB> b(z, o->n_iter);
    const int64_t dim = z.dim;
    // V_0 from the pivot block
    hip_check(hipMemcpyAsync(z.w, pivot, (size_t)dim * NB * 8, hipMemcpyDeviceToDevice, st), "pivot copy");
    if (!b.first_block()) fail(FOTCI_EINVAL, "pivot block columns are linearly dependent");
    std::vector<std::vector<double>> As, Bs;
    double tnorm = 0.0;
    int done = 0, fills = 0;
    for (int n = 0; n < o->n_iter; ++n) {
        launch_apply_nb(h, z.mode, NB, b.blk(n), z.y, st);
        hipLaunchKernelGGL(k_widen<T>, dim3(stream_blocks(dim * NB)), dim3(kThreads), 0, st, (const T *)z.y, z.w,
                           dim * NB);
        b.template multidot<T>(b.blk(n), b.ldb, 1, b.c3 + NQ);   // A_n
        if (n > 0) {
            std::vector<double> Bt(NQ);
            for (int v = 0; v < NB; ++v)
                for (int u = 0; u < NB; ++u) Bt[v * NB + u] = Bs[n - 1][u * NB + v];
            b.to_dev(b.c3, Bt.data(), NQ);
            b.subtract(n - 1, 2, b.c3);   // blocks n-1, n: coefficients B_{n-1}^T, A_n
        } else {
            b.subtract(0, 1, b.c3 + NQ);
        }
        for (int pass = 0; pass < 2; ++pass) {
            b.template multidot<T>(b.blk(0), b.ldb, n + 1, b.cg);
            b.subtract(0, n + 1, b.cg);
        }
        std::vector<double> A(NQ);
        b.to_host(A.data(), b.c3 + NQ, NQ);
        hip_check(hipStreamSynchronize(st), "block sync");
        for (int v = 0; v < NB; ++v)
            for (int u = 0; u < v; ++u) A[v * NB + u] = A[u * NB + v] = 0.5 * (A[v * NB + u] + A[u * NB + v]);
        As.push_back(A);
        done = n + 1;
        if (n == o->n_iter - 1) break;
        const double side = n > 0 ? frob(Bs[n - 1]) : 0.0;
        tnorm = std::max(tnorm, frob(A) + side);
        std::vector<double> Bn;
        if (!b.next_block(tnorm, n + 1, fills, Bn)) break;   // invariant block Krylov space
        Bs.push_back(Bn);
        tnorm = std::max(tnorm, frob(A) + side + frob(Bn));
    }
    const int m = done * NB;
    if (m < o->n_keep) fail(FOTCI_ENOTCONV, "block Krylov space smaller than n_keep");
    std::vector<double> Tm((size_t)m * m, 0.0);
    for (int j = 0; j < done; ++j)
        for (int a = 0; a < NB; ++a)
            for (int c = 0; c < NB; ++c) Tm[(size_t)(j * NB + a) * m + j * NB + c] = As[j][a * NB + c];
    for (int j = 0; j + 1 < done; ++j)
        for (int a = 0; a < NB; ++a)
            for (int c = 0; c < NB; ++c) {
                Tm[(size_t)((j + 1) * NB + a) * m + j * NB + c] = Bs[j][a * NB + c];
                Tm[(size_t)(j * NB + c) * m + (j + 1) * NB + a] = Bs[j][a * NB + c];
            }
    std::vector<double> theta, Zm;
    sym_eig(m, Tm, theta, Zm);
    const int nk = o->n_keep;
    std::vector<double> S((size_t)m * nk);
    for (int l = 0; l < m; ++l)
        for (int c = 0; c < nk; ++c) S[(size_t)l * nk + c] = Zm[(size_t)l * m + c];
    hip_check(hipMemcpyAsync(z.Sd, S.data(), S.size() * 8, hipMemcpyHostToDevice, st), "coefficient copy");
    for (int c0 = 0; c0 < nk; c0 += 16) {
        const int nc = std::min(16, nk - c0);
        hipLaunchKernelGGL((k_britz<T, NB>), dim3((int)((dim + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                           (const T *)b.blk(0), b.ldb, done, (const double *)z.Sd, nk, c0, nc, z.ritz + c0 * dim,
                           dim);
    }
    hip_check(hipGetLastError(), "ritz launch");
    z.finish_ritz(theta, nk, o->refine != 0, evals, resid);
    if (n_done) *n_done = done;
}

template <typename T>
void run_block_nb(const fotci_ham *h, const fotci_block_lanczos_opts *o, const double *pivot, char *work,
                  double *evals, double *resid, double *evecs, int32_t *n_done, hipStream_t st) {
    switch (o->n_block) {
        case 1: run_block<T, 1>(h, o, pivot, work, evals, resid, evecs, n_done, st); break;
        case 2: run_block<T, 2>(h, o, pivot, work, evals, resid, evecs, n_done, st); break;
        case 4: run_block<T, 4>(h, o, pivot, work, evals, resid, evecs, n_done, st); break;
        default: run_block<T, 8>(h, o, pivot, work, evals, resid, evecs, n_done, st); break;
    }
}

}  // namespace

int64_t lanczos_bytes(const fotci_ham *h, const fotci_lanczos_opts *o) { return standard_layout(h, o).total; }

void lanczos_run(const fotci_ham *h, const fotci_lanczos_opts *o, const double *pivot, void *work, int64_t work_bytes,
                 double *evals, double *resid, double *evecs, double *alpha, double *beta, void *stream) {
    if (o->n_keep < 1 || o->n_keep > 16) fail(FOTCI_EINVAL, "n_keep must be in 1..16");
    if (o->n_iter < o->n_keep || o->n_iter > kMaxIter) fail(FOTCI_EINVAL, "n_iter must be in n_keep..4096");
    if (o->reorth != FOTCI_REORTH_CGS2 && o->reorth != FOTCI_REORTH_DGKS) fail(FOTCI_EINVAL, "unknown reorth");
    if (work_bytes < lanczos_bytes(h, o)) fail(FOTCI_ENOMEM, "Lanczos workspace too small");
    if (((uintptr_t)work & 255u) != 0) fail(FOTCI_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    switch (o->mode) {
        case FOTCI_MODE_F64_PLAIN:
        case FOTCI_MODE_F64:
            run<double>(h, o, pivot, (char *)work, evals, resid, evecs, alpha, beta, st);
            break;
        case FOTCI_MODE_F32:
            run<float>(h, o, pivot, (char *)work, evals, resid, evecs, alpha, beta, st);
            break;
        default:
            fail(FOTCI_EINVAL, "unknown mode");
    }
}

void check_trlan_opts(const fotci_trlan_opts *o) {
    if (o->n_keep < 1 || o->n_keep > 16) fail(FOTCI_EINVAL, "n_keep must be in 1..16");
    if (o->n_thick < o->n_keep) fail(FOTCI_EINVAL, "n_thick must be at least n_keep");
    if (o->n_basis < o->n_thick + 2 || o->n_basis + 1 > kMaxIter)
        fail(FOTCI_EINVAL, "n_basis must be in n_thick+2..4095");
    if (o->max_restarts < 0) fail(FOTCI_EINVAL, "max_restarts must be >= 0");
    if (!(o->tol > 0.0)) fail(FOTCI_EINVAL, "tol must be positive");
    if (o->reorth != FOTCI_REORTH_CGS2 && o->reorth != FOTCI_REORTH_DGKS) fail(FOTCI_EINVAL, "unknown reorth");
    if (o->mode != FOTCI_MODE_F64 && o->mode != FOTCI_MODE_F64_PLAIN && o->mode != FOTCI_MODE_F32)
        fail(FOTCI_EINVAL, "unknown mode");
}

int64_t trlan_bytes(const fotci_ham *h, const fotci_trlan_opts *o) {
    check_trlan_opts(o);
    return trlan_layout(h, o).total;
}

void trlan_run(const fotci_ham *h, const fotci_trlan_opts *o, const double *pivot, void *work, int64_t work_bytes,
               double *evals, double *resid, double *evecs, int32_t *stats, void *stream) {
    check_trlan_opts(o);
    if (work_bytes < trlan_bytes(h, o)) fail(FOTCI_ENOMEM, "Lanczos workspace too small");
    if (((uintptr_t)work & 255u) != 0) fail(FOTCI_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    if (o->mode == FOTCI_MODE_F32)
        run_trlan<float>(h, o, pivot, (char *)work, evals, resid, evecs, stats, st);
    else
        run_trlan<double>(h, o, pivot, (char *)work, evals, resid, evecs, stats, st);
}

void check_block_opts(const fotci_block_lanczos_opts *o) {
    if (o->n_keep < 1 || o->n_keep > 16) fail(FOTCI_EINVAL, "n_keep must be in 1..16");
    if (o->n_block != 1 && o->n_block != 2 && o->n_block != 4 && o->n_block != 8)
        fail(FOTCI_EINVAL, "n_block must be 1, 2, 4 or 8");
    if (o->n_iter < 1 || (int64_t)o->n_iter * o->n_block > kMaxIter)
        fail(FOTCI_EINVAL, "n_iter must be >= 1 with n_iter * n_block <= 4096");
    if (o->mode != FOTCI_MODE_F64 && o->mode != FOTCI_MODE_F32)
        fail(FOTCI_EINVAL, "block Lanczos needs FOTCI_MODE_F64 or FOTCI_MODE_F32");
}

int64_t block_lanczos_bytes(const fotci_ham *h, const fotci_block_lanczos_opts *o) {
    check_block_opts(o);
    return block_layout(h, o).total;
}

void block_lanczos_run(const fotci_ham *h, const fotci_block_lanczos_opts *o, const double *pivot, void *work,
                       int64_t work_bytes, double *evals, double *resid, double *evecs, int32_t *n_done,
                       void *stream) {
    check_block_opts(o);
    if (work_bytes < block_lanczos_bytes(h, o)) fail(FOTCI_ENOMEM, "Lanczos workspace too small");
    if (((uintptr_t)work & 255u) != 0) fail(FOTCI_EINVAL, "workspace must be 256-byte aligned");
    if (((uintptr_t)pivot & 15u) != 0) fail(FOTCI_EINVAL, "pivot block must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    if (o->mode == FOTCI_MODE_F32)
        run_block_nb<float>(h, o, pivot, (char *)work, evals, resid, evecs, n_done, st);
    else
        run_block_nb<double>(h, o, pivot, (char *)work, evals, resid, evecs, n_done, st);
}

}  // namespace fotci
