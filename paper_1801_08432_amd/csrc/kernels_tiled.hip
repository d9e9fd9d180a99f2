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
//            source neutron columns jn, K = proton jumps), staged in LDS 128
//            source columns at a time; the neutron one-body jumps whose
//            source lies in that chunk (pre-grouped by chunk, read coalesced)
//            then add phase_l R[B_l, jn_l] into the output row held in LDS.
//            This is the proton-first grouping of sum_{A,B} V_AB P_A X N_B^T:
//            the contraction over B is dense, so the matrix cores execute
//            about n_B / (neutron jumps per column) ~ 5 times the useful
//            multiply-adds of the pn part. Adds to y.
#include <hip/hip_runtime.h>

#include "fotci_internal.h"

namespace fotci {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;      // threads per workgroup (4 waves)
constexpr int kTile = 8;     // rows (nn kernel) / columns (pp kernel) per tile
constexpr int kCH = 128;     // source columns per LDS chunk of R
constexpr int kNB = 64;      // max neutron labels per class (rows of R)
constexpr int kKB = 32;      // proton jumps per contraction batch
constexpr int kLdsTile = 65536;  // bytes of LDS for a staged tile

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
    static __device__ __forceinline__ const double *nn_ell(const DevTiled &t) { return t.nn_ell_v64; }
    static __device__ __forceinline__ const double *pp_ell(const DevTiled &t) { return t.pp_ell_v64; }
};
template <>
struct TabT<float> {
    static __device__ __forceinline__ const float *diag(const DevSpecies &s) { return s.d32; }
    static __device__ __forceinline__ const float *vq(const DevHam &h) { return h.vq32; }
    static __device__ __forceinline__ const float *nn_ell(const DevTiled &t) { return t.nn_ell_v32; }
    static __device__ __forceinline__ const float *pp_ell(const DevTiled &t) { return t.pp_ell_v32; }
};

__global__ __launch_bounds__(kT) void k_ell_values(const int32_t *__restrict__ ent, const double *__restrict__ off,
                                                   double *__restrict__ v64, float *__restrict__ v32, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const int e = ent[i];
    const double v = e >= 0 ? off[e] : 0.0;
    v64[i] = v;
    v32[i] = (float)v;
}

// ------------------------------------------------------------ diagonal + nn
// RT rows are staged per pass (RT * max_nn * sizeof(T) <= 64 KiB).
template <typename T, int RT>
__global__ __launch_bounds__(kT) void k_nn_diag(DevHam P, DevTiled TT, const T *__restrict__ x, T *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *Xl = reinterpret_cast<T *>(smem_raw);   // Xl[c * RT + r]
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
        const T *xs = x + off + (int64_t)r0 * nn;
        __syncthreads();
        for (int idx = tid; idx < RT * nn; idx += kT) {
            const int r = idx / nn, c = idx - r * nn;
            Xl[c * RT + r] = r < nr ? xs[(int64_t)r * nn + c] : T(0);
        }
        T dp[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) dp[r] = r < nr ? dpa[pf + r0 + r] : T(0);
        __syncthreads();
        for (int c = tid; c < nn; c += kT) {
            T acc[RT];
            const T dnc = dn[nf + c];
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = (dp[r] + dnc) * Xl[c * RT + r];
            for (int e = 0; e < E; ++e) {
                const int64_t k = eb + (int64_t)e * nn + c;
                const int src = TT.nn_ell_src[k];
                const T v = ev[k];
                const T *xr = Xl + src * RT;
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r] += v * xr[r];
            }
#pragma unroll
            for (int r = 0; r < RT; ++r)
                if (r < nr) y[off + (int64_t)(r0 + r) * nn + c] = acc[r];
        }
    }
}

// ---------------------------------------------------------------------- pp
// CT columns are staged per pass (max_np * CT * sizeof(T) <= 64 KiB).
template <typename T, int CT>
__global__ __launch_bounds__(kT) void k_pp(DevHam P, DevTiled TT, const T *__restrict__ x, T *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *Xl = reinterpret_cast<T *>(smem_raw);   // Xl[r * CT + c]
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
        for (int idx = tid; idx < np * CT; idx += kT) {
            const int r = idx / CT, c = idx - r * CT;
            Xl[idx] = c < nc ? x[off + (int64_t)r * nn + c0 + c] : T(0);
        }
        __syncthreads();
        for (int r = tid; r < np; r += kT) {
            T acc[CT];
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[c] = 0;
            for (int e = 0; e < E; ++e) {
                const int64_t k = eb + (int64_t)e * np + r;
                const int src = TT.pp_ell_src[k];
                const T v = ev[k];
                const T *xr = Xl + src * CT;
#pragma unroll
                for (int c = 0; c < CT; ++c) acc[c] += v * xr[c];
            }
            T *yr = y + off + (int64_t)r * nn + c0;
#pragma unroll
            for (int c = 0; c < CT; ++c)
                if (c < nc) yr[c] += acc[c];
        }
    }
}

// ---------------------------------------------------------------------- pn
template <typename T>
__global__ __launch_bounds__(kT) void k_pn(DevHam P, DevTiled TT, const T *__restrict__ x, T *__restrict__ y) {
    typedef typename Mma<T>::acc_t acc_t;
    __shared__ T R[kNB * kCH];
    __shared__ T C[kNB * kKB];
    __shared__ int64_t srcb[kKB];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *yl = reinterpret_cast<T *>(smem_raw);   // output row [nn]

    const int ip = TT.order[blockIdx.x];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int s = P.p_sector[ip];
    const int nn = P.sec_nn[s];
    const int64_t base = P.p_pstart[ip];
    const int nq = P.nq;
    const int nch = TT.n_chunk;
    const T *vq = TabT<T>::vq(P);
    for (int c = tid; c < nn; c += kT) yl[c] = 0;
    bool any = false;
    for (int q = 0; q < nq; ++q) {
        const int a0 = P.p.ob_ptr[(int64_t)ip * nq + q], a1 = P.p.ob_ptr[(int64_t)ip * nq + q + 1];
        if (a0 == a1) continue;   // uniform across the workgroup
        any = true;
        const int qn = P.conjq[q];
        const int nB = P.vq_nb[q];
        const int nbt = (nB + 15) >> 4;
        const T *V = vq + P.vq_off[q];
        const int nns = P.sec_nn[P.p_sector[P.p.ob_src[a0]]];
        const int64_t pslot = ((int64_t)s * nq + qn) * nch;
        const int kp = a1 - a0;
        const int nbat = (kp + kKB - 1) / kKB;
        // stage the contraction operand C[B][k] = phase_k V^q[A_k, B] and the
        // source row offsets of one batch of proton jumps
        auto stage = [&](int kb0, int kn) {
            __syncthreads();
            for (int t = tid; t < kn; t += kT) srcb[t] = TT.p_ob_base[kb0 + t];
            for (int idx = tid; idx < kNB * kKB; idx += kT) {
                const int B = idx / kKB, k = idx - B * kKB;
                T v = 0;
                if (B < nB && k < kn) {
                    const int code = P.p.ob_code[kb0 + k];
                    v = V[(code >> 1) * nB + B];
                    if (code & 1) v = -v;
                }
                C[idx] = v;
            }
            __syncthreads();
        };
        if (nbat == 1) stage(a0, kp);
        for (int c0 = 0, ch = 0; c0 < nns; c0 += kCH, ++ch) {
            const int e0 = TT.pn_ptr[pslot + ch], e1 = TT.pn_ptr[pslot + ch + 1];
            if (e0 == e1) continue;   // no neutron jump starts in this chunk (uniform)
            acc_t t0[4], t1[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) t0[b] = t1[b] = Mma<T>::zero();
            for (int bat = 0; bat < nbat; ++bat) {
                const int kb0 = a0 + bat * kKB;
                const int kn = min(kKB, a1 - kb0);
                if (nbat > 1) stage(kb0, kn);
                const int ksteps = (kn + 3) >> 2;
                const int col0 = c0 + 16 * wid + (lane & 15);
                const int col1 = col0 + 64;
                for (int ks = 0; ks < ksteps; ++ks) {
                    const int k = 4 * ks + (lane >> 4);
                    T b0 = 0, b1 = 0;
                    if (k < kn) {
                        const int64_t sb = srcb[k];
                        if (col0 < nns) b0 = x[sb + col0];
                        if (col1 < nns) b1 = x[sb + col1];
                    }
#pragma unroll
                    for (int bt = 0; bt < 4; ++bt) {
                        if (bt < nbt) {
                            const T a = C[(16 * bt + (lane & 15)) * kKB + k];
                            t0[bt] = Mma<T>::mma(a, b0, t0[bt]);
                            t1[bt] = Mma<T>::mma(a, b1, t1[bt]);
                        }
                    }
                }
            }
            __syncthreads();   // the previous chunk's gather has finished reading R
#pragma unroll
            for (int bt = 0; bt < 4; ++bt) {
                if (bt < nbt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * bt + Mma<T>::row(lane, r);
                        R[row * kCH + 16 * wid + (lane & 15)] = t0[bt][r];
                        R[row * kCH + 64 + 16 * wid + (lane & 15)] = t1[bt][r];
                    }
                }
            }
            __syncthreads();
            for (int e = e0 + tid; e < e1; e += kT) {
                const uint32_t code = TT.pn_code[e];
                const T v = R[((code >> 1) & 63u) * kCH + ((code >> 7) & 127u)];
                atomicAdd(&yl[code >> 14], (code & 1u) ? -v : v);
            }
        }
    }
    if (!any) return;
    __syncthreads();
    for (int c = tid; c < nn; c += kT) y[base + c] += yl[c];
}

inline int pick_tile(int max_len, int elem) {
    int t = kTile;
    while (t > 1 && (int64_t)t * max_len * elem > kLdsTile) t >>= 1;
    return t;
}

template <typename T>
void launch_all(const DevHam &d, const DevTiled &t, const T *x, T *y, hipStream_t st) {
    const int rt = pick_tile(t.max_nn, sizeof(T));
    const size_t lds_nn = (size_t)rt * t.max_nn * sizeof(T);
    switch (rt) {
        case 8: hipLaunchKernelGGL((k_nn_diag<T, 8>), dim3(t.n_rtiles), dim3(kT), lds_nn, st, d, t, x, y); break;
        case 4: hipLaunchKernelGGL((k_nn_diag<T, 4>), dim3(t.n_rtiles), dim3(kT), lds_nn, st, d, t, x, y); break;
        case 2: hipLaunchKernelGGL((k_nn_diag<T, 2>), dim3(t.n_rtiles), dim3(kT), lds_nn, st, d, t, x, y); break;
        default: hipLaunchKernelGGL((k_nn_diag<T, 1>), dim3(t.n_rtiles), dim3(kT), lds_nn, st, d, t, x, y); break;
    }
    const int ct = pick_tile(t.max_np, sizeof(T));
    const size_t lds_pp = (size_t)ct * t.max_np * sizeof(T);
    switch (ct) {
        case 8: hipLaunchKernelGGL((k_pp<T, 8>), dim3(t.n_ctiles), dim3(kT), lds_pp, st, d, t, x, y); break;
        case 4: hipLaunchKernelGGL((k_pp<T, 4>), dim3(t.n_ctiles), dim3(kT), lds_pp, st, d, t, x, y); break;
        case 2: hipLaunchKernelGGL((k_pp<T, 2>), dim3(t.n_ctiles), dim3(kT), lds_pp, st, d, t, x, y); break;
        default: hipLaunchKernelGGL((k_pp<T, 1>), dim3(t.n_ctiles), dim3(kT), lds_pp, st, d, t, x, y); break;
    }
    hipLaunchKernelGGL(k_pn<T>, dim3(d.p.n_sd), dim3(kT), (size_t)t.max_nn * sizeof(T), st, d, t, x, y);
}

}  // namespace

void launch_materialize_tiled(const DevHam &d, const DevTiled &t, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (t.nn_ell_len > 0)
        hipLaunchKernelGGL(k_ell_values, dim3((unsigned)((t.nn_ell_len + kT - 1) / kT)), dim3(kT), 0, st,
                           t.nn_ell_ent, (const double *)d.n.off_val64, t.nn_ell_v64, t.nn_ell_v32, t.nn_ell_len);
    if (t.pp_ell_len > 0)
        hipLaunchKernelGGL(k_ell_values, dim3((unsigned)((t.pp_ell_len + kT - 1) / kT)), dim3(kT), 0, st,
                           t.pp_ell_ent, (const double *)d.p.off_val64, t.pp_ell_v64, t.pp_ell_v32, t.pp_ell_len);
    hip_check(hipGetLastError(), "materialize launch");
}

void launch_apply_tiled(const DevHam &d, const DevTiled &t, int mode, const void *x, void *y, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (d.p.n_sd == 0) return;
    if (!t.ok) fail(FOTCI_EINVAL, "basis too large for the tiled kernels (use FOTCI_MODE_F64_PLAIN)");
    if (mode == FOTCI_MODE_F64)
        launch_all<double>(d, t, (const double *)x, (double *)y, st);
    else
        launch_all<float>(d, t, (const float *)x, (float *)y, st);
    hip_check(hipGetLastError(), "apply launch");
}

}  // namespace fotci
