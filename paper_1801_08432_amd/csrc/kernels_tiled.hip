// Tiled apply_H for gfx950: one workgroup per destination proton SD, every
// part of H fused so that each output element is written once.
//
// For a destination row ip' (basis sector s', neutron columns jn' of the
// conjugate sector) the kernel accumulates, per output column:
//   diagonal  (d_p[ip'] + d_n[jn']) x[ip', jn'];
//   pp        sum over proton two-body entries into ip' of h x[ip, jn']
//             (whole-row, coalesced loads: neutrons are spectators);
//   nn        sum over neutron two-body entries into jn' of h x[ip', jn];
//   pn        for every operator class q (Jz change Delta of the proton
//             one-body operator, the neutron one opposite):
//               R[B, jn] = sum_k (phase_k V^q[A_k, B]) x[ip_k, jn]
//             over the K_p proton one-body jumps (ip_k -> ip', label A_k),
//             a dense contraction on the matrix cores (M = neutron labels B,
//             N = source neutron columns jn, K = proton jumps), staged in LDS
//             128 source columns at a time; then each output column gathers
//               y[ip', jn'] += sum_l phase_l R[B_l, jn_l]
//             over its neutron one-body jumps (jn_l -> jn', label B_l).
// This is the proton-first grouping of y += sum_{A,B} V_AB P_A X N_B^T
// (Ch. 2, "Representation of the Hamiltonian": the pn matrix element is
// rebuilt from one proton and one neutron jump). The contraction over B is
// dense, so the matrix cores execute about n_B / (neutron jumps per column)
// ~ 5 times the useful multiply-adds; the gathers read LDS only.
#include <hip/hip_runtime.h>

#include "fotci_internal.h"

namespace fotci {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;          // threads per workgroup (4 waves)
constexpr int kCols = 8;         // output columns per thread per column group
constexpr int kGroup = kT * kCols;
constexpr int kCH = 128;         // source columns per LDS chunk of R
constexpr int kNB = 64;          // max neutron labels per class (rows of R)
constexpr int kKB = 32;          // proton jumps per contraction batch

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
    static __device__ __forceinline__ const double *off(const DevSpecies &s) { return s.off_val64; }
    static __device__ __forceinline__ const double *diag(const DevSpecies &s) { return s.d64; }
    static __device__ __forceinline__ const double *vq(const DevHam &h) { return h.vq64; }
};
template <>
struct TabT<float> {
    static __device__ __forceinline__ const float *off(const DevSpecies &s) { return s.off_val32; }
    static __device__ __forceinline__ const float *diag(const DevSpecies &s) { return s.d32; }
    static __device__ __forceinline__ const float *vq(const DevHam &h) { return h.vq32; }
};

template <typename T>
__global__ __launch_bounds__(kT) void k_apply_tiled(DevHam P, DevTiled TT, const T *__restrict__ x,
                                                    T *__restrict__ y) {
    typedef typename Mma<T>::acc_t acc_t;
    __shared__ T R[kNB * kCH];
    __shared__ T C[kNB * kKB];
    __shared__ int64_t srcb[kKB];

    const int ip = TT.order ? TT.order[blockIdx.x] : blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int s = P.p_sector[ip];
    const int nn = P.sec_nn[s], nf = P.sec_nfirst[s];
    const int64_t base = P.p_pstart[ip];
    const int nq = P.nq;
    const T *offp = TabT<T>::off(P.p);
    const T *offn = TabT<T>::off(P.n);
    const T *dn = TabT<T>::diag(P.n);
    const T *vq = TabT<T>::vq(P);
    const T dpi = TabT<T>::diag(P.p)[ip];
    const int pp0 = P.p.off_rowptr[ip], pp1 = P.p.off_rowptr[ip + 1];

    for (int g0 = 0; g0 < nn; g0 += kGroup) {
        T acc[kCols];
        // diagonal, pp and nn
#pragma unroll
        for (int i = 0; i < kCols; ++i) {
            const int c = g0 + tid + i * kT;
            acc[i] = 0;
            if (c < nn) {
                const int jn = nf + c;
                T a = (dpi + dn[jn]) * x[base + c];
                const int n0 = P.n.off_rowptr[jn], n1 = P.n.off_rowptr[jn + 1];
                for (int k = n0; k < n1; ++k) a += offn[k] * x[base + TT.n_off_local[k]];
                acc[i] = a;
            }
        }
        for (int k = pp0; k < pp1; ++k) {
            const T h = offp[k];
            const int64_t sb = TT.p_off_base[k];
#pragma unroll
            for (int i = 0; i < kCols; ++i) {
                const int c = g0 + tid + i * kT;
                if (c < nn) acc[i] += h * x[sb + c];
            }
        }
        // pn, class by class
        for (int q = 0; q < nq; ++q) {
            const int a0 = P.p.ob_ptr[(int64_t)ip * nq + q], a1 = P.p.ob_ptr[(int64_t)ip * nq + q + 1];
            if (a0 == a1) continue;   // uniform across the workgroup
            const int qn = P.conjq[q];
            const int nB = P.vq_nb[q];
            const int nbt = (nB + 15) >> 4;
            const T *V = vq + P.vq_off[q];
            const int ssrc = P.p_sector[P.p.ob_src[a0]];
            const int nns = P.sec_nn[ssrc];
            int pb[kCols], pe[kCols];
#pragma unroll
            for (int i = 0; i < kCols; ++i) {
                const int c = g0 + tid + i * kT;
                pb[i] = pe[i] = 0;
                if (c < nn) {
                    const int64_t r = (int64_t)(nf + c) * nq + qn;
                    pb[i] = P.n.ob_ptr[r];
                    pe[i] = P.n.ob_ptr[r + 1];
                }
            }
            const int kp = a1 - a0;
            const int nbat = (kp + kKB - 1) / kKB;
            for (int c0 = 0; c0 < nns; c0 += kCH) {
                acc_t t0[4], t1[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) t0[b] = t1[b] = Mma<T>::zero();
                for (int bat = 0; bat < nbat; ++bat) {
                    const int kb0 = a0 + bat * kKB;
                    const int kn = min(kKB, a1 - kb0);
                    if (nbat > 1 || c0 == 0) {
                        __syncthreads();
                        for (int t = tid; t < kn; t += kT) srcb[t] = TT.p_ob_base[kb0 + t];
                        for (int idx = tid; idx < kNB * kKB; idx += kT) {
                            const int B = idx / kKB, k = idx % kKB;
                            T v = 0;
                            if (B < nB && k < kn) {
                                const int code = P.p.ob_code[kb0 + k];
                                v = V[(code >> 1) * nB + B];
                                if (code & 1) v = -v;
                            }
                            C[idx] = v;
                        }
                        __syncthreads();
                    }
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
                // R[B][jn - c0]: each lane holds four rows of a 16x16 block, column lane%16
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
                const int cend = c0 + kCH;
#pragma unroll
                for (int i = 0; i < kCols; ++i) {
                    T a = 0;
                    int p = pb[i];
                    while (p < pe[i]) {
                        const int code = TT.n_ob_code[p];
                        const int src = code >> 11;
                        if (src >= cend) break;
                        const T v = R[((code >> 1) & 1023) * kCH + (src - c0)];
                        a += (code & 1) ? -v : v;
                        ++p;
                    }
                    pb[i] = p;
                    acc[i] += a;
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int i = 0; i < kCols; ++i) {
            const int c = g0 + tid + i * kT;
            if (c < nn) y[base + c] = acc[i];
        }
    }
}

}  // namespace

void launch_apply_tiled(const DevHam &d, const DevTiled &t, int mode, const void *x, void *y, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int grid = d.p.n_sd;
    if (grid == 0) return;
    if (!t.ok) fail(FOTCI_EINVAL, "operator classes too large for the tiled kernels (use FOTCI_MODE_F64_PLAIN)");
    if (mode == FOTCI_MODE_F64)
        hipLaunchKernelGGL(k_apply_tiled<double>, dim3(grid), dim3(kT), 0, st, d, t, (const double *)x, (double *)y);
    else
        hipLaunchKernelGGL(k_apply_tiled<float>, dim3(grid), dim3(kT), 0, st, d, t, (const float *)x, (float *)y);
    hip_check(hipGetLastError(), "apply launch");
}

}  // namespace fotci
