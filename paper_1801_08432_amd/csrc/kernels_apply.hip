// apply_H kernels for gfx950 and the on-device formation of matrix elements.
//
// y = H x in the factorised basis (Ch. 2 "Representation of the Hamiltonian";
// Ch. 8 "Opbundles and optypes"): a sector block of x is the dense matrix
// X_s (np_s x nn_s, neutron index contiguous) and
//   Y_s = (d_p + d_n) o X_s                      diagonal (spe + diagonal pp/nn)
//       + H_pp^s X_s                             proton jumps, neutrons spectators
//       + X_s H_nn^{s T}                         neutron jumps, protons spectators
//       + sum_{A,B} V_AB P_A X_{s-Delta} N_B^T   pairs of one-body jumps (pn)
// Every kernel is destination-ordered: a thread owns output elements and
// gathers its inputs, so no atomics are needed and results are deterministic
// (the paper orders the final index to avoid races between threads; gathering
// through jumps stored in both directions is the GPU form of that).
#include <hip/hip_runtime.h>

#include "fotci_internal.h"

namespace fotci {

namespace {

// --------------------------------------------------------- materialisation
// merged off-diagonal pp/nn matrix element of one (dst, src) pair: the sum of
// phase x V[label] over the two-body jumps linking the two SDs.
__global__ __launch_bounds__(256) void k_mat_off(DevSpecies S) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S.n_off) return;
    double v = 0.0;
    for (int j = S.off_j0[k]; j < S.off_j1[k]; ++j) {
        const int c = S.code2[j];
        const double m = S.v2[c >> 1];
        v += (c & 1) ? -m : m;
    }
    S.off_val64[k] = v;
    S.off_val32[k] = (float)v;
}

// diagonal of one species: single-particle energies of the occupied m-states
// plus the diagonal two-body jumps.
__global__ __launch_bounds__(256) void k_mat_diag(DevSpecies S, int ns) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.n_sd) return;
    const uint32_t m = S.masks[i];
    double v = 0.0;
    for (int b = 0; b < ns; ++b)
        if ((m >> b) & 1u) v += S.eps[b];
    for (int j = S.diag_j0[i]; j < S.diag_j1[i]; ++j) {
        const int c = S.code2[j];
        const double x = S.v2[c >> 1];
        v += (c & 1) ? -x : x;
    }
    S.d64[i] = v;
    S.d32[i] = (float)v;
}

__global__ __launch_bounds__(256) void k_to_f32(const double *a, float *b, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------ plain apply
template <typename T>
struct Tab;
template <>
struct Tab<double> {
    static __device__ __forceinline__ const double *off(const DevSpecies &s) { return s.off_val64; }
    static __device__ __forceinline__ const double *diag(const DevSpecies &s) { return s.d64; }
    static __device__ __forceinline__ const double *vq(const DevHam &h) { return h.vq64; }
};
template <>
struct Tab<float> {
    static __device__ __forceinline__ const float *off(const DevSpecies &s) { return s.off_val32; }
    static __device__ __forceinline__ const float *diag(const DevSpecies &s) { return s.d32; }
    static __device__ __forceinline__ const float *vq(const DevHam &h) { return h.vq32; }
};

// One workgroup per destination proton SD ip; its threads stride over the
// neutron SDs jn of the conjugate sector and each computes y[pstart(ip)+jn]
// from the definition: diagonal, proton jumps into ip (whole-row gathers),
// neutron jumps into jn (gathers inside row ip), and every pair (proton
// one-body jump into ip) x (neutron one-body jump into jn) of conjugate
// classes (gathers anywhere in the source sector).
template <typename T>
__global__ __launch_bounds__(256) void k_apply_plain(DevHam P, const T *__restrict__ x, T *__restrict__ y) {
    const int ip = blockIdx.x;
    const int s = P.p_sector[ip];
    const int nn = P.sec_nn[s];
    const int nf = P.sec_nfirst[s];
    const int64_t base = P.p_pstart[ip];
    const T *offp = Tab<T>::off(P.p);
    const T *offn = Tab<T>::off(P.n);
    const T *dn = Tab<T>::diag(P.n);
    const T *vq = Tab<T>::vq(P);
    const T dpi = Tab<T>::diag(P.p)[ip];
    const int pp0 = P.p.off_rowptr[ip], pp1 = P.p.off_rowptr[ip + 1];
    const int nq = P.nq;
    for (int c = threadIdx.x; c < nn; c += blockDim.x) {
        const int jn = nf + c;
        T acc = (dpi + dn[jn]) * x[base + c];
        for (int k = pp0; k < pp1; ++k) acc += offp[k] * x[P.p_pstart[P.p.off_col[k]] + c];
        const int n0 = P.n.off_rowptr[jn], n1 = P.n.off_rowptr[jn + 1];
        for (int k = n0; k < n1; ++k) acc += offn[k] * x[base + P.n_local[P.n.off_col[k]]];
        for (int q = 0; q < nq; ++q) {
            const int a0 = P.p.ob_ptr[(int64_t)ip * nq + q], a1 = P.p.ob_ptr[(int64_t)ip * nq + q + 1];
            if (a0 == a1) continue;
            const int qn = P.conjq[q];
            const int b0 = P.n.ob_ptr[(int64_t)jn * nq + qn], b1 = P.n.ob_ptr[(int64_t)jn * nq + qn + 1];
            if (b0 == b1) continue;
            const T *V = vq + P.vq_off[q];
            const int nb = P.vq_nb[q];
            for (int ka = a0; ka < a1; ++ka) {
                const int ca = P.p.ob_code[ka];
                const T *Vrow = V + (ca >> 1) * nb;
                const int64_t rowbase = P.p_pstart[P.p.ob_src[ka]];
                T part = 0;
                for (int kb = b0; kb < b1; ++kb) {
                    const int cb = P.n.ob_code[kb];
                    const T v = Vrow[cb >> 1];
                    const T xv = x[rowbase + P.n_local[P.n.ob_src[kb]]];
                    part += (cb & 1) ? -v * xv : v * xv;
                }
                acc += (ca & 1) ? -part : part;
            }
        }
        y[base + c] = acc;
    }
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_materialize(const fotci_ham *h, void *stream) {
    const DevHam &d = h->dev;
    hipStream_t st = (hipStream_t)stream;
    for (const DevSpecies *s : {&d.p, &d.n}) {
        if (s->n_off > 0) hipLaunchKernelGGL(k_mat_off, dim3(blocks_for(s->n_off, 256)), dim3(256), 0, st, *s);
        if (s->n_sd > 0) hipLaunchKernelGGL(k_mat_diag, dim3(blocks_for(s->n_sd, 256)), dim3(256), 0, st, *s, d.ns);
    }
    if (d.n_vq > 0)
        hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(d.n_vq, 256)), dim3(256), 0, st, d.vq64, d.vq32, d.n_vq);
    hip_check(hipGetLastError(), "materialize launch");
    launch_materialize_tiled(d, h->dev_tiled, stream);
}

// The plain kernel in float64 (FOTCI_MODE_F64_PLAIN) or float32 (used for
// reference timings only).
void launch_apply_plain(const DevHam &d, int mode, const void *x, void *y, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int grid = d.p.n_sd;
    if (grid == 0) return;
    if (mode == FOTCI_MODE_F64_PLAIN)
        hipLaunchKernelGGL(k_apply_plain<double>, dim3(grid), dim3(256), 0, st, d, (const double *)x, (double *)y);
    else
        hipLaunchKernelGGL(k_apply_plain<float>, dim3(grid), dim3(256), 0, st, d, (const float *)x, (float *)y);
    hip_check(hipGetLastError(), "apply launch");
}

void launch_apply(const fotci_ham *h, int mode, const void *x, void *y, void *stream) {
    auto &pr = h->prof;
    void **ev = nullptr;
    if (pr.on && pr.calls < pr.max_calls) ev = &pr.events[(size_t)pr.calls * 5];
    switch (mode) {
        case FOTCI_MODE_F64_PLAIN:
            if (ev) hip_check(hipEventRecord((hipEvent_t)ev[0], (hipStream_t)stream), "event");
            launch_apply_plain(h->dev, mode, x, y, stream);
            if (ev) {
                hip_check(hipEventRecord((hipEvent_t)ev[1], (hipStream_t)stream), "event");
                pr.n_kernels = 1;
                pr.names[0] = "k_apply_plain";
            }
            break;
        case FOTCI_MODE_F64:
        case FOTCI_MODE_F32:
            launch_apply_tiled(h->dev, h->dev_tiled, mode, x, y, stream, ev);
            if (ev) {
                pr.n_kernels = 3;
                pr.names[0] = "k_nn_diag";
                pr.names[1] = "k_pp";
                pr.names[2] = "k_pn";
            }
            break;
        default:
            fail(FOTCI_EINVAL, "unknown or unsupported mode");
    }
    if (ev) pr.calls++;
}

void launch_apply_nb(const fotci_ham *h, int mode, int nb, const void *x, void *y, void *stream) {
    if (nb == 1) {
        launch_apply(h, mode, x, y, stream);
        return;
    }
    auto &pr = h->prof;
    void **ev = nullptr;
    if (pr.on && pr.calls < pr.max_calls) ev = &pr.events[(size_t)pr.calls * 5];
    launch_apply_block(h->dev, h->dev_tiled, mode, nb, x, y, stream, ev);
    if (ev) {
        pr.n_kernels = 3;
        pr.names[0] = "k_nn_diag_blk";
        pr.names[1] = "k_pp_blk";
        pr.names[2] = "k_pn";
        pr.calls++;
    }
}

}  // namespace fotci
