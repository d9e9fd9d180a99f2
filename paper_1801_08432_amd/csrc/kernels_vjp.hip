// Adjoint of y = H(V) x for a scalar loss L = <g, y> (float64).
//
//   dL/dx = H g, since H is real symmetric;
//   dL/dV[label] = <g| O_label |x>: the label-wise transition density of the
//   operator string that V[label] multiplies (the m-scheme analogue of the
//   paper's two-body densities, Ch. 5 "Two-body densities": the expectation
//   value of a Hamiltonian with exactly one matrix element set to one).
// Each density is a sum over the same jumps apply_H uses:
//   pp: phase * <g row dst, x row src> per proton two-body jump;
//   nn: phase * <g column dst, x column src> per neutron two-body jump;
//   pn: phase_p phase_n g[ip',jn'] x[ip,jn] per pair of one-body jumps;
//   spe: <g, n_orbit x> from the row/column dots of the diagonal.
// Label bins receive float64 atomic adds (several jumps share a label).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fotci_internal.h"

namespace fotci {

namespace {

constexpr int kT = 256;

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

// Proton side, one block per destination proton SD ip: row dots against every
// source row of its two-body entries (diagonal included), the diagonal row dot
// for the proton single-particle energies, and the per-element products for
// the neutron diagonal (column sums, atomically).
__global__ __launch_bounds__(kT) void k_vjp_proton(DevHam P, const double *__restrict__ x,
                                                   const double *__restrict__ g, double *d_spe_p,
                                                   double *d_v_pp, double *dcol_n) {
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
    if (!d_v_pp) return;
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

// Neutron side, one block per destination neutron SD jn: column dots over the
// proton rows of its basis sector.
__global__ __launch_bounds__(kT) void k_vjp_neutron(DevHam P, const double *__restrict__ x,
                                                    const double *__restrict__ g, const double *dcol_n,
                                                    double *d_spe_n, double *d_v_nn) {
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
    if (!d_v_nn) return;
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

void launch_vjp(const DevHam &d, const fotci_ham *h, const double *x, const double *g, double *dx, double *d_spe_p,
                double *d_spe_n, double *d_v_pp, double *d_v_nn, double *d_v_pn, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (dx) launch_apply(h, FOTCI_MODE_F64, g, dx, stream);
    double *dcol = nullptr;
    const bool need_n = d_spe_n || d_v_nn;
    if (need_n) {
        // column sums of g o x per neutron SD, in the Hamiltonian's workspace
        dcol = d.scratch_ncol;
        hipLaunchKernelGGL(k_zero, dim3((d.n.n_sd + kT - 1) / kT), dim3(kT), 0, st, dcol, d.n.n_sd);
    }
    if (d_spe_p || d_v_pp || need_n)
        hipLaunchKernelGGL(k_vjp_proton, dim3(d.p.n_sd), dim3(kT), 0, st, d, x, g, d_spe_p, d_v_pp, dcol);
    if (need_n) hipLaunchKernelGGL(k_vjp_neutron, dim3(d.n.n_sd), dim3(kT), 0, st, d, x, g, (const double *)dcol,
                                   d_spe_n, d_v_nn);
    if (d_v_pn) {
        for (int q = 0; q < d.nq; ++q)
            if ((int64_t)h->j->cls.ops[q].size() * h->vq_nb[q] > kMaxBins)
                fail(FOTCI_EINVAL, "pn operator class too large for the adjoint kernel");
        hipLaunchKernelGGL(k_vjp_pn, dim3(d.p.n_sd * d.nq), dim3(kT), 0, st, d, x, g, d_v_pn);
    }
    hip_check(hipGetLastError(), "vjp launch");
}

}  // namespace fotci
