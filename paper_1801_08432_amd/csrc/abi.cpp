// extern "C" entry points of libfotci: argument checks, error capture (no C++
// exception crosses the ABI) and dispatch to the host setup and device code.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>

#include "fotci_internal.h"

namespace fotci {

namespace {
thread_local std::string g_last_error;
}

struct Thrown {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg) { throw Thrown{code, msg}; }
void set_error(const std::string &msg) { g_last_error = msg; }

template <typename F>
int guard(F &&f) {
    try {
        return f();
    } catch (const Thrown &t) {
        g_last_error = t.msg;
        return t.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return FOTCI_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return FOTCI_EINVAL;
    } catch (...) {
        g_last_error = "unknown error";
        return FOTCI_EINVAL;
    }
}

}  // namespace fotci

using namespace fotci;

extern "C" int fotci_build_basis_impl(int32_t, const int32_t *, const int32_t *, int32_t, int32_t, int32_t, int32_t,
                                      fotci_basis **);
extern "C" int fotci_build_jumps_impl(const fotci_basis *, fotci_jumps **);
extern "C" int fotci_set_interaction_impl(const fotci_jumps *, const double *, const double *, const double *,
                                          const double *, const double *, fotci_ham **);
extern "C" int64_t fotci_ham_workspace_bytes_impl(const fotci_ham *);
extern "C" int fotci_ham_upload_impl(fotci_ham *, void *, int64_t, void *);
extern "C" int fotci_ham_set_values_impl(fotci_ham *, const double *, const double *, const double *, const double *,
                                         const double *, void *);
extern "C" int fotci_ham_op_counts_impl(const fotci_ham *, int64_t *, int64_t *, int64_t *, int64_t *);
extern "C" int fotci_ham_pn_work_impl(const fotci_ham *, int32_t, int64_t *, int64_t *, int64_t *);
extern "C" int fotci_decouple_tbme_impl(int32_t, const int32_t *, const int32_t *, int32_t, const fotci_tbme *, int32_t,
                                        const fotci_tbme *, int32_t, const fotci_tbme *, double *, double *, double *);
extern "C" int fotci_ham_set_pn_private_rows_impl(fotci_ham *, int32_t);

extern "C" {

const char *fotci_last_error(void) { return g_last_error.c_str(); }
const char *fotci_version(void) { return "fotci 0.1 (gfx950)"; }

int fotci_build_basis(int32_t n_orbits, const int32_t *two_j, const int32_t *parity, int32_t Z, int32_t N,
                      int32_t two_M, int32_t parity_total, fotci_basis **out) {
    return guard([&] { return fotci_build_basis_impl(n_orbits, two_j, parity, Z, N, two_M, parity_total, out); });
}

void fotci_free_basis(fotci_basis *b) { delete b; }

int fotci_basis_info(const fotci_basis *b, int64_t *dim, int32_t *n_sectors, int32_t *n_psd, int32_t *n_nsd,
                     int32_t *n_states) {
    return guard([&] {
        if (!b) fail(FOTCI_EINVAL, "NULL handle");
        if (dim) *dim = b->dim;
        if (n_sectors) *n_sectors = (int32_t)b->sectors.size();
        if (n_psd) *n_psd = (int32_t)b->p.sd.size();
        if (n_nsd) *n_nsd = (int32_t)b->n.sd.size();
        if (n_states) *n_states = (int32_t)b->ms.size();
        return FOTCI_OK;
    });
}

int fotci_basis_export(const fotci_basis *b, uint32_t *p_bits, uint32_t *n_bits, int64_t *pstart, int64_t *nstart,
                       int64_t *sector_table) {
    return guard([&] {
        if (!b) fail(FOTCI_EINVAL, "NULL handle");
        if (p_bits) std::memcpy(p_bits, b->p.sd.data(), b->p.sd.size() * 4);
        if (n_bits) std::memcpy(n_bits, b->n.sd.data(), b->n.sd.size() * 4);
        if (pstart) std::memcpy(pstart, b->pstart.data(), b->pstart.size() * 8);
        if (nstart) std::memcpy(nstart, b->nstart.data(), b->nstart.size() * 8);
        if (sector_table)
            for (size_t s = 0; s < b->sectors.size(); ++s) {
                const auto &x = b->sectors[s];
                int64_t *r = sector_table + 7 * s;
                r[0] = x.two_mp;
                r[1] = x.parity_p;
                r[2] = x.p_first;
                r[3] = x.np;
                r[4] = x.n_first;
                r[5] = x.nn;
                r[6] = x.offset;
            }
        return FOTCI_OK;
    });
}

int fotci_build_jumps(const fotci_basis *b, fotci_jumps **out) {
    return guard([&] { return fotci_build_jumps_impl(b, out); });
}

void fotci_free_jumps(fotci_jumps *j) { delete j; }

int fotci_jumps_count(const fotci_jumps *j, int32_t kind, int64_t *count) {
    return guard([&] {
        if (!j || !count) fail(FOTCI_EINVAL, "NULL argument");
        if (kind < 0 || kind > 3) fail(FOTCI_EINVAL, "unknown jump kind");
        *count = (int64_t)j->rec[kind].size();
        return FOTCI_OK;
    });
}

int fotci_jumps_export(const fotci_jumps *j, int32_t kind, int32_t *src, int32_t *dst, int8_t *phase,
                       int32_t *label) {
    return guard([&] {
        if (!j) fail(FOTCI_EINVAL, "NULL handle");
        if (kind < 0 || kind > 3) fail(FOTCI_EINVAL, "unknown jump kind");
        const auto &r = j->rec[kind];
        for (size_t k = 0; k < r.size(); ++k) {
            if (src) src[k] = r[k].src;
            if (dst) dst[k] = r[k].dst;
            if (phase) phase[k] = r[k].phase;
            if (label) label[k] = r[k].label;
        }
        return FOTCI_OK;
    });
}

int fotci_set_interaction(const fotci_jumps *j, const double *spe_p, const double *spe_n, const double *v_pp,
                          const double *v_nn, const double *v_pn, fotci_ham **out) {
    return guard([&] { return fotci_set_interaction_impl(j, spe_p, spe_n, v_pp, v_nn, v_pn, out); });
}

void fotci_free_ham(fotci_ham *h) { delete h; }

int fotci_ham_set_values(fotci_ham *h, const double *spe_p, const double *spe_n, const double *v_pp,
                         const double *v_nn, const double *v_pn, void *stream) {
    return guard([&] { return fotci_ham_set_values_impl(h, spe_p, spe_n, v_pp, v_nn, v_pn, stream); });
}

int64_t fotci_ham_workspace_bytes(const fotci_ham *h) {
    int64_t r = 0;
    int rc = guard([&] {
        r = fotci_ham_workspace_bytes_impl(h);
        return FOTCI_OK;
    });
    return rc == FOTCI_OK ? r : rc;
}

int fotci_ham_upload(fotci_ham *h, void *ws, int64_t bytes, void *stream) {
    return guard([&] { return fotci_ham_upload_impl(h, ws, bytes, stream); });
}

int fotci_apply_H(const fotci_ham *h, int32_t mode, const void *x, void *y, void *stream) {
    return guard([&] {
        if (!h || !x || !y) fail(FOTCI_EINVAL, "NULL argument");
        if (!h->uploaded) fail(FOTCI_ESTATE, "Hamiltonian not uploaded");
        if (x == y) fail(FOTCI_EINVAL, "x and y must not overlap");
        launch_apply(h, mode, x, y, stream);
        return FOTCI_OK;
    });
}

int fotci_apply_H_block(const fotci_ham *h, int32_t mode, int32_t n_block, const void *x, void *y, void *stream) {
    return guard([&] {
        if (!h || !x || !y) fail(FOTCI_EINVAL, "NULL argument");
        if (n_block != 1 && n_block != 2 && n_block != 4 && n_block != 8)
            fail(FOTCI_EINVAL, "n_block must be 1, 2, 4 or 8");
        if (mode != FOTCI_MODE_F64 && mode != FOTCI_MODE_F32 && !(mode == FOTCI_MODE_F64_PLAIN && n_block == 1))
            fail(FOTCI_EINVAL, "block apply_H needs FOTCI_MODE_F64 or FOTCI_MODE_F32");
        if (!h->uploaded) fail(FOTCI_ESTATE, "Hamiltonian not uploaded");
        const int64_t es = mode == FOTCI_MODE_F32 ? 4 : 8;
        const int64_t bytes = h->j->b->dim * n_block * es;
        const char *xa = (const char *)x, *ya = (const char *)y;
        if (xa < ya + bytes && ya < xa + bytes) fail(FOTCI_EINVAL, "x and y must not overlap");
        launch_apply_nb(h, mode, n_block, x, y, stream);
        return FOTCI_OK;
    });
}

int fotci_apply_H_vjp(const fotci_ham *h, const double *x, const double *g, double *dx, double *d_spe_p,
                      double *d_spe_n, double *d_v_pp, double *d_v_nn, double *d_v_pn, void *stream) {
    return guard([&] {
        if (!h || !x || !g) fail(FOTCI_EINVAL, "NULL argument");
        if (!h->uploaded) fail(FOTCI_ESTATE, "Hamiltonian not uploaded");
        launch_vjp(h->dev, h, x, g, dx, d_spe_p, d_spe_n, d_v_pp, d_v_nn, d_v_pn, stream);
        return FOTCI_OK;
    });
}

int fotci_apply_H_vjp_static(const fotci_ham *h, const double *x, const double *g, double *dx, double *d_spe_p,
                             double *d_spe_n, double *d_v_pp, double *d_v_nn, double *d_v_pn, void *stream) {
    return guard([&] {
        if (!h || !x || !g) fail(FOTCI_EINVAL, "NULL argument");
        const int64_t n_nsd = (int64_t)h->j->b->n.sd.size();
        if (n_nsd > kStaticNcolMax)
            fail(FOTCI_EINVAL, "fotci_apply_H_vjp_static: " + std::to_string(n_nsd) +
                                   " neutron SDs exceed the static scratch of " + std::to_string(kStaticNcolMax) +
                                   " (use fotci_apply_H_vjp)");
        if (!h->uploaded) fail(FOTCI_ESTATE, "Hamiltonian not uploaded");
        double *ncol = static_ncol_scratch();
        launch_vjp(h->dev, h, x, g, dx, d_spe_p, d_spe_n, d_v_pp, d_v_nn, d_v_pn, stream, ncol);
        return FOTCI_OK;
    });
}

int fotci_one_body_density(const fotci_ham *h, const double *g, const double *x, double *rho_p, double *rho_n,
                           void *stream) {
    return guard([&] {
        if (!h || !x || !g) fail(FOTCI_EINVAL, "NULL argument");
        if (!h->uploaded) fail(FOTCI_ESTATE, "Hamiltonian not uploaded");
        const auto &cl = h->j->cls;
        int q0 = -1;
        for (int q = 0; q < cl.nq; ++q)
            if (cl.delta[q] == 0 && cl.rho[q] == 1) q0 = q;
        if (q0 < 0) fail(FOTCI_EINVAL, "no operator class conserves m and parity");
        launch_one_body_density(h->dev, h->tc.sec_np, q0, g, x, rho_p, rho_n, stream);
        return FOTCI_OK;
    });
}

int64_t fotci_lanczos_workspace_bytes(const fotci_ham *h, const fotci_lanczos_opts *o) {
    int64_t r = 0;
    int rc = guard([&] {
        if (!h || !o) fail(FOTCI_EINVAL, "NULL argument");
        if (o->n_iter < 1 || o->n_keep < 1) fail(FOTCI_EINVAL, "n_iter and n_keep must be positive");
        r = lanczos_bytes(h, o);
        return FOTCI_OK;
    });
    return rc == FOTCI_OK ? r : rc;
}

int fotci_lanczos_lowest(const fotci_ham *h, const fotci_lanczos_opts *o, const double *pivot, void *work,
                         int64_t work_bytes, double *evals, double *resid, double *evecs, double *alpha,
                         double *beta, void *stream) {
    return guard([&] {
        if (!h || !o || !pivot || !work || !evals || !resid) fail(FOTCI_EINVAL, "NULL argument");
        if (!h->uploaded) fail(FOTCI_ESTATE, "Hamiltonian not uploaded");
        lanczos_run(h, o, pivot, work, work_bytes, evals, resid, evecs, alpha, beta, stream);
        return FOTCI_OK;
    });
}

int64_t fotci_trlan_workspace_bytes(const fotci_ham *h, const fotci_trlan_opts *o) {
    int64_t r = 0;
    int rc = guard([&] {
        if (!h || !o) fail(FOTCI_EINVAL, "NULL argument");
        r = trlan_bytes(h, o);
        return FOTCI_OK;
    });
    return rc == FOTCI_OK ? r : rc;
}

int fotci_lanczos_thick_restart(const fotci_ham *h, const fotci_trlan_opts *o, const double *pivot, void *work,
                                int64_t work_bytes, double *evals, double *resid, double *evecs, int32_t *stats,
                                void *stream) {
    return guard([&] {
        if (!h || !o || !pivot || !work || !evals || !resid) fail(FOTCI_EINVAL, "NULL argument");
        if (!h->uploaded) fail(FOTCI_ESTATE, "Hamiltonian not uploaded");
        trlan_run(h, o, pivot, work, work_bytes, evals, resid, evecs, stats, stream);
        return FOTCI_OK;
    });
}

int64_t fotci_block_lanczos_workspace_bytes(const fotci_ham *h, const fotci_block_lanczos_opts *o) {
    int64_t r = 0;
    int rc = guard([&] {
        if (!h || !o) fail(FOTCI_EINVAL, "NULL argument");
        r = block_lanczos_bytes(h, o);
        return FOTCI_OK;
    });
    return rc == FOTCI_OK ? r : rc;
}

int fotci_lanczos_block(const fotci_ham *h, const fotci_block_lanczos_opts *o, const double *pivot, void *work,
                        int64_t work_bytes, double *evals, double *resid, double *evecs, int32_t *n_done,
                        void *stream) {
    return guard([&] {
        if (!h || !o || !pivot || !work || !evals || !resid) fail(FOTCI_EINVAL, "NULL argument");
        if (!h->uploaded) fail(FOTCI_ESTATE, "Hamiltonian not uploaded");
        block_lanczos_run(h, o, pivot, work, work_bytes, evals, resid, evecs, n_done, stream);
        return FOTCI_OK;
    });
}

int fotci_ham_op_counts(const fotci_ham *h, int64_t *ops_pp, int64_t *ops_nn, int64_t *ops_pn, int64_t *ops_diag) {
    return guard([&] { return fotci_ham_op_counts_impl(h, ops_pp, ops_nn, ops_pn, ops_diag); });
}

int fotci_decouple_tbme(int32_t n_orbits, const int32_t *two_j, const int32_t *parity, int32_t n_pp,
                        const fotci_tbme *pp, int32_t n_nn, const fotci_tbme *nn, int32_t n_pn, const fotci_tbme *pn,
                        double *v_pp, double *v_nn, double *v_pn) {
    return guard(
        [&] { return fotci_decouple_tbme_impl(n_orbits, two_j, parity, n_pp, pp, n_nn, nn, n_pn, pn, v_pp, v_nn, v_pn); });
}

int fotci_ham_pn_work(const fotci_ham *h, int32_t mode, int64_t *tile_visits, int64_t *mfma_instr,
                      int64_t *gather_slots) {
    return guard([&] { return fotci_ham_pn_work_impl(h, mode, tile_visits, mfma_instr, gather_slots); });
}

int fotci_ham_set_pn_private_rows(fotci_ham *h, int32_t enable) {
    return guard([&] { return fotci_ham_set_pn_private_rows_impl(h, enable); });
}

int fotci_profile_start(fotci_ham *h, int32_t max_calls) {
    return guard([&] {
        if (!h || max_calls < 1) fail(FOTCI_EINVAL, "bad argument");
        auto &pr = h->prof;
        for (void *e : pr.events) (void)hipEventDestroy((hipEvent_t)e);
        pr.events.assign((size_t)max_calls * 5, nullptr);
        for (auto &e : pr.events) {
            hipEvent_t ev;
            hip_check(hipEventCreate(&ev), "hipEventCreate");
            e = (void *)ev;
        }
        pr.max_calls = max_calls;
        pr.calls = 0;
        pr.n_kernels = 0;
        pr.on = true;
        return FOTCI_OK;
    });
}

int fotci_profile_stop(fotci_ham *h, double *avg_ms, const char **names, int32_t *n_kernels, int32_t *n_calls) {
    return guard([&] {
        if (!h) fail(FOTCI_EINVAL, "NULL handle");
        auto &pr = h->prof;
        pr.on = false;
        double acc[4] = {0, 0, 0, 0};
        for (int c = 0; c < pr.calls; ++c) {
            void **ev = &pr.events[(size_t)c * 5];
            hip_check(hipEventSynchronize((hipEvent_t)ev[pr.n_kernels]), "hipEventSynchronize");
            for (int k = 0; k < pr.n_kernels; ++k) {
                float ms = 0.f;
                hip_check(hipEventElapsedTime(&ms, (hipEvent_t)ev[k], (hipEvent_t)ev[k + 1]), "hipEventElapsedTime");
                acc[k] += ms;
            }
        }
        for (int k = 0; k < pr.n_kernels; ++k) {
            if (avg_ms) avg_ms[k] = pr.calls ? acc[k] / pr.calls : 0.0;
            if (names) names[k] = pr.names[k];
        }
        if (n_kernels) *n_kernels = pr.n_kernels;
        if (n_calls) *n_calls = pr.calls;
        for (void *e : pr.events) (void)hipEventDestroy((hipEvent_t)e);
        pr.events.clear();
        pr.calls = 0;
        return FOTCI_OK;
    });
}

int fotci_tridiag_eigh(int32_t n, const double *diag, const double *offdiag, double *evals, double *evecs) {
    return guard([&] {
        if (n < 1 || !diag || !evals) fail(FOTCI_EINVAL, "bad argument");
        std::vector<double> d(diag, diag + n), e(n > 1 ? n - 1 : 0), z;
        for (int i = 0; i + 1 < n; ++i) e[i] = offdiag[i];
        tridiag_eig(n, d, e, z);
        std::memcpy(evals, d.data(), (size_t)n * 8);
        if (evecs) std::memcpy(evecs, z.data(), (size_t)n * n * 8);
        return FOTCI_OK;
    });
}

int fotci_sym_eigh(int32_t n, const double *a, double *evals, double *evecs) {
    return guard([&] {
        if (n < 1 || !a || !evals) fail(FOTCI_EINVAL, "bad argument");
        std::vector<double> m(a, a + (size_t)n * n), d, z;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < i; ++j)
                if (m[(size_t)i * n + j] != m[(size_t)j * n + i]) fail(FOTCI_EINVAL, "matrix not symmetric");
        sym_eig(n, m, d, z);
        std::memcpy(evals, d.data(), (size_t)n * 8);
        if (evecs) std::memcpy(evecs, z.data(), (size_t)n * n * 8);
        return FOTCI_OK;
    });
}

}  // extern "C"
