/*
 * CPU oracle, C part -- TEST INFRASTRUCTURE ONLY (tests, smoke check and the
 * benchmark's CPU-baseline leg). The GPU library never links or calls it.
 *
 * The same definitions as oracle/hamiltonian.py, in plain C with OpenMP, for
 * workloads too large for Python loops:
 *
 *   H = sum_i eps_p[i] n_i(p) + sum_i eps_n[i] n_i(n)
 *     + sum_{a<b,c<d} V_pp[(ab),(cd)] p+_a p+_b p_d p_c   (and nn alike)
 *     + sum_{abcd} V_pn[(a b),(c d)] (p+_a p_c)(n+_b n_d)
 *
 * (the M-scheme form of the standard one- plus two-body Hamiltonian, eq.
 * hamdef of App. A), acting on occupation bit strings with the fermion sign
 * (-1)^(occupied states of lower index) (Ch. 2, "Representation of the
 * basis"). The basis is the factorised proton x neutron one: index =
 * pstart(ip) + nstart(jn) (Ch. 2 "factorization of the basis", Ch. 6 ".bas"
 * pseudocode); the caller passes the kept SDs and the sector table.
 *
 * orc_apply_h: y[t] = sum_s <t|H|s> x[s] for rows t in [row0,row1). Each row
 *   applies H to |t> and uses <t|H|s> = <s|H|t>, which holds because the
 *   caller passes exactly symmetric real V (checked on the Python side).
 * orc_densities: for every operator string O_L of H (each label L of each
 *   term), bins[L] += <g|O_L|x>, pushing column by column with per-thread
 *   bins. Labels that conserve 2M and parity are all visited, whatever V is.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static inline int sgn_below(uint32_t m, int i)
{
    return (__builtin_popcount(m & ((1u << i) - 1u)) & 1) ? -1 : 1;
}

/* p+_a p+_b p_d p_c |m> : returns sign (0 when the result vanishes). */
static inline int op_two_body(uint32_t m, int a, int b, int c, int d, uint32_t *out)
{
    int s;
    if (!((m >> c) & 1u)) return 0;
    s = sgn_below(m, c); m &= ~(1u << c);
    if (!((m >> d) & 1u)) return 0;
    s *= sgn_below(m, d); m &= ~(1u << d);
    if ((m >> b) & 1u) return 0;
    s *= sgn_below(m, b); m |= 1u << b;
    if ((m >> a) & 1u) return 0;
    s *= sgn_below(m, a); m |= 1u << a;
    *out = m;
    return s;
}

/* p+_a p_c |m> */
static inline int op_one_body(uint32_t m, int a, int c, uint32_t *out)
{
    int s;
    if (!((m >> c) & 1u)) return 0;
    s = sgn_below(m, c); m &= ~(1u << c);
    if ((m >> a) & 1u) return 0;
    s *= sgn_below(m, a); m |= 1u << a;
    *out = m;
    return s;
}

typedef struct {
    int ns, npairs;
    int *pa, *pb;          /* pair r -> (a, b), a<b */
    int *pidx;             /* ns*ns -> pair index or -1 */
    int32_t *p_rank, *n_rank;   /* mask -> kept SD index or -1, size 2^ns */
    int64_t *pstart, *nstart;
    int n_sectors;
    const int64_t *sectab; /* n_sectors x 7: 2Mp, par, pf, np, nf, nn, off */
} ctx_t;

static int ctx_init(ctx_t *c, int ns, int n_sectors, const int64_t *sectab,
                    int n_psd, const uint32_t *p_masks, int n_nsd, const uint32_t *n_masks)
{
    int r = 0;
    c->ns = ns;
    c->npairs = ns * (ns - 1) / 2;
    c->pa = (int *)malloc(sizeof(int) * (size_t)c->npairs);
    c->pb = (int *)malloc(sizeof(int) * (size_t)c->npairs);
    c->pidx = (int *)malloc(sizeof(int) * (size_t)ns * ns);
    c->p_rank = (int32_t *)malloc(sizeof(int32_t) * ((size_t)1 << ns));
    c->n_rank = (int32_t *)malloc(sizeof(int32_t) * ((size_t)1 << ns));
    c->pstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_psd > 0 ? n_psd : 1));
    c->nstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_nsd > 0 ? n_nsd : 1));
    c->n_sectors = n_sectors;
    c->sectab = sectab;
    for (int i = 0; i < ns * ns; ++i) c->pidx[i] = -1;
    for (int a = 0; a < ns; ++a)
        for (int b = a + 1; b < ns; ++b) {
            c->pa[r] = a; c->pb[r] = b;
            c->pidx[a * ns + b] = r;
            ++r;
        }
    for (size_t m = 0; m < ((size_t)1 << ns); ++m) { c->p_rank[m] = -1; c->n_rank[m] = -1; }
    for (int i = 0; i < n_psd; ++i) c->p_rank[p_masks[i]] = i;
    for (int i = 0; i < n_nsd; ++i) c->n_rank[n_masks[i]] = i;
    for (int s = 0; s < n_sectors; ++s) {
        const int64_t *t = sectab + 7 * s;
        for (int64_t k = 0; k < t[3]; ++k) c->pstart[t[2] + k] = t[6] + k * t[5];
        for (int64_t k = 0; k < t[5]; ++k) c->nstart[t[4] + k] = k;
    }
    return 0;
}

static void ctx_free(ctx_t *c)
{
    free(c->pa); free(c->pb); free(c->pidx); free(c->p_rank); free(c->n_rank);
    free(c->pstart); free(c->nstart);
}

static inline int find_sector(const ctx_t *c, int64_t t)
{
    int lo = 0, hi = c->n_sectors - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (c->sectab[7 * mid + 6] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Column lists of nonzero V entries: for column col, rows list[ptr[col]..ptr[col+1]). */
static void nz_columns(const double *v, int n, int **ptr_out, int **rows_out)
{
    int *ptr = (int *)calloc((size_t)n + 1, sizeof(int));
    int cnt = 0;
    for (int col = 0; col < n; ++col) {
        ptr[col] = cnt;
        for (int row = 0; row < n; ++row) if (v[(size_t)row * n + col] != 0.0) ++cnt;
    }
    ptr[n] = cnt;
    int *rows = (int *)malloc(sizeof(int) * (size_t)(cnt > 0 ? cnt : 1));
    cnt = 0;
    for (int col = 0; col < n; ++col)
        for (int row = 0; row < n; ++row) if (v[(size_t)row * n + col] != 0.0) rows[cnt++] = row;
    *ptr_out = ptr;
    *rows_out = rows;
}

int orc_apply_h(int ns, const double *eps_p, const double *eps_n,
                const double *v_pp, const double *v_nn, const double *v_pn,
                int n_sectors, const int64_t *sectab,
                int n_psd, const uint32_t *p_masks, int n_nsd, const uint32_t *n_masks,
                const double *x, double *y, int64_t row0, int64_t row1, int nthreads)
{
    ctx_t c;
    int *pp_ptr, *pp_rows, *nn_ptr, *nn_rows, *pn_ptr, *pn_rows;
    int bad = 0;
    ctx_init(&c, ns, n_sectors, sectab, n_psd, p_masks, n_nsd, n_masks);
    nz_columns(v_pp, c.npairs, &pp_ptr, &pp_rows);
    nz_columns(v_nn, c.npairs, &nn_ptr, &nn_rows);
    nz_columns(v_pn, ns * ns, &pn_ptr, &pn_rows);
    if (nthreads > 0) omp_set_num_threads(nthreads);

#pragma omp parallel for schedule(dynamic, 256) reduction(|:bad)
    for (int64_t t = row0; t < row1; ++t) {
        int s = find_sector(&c, t);
        const int64_t *st = sectab + 7 * s;
        int64_t loc = t - st[6];
        int ip = (int)(st[2] + loc / st[5]);
        int jn = (int)(st[4] + loc % st[5]);
        uint32_t pm = p_masks[ip], nm = n_masks[jn];
        double acc = 0.0, d = 0.0;
        int occp[32], occn[32], np_ = 0, nn_ = 0;
        for (int i = 0; i < ns; ++i) {
            if ((pm >> i) & 1u) { occp[np_++] = i; d += eps_p[i]; }
            if ((nm >> i) & 1u) { occn[nn_++] = i; d += eps_n[i]; }
        }
        acc = d * x[t];
        /* pp */
        for (int i1 = 0; i1 < np_; ++i1)
            for (int i2 = i1 + 1; i2 < np_; ++i2) {
                int col = c.pidx[occp[i1] * ns + occp[i2]];
                for (int k = pp_ptr[col]; k < pp_ptr[col + 1]; ++k) {
                    int row = pp_rows[k];
                    uint32_t m2;
                    int sg = op_two_body(pm, c.pa[row], c.pb[row], occp[i1], occp[i2], &m2);
                    if (!sg) continue;
                    int r = c.p_rank[m2];
                    if (r < 0) { bad = 1; continue; }
                    acc += sg * v_pp[(size_t)row * c.npairs + col] * x[c.pstart[r] + c.nstart[jn]];
                }
            }
        /* nn */
        for (int i1 = 0; i1 < nn_; ++i1)
            for (int i2 = i1 + 1; i2 < nn_; ++i2) {
                int col = c.pidx[occn[i1] * ns + occn[i2]];
                for (int k = nn_ptr[col]; k < nn_ptr[col + 1]; ++k) {
                    int row = nn_rows[k];
                    uint32_t m2;
                    int sg = op_two_body(nm, c.pa[row], c.pb[row], occn[i1], occn[i2], &m2);
                    if (!sg) continue;
                    int r = c.n_rank[m2];
                    if (r < 0) { bad = 1; continue; }
                    acc += sg * v_nn[(size_t)row * c.npairs + col] * x[c.pstart[ip] + c.nstart[r]];
                }
            }
        /* pn */
        for (int i1 = 0; i1 < np_; ++i1)
            for (int i2 = 0; i2 < nn_; ++i2) {
                int cp = occp[i1], dn = occn[i2];
                int col = cp * ns + dn;
                for (int k = pn_ptr[col]; k < pn_ptr[col + 1]; ++k) {
                    int row = pn_rows[k];
                    int a = row / ns, b = row % ns;
                    uint32_t pm2, nm2;
                    int sp = op_one_body(pm, a, cp, &pm2);
                    if (!sp) continue;
                    int sn = op_one_body(nm, b, dn, &nm2);
                    if (!sn) continue;
                    int rp = c.p_rank[pm2], rn = c.n_rank[nm2];
                    if (rp < 0 || rn < 0) { bad = 1; continue; }
                    acc += sp * sn * v_pn[(size_t)row * ns * ns + col] * x[c.pstart[rp] + c.nstart[rn]];
                }
            }
        y[t - row0] = acc;
    }
    free(pp_ptr); free(pp_rows); free(nn_ptr); free(nn_rows); free(pn_ptr); free(pn_rows);
    ctx_free(&c);
    return bad ? -1 : 0;
}

/* bins layout: [eps_p: ns][eps_n: ns][v_pp: npairs^2][v_nn: npairs^2][v_pn: ns^4] */
int orc_densities(int ns, const int *two_m, const int *par,
                  int n_sectors, const int64_t *sectab,
                  int n_psd, const uint32_t *p_masks, int n_nsd, const uint32_t *n_masks,
                  const double *g, const double *x, double *bins, int nthreads)
{
    ctx_t c;
    int bad = 0;
    ctx_init(&c, ns, n_sectors, sectab, n_psd, p_masks, n_nsd, n_masks);
    const int np2 = c.npairs * c.npairs;
    const size_t nbins = (size_t)2 * ns + 2 * (size_t)np2 + (size_t)ns * ns * ns * ns;
    const int64_t dim = sectab[7 * (n_sectors - 1) + 6] + sectab[7 * (n_sectors - 1) + 3] * sectab[7 * (n_sectors - 1) + 5];
    if (nthreads > 0) omp_set_num_threads(nthreads);
    memset(bins, 0, sizeof(double) * nbins);

#pragma omp parallel reduction(|:bad)
    {
        double *loc = (double *)calloc(nbins, sizeof(double));
        double *b_ep = loc, *b_en = loc + ns, *b_pp = loc + 2 * ns, *b_nn = b_pp + np2, *b_pn = b_nn + np2;
#pragma omp for schedule(dynamic, 256)
        for (int64_t s = 0; s < dim; ++s) {
            double xs = x[s];
            if (xs == 0.0) continue;
            int sec = find_sector(&c, s);
            const int64_t *st = sectab + 7 * sec;
            int64_t l = s - st[6];
            int ip = (int)(st[2] + l / st[5]);
            int jn = (int)(st[4] + l % st[5]);
            uint32_t pm = p_masks[ip], nm = n_masks[jn];
            int occp[32], occn[32], np_ = 0, nn_ = 0;
            for (int i = 0; i < ns; ++i) {
                if ((pm >> i) & 1u) { occp[np_++] = i; b_ep[i] += g[s] * xs; }
                if ((nm >> i) & 1u) { occn[nn_++] = i; b_en[i] += g[s] * xs; }
            }
            for (int i1 = 0; i1 < np_; ++i1)
                for (int i2 = i1 + 1; i2 < np_; ++i2) {
                    int cc = occp[i1], dd = occp[i2];
                    int col = c.pidx[cc * ns + dd];
                    for (int row = 0; row < c.npairs; ++row) {
                        int a = c.pa[row], b = c.pb[row];
                        if (two_m[a] + two_m[b] != two_m[cc] + two_m[dd]) continue;
                        if (par[a] * par[b] != par[cc] * par[dd]) continue;
                        uint32_t m2;
                        int sg = op_two_body(pm, a, b, cc, dd, &m2);
                        if (!sg) continue;
                        int r = c.p_rank[m2];
                        if (r < 0) { bad = 1; continue; }
                        b_pp[(size_t)row * c.npairs + col] += sg * g[c.pstart[r] + c.nstart[jn]] * xs;
                    }
                }
            for (int i1 = 0; i1 < nn_; ++i1)
                for (int i2 = i1 + 1; i2 < nn_; ++i2) {
                    int cc = occn[i1], dd = occn[i2];
                    int col = c.pidx[cc * ns + dd];
                    for (int row = 0; row < c.npairs; ++row) {
                        int a = c.pa[row], b = c.pb[row];
                        if (two_m[a] + two_m[b] != two_m[cc] + two_m[dd]) continue;
                        if (par[a] * par[b] != par[cc] * par[dd]) continue;
                        uint32_t m2;
                        int sg = op_two_body(nm, a, b, cc, dd, &m2);
                        if (!sg) continue;
                        int r = c.n_rank[m2];
                        if (r < 0) { bad = 1; continue; }
                        b_nn[(size_t)row * c.npairs + col] += sg * g[c.pstart[ip] + c.nstart[r]] * xs;
                    }
                }
            for (int i1 = 0; i1 < np_; ++i1)
                for (int i2 = 0; i2 < nn_; ++i2) {
                    int cp = occp[i1], dn = occn[i2];
                    for (int a = 0; a < ns; ++a) {
                        uint32_t pm2;
                        int sp = op_one_body(pm, a, cp, &pm2);
                        if (!sp) continue;
                        for (int b = 0; b < ns; ++b) {
                            if (two_m[a] + two_m[b] != two_m[cp] + two_m[dn]) continue;
                            if (par[a] * par[b] != par[cp] * par[dn]) continue;
                            uint32_t nm2;
                            int sn = op_one_body(nm, b, dn, &nm2);
                            if (!sn) continue;
                            int rp = c.p_rank[pm2], rn = c.n_rank[nm2];
                            if (rp < 0 || rn < 0) { bad = 1; continue; }
                            b_pn[((size_t)a * ns + b) * ns * ns + (size_t)cp * ns + dn] +=
                                sp * sn * g[c.pstart[rp] + c.nstart[rn]] * xs;
                        }
                    }
                }
        }
#pragma omp critical
        for (size_t k = 0; k < nbins; ++k) bins[k] += loc[k];
        free(loc);
    }
    ctx_free(&c);
    return bad ? -1 : 0;
}

/* One-body transition densities rho_p[a*ns + c] = <g| p+_a p_c |x> and
 * rho_n likewise (Ch. 5, "One-body density matrices", before J coupling):
 * every basis state, every occupied c and every a with the same 2m and
 * parity, by direct operator action. */
int orc_one_body_densities(int ns, const int *two_m, const int *par,
                           int n_sectors, const int64_t *sectab,
                           int n_psd, const uint32_t *p_masks, int n_nsd, const uint32_t *n_masks,
                           const double *g, const double *x, double *rho_p, double *rho_n, int nthreads)
{
    ctx_t c;
    int bad = 0;
    ctx_init(&c, ns, n_sectors, sectab, n_psd, p_masks, n_nsd, n_masks);
    const int64_t dim = sectab[7 * (n_sectors - 1) + 6] + sectab[7 * (n_sectors - 1) + 3] * sectab[7 * (n_sectors - 1) + 5];
    if (nthreads > 0) omp_set_num_threads(nthreads);
    memset(rho_p, 0, sizeof(double) * ns * ns);
    memset(rho_n, 0, sizeof(double) * ns * ns);

#pragma omp parallel reduction(|:bad)
    {
        double *lp = (double *)calloc((size_t)2 * ns * ns, sizeof(double));
        double *ln = lp + ns * ns;
#pragma omp for schedule(dynamic, 256)
        for (int64_t s = 0; s < dim; ++s) {
            double xs = x[s];
            if (xs == 0.0) continue;
            int sec = find_sector(&c, s);
            const int64_t *st = sectab + 7 * sec;
            int64_t l = s - st[6];
            int ip = (int)(st[2] + l / st[5]);
            int jn = (int)(st[4] + l % st[5]);
            uint32_t pm = p_masks[ip], nm = n_masks[jn];
            for (int cc = 0; cc < ns; ++cc)
                for (int a = 0; a < ns; ++a) {
                    if (two_m[a] != two_m[cc] || par[a] != par[cc]) continue;
                    uint32_t m2;
                    int sg;
                    if ((pm >> cc) & 1u) {
                        sg = op_one_body(pm, a, cc, &m2);
                        if (sg) {
                            int r = c.p_rank[m2];
                            if (r < 0) bad = 1;
                            else lp[a * ns + cc] += sg * g[c.pstart[r] + c.nstart[jn]] * xs;
                        }
                    }
                    if ((nm >> cc) & 1u) {
                        sg = op_one_body(nm, a, cc, &m2);
                        if (sg) {
                            int r = c.n_rank[m2];
                            if (r < 0) bad = 1;
                            else ln[a * ns + cc] += sg * g[c.pstart[ip] + c.nstart[r]] * xs;
                        }
                    }
                }
        }
#pragma omp critical
        for (int k = 0; k < ns * ns; ++k) {
            rho_p[k] += lp[k];
            rho_n[k] += ln[k];
        }
        free(lp);
    }
    ctx_free(&c);
    return bad ? -1 : 0;
}
