/*
 * fotci -- factorized on-the-fly configuration interaction on MI355X (gfx950).
 *
 * C-ABI of the library (libfotci.so). The library computes the Hamiltonian
 * times a vector in the M-scheme basis of proton Slater determinants (SDs)
 * times neutron SDs, reconstructing matrix elements on the fly from
 * precomputed one-species "jumps", and the lowest eigenvalues of H by Lanczos
 * with full reorthogonalisation.
 *
 * Conventions shared by every entry point:
 *  - Return value 0 = success; a negative FOTCI_E* code on failure, with a
 *    message from fotci_last_error() (thread-local; valid until the next call
 *    on the same thread). No C++ exception crosses the ABI.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are GPU
 *    memory owned by the caller (e.g. a torch tensor's data_ptr()). The
 *    library never allocates device memory: the caller passes workspaces of
 *    the size the matching *_bytes query returns.
 *  - stream arguments are hipStream_t passed as void* (NULL = null stream).
 *    Device work is enqueued asynchronously unless a call says otherwise.
 *  - Handles (fotci_basis, fotci_jumps, fotci_ham) are library-owned host
 *    objects, released with the matching fotci_free_*; a fotci_jumps keeps
 *    its fotci_basis alive by reference, so free in reverse order of creation.
 */
#ifndef FOTCI_H
#define FOTCI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FOTCI_OK 0
#define FOTCI_EINVAL (-1)    /* invalid argument or inconsistent input */
#define FOTCI_ENOMEM (-2)    /* workspace too small / host allocation failed */
#define FOTCI_EHIP (-3)      /* a HIP runtime call or kernel launch failed */
#define FOTCI_ENOTCONV (-4)  /* Lanczos could not produce the requested states */
#define FOTCI_ESTATE (-5)    /* call out of order (e.g. apply before upload) */

/* Arithmetic modes of apply_H / lanczos_lowest. */
#define FOTCI_MODE_F64_PLAIN 0  /* float64 vectors; straightforward gather kernel */
#define FOTCI_MODE_F64 1        /* float64 vectors; tiled kernels */
#define FOTCI_MODE_F32 2        /* float32 vectors and matrix elements (pn on f32 MFMA) */

/* Reorthogonalisation of each new Lanczos vector against all stored ones
 * (classical Gram-Schmidt with float64 sums): */
#define FOTCI_REORTH_CGS2 0     /* two passes, always */
#define FOTCI_REORTH_DGKS 1     /* a second pass only when the first shrank the vector below
                                   1/sqrt(2) of its norm (the Daniel-Gragg-Kaufman-Stewart test) */

/* Jump kinds for fotci_jumps_count / fotci_jumps_export. */
#define FOTCI_JUMP_PP2 0  /* proton two-body jumps */
#define FOTCI_JUMP_NN2 1  /* neutron two-body jumps */
#define FOTCI_JUMP_P1 2   /* proton one-body jumps */
#define FOTCI_JUMP_N1 3   /* neutron one-body jumps */

typedef struct fotci_basis fotci_basis;
typedef struct fotci_jumps fotci_jumps;
typedef struct fotci_ham fotci_ham;

const char *fotci_last_error(void);
const char *fotci_version(void);

/*
 * fotci_build_basis -- the factorised M-scheme basis (Ch. 2, "Use of quantum
 * numbers: factorization of the basis"; Ch. 6, "Writing out the basis").
 *
 *  n_orbits, two_j[n_orbits], parity[n_orbits] (host): the single-particle
 *    orbits, identical for protons and neutrons; 2j odd and > 0, parity +1 or
 *    -1. m-states are numbered orbit by orbit, 2m ascending inside an orbit;
 *    m-state i is bit i of an SD mask, so the total N_s must be <= 32.
 *  Z, N: valence protons and neutrons (0 <= Z, N <= N_s).
 *  two_M: twice the total Jz; its parity must equal that of Z + N.
 *  parity_total: +1 or -1.
 *  Proton sectors are ordered by 2M_p ascending (parity +1 before -1); a
 *  species sector whose conjugate sector is empty is dropped; SDs inside a
 *  sector ascend by mask value; basis index = pstart[ip] + nstart[jn] with
 *  the neutron index fastest.
 *  *out receives a new handle. FOTCI_EINVAL on bad arguments or an empty
 *  basis.
 */
int fotci_build_basis(int32_t n_orbits, const int32_t *two_j, const int32_t *parity,
                      int32_t Z, int32_t N, int32_t two_M, int32_t parity_total,
                      fotci_basis **out);
void fotci_free_basis(fotci_basis *b);

/* Sizes of the basis (any output pointer may be NULL). */
int fotci_basis_info(const fotci_basis *b, int64_t *dim, int32_t *n_sectors,
                     int32_t *n_psd, int32_t *n_nsd, int32_t *n_states);

/*
 * fotci_basis_export -- copy the basis tables into caller-allocated host
 * arrays (any may be NULL): p_bits[n_psd], n_bits[n_nsd] (SD masks in basis
 * order), pstart[n_psd], nstart[n_nsd], and sector_table[n_sectors*7] with
 * rows (2M_p, parity_p, first pSD, #pSDs, first nSD, #nSDs, offset).
 */
int fotci_basis_export(const fotci_basis *b, uint32_t *p_bits, uint32_t *n_bits,
                       int64_t *pstart, int64_t *nstart, int64_t *sector_table);

/*
 * fotci_build_jumps -- one-species jumps (Ch. 2, "Representation of the
 * Hamiltonian"; Ch. 8, "Opbundles and optypes"): the nonzero results of
 * p+_a p+_b p_d p_c (two-body; a<b, c<d conserving 2M and parity, diagonal
 * included; label = pair(a,b) * n_pairs + pair(c,d), pairs (a<b) numbered
 * lexicographically) and of p+_a p_c (one-body; any a, c; label = a*N_s + c;
 * the destination must be a kept SD) on every kept SD of each species, with
 * the fermion phase (-1)^(occupied states below the index) of each operator.
 * The basis must outlive the jumps.
 */
int fotci_build_jumps(const fotci_basis *b, fotci_jumps **out);
void fotci_free_jumps(fotci_jumps *j);

/* Number of records of one kind (FOTCI_JUMP_*). */
int fotci_jumps_count(const fotci_jumps *j, int32_t kind, int64_t *count);

/*
 * Copy one kind's records, sorted by (dst, src, label), into caller-allocated
 * host arrays of length count (any may be NULL). src/dst are species SD
 * indices in basis order; phase is +1 or -1.
 */
int fotci_jumps_export(const fotci_jumps *j, int32_t kind, int32_t *src, int32_t *dst,
                       int8_t *phase, int32_t *label);

/*
 * fotci_set_interaction -- the one- plus two-body Hamiltonian in M-scheme
 * form (App. A, "The Hamiltonian and other operators in second
 * quantization", eq. hamdef, with V already uncoupled):
 *   H = sum_i eps_p[orb i] n_i(p) + sum_i eps_n[orb i] n_i(n)
 *     + sum_{a<b,c<d} v_pp[(ab),(cd)] p+_a p+_b p_d p_c   (v_nn alike)
 *     + sum_{abcd} v_pn[(a b),(c d)] (p+_a p_c)(n+_b n_d).
 *  spe_p, spe_n: host [n_orbits]; v_pp, v_nn: host [n_pairs*n_pairs]
 *  row-major; v_pn: host [(N_s*N_s)^2], row index a*N_s+b (proton a,
 *  neutron b). Arrays are copied. Every array must be exactly symmetric and
 *  zero wherever 2M or parity would change, else FOTCI_EINVAL. The jumps must
 *  outlive the Hamiltonian.
 */
int fotci_set_interaction(const fotci_jumps *j, const double *spe_p, const double *spe_n,
                          const double *v_pp, const double *v_nn, const double *v_pn,
                          fotci_ham **out);
void fotci_free_ham(fotci_ham *h);

/* Replace the interaction values (same rules as fotci_set_interaction). If
 * the Hamiltonian is uploaded, the device copy is refreshed on `stream`. */
int fotci_ham_set_values(fotci_ham *h, const double *spe_p, const double *spe_n,
                         const double *v_pp, const double *v_nn, const double *v_pn,
                         void *stream);

/* Bytes of device workspace fotci_ham_upload needs (>= 0), or a negative code. */
int64_t fotci_ham_workspace_bytes(const fotci_ham *h);

/* One J-coupled two-body matrix element V_J(ab, cd) in MeV: orbit indices
 * (0-based, in the orbit order of the basis) and 2J. */
typedef struct {
    int32_t a, b, c, d;
    int32_t two_J;
    double v;
} fotci_tbme;

/*
 * fotci_decouple_tbme -- the m-scheme arrays fotci_set_interaction takes,
 * from J-coupled two-body matrix elements between normalised two-body states
 * of good J (App. A, "The Hamiltonian and other operators in second
 * quantization", eq. hamdef). For like particles (al < be, ga < de m-states
 * of orbits a <= b, c <= d):
 *   V[(al be),(ga de)] = sum_J zeta_ab zeta_cd V_J(ab,cd)
 *                        (j_a m_al j_b m_be | J M) (j_c m_ga j_d m_de | J M),
 * zeta_ab = sqrt(2) if a == b else 1; for a proton-neutron pair (a, c proton
 * orbits, b, d neutron orbits) the same product-state sum without zeta.
 * two_j[n_orbits], parity[n_orbits] (NULL: all +1) define the m-states as in
 * fotci_build_basis. Each (ab, cd) is given once and (cd, ab) is implied;
 * repeated elements add. Outputs (host, overwritten, exactly symmetric; each
 * may be NULL): v_pp, v_nn [n_pairs^2], v_pn [N_s^4]. FOTCI_EINVAL for an
 * orbit index out of range, a > b or c > d for like particles, 2J outside the
 * coupling range of a pair, a parity change, a nonzero odd-J element of two
 * like particles in one orbit, or a non-finite value. Host only.
 */
int fotci_decouple_tbme(int32_t n_orbits, const int32_t *two_j, const int32_t *parity, int32_t n_pp,
                        const fotci_tbme *pp, int32_t n_nn, const fotci_tbme *nn, int32_t n_pn,
                        const fotci_tbme *pn, double *v_pp, double *v_nn, double *v_pn);

/*
 * fotci_ham_upload -- copy the jump tables and interaction into the
 * caller-owned device workspace (256-byte aligned, `bytes` >= the size from
 * fotci_ham_workspace_bytes, else FOTCI_ENOMEM) and form the per-jump matrix
 * element values on the device. The workspace must stay allocated and
 * untouched while the Hamiltonian is used. Synchronises `stream` before
 * returning.
 */
int fotci_ham_upload(fotci_ham *h, void *dev_workspace, int64_t bytes, void *stream);

/*
 * fotci_apply_H -- y = H x (overwrite), the on-the-fly matrix-vector product
 * (Ch. 2, "Representation of the Hamiltonian"; Ch. 8, "Mode times": pp, nn
 * and pn parts plus single-particle energies). x, y: device vectors of length
 * dim in basis order, float64 for the F64 modes and float32 otherwise; x and
 * y must not overlap. Asynchronous on `stream`.
 */
int fotci_apply_H(const fotci_ham *h, int32_t mode, const void *x, void *y, void *stream);

/*
 * fotci_apply_H_block -- Y = H X for a block of n_block vectors stored
 * row-wise (Ch. "Block Lanczos": the Hamiltonian applied to a block whose
 * vectors are adjacent in memory element by element, so every matrix element
 * reconstructed serves the whole block). X, Y: device arrays of dim * n_block
 * elements, element i of vector v at [i * n_block + v] (a row-major
 * dim x n_block matrix), float64 for FOTCI_MODE_F64 and float32 for
 * FOTCI_MODE_F32, 16-byte aligned, not overlapping; Y is overwritten.
 * n_block: 1, 2, 4 or 8 (1 is fotci_apply_H, which also takes
 * FOTCI_MODE_F64_PLAIN). Each vector's result is fotci_apply_H of that vector
 * with the same per-element arithmetic. FOTCI_EINVAL for another n_block,
 * FOTCI_MODE_F64_PLAIN with n_block > 1, misaligned pointers, a block of more
 * than 2^31 - 2^20 bytes (32-bit buffer offsets), or sectors too large for
 * the kernels' LDS tiles; FOTCI_ESTATE if the Hamiltonian is not uploaded.
 * Asynchronous on `stream`; fotci_profile_start records its kernels too.
 */
int fotci_apply_H_block(const fotci_ham *h, int32_t mode, int32_t n_block, const void *x, void *y, void *stream);

/*
 * fotci_apply_H_vjp_static -- fotci_apply_H_vjp for callers that cannot
 * allocate or must not depend on per-call device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc).
 * Same arguments, results and accumulation rules as fotci_apply_H_vjp; the
 * per-neutron-SD column sums it needs go to a static device array of the
 * library (65,536 doubles = 512 KiB per GPU, held from the first call on a
 * device until the process ends) instead of the Hamiltonian's workspace. It
 * calls no device or host allocator; the kernels clear the array before use.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (different streams or threads) race and give wrong results.
 * FOTCI_EINVAL if the basis has more than 65,536 neutron SDs (use
 * fotci_apply_H_vjp), FOTCI_ESTATE if the Hamiltonian is not uploaded,
 * FOTCI_EHIP if the array's device address cannot be obtained.
 */
int fotci_apply_H_vjp_static(const fotci_ham *h, const double *x, const double *g, double *dx,
                             double *d_spe_p, double *d_spe_n, double *d_v_pp, double *d_v_nn,
                             double *d_v_pn, void *stream);

/*
 * fotci_one_body_density -- m-scheme one-body transition densities of two
 * vectors of the basis (Ch. 5, "One-body density matrices", in the
 * proton-neutron form the reduced densities are coupled from):
 *   rho_p[a*N_s + c] = <g| p+_a p_c |x>,  rho_n[a*N_s + c] = <g| n+_a n_c |x>.
 * Only entries with equal 2m and parity of a and c can be nonzero. For
 * g = x = psi (unit norm) the diagonals are the m-state occupations (Ch. 4,
 * "Single-particle occupations"). g, x: device float64 [dim]; rho_p, rho_n:
 * device float64 [N_s^2], overwritten; either may be NULL. Asynchronous on
 * `stream`. FOTCI_ESTATE if the Hamiltonian is not uploaded.
 */
int fotci_one_body_density(const fotci_ham *h, const double *g, const double *x, double *rho_p, double *rho_n,
                           void *stream);

/*
 * fotci_apply_H_vjp -- adjoint of y = H(v) x for L = <g, y> (float64 only):
 *   dx = H g  (H is symmetric), written to dx (device, length dim) if non-NULL;
 *   d_v_pp[(ab),(cd)] += <g| p+_a p+_b p_d p_c |x>  (device [n_pairs^2]), and
 *   d_v_nn, d_v_pn [(N_s^2)^2] alike, d_spe_p/d_spe_n [n_orbits] += <g|n_orbit|x>:
 *   the label-wise transition densities (Ch. 5, "Two-body densities").
 * Gradient buffers are accumulated into (the caller zeroes them); each may be
 * NULL. Entries (r,c) and (c,r) are separate (unsymmetrised).
 */
int fotci_apply_H_vjp(const fotci_ham *h, const double *x, const double *g, double *dx,
                      double *d_spe_p, double *d_spe_n, double *d_v_pp, double *d_v_nn,
                      double *d_v_pn, void *stream);

typedef struct {
    int32_t n_keep;   /* number of lowest eigenpairs wanted (>= 1) */
    int32_t n_iter;   /* Lanczos iterations (Krylov dimension), n_keep <= n_iter */
    int32_t mode;     /* FOTCI_MODE_*: storage/arithmetic of vectors and apply_H */
    int32_t refine;   /* 1: float64 Rayleigh-quotient refinement of the Ritz vectors */
    int32_t reorth;   /* FOTCI_REORTH_* */
} fotci_lanczos_opts;

/* Bytes of device workspace fotci_lanczos_lowest needs for these options. */
int64_t fotci_lanczos_workspace_bytes(const fotci_ham *h, const fotci_lanczos_opts *o);

/*
 * fotci_lanczos_lowest -- lowest eigenvalues by Lanczos with full
 * reorthogonalisation (Ch. 7, "Standard Lanczos algorithm": alpha first, then
 * classical Gram-Schmidt twice against every earlier vector, float64
 * accumulation). Lanczos vectors are stored in the mode's precision; alpha,
 * beta, reorthogonalisation coefficients and the tridiagonal eigenproblem are
 * float64.
 *  pivot: device float64 [dim], the starting vector (normalised internally).
 *  work: device workspace of the queried size (FOTCI_ENOMEM if smaller).
 *  evals, resid: host [n_keep]; resid = ||H y - theta y|| / ||y|| in float64.
 *  evecs: device float64 [n_keep*dim] Ritz vectors (unit norm), or NULL.
 *  alpha, beta: host [n_iter] copies of the recurrence, or NULL.
 * With refine = 1, theta is the float64 Rayleigh quotient of each Ritz vector.
 * Synchronous (returns after the stream drained). FOTCI_ENOTCONV when the
 * Krylov space breaks down before n_keep Ritz values exist.
 */
int fotci_lanczos_lowest(const fotci_ham *h, const fotci_lanczos_opts *o, const double *pivot,
                         void *work, int64_t work_bytes, double *evals, double *resid,
                         double *evecs, double *alpha, double *beta, void *stream);

/*
 * Thick-restart Lanczos (Ch. 7, "Thick-restart Lanczos"): the basis is held
 * to n_basis + 1 vectors. When a cycle has reached n_basis vectors, the
 * projected matrix is diagonalised; unless the lowest n_keep Ritz pairs have
 * converged (|beta_last L[last, mu]| <= tol * max(1, |E_mu|)), the n_thick
 * lowest Ritz vectors and the last Lanczos vector start the next cycle.
 * Every step reorthogonalises fully (classical Gram-Schmidt, twice, float64
 * sums), vectors are stored in the mode's precision as in
 * fotci_lanczos_lowest, and the final Ritz vectors are refined in float64.
 */
typedef struct {
    int32_t n_keep;        /* lowest eigenpairs wanted, 1..16 */
    int32_t n_thick;       /* Ritz vectors kept at a restart, n_keep <= n_thick */
    int32_t n_basis;       /* Lanczos vectors per cycle, n_thick + 2 <= n_basis <= 4095 */
    int32_t max_restarts;  /* restarts allowed (>= 0) */
    int32_t mode;          /* FOTCI_MODE_* */
    int32_t refine;        /* 1: float64 Rayleigh-quotient refinement of the Ritz vectors */
    int32_t reorth;        /* FOTCI_REORTH_* */
    double tol;            /* convergence threshold (> 0), relative to max(1, |E|) */
} fotci_trlan_opts;

/* Bytes of device workspace fotci_lanczos_thick_restart needs (negative
 * error code for invalid options). */
int64_t fotci_trlan_workspace_bytes(const fotci_ham *h, const fotci_trlan_opts *o);

/*
 * pivot: device float64 [dim]; work: device workspace (256-byte aligned) of
 * at least the queried size; evals, resid: host [n_keep]; evecs: device
 * float64 [n_keep*dim] Ritz vectors or NULL; stats: host int32[3] =
 * {restarts, apply_H calls in the cycles, converged (0/1)} or NULL. The
 * cycles stop when the recurrence's estimate meets tol (or max_restarts is
 * exhausted); converged is then 1 only if every returned resid[mu] (the true
 * ||H y - E y|| of the float64 Ritz vector, H applied in float64) is
 * <= tol * max(1, |E_mu|). With FOTCI_MODE_F32 the stored basis limits that
 * residual to roughly 1e-7 * ||H|| (float32 rounding of the vectors), so a
 * tol below that returns converged = 0 with the best pairs found. A run that
 * exhausts max_restarts returns FOTCI_OK with stats[2] = 0 and the current
 * Ritz pairs. Synchronous. FOTCI_ENOTCONV if the Krylov space breaks
 * down before n_keep Ritz values exist.
 */
int fotci_lanczos_thick_restart(const fotci_ham *h, const fotci_trlan_opts *o, const double *pivot, void *work,
                                int64_t work_bytes, double *evals, double *resid, double *evecs, int32_t *stats,
                                void *stream);

/*
 * Block Lanczos (Ch. "Block Lanczos"): H V_n = V_{n-1} B_{n-1}^T + V_n A_n +
 * V_{n+1} B_n for blocks V_n of n_block orthonormal vectors. Per block
 * iteration: W = H V_n (fotci_apply_H_block); A_n = V_n^T W;
 * W -= V_n A_n + V_{n-1} B_{n-1}^T; classical Gram-Schmidt of W against every
 * block so far, twice (float64 sums); the overlap W^T W = U Lambda U^T gives
 * B_n = Lambda^{1/2} U^T and V_{n+1} = W U Lambda^{-1/2} (repeated once on
 * the new block, B_n the product of both factors). The block-tridiagonal
 * matrix of the A_n and B_n is diagonalised on the host in float64 (Jacobi
 * rotations); Ritz vectors and refinement as in fotci_lanczos_lowest. Blocks
 * are stored row-wise in the mode's precision; W and every sum are float64.
 */
typedef struct {
    int32_t n_keep;   /* lowest eigenpairs wanted, 1..16 */
    int32_t n_block;  /* vectors per block: 1, 2, 4 or 8 */
    int32_t n_iter;   /* block iterations, >= 1, with n_iter * n_block <= 4096 */
    int32_t mode;     /* FOTCI_MODE_F64 or FOTCI_MODE_F32 */
    int32_t refine;   /* 1: float64 Rayleigh-quotient refinement of the Ritz vectors */
} fotci_block_lanczos_opts;

/* Bytes of device workspace fotci_lanczos_block needs (negative error code
 * for invalid options). */
int64_t fotci_block_lanczos_workspace_bytes(const fotci_ham *h, const fotci_block_lanczos_opts *o);

/*
 * pivot: device float64 [dim * n_block], the starting block, row-wise as in
 * fotci_apply_H_block, 16-byte aligned (orthonormalised internally;
 * FOTCI_EINVAL if its columns are linearly dependent). work: device
 * workspace (256-byte aligned) of at least the queried size. evals, resid:
 * host [n_keep]; evecs: device float64 [n_keep*dim] Ritz vectors (one after
 * another, unit norm) or NULL; n_done: host, the block iterations carried
 * out, or NULL. A column of a new block whose overlap eigenvalue has
 * sqrt(lambda) <= 1e-7 times the norm of the block-tridiagonal matrix
 * (dependent on the basis to the resolution of the overlap) is replaced by a
 * new vector: the basis vector e_k, k = ((r * n_block + column) * 2654435761)
 * mod dim at the r-th replacement of the run, orthogonalised against the
 * basis. The iteration stops early when every column of a new block is
 * dependent (the block Krylov space is invariant to rounding) or a new vector
 * lies in the span. Synchronous. FOTCI_ENOTCONV if fewer than n_keep Ritz
 * values exist.
 */
int fotci_lanczos_block(const fotci_ham *h, const fotci_block_lanczos_opts *o, const double *pivot, void *work,
                        int64_t work_bytes, double *evals, double *resid, double *evecs, int32_t *n_done,
                        void *stream);

/* Counts of the work in one apply_H (host; no device needed): multiply-adds
 * of the pp, nn and pn parts and of the diagonal, as the paper counts
 * "operations" (Ch. 8, "Jump storage"). */
int fotci_ham_op_counts(const fotci_ham *h, int64_t *ops_pp, int64_t *ops_nn, int64_t *ops_pn,
                        int64_t *ops_diag);

/* Work of the pn kernel that fotci_apply_H runs in `mode` (FOTCI_MODE_F32 or
 * FOTCI_MODE_F64) in one apply_H (host; no device needed), counted from the
 * tables the kernel walks: visited (destination row, operator class,
 * 32-column source tile) triples, 16x16x4 matrix-core instructions, and
 * gather slots including the padding of the 64-entry rounds. The float32
 * kernel with a shared output row per pair of waves works through pairs of
 * source tiles and contracts both tiles of a pair that has any jump; the
 * others skip every tile without jumps. Each output may be NULL.
 * FOTCI_EINVAL for another mode, FOTCI_ESTATE when the tiled kernels are not
 * available for this basis. */
int fotci_ham_pn_work(const fotci_ham *h, int32_t mode, int64_t *tile_visits, int64_t *mfma_instr,
                      int64_t *gather_slots);

/* Output-row policy of the float32 pn kernel (FOTCI_MODE_F32, one vector and
 * blocks): 1 (default) has the two waves of a workgroup take the source tiles
 * in pairs and own the destination columns of one parity each, so the row is
 * updated by plain LDS read-modify-write (when the row fits); 0 lets both
 * waves add to the row with LDS atomics, as the float64 kernel does. Both
 * give the same sums up to rounding order; the choice changes speed only.
 * FOTCI_EINVAL unless enable is 0 or 1. */
int fotci_ham_set_pn_private_rows(fotci_ham *h, int32_t enable);

/*
 * fotci_profile_start / fotci_profile_stop -- per-kernel timing of apply_H
 * (the per-part timings of Ch. 8, taken with HIP events). Between start and
 * stop, every fotci_apply_H call on this Hamiltonian records a HIP event on
 * its stream before its first kernel and after each kernel (max_calls calls at
 * most; later calls are not recorded). stop synchronises on the events and
 * writes, for each kernel of the last recorded mode, the mean duration in
 * milliseconds (avg_ms[k], k < *n_kernels <= 4) and its name (names[k],
 * static strings; names may be NULL); *n_calls = calls recorded. The events
 * are host-side HIP objects created by start and destroyed by stop.
 */
int fotci_profile_start(fotci_ham *h, int32_t max_calls);
int fotci_profile_stop(fotci_ham *h, double *avg_ms, const char **names, int32_t *n_kernels, int32_t *n_calls);

/*
 * Host utility: eigenvalues (ascending) and orthonormal eigenvectors of the
 * symmetric tridiagonal matrix with diagonal diag[n] and off-diagonal
 * offdiag[n-1] in float64 (the tridiagonal step of Lanczos; implicit QL).
 * evecs: host [n*n] row-major, column k = eigenvector k, or NULL.
 */
int fotci_tridiag_eigh(int32_t n, const double *diag, const double *offdiag, double *evals, double *evecs);

/*
 * Host utility: eigenvalues (ascending) and orthonormal eigenvectors of a
 * dense symmetric float64 matrix a[n*n] (row-major; FOTCI_EINVAL unless
 * exactly symmetric), by cyclic Jacobi rotations -- the projected-matrix step
 * of thick-restart Lanczos. evecs: host [n*n] row-major, column k =
 * eigenvector k, or NULL.
 */
int fotci_sym_eigh(int32_t n, const double *a, double *evals, double *evecs);

#ifdef __cplusplus
}
#endif
#endif /* FOTCI_H */
