// Internal types of libfotci: host-side basis, jumps and Hamiltonian tables,
// and the device view the kernels read.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fotci.h"

namespace fotci {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg);
void set_error(const std::string &msg);

// -------------------------------------------------------------- m-states
struct MState {
    int orbit, two_j, two_m, parity;
};

// One species' kept SDs, grouped into (2M, parity) sectors.
struct SpeciesBasis {
    int n = 0;                       // particles
    std::vector<uint32_t> sd;        // kept SD masks, basis order
    std::vector<int32_t> sd_sector;  // species sector of each SD
    std::vector<int32_t> sd_local;   // rank inside its species sector
    struct Sector {
        int two_m, parity, first, count;
    };
    std::vector<Sector> sectors;
    // index of a mask among the kept SDs, or -1
    int32_t find(uint32_t mask, const std::vector<MState> &ms) const;
};

struct BasisSector {
    int two_mp, parity_p;
    int p_sector, n_sector;          // species sector indices
    int p_first, np, n_first, nn;
    int64_t offset;
};

}  // namespace fotci

struct fotci_basis {
    std::vector<fotci::MState> ms;
    int n_orbits = 0;
    int two_M = 0, parity = 1;
    fotci::SpeciesBasis p, n;
    std::vector<fotci::BasisSector> sectors;
    std::vector<int32_t> p_basis_sector;   // per proton SD: basis sector
    std::vector<int64_t> pstart, nstart;
    int64_t dim = 0;
};

namespace fotci {

struct JumpRec {
    int32_t src, dst;
    int32_t label;
    int8_t phase;
};

// One-body operator classes: a+_a a_c grouped by (Delta = 2m_a - 2m_c,
// rho = parity_a * parity_c). A proton class q pairs with the neutron class
// conj[q] of opposite Delta and the same rho.
struct OpClasses {
    int nq = 0;
    std::vector<int> delta, rho, conj;
    std::vector<std::vector<int>> ops;   // labels a*ns+c in the class, ascending
    std::vector<int> class_of;           // label -> class
    std::vector<int> local_of;           // label -> position in its class
};

}  // namespace fotci

struct fotci_jumps {
    const fotci_basis *b = nullptr;
    int ns = 0, npairs = 0;
    std::vector<fotci::JumpRec> rec[4];  // FOTCI_JUMP_* order, canonical sort
    fotci::OpClasses cls;
};

namespace fotci {

// Device-side view of one species' tables.
struct DevSpecies {
    const uint32_t *masks;     // [n_sd]
    const int32_t *code2;      // [n_jump2] two-body jump codes: label*2 + (phase<0)
    const int32_t *off_rowptr; // [n_sd+1] off-diagonal merged entries by dst
    const int32_t *off_col;    // [n_off] source SD
    const int32_t *off_j0;     // [n_off] jump range of the entry
    const int32_t *off_j1;
    const int32_t *diag_j0;    // [n_sd] diagonal jump range (j0 == j1: none)
    const int32_t *diag_j1;
    const int32_t *ob_ptr;     // [n_sd*nq+1] one-body jumps by (dst, class)
    const int32_t *ob_src;     // [n_ob] source SD
    const int32_t *ob_code;    // [n_ob] local op index*2 + (phase<0)
    const double *eps;         // [ns] single-particle energy per m-state
    const double *v2;          // [npairs^2] two-body matrix elements
    double *off_val64;         // [n_off] merged matrix elements
    float *off_val32;
    double *d64;               // [n_sd] diagonal: spe + diagonal two-body
    float *d32;
    int32_t n_sd, n_off;
};

struct DevHam {
    int32_t ns, npairs, nq, n_sectors;
    int32_t n_vq;              // length of the blocked pn element array
    int64_t dim;
    const int32_t *p_sector;   // [n_psd] basis sector of each proton SD
    const int64_t *p_pstart;   // [n_psd]
    const int32_t *n_local;    // [n_nsd] nstart
    const int32_t *sec_nn;     // [n_sectors]
    const int32_t *sec_nfirst; // [n_sectors]
    const int32_t *sec_pfirst; // [n_sectors]
    const int32_t *sec_np;     // [n_sectors]
    const int64_t *sec_off;    // [n_sectors]
    const int32_t *conjq;      // [nq]
    const int32_t *ms_orbit;   // [ns] orbit of each m-state
    const int32_t *n_bsector;  // [n_nsd] basis sector of each neutron SD
    const int32_t *cls_off;    // [nq+1] class q's op labels are cls_ops[cls_off[q]..cls_off[q+1])
    const int32_t *cls_ops;    // [ns*ns] op labels a*ns+c grouped by class
    const int32_t *vq_off;     // [nq] offset of V^q in vq64/vq32
    const int32_t *vq_nb;      // [nq] columns of V^q (= #ops of the neutron class)
    const double *vq64;
    float *vq32;
    double *scratch_ncol;      // [n_nsd] adjoint scratch: per-neutron-SD column sums
    DevSpecies p, n;
};

// One ELL entry of the nn / pp kernels: the local source index and the merged
// matrix element, read with a single 8- or 12-byte load (the float64 value as
// two 32-bit words, low first).
struct alignas(8) EllE32 {
    int32_t src;
    float v;
};
struct alignas(4) EllE64 {
    int32_t src;
    uint32_t v_lo, v_hi;
};

// Extra device tables of the tiled kernels (indexed by basis sector s; each
// basis sector owns one proton and one neutron species sector).
struct DevTiled {
    const int32_t *order;        // [n_psd] pn workgroup -> destination proton SD (largest rows first)
    const int64_t *p_ob_base;    // [proton one-body jumps] pstart of the source SD
    // nn: per sector an ELL table over destination neutron columns, entry e of
    // column c at ell_base[s] + e*nn_s + c (padding: src 0, value 0)
    const int64_t *nn_ell_base;  // [n_sectors]
    const int32_t *nn_ell_E;     // [n_sectors]
    const int32_t *nn_ell_src;   // local source column
    const int32_t *nn_ell_ent;   // merged neutron entry index, -1 for padding
    // the entries the kernels walk, source and value side by side (one load each)
    EllE32 *nn_ell_e32;
    EllE64 *nn_ell_e64;
    // pp: per sector an ELL table over destination proton rows (e*np_s + r)
    const int64_t *pp_ell_base;
    const int32_t *pp_ell_E;
    const int32_t *pp_ell_src;   // local source row
    const int32_t *pp_ell_ent;
    EllE32 *pp_ell_e32;
    EllE64 *pp_ell_e64;
    int64_t nn_ell_len, pp_ell_len;
    // nn / pp workgroup tiles
    const int32_t *rt_sec, *rt_r0;   // [n_rtiles] row tiles (nn kernel)
    const int32_t *ct_sec, *ct_c0;   // [n_ctiles] column tiles (pp kernel)
    int32_t n_rtiles, n_ctiles, rt_rows, ct_cols;
    // pn neutron gather lists grouped by (destination sector, neutron class, 16-column source tile)
    const int32_t *pn_ptr;       // [(n_sectors*nq)*n_t16 + 1]
    const uint32_t *pn_code;     // (phase < 0) << 31 | last << 30 | dst col << kPnRBits | R element; rounds of
                                 // 64 entries, each destination owned by one lane (its entries consecutive
                                 // there, `last` on the final one), padded with pn_null (R element 0, dst
                                 // col max_nn, not last)
    int64_t n_pn_code;           // entries of pn_code (a multiple of 64)
    // the same jumps for the float32 one-vector kernel (k_pn2), one list per (destination sector, neutron
    // class, pair of source tiles, destination-column parity): slot ((s*nq + qn)*n_s2 + pair)*2 + parity;
    // codes as above with the R element (tile of the pair)*kPnTile*kPnRStride + col*kPnRStride + B in the
    // low kPn2RBits bits and the destination column above them
    const int32_t *pn2_ptr;      // [(n_sectors*nq)*n_s2*2 + 1]
    const uint32_t *pn2_code;
    int64_t n_pn2_code;
    uint32_t pn2_null;           // padding code: R element 0, dst col max_nn, not last
    int32_t n_s2;                // tile pairs per sector slot
    const int8_t *pn_ndiag;      // [n_psd * nq] proton jumps of (row, class) that leave the SD unchanged; they
                                 // lead the row's list for the class and the pn kernels contract them as one
    uint32_t pn_null;            // padding code
    int32_t n_t16;               // tiles per sector slot (ceil(max nn / kPnTile))
    int32_t kp_pad;              // max proton one-body jumps into a row per class, rounded up to 4
    int32_t max_nn, max_np;
    int32_t ok;
    int32_t pn_priv;             // float pn kernel: 1 = a private output row per wave when it fits, 0 = shared row
};

// The pn kernel's per-wave tile R holds, for the kPnTile source columns of a
// tile and up to 64 neutron labels B, the partial sums R[B][col] column-major
// with column stride kPnRStride; a gather code names its R element
// col * kPnRStride + B in its low kPnRBits bits, the destination column in
// the bits above, and the phase in bit 31.
constexpr int kPnTile = 32;                 // source columns per tile (a multiple of 16)
constexpr int kPnRStride = 68;
constexpr int kPnRBits = 12;                // kPnTile * kPnRStride <= 1 << kPnRBits
constexpr int kPnDstBits = 30 - kPnRBits;   // bit 30: last entry of its destination in its lane
constexpr uint32_t kPnFlush = 1u << 30;
constexpr int kPn2RBits = 13;               // 2 * kPnTile * kPnRStride <= 1 << kPn2RBits
constexpr int kPn2DstBits = 30 - kPn2RBits;
constexpr int kPnWaves = 2;                 // waves per pn workgroup
// float32 pn: the row split between the two waves by column parity (k_pn2)
// is used while its LDS (two R tiles, the row with one padding column and 64
// scratch words per wave) fits the 64 KiB a workgroup may hold
inline bool pn_split_row_fits(int max_nn) {
    return ((int64_t)kPnWaves * kPnTile * kPnRStride + max_nn + 1 + 64 * kPnWaves) * 4 <= 65536;
}

struct HostTiled {
    std::vector<int32_t> order, nn_ell_E, nn_ell_src, nn_ell_ent, pp_ell_E, pp_ell_src, pp_ell_ent;
    std::vector<int64_t> p_ob_base, nn_ell_base, pp_ell_base;
    std::vector<int32_t> rt_sec, rt_r0, ct_sec, ct_c0, pn_ptr, pn2_ptr;
    std::vector<uint32_t> pn_code, pn2_code;
    std::vector<int8_t> pn_ndiag;
    int n_t16 = 0, n_s2 = 0, kp_pad = 4, max_nn = 0, max_np = 0;
    bool ok = false;
};

// Host-side tables (built once per jumps + interaction layout).
struct HostCommonTables {
    std::vector<int32_t> p_sector, n_local, sec_nn, sec_nfirst, sec_pfirst, sec_np, conjq;
    std::vector<int32_t> ms_orbit, n_bsector, cls_off, cls_ops;
    std::vector<int64_t> sec_off;
};

struct HostSpeciesTables {
    std::vector<uint32_t> masks;
    std::vector<int32_t> code2, off_rowptr, off_col, off_j0, off_j1, diag_j0, diag_j1;
    std::vector<int32_t> ob_ptr, ob_src, ob_code;
    std::vector<double> eps, v2;
};

}  // namespace fotci

struct fotci_ham {
    const fotci_jumps *j = nullptr;
    std::vector<double> spe_p, spe_n, v_pp, v_nn, v_pn;
    std::vector<double> vq;               // blocked pn matrix elements
    std::vector<int32_t> vq_off, vq_nb;
    fotci::HostSpeciesTables tp, tn;
    fotci::HostCommonTables tc;
    fotci::HostTiled tt;
    fotci::DevTiled dev_tiled{};
    int32_t pn_priv = 1;                  // see fotci_ham_set_pn_private_rows
    // device
    bool uploaded = false;
    void *ws = nullptr;
    int64_t ws_bytes = 0;
    fotci::DevHam dev{};
    // per-kernel timing (fotci_profile_start/stop)
    struct Profile {
        bool on = false;
        int max_calls = 0, calls = 0, n_kernels = 0;
        std::vector<void *> events;   // hipEvent_t, (max_calls * 5)
        const char *names[4] = {nullptr, nullptr, nullptr, nullptr};
    };
    mutable Profile prof;
    // layout (offsets in bytes from ws), filled by layout()
    std::vector<std::pair<std::string, int64_t>> layout_offsets;
    int64_t layout_total = 0;
};

namespace fotci {
// host helpers
int pair_index(int a, int b, int ns);
void build_species_tables(const fotci_jumps *j, int species, HostSpeciesTables &t);
void block_pn(fotci_ham *h);
void fill_species_values(fotci_ham *h);

// device helpers (kernels_*.hip)
void launch_materialize(const fotci_ham *h, void *stream);
void launch_materialize_tiled(const DevHam &d, const DevTiled &t, void *stream);
void launch_apply(const fotci_ham *h, int mode, const void *x, void *y, void *stream);
void launch_apply_plain(const DevHam &d, int mode, const void *x, void *y, void *stream);
void launch_apply_tiled(const DevHam &d, const DevTiled &t, int mode, const void *x, void *y, void *stream,
                        void **events = nullptr);
void launch_apply_block(const DevHam &d, const DevTiled &t, int mode, int nb, const void *x, void *y, void *stream,
                        void **events = nullptr);
// pn part of the block apply (nb 2, 4 or 8; adds to y): the one-vector pn kernel with a vector stride
void launch_pn_block(const DevHam &d, const DevTiled &t, int mode, int nb, const void *x, void *y, void *stream);
// block apply with the per-kernel timing of launch_apply; nb == 1 is launch_apply
void launch_apply_nb(const fotci_ham *h, int mode, int nb, const void *x, void *y, void *stream);
void build_tiled_tables(fotci_ham *h);
void launch_one_body_density(const DevHam &d, const std::vector<int32_t> &h_sec_np, int q0, const double *g,
                             const double *x, double *rho_p, double *rho_n, void *stream);
// ncol: device buffer of n_nsd doubles for the neutron column sums, or NULL
// for the one in the Hamiltonian's workspace
void launch_vjp(const DevHam &d, const fotci_ham *h, const double *x, const double *g,
                double *dx, double *d_spe_p, double *d_spe_n, double *d_v_pp, double *d_v_nn,
                double *d_v_pn, void *stream, double *ncol = nullptr);
// The allocation-free adjoint's scratch: a static device array of
// kStaticNcolMax doubles; its address on the current device (looked up once
// per device).
constexpr int kStaticNcolMax = 1 << 16;
double *static_ncol_scratch();
int64_t lanczos_bytes(const fotci_ham *h, const fotci_lanczos_opts *o);
void lanczos_run(const fotci_ham *h, const fotci_lanczos_opts *o, const double *pivot, void *work,
                 int64_t work_bytes, double *evals, double *resid, double *evecs, double *alpha,
                 double *beta, void *stream);
int64_t trlan_bytes(const fotci_ham *h, const fotci_trlan_opts *o);
void trlan_run(const fotci_ham *h, const fotci_trlan_opts *o, const double *pivot, void *work, int64_t work_bytes,
               double *evals, double *resid, double *evecs, int32_t *stats, void *stream);
int64_t block_lanczos_bytes(const fotci_ham *h, const fotci_block_lanczos_opts *o);
void block_lanczos_run(const fotci_ham *h, const fotci_block_lanczos_opts *o, const double *pivot, void *work,
                       int64_t work_bytes, double *evals, double *resid, double *evecs, int32_t *n_done,
                       void *stream);
void hip_check(int err, const char *what);

// tridiagonal symmetric eigenproblem (host, float64): implicit QL with
// Wilkinson shifts; eigenvalues ascending in d, eigenvectors in z (n x n,
// column k = eigenvector k, row-major storage z[i*n+k]).
void tridiag_eig(int n, std::vector<double> &d, std::vector<double> e, std::vector<double> &z);
// dense symmetric eigenproblem (host, float64), cyclic Jacobi; a: n x n
// row-major; same output layout as tridiag_eig
void sym_eig(int n, std::vector<double> a, std::vector<double> &d, std::vector<double> &z);

}  // namespace fotci
