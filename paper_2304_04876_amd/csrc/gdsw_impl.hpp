// Internal state of a GDSW handle: host symbolic data (built by the analysis
// in symbolic.cpp) and the device buffers of the numerical setup and solve
// phases (device.hip).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gdsw.h"

namespace gdsw {

// A dense block of the coarse basis Phi: rows are global dofs, columns are
// coarse columns; values are stored column-major (nr x k).  Row sets of
// different blocks are disjoint, so Phi is the union of its blocks.
struct PhiBlocks {
    std::vector<int64_t> row_ptr;   // [nb+1] offsets into rows
    std::vector<int32_t> rows;      // global dofs
    std::vector<int64_t> col_ptr;   // [nb+1] offsets into cols (= partial index base)
    std::vector<int32_t> cols;      // coarse columns (ascending within a block)
    std::vector<int64_t> val_off;   // [nb+1] offsets into the value array
    std::vector<int32_t> kind;      // 0 = interior of a subdomain, 1 = interface component
    std::vector<int32_t> owner;     // subdomain or component id
    int32_t nb = 0;
};

// Nested-dissection supernodal factor of the local matrices (exact local
// solver with exact_order = GDSW_ORDER_ND).  Per subdomain the rows are
// renumbered by recursive vertex-separator bisection (new local index p:
// old local row perm[ov_ptr[i] + p]); a supernode is a leaf part or a
// separator, columns [first, first + ncol) of the new numbering, ordered
// children before parents.  Its panel holds L's columns first..first+ncol-1
// on the rows first..first+ncol-1 and then on its struct rows (ascending
// new indices, all beyond the supernode), column-major with leading
// dimension nrow = ncol + |struct|.
// LDS bytes of the supernodal solve (k_nd_apply) for subdomains of at most
// `rows` rows, `trows` rows of one height above the leaves and `nsn`
// supernodes with accumulators of `acc` bytes: the vector (rows), the pass
// results of one height (trows; the leaves need none), each rounded up to
// 4, the supernode table (16 B each), the struct offsets (nsn + 1 ints) and
// each row's supernode (16-bit).  A subdomain takes the supernodal factor
// only if it has at most ND_MAX_SUPERNODES supernodes, at most ND_MAX_TROWS
// rows of one height above the leaves and nd_lds_bytes(rows, ND_MAX_TROWS,
// ND_MAX_SUPERNODES, acc) fits a compute unit's 160 KiB, so that any set of
// such subdomains fits one launch (FP64 accumulators: up to 10,648 rows;
// FP32: up to 19,112).
constexpr int ND_MAX_SUPERNODES = 2048;
constexpr int ND_MAX_TROWS = 2048;
// leaf parts of the dissection: at most this many rows (at most 64, one
// wavefront's rows; on the 128^3 workload leaves of 32, 40, 48, 56 and 64
// rows gave 1.85, 1.32, 1.33, 1.38 and 1.44 ms per launch inside the apply,
// and 48 the most applies/s and batch solves/s)
constexpr int ND_LEAF = 48;
inline size_t nd_lds_bytes(int rows, int trows, int nsn, size_t acc) {
    const size_t r4 = (size_t(rows) + 3) / 4 * 4, t4 = (size_t(trows) + 3) / 4 * 4;
    return acc * (r4 + t4) + 16 * size_t(nsn) + 4 * (size_t(nsn) + 1) + 2 * r4;
}

struct NDSym {
    std::vector<int32_t> perm;        // [sum n_i]
    std::vector<int64_t> sn_ptr;      // [np+1] supernodes of each subdomain (global ids)
    std::vector<int32_t> first, ncol, nrow, height;   // [nsn]
    std::vector<int64_t> voff;        // [nsn+1] panel value offsets (all subdomains)
    std::vector<int64_t> st_ptr;      // [nsn+1] struct rows
    std::vector<int32_t> st_row;      //   new local indices
    std::vector<int32_t> row_sn;      // [sum n_i] supernode (global id) holding each new row
    // forward solve: each row gathers the products of the earlier supernodes
    // whose struct holds it (contributor K, row position in K's panel)
    std::vector<int64_t> rc_ptr;      // [sum n_i + 1]
    std::vector<int32_t> rc_sn, rc_pos;
    // the same gathers as struct entries relative to the subdomain's first
    // (the solve keeps each struct product in a vector laid out like st_row)
    std::vector<int32_t> rc_w;
    std::vector<int32_t> st_sn;       // [struct entries] supernode holding each
    // rows by height of their supernode (leaves 0): per subdomain a list of
    // level offsets into its slice of lv_rows (slice i starts at ov_ptr[i])
    std::vector<int64_t> lv_base;     // [np+1] offsets into lv_ptr (nlev_i + 1 each)
    std::vector<int32_t> lv_ptr;
    std::vector<int32_t> lv_rows;     // [sum n_i] new local rows (supernodes are
                                      // numbered by height: the identity)
    // per lv_ptr entry: {first struct entry of the height's supernodes
    // (relative to the subdomain's first), multiply-adds of their diagonal
    // blocks, of their struct parts, 0}
    std::vector<int32_t> lv_info;
    // the leaves' rows in chunks of at most 64 rows that split no leaf (the
    // leaves are numbered first): chunk boundaries of subdomain i at
    // ch_row[ch_base[i] .. ch_base[i+1]) (a leading 0, then each chunk's end;
    // an empty slice for band subdomains)
    std::vector<int64_t> ch_base;     // [np+1]
    std::vector<int32_t> ch_row;
    // left-looking factor: the earlier supernodes K updating J (ascending K):
    // struct(K) from index s0 on lies in J's panel rows (the first n1 of them
    // in J's columns), at panel rows rel[rel_off .. + |struct(K)| - s0)
    std::vector<int64_t> up_ptr;      // [nsn+1]
    std::vector<int32_t> up_k, up_s0, up_n1;
    std::vector<int64_t> up_rel;
    std::vector<int32_t> rel;
    // assembly: lower entries of A_i -> panel values
    std::vector<int64_t> asm_src;     // position in A's CSR
    std::vector<int64_t> asm_dst;     // panel value index
    int32_t max_ncol = 0, max_levels = 0, max_sn = 0;
    int32_t max_t = 0;                // most rows of one height above the leaves
    int64_t nsn = 0;
};

struct Symbolic {
    // ---- input copy -----------------------------------------------------
    int64_t n = 0, nn = 0, nnz = 0;
    int32_t dpn = 1, np = 1;
    gdsw_options opt{};
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<int32_t> part;      // [nn]
    // optional sharing sets (gdsw_analyze_sharing): the subdomains whose
    // elements hold each node; empty for the algebraic interface
    std::vector<int64_t> share_ptr; // [nn+1]
    std::vector<int32_t> share_sub;
    std::vector<double> Z;          // [n x n_null] column-major
    int32_t n_null = 1;

    // ---- node graph --------------------------------------------------------
    std::vector<int64_t> gptr;      // [nn+1]
    std::vector<int32_t> gadj;

    // ---- overlapping subdomains ---------------------------------------------
    std::vector<int64_t> ov_ptr;    // [np+1] dof offsets (local row p = ov_ptr[i] + l)
    std::vector<int32_t> ov_idx;    // global dofs, ascending per subdomain
    int32_t max_ni = 0;

    // transpose of the restriction maps: for dof d the local rows p that
    // hold it, in ascending subdomain order
    std::vector<int64_t> t_ptr;     // [n+1]
    std::vector<int32_t> t_pos;     // local rows p (int32: sum |Omega'| < 2^31)

    // ---- interface ------------------------------------------------------------
    std::vector<int8_t> is_gamma;       // [nn]
    std::vector<int32_t> comp_of_node;  // [nn], -1 interior
    std::vector<int64_t> comp_ptr;      // [nc+1]
    std::vector<int32_t> comp_nodes;
    std::vector<int32_t> comp_rank;     // coarse columns touching each component (k_c)
    std::vector<int64_t> ccol_ptr;      // [nc+1]
    std::vector<int32_t> ccol;          // those columns, ascending (GDSW: the component's own)
    std::vector<int32_t> col_comp;      // [n0] component a coarse column belongs to (its coarse node)
    std::vector<int64_t> phig_off;      // [nc+1] offsets of the interface blocks
    std::vector<double> phig;           // column-major (|c|*dpn x k_c) blocks
    int32_t nc = 0, n0 = 0;
    int64_t n_gamma_nodes = 0;

    // ---- interior sets and the extension ------------------------------------------
    std::vector<int64_t> int_ptr;   // [np+1] offsets of interior dofs
    std::vector<int32_t> int_idx;   // global interior dofs, ascending per subdomain
    std::vector<int64_t> scol_ptr;  // [np+1] coarse columns adjacent to I_i
    std::vector<int32_t> scol;
    // couplings A_{I_i, Gamma}: per interior row (global interior row index q)
    std::vector<int64_t> cpl_ptr;   // [n_int+1]
    std::vector<int64_t> cpl_apos;  // position in A's CSR
    std::vector<int64_t> cpl_phi;   // offset of the Phi_G row of the Gamma dof
    std::vector<int32_t> cpl_stride;// rows of that component block
    std::vector<int32_t> cpl_rank;  // columns of that component block
    std::vector<int32_t> cpl_slot;  // start in cpl_slotmap of the slots of those columns in scol of i
    std::vector<int32_t> cpl_slotmap;   // per (subdomain, adjacent component): slot of each block column
    // extension value offsets (column-major n_Ii x k_i per subdomain)
    std::vector<int64_t> ext_off;   // [np+1]

    // ---- local matrices ---------------------------------------------------------------
    // A_i in CSR over local rows p (all subdomains concatenated)
    std::vector<int64_t> lrowptr;   // [sum n_i + 1]
    std::vector<int32_t> lcol;      // local column within the subdomain
    std::vector<int64_t> lgpos;     // position in A's CSR
    // nested-dissection supernodal factors (exact local solver): the
    // subdomains that take it (1) instead of the band (0)
    NDSym nd;
    std::vector<uint8_t> nd_mask;
    // band Cholesky profiles (exact local solver, natural order)
    std::vector<int32_t> bw;        // [np] lower bandwidth b_i of A_i
    std::vector<int64_t> band_off;  // [np+1] offsets, row-major (b_i+1) per row
    std::vector<int64_t> bscat_dst; // band positions of the lower entries of A_i
    std::vector<int64_t> bscat_src; // their positions in A's CSR
    // same for A_{I_i I_i}
    std::vector<int32_t> ibw;
    std::vector<int64_t> iband_off;
    std::vector<int64_t> ibscat_dst;
    std::vector<int64_t> ibscat_src;
    int32_t max_bw = 0, max_ibw = 0, max_nii = 0;

    // ---- ILU(0) level schedule and sweep layout -----------------------------------------
    std::vector<int64_t> lvl_base;  // [np+1] offsets into lvl_ptr (each subdomain has nl_i+1)
    std::vector<int32_t> lvl_ptr;   // local offsets into the subdomain's lvl_rows slice
    std::vector<int32_t> lvl_rows;  // local rows by level, slice i starts at ov_ptr[i]
    std::vector<int32_t> ldiag;     // [sum n_i] position (relative to lrowptr) of the diagonal
    int32_t KL = 0, KU = 0;         // max strictly lower / upper entries per row
    std::vector<int64_t> ell_off;   // [np+1] padded row offsets
    int64_t ell_rows = 0;
    // FastILU: per local entry its product pairs (positions into the local
    // values, two int32 each) and the pivot position of a lower entry (-1)
    std::vector<int64_t> fi_ptr;
    std::vector<int32_t> fi_pairs;
    std::vector<int32_t> fi_dpos;

    // ---- coarse space ---------------------------------------------------------------
    PhiBlocks blk;
    std::vector<int64_t> red_ptr;   // [n0+1] partials of each coarse column
    std::vector<int32_t> red_idx;
    std::vector<int32_t> dof_blk;   // [n] block holding the Phi row of d, -1 none
    std::vector<int32_t> dof_lr;    // [n] row within that block
    // A_0 assembly: interface-interface pairs
    std::vector<int32_t> pair_c, pair_d;      // component pairs (c, d)
    std::vector<int64_t> pair_off;            // [npairs+1] offsets of their r_c x r_d blocks
    std::vector<int64_t> pair_eptr;           // [npairs+1] entry lists
    std::vector<int64_t> pair_apos;
    std::vector<int32_t> pair_lr_c, pair_lr_d;
    // subdomain contributions E_i^T X_i scattered into A_0
    std::vector<int64_t> t1_off;              // [np+1] offsets of the k_i x k_i blocks
    std::vector<int64_t> a0seg_tgt;           // target index a*n0+b of each segment
    std::vector<int64_t> a0seg_ptr;           // [nseg+1]
    std::vector<int64_t> a0seg_src;           // index into the T1 buffer
    std::vector<int64_t> a0pair_tgt;          // target of every T2 value (same order as values)
    std::vector<int64_t> a0seg2_tgt;          // T2 values added by target (several pairs may
    std::vector<int64_t> a0seg2_ptr;          //   share a target when components share
    std::vector<int64_t> a0seg2_src;          //   coarse columns), ascending pair order

    // ---- independent problems packed in one handle (block-diagonal A) ----------
    int32_t nprob = 1;
    std::vector<int64_t> prob_ptr;  // [nprob+1] dof offsets
    std::vector<int32_t> prob_sub;  // [nprob+1] subdomain offsets
    std::vector<int32_t> prob_c0;   // [nprob+1] coarse column offsets
    std::vector<int64_t> a0_off;    // [nprob+1] offsets of the dense A_0 blocks
    std::vector<int32_t> cprob;     // [n0] problem of each coarse column
    std::vector<int32_t> sub_prob;  // [np] problem of each subdomain

    double t_analyze = 0.0;
};

struct Device;   // device buffers (device.hip)

}  // namespace gdsw

struct gdsw_handle_s {
    gdsw::Symbolic sym;
    gdsw::Device *dev = nullptr;
    std::string err;
    bool analyzed = false;
    bool factored = false;
    double t_factor = 0.0;
    double t_refactor = 0.0;   // last numeric re-setup
};

namespace gdsw {
// symbolic.cpp
gdsw_status analyze(gdsw_handle_s *h, const gdsw_csr *A, const int32_t *part, int32_t n_parts,
                    int32_t dpn, const double *Z, int32_t n_null, const gdsw_options *opt,
                    const int64_t *share_ptr = nullptr, const int32_t *share_sub = nullptr);
gdsw_status analyze_batch(gdsw_handle_s *h, int32_t count, const gdsw_csr *A, const int32_t *const *part,
                          const int32_t *n_parts, int32_t dpn, const double *const *Z, int32_t n_null,
                          const gdsw_options *opt);
// nd.cpp: the nested-dissection supernodal structure of every A_i (needs
// the local CSR of build_local)
void build_nd(Symbolic &s);
// device.hip
gdsw_status factor(gdsw_handle_s *h, void *stream);
gdsw_status refactor(gdsw_handle_s *h, const double *val, void *stream);
gdsw_status apply(gdsw_handle_s *h, const double *r, double *z, int which, void *stream);
gdsw_status apply_static(gdsw_handle_s *h, const double *r, double *z, void *stream);
int64_t slot_bytes(const gdsw_handle_s *h);
gdsw_status spmv(gdsw_handle_s *h, const double *x, double *y, void *stream);
gdsw_status solve(gdsw_handle_s *h, const double *b, double *x, int krylov, int restart,
                  double rtol, int maxit, int fixed_iters, gdsw_solve_info *info, int ninfo, void *stream);
gdsw_status slots_begin(gdsw_handle_s *h, const double *b, double *x, double rtol, int maxit, void *stream);
gdsw_status slot_start(gdsw_handle_s *h, int slot, void *stream);
gdsw_status slots_step(gdsw_handle_s *h, int iters, int32_t *state, void *stream);
gdsw_status slot_finish(gdsw_handle_s *h, int slot, gdsw_solve_info *info, void *stream);
gdsw_status autotune(gdsw_handle_s *h, int reps, float *times, void *stream);
gdsw_status profile_local(gdsw_handle_s *h, int enable);
gdsw_status profile_read(gdsw_handle_s *h, float *ms, int max, int *count);
gdsw_status set_launch(gdsw_handle_s *h, int local_variant, int gemv_variant, int apply_streams, int prolong_variant,
                       void *stream);
int tuned_variant(const gdsw_handle_s *h, int which);
gdsw_status set_size_classes(gdsw_handle_s *h, int split);
void destroy_device(gdsw_handle_s *h);
int64_t device_bytes(const gdsw_handle_s *h);
gdsw_status copy_device_map(gdsw_handle_s *h, int map, void *out);
}  // namespace gdsw
