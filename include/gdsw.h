/*
 * gdsw.h -- C ABI of the GDSW two-level overlapping Schwarz preconditioner
 * for AMD Instinct MI355X (gfx950).
 *
 * The library applies
 *
 *     M^{-1} r = sum_i R_i^T A_i^{-1} R_i r + Phi A_0^{-1} Phi^T r        (paper eq. (1))
 *
 * with the energy-minimising GDSW coarse basis
 *
 *     Phi = [ -A_II^{-1} A_IG ; I ] Phi_G,     A_0 = Phi^T A Phi           (paper eq. (2))
 *
 * inside preconditioned CG or GMRES, in the paper's three phases (Sec. V-A,
 * "Software Structure"): a host-side symbolic analysis (gdsw_analyze), a
 * device-side numerical setup (gdsw_factor) and device-side applies/solves.
 *
 * Conventions shared by every entry point:
 *  - Host pointers are read during the call only; the caller keeps ownership
 *    and may free them afterwards.  Device pointers (suffix _dev) are HIP
 *    device addresses; the caller owns them and they must stay valid until
 *    the work queued on `stream` has finished.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is queued on it; entry points do not synchronise except where
 *    stated (gdsw_factor, gdsw_solve poll the device for convergence).
 *  - Every entry point returns a gdsw_status and never aborts.  On error the
 *    handle (when there is one) keeps a message for gdsw_last_error.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Sizes are int64_t; matrix column indices are int32_t (n < 2^31).
 */
#ifndef GDSW_H
#define GDSW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gdsw_handle_s *gdsw_handle;

typedef enum {
    GDSW_OK = 0,
    GDSW_ERR_INVALID_ARG = 1,   /* bad shape, index, option or non-finite value   */
    GDSW_ERR_SINGULAR = 2,      /* non-positive pivot in a Cholesky / zero ILU pivot */
    GDSW_ERR_BREAKDOWN = 3,     /* Krylov breakdown (NaN/Inf or zero denominator)   */
    GDSW_ERR_NOT_CONVERGED = 4, /* maxit reached before the tolerance              */
    GDSW_ERR_BUDGET = 5,        /* device memory budget exceeded / allocation failed */
    GDSW_ERR_HIP = 6,           /* a HIP runtime call failed                        */
    GDSW_ERR_STATE = 7,         /* call out of order (e.g. apply before factor)     */
    GDSW_ERR_INTERNAL = 8
} gdsw_status;

/* Coarse space of eq. (1): none (one-level), GDSW (eq. (2); one block of
 * the null space per interface component), or the reduced GDSW variant the
 * paper's experiments use (Sec. III, variants of GDSW; Sec. VII): coarse
 * functions only for the interface components whose set of meeting
 * subdomains is not contained in another component's (the cross points of a
 * box partition with a 27-point coupling); every other component is shared
 * among the coarse nodes whose sets strictly contain its own, each with
 * weight 1 / (their number), and each coarse node's functions are the
 * weighted null space over its support, orthonormalised, then extended by
 * eq. (2). */
enum { GDSW_COARSE_NONE = 0, GDSW_COARSE_GDSW = 1, GDSW_COARSE_RGDSW = 2 };

/* Local solver for A_i^{-1}: exact (banded Cholesky, A_i must be SPD;
 * Sec. V-B "Sparse Direct Matrix Factorization") or ILU(0) in the natural
 * order with Jacobi-sweep triangular solves (Sec. V-B "Incomplete Local
 * Solver"). */
enum { GDSW_LOCAL_EXACT = 0, GDSW_LOCAL_ILU0 = 1 };

/* Storage precision of the local factors and the coarse basis Phi.
 * Arithmetic is FP32 for the reduced formats and FP64 for GDSW_FP64; the
 * coarse matrix, its inverse and all Krylov vectors stay FP64 (the paper's
 * half-precision preconditioner, Sec. V-A "Lower Precision Preconditioning",
 * applied to the local parts only). */
enum { GDSW_FP64 = 0, GDSW_FP32 = 1, GDSW_BF16 = 2, GDSW_FP16 = 3 };

/* Option flags.  GDSW_FLAG_GRAPHS: CG iterations (gdsw_solve, gdsw_solve_batch,
 * gdsw_slots_step) are queued as captured HIP graphs of k iterations, one
 * graph per (x pointer, k) kept by the handle and replayed on the caller's
 * stream, instead of kernel by kernel; results are bit-identical. */
enum { GDSW_FLAG_GRAPHS = 1 };

/* Krylov method of gdsw_solve. */
enum { GDSW_KRYLOV_CG = 0, GDSW_KRYLOV_GMRES = 1, GDSW_KRYLOV_GMRES_SR = 2 };

typedef struct {
    int32_t overlap;          /* layers of graph overlap (>= 0); paper: 1        */
    int32_t coarse;           /* GDSW_COARSE_*                                    */
    int32_t local;            /* GDSW_LOCAL_*                                     */
    int32_t jacobi_sweeps;    /* sweeps per triangle for ILU(0); paper: 5         */
    int32_t local_prec;       /* GDSW_FP64 / FP32 / BF16 / FP16                   */
    int32_t basis_prec;       /* GDSW_FP64 / FP32 (storage of Phi)                */
    int64_t hbm_budget_bytes; /* device bytes the handle may allocate; 0 = no cap */
    uint64_t flags;           /* GDSW_FLAG_* bits, 0 by default                   */
    int32_t ilu_level;        /* GDSW_LOCAL_ILU0 only: level of fill k of ILU(k)
                                 (Sec. V-B, levels varied in Sec. VII-C); 0..8,
                                 default 0                                         */
    int32_t ilu_factor_sweeps;/* GDSW_LOCAL_ILU0 only: 0 = exact incomplete
                                 factors (level-scheduled, row by row); s > 0 =
                                 the iterative FastILU variant, s Jacobi sweeps
                                 over the factor entries (Sec. V-B; the paper's
                                 experiments use 3); default 0                    */
    int32_t slots;            /* right-hand-side slots per problem (>= 1; 0 is read
                                 as 1): the handle keeps one factored operator
                                 and preconditions `slots` right-hand sides of
                                 every problem with it.  Vectors passed to
                                 gdsw_apply, gdsw_spmv, gdsw_solve(_batch) and
                                 gdsw_slots_begin then hold the slots one after
                                 another (length slots * n; dof d of slot k at
                                 k n + d); slot k of problem p is the Krylov
                                 problem k * n_problems + p (its dof range from
                                 gdsw_problem_offsets).  Only the per-slot
                                 vectors and intermediate results are
                                 allocated per slot; slots * n < 2^31.
                                 GMRES needs slots = 1.  Default 1.              */
    int32_t exact_order;      /* GDSW_LOCAL_EXACT only: GDSW_ORDER_NATURAL (band
                                 Cholesky in the natural local order),
                                 GDSW_ORDER_ND (nested dissection by vertex
                                 separators, supernodal Cholesky; Sec. V-B,
                                 sparse direct factorization) for every
                                 subdomain whose solve fits the 160 KiB of
                                 LDS (at most 10,648 local rows with FP64
                                 factors, 19,112 otherwise, 2,048 supernodes
                                 and 2,048 rows of one height above the
                                 leaves), the band for the others, or
                                 GDSW_ORDER_AUTO (per subdomain whichever of
                                 the two stores fewer factor values, when its
                                 supernodal solve fits LDS; the choice depends
                                 on the subdomain alone, gdsw_info.nd_subdomains
                                 counts the supernodal ones).  Default NATURAL */
} gdsw_options;

/* Orderings of the exact local factor (options.exact_order). */
enum { GDSW_ORDER_NATURAL = 0, GDSW_ORDER_ND = 1, GDSW_ORDER_AUTO = 2 };

/* Square sparse matrix in CSR form, HOST pointers: rowptr[n+1] (int64),
 * col[nnz] (int32, sorted ascending within each row), val[nnz] (FP64). */
typedef struct {
    int64_t n;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
} gdsw_csr;

typedef struct {
    int32_t iterations;       /* Krylov iterations performed                     */
    int32_t converged;        /* 1 if the tolerance was met                       */
    double rel_res_recursive; /* ||r_k|| / ||b|| as tracked by the iteration      */
    double rel_res_true;      /* ||b - A x|| / ||b|| recomputed at the end        */
    double seconds;           /* wall time of the call                            */
} gdsw_solve_info;

typedef struct {
    int64_t n;                /* dofs                                             */
    int64_t n_nodes;
    int32_t dpn;              /* dofs per node                                    */
    int32_t n_parts;          /* subdomains                                       */
    int64_t sum_overlap_dofs; /* sum_i |Omega_i'| * dpn                           */
    int64_t n_gamma_nodes;    /* interface nodes                                  */
    int32_t n_components;     /* interface components                             */
    int32_t n0;               /* coarse dimension                                 */
    int64_t local_factor_entries;  /* stored local-factor values (all subdomains) */
    int64_t phi_entries;      /* stored coarse-basis values                       */
    int64_t device_bytes;     /* device memory held by the handle                 */
    int32_t max_local_rows;   /* largest overlapping subdomain (dofs)             */
    int32_t max_bandwidth;    /* largest local bandwidth (exact solver)           */
    double t_analyze;         /* seconds: host symbolic analysis                  */
    double t_factor;          /* seconds: device numerical setup (synchronised)   */
    int32_t n_problems;       /* independent problems packed in the handle        */
    int32_t local_variant;    /* launch configuration of the local solves (-1 = fixed rule) */
    int32_t gemv_variant;     /* coarse GEMV: -1 fixed rule, 0 wavefront, 1 workgroup per row */
    int32_t apply_streams;    /* coarse part of the apply: -1 fixed rule (second stream when
                                 the subdomains do not fill the compute units), 1 same stream
                                 as the local solves, 2 second stream                */
    int32_t prolong_variant;  /* coarse part of the prolongation: -1 fixed rule (by blocks
                                 when Phi holds >= 16 values per dof), 0 per dof,
                                 1 by blocks                                         */
    double t_refactor;        /* seconds: last numeric re-setup (gdsw_refactor,
                                 synchronised); 0 if there was none             */
    int32_t slots;            /* right-hand-side slots per problem (options.slots) */
    int64_t slot_bytes;       /* of device_bytes, the bytes held per slot (its
                                 vectors and intermediate results); the rest is
                                 the factored operator, held once            */
    int32_t exact_order;      /* options.exact_order                              */
    int32_t nd_subdomains;    /* subdomains with the supernodal (nested-dissection)
                                 exact factor; the others keep the band       */
    int32_t local_classes;    /* size classes the local solves run in (1, or
                                 more when gdsw_autotune found the split by
                                 size faster)                                 */
    int64_t local_solve_bytes;/* algorithmic bytes of one launch of the local
                                 solves (every stored factor value read once
                                 per pass, the index data once, per local row
                                 the restriction index, the gathered r and the
                                 local result)                                 */
} gdsw_info;

/* Integer maps that can be copied out for inspection (gdsw_map_size /
 * gdsw_copy_map).  All are produced by gdsw_analyze. */
enum {
    GDSW_MAP_OV_PTR = 0,       /* int64 [n_parts+1]: offsets into OV_IDX          */
    GDSW_MAP_OV_IDX = 1,       /* int64 [sum_overlap_dofs]: dofs of Omega_i', ascending */
    GDSW_MAP_IS_GAMMA = 2,     /* int8  [n_nodes]: 1 on the interface             */
    GDSW_MAP_COMP_OF_NODE = 3, /* int32 [n_nodes]: interface component, -1 if interior */
    GDSW_MAP_COMP_RANK = 4,    /* int32 [n_components]: coarse columns of each component */
    GDSW_MAP_PHI_ROWPTR = 5,   /* int64 [n+1]: CSR of Phi (after gdsw_factor)     */
    GDSW_MAP_PHI_COL = 6,      /* int32 [phi_entries]                             */
    GDSW_MAP_PHI_VAL = 7,      /* FP64  [phi_entries]  (after gdsw_factor)        */
    GDSW_MAP_A0 = 8,           /* FP64  coarse matrix, row-major (after gdsw_factor): [n0*n0]
                                  for one problem, the dense diagonal blocks one after
                                  another for a batch */
    GDSW_MAP_LOCAL_ROWPTR = 9, /* int64 [sum_overlap_dofs+1]: CSR row pointers of the
                                  local matrices' patterns (ILU(k) patterns with fill
                                  for GDSW_LOCAL_ILU0), subdomains one after another */
    GDSW_MAP_LOCAL_COL = 10,   /* int32 [local entries]: local column indices        */
    /* the nested-dissection supernodal structure (exact_order = ND; empty
     * otherwise): new local numbering, supernodes (children before parents),
     * their panels, the forward-solve row gathers, the rows by height, the
     * left-looking update lists and the assembly map */
    GDSW_MAP_ND_PERM = 11,     /* int32 [sum_overlap_dofs]: old local row of new row p  */
    GDSW_MAP_ND_SN_PTR = 12,   /* int64 [n_parts+1]: supernodes of each subdomain       */
    GDSW_MAP_ND_SN = 13,       /* int32 [4 nsn]: first column, columns, panel rows, height */
    GDSW_MAP_ND_VOFF = 14,     /* int64 [nsn+1]: panel value offsets                   */
    GDSW_MAP_ND_ST_PTR = 15,   /* int64 [nsn+1]                                        */
    GDSW_MAP_ND_ST_ROW = 16,   /* int32: struct rows (new local indices)                */
    GDSW_MAP_ND_RC_PTR = 17,   /* int64 [sum_overlap_dofs+1]                            */
    GDSW_MAP_ND_RC = 18,       /* int32 [2 nrc]: contributor supernode, panel row       */
    GDSW_MAP_ND_LV_BASE = 19,  /* int64 [n_parts+1]: offsets into ND_LV_PTR (nlev_i+1 each) */
    GDSW_MAP_ND_LV_PTR = 20,   /* int32: level offsets into the subdomain's rows by level */
    GDSW_MAP_ND_LV_ROWS = 21,  /* int32 [sum_overlap_dofs]: new rows by level, subdomains
                                  one after another (supernodes are numbered by height,
                                  so each slice is the identity)                         */
    GDSW_MAP_ND_UP_PTR = 22,   /* int64 [nsn+1]                                         */
    GDSW_MAP_ND_UP = 23,       /* int64 [4 nup]: K, s0, n1, offset into ND_REL          */
    GDSW_MAP_ND_REL = 24,      /* int32: panel rows of the update lists                 */
    GDSW_MAP_ND_ASM = 25,      /* int64 [2 nasm]: A CSR position, panel value index     */
    GDSW_MAP_ND_RC_W = 26,     /* int32 [nrc]: the gather entries as struct entries,
                                  relative to the subdomain's first                     */
    GDSW_MAP_ND_ST_SN = 27,    /* int32: supernode holding each struct entry            */
    GDSW_MAP_ND_LV_INFO = 28,  /* int32 [4 per ND_LV_PTR entry]: first struct entry of
                                  the height's supernodes (relative), multiply-adds of
                                  their diagonal blocks, of their struct parts, 0        */
    GDSW_MAP_ND_CH_BASE = 29,  /* int64 [n_parts+1]: offsets into ND_CH_ROW             */
    GDSW_MAP_ND_CH_ROW = 30    /* int32: per subdomain 0 and the end row of each chunk of
                                  whole leaves (at most 64 rows; one wavefront each)    */
};

/* Fills `opt` with the paper's defaults: overlap 1, GDSW coarse space,
 * exact local solver, 5 Jacobi sweeps, FP64 storage, no budget. */
void gdsw_default_options(gdsw_options *opt);

/* Phase (a), symbolic, host only (no device is touched).
 *   A        : the matrix (host CSR).  Values are copied for gdsw_factor.
 *   part     : [n/dpn] nonoverlapping subdomain of every node, in [0, n_parts).
 *   n_parts  : number of subdomains (>= 1).
 *   dpn      : dofs per node (dof = dpn*node + component), n % dpn == 0.
 *   Z        : [n x n_null] column-major null-space basis of the Neumann
 *              operator (Sec. III item 3), or NULL for the constants (then
 *              n_null must be 0 or 1).
 * Builds the node graph, the overlapping subdomains, the interface and its
 * components, the interface basis Phi_G (orthonormal per component), the
 * local orderings, band profiles, level schedules and all index maps.
 * Errors: INVALID_ARG for malformed input. */
gdsw_status gdsw_analyze(const gdsw_csr *A, const int32_t *part, int32_t n_parts,
                         int32_t dpn, const double *Z, int32_t n_null,
                         const gdsw_options *opt, gdsw_handle *out);

/* Phase (a) as gdsw_analyze, with the interface taken from given sharing
 * sets instead of the node graph: the geometric interface of a
 * decomposition into subdomains of elements (Sec. III: Gamma is the set of
 * nodes shared by two or more subdomains, its components are grouped by the
 * set of subdomains sharing them).
 *   share_ptr: [n/dpn + 1] int64, share_ptr[0] = 0, ascending (host);
 *   share_sub: [share_ptr[n/dpn]] int32 (host): for node v the subdomains
 *              whose elements contain v, at share_sub[share_ptr[v] ..
 *              share_ptr[v+1]) in any order (duplicates allowed).
 * Both are read during the call only.  Every node's set must contain
 * part[v]; a node with a set of one subdomain is interior, and each of its
 * graph neighbours must be shared by that subdomain (A_II block diagonal,
 * eq. (2)).  The overlapping subdomains still come from `part` and the
 * graph.  Errors: INVALID_ARG (NULL arrays, ids out of range, a set
 * without the node's own subdomain, an interior node coupled outside its
 * subdomain), otherwise as gdsw_analyze. */
gdsw_status gdsw_analyze_sharing(const gdsw_csr *A, const int32_t *part, int32_t n_parts,
                                 int32_t dpn, const double *Z, int32_t n_null,
                                 const int64_t *share_ptr, const int32_t *share_sub,
                                 const gdsw_options *opt, gdsw_handle *out);

/* Phase (b), numeric, on the current HIP device: uploads the maps, gathers
 * the local matrices, factors them, computes the extension Phi_I, assembles
 * A_0 and inverts it.  Synchronises `stream` before returning (so that
 * singular pivots are reported).  Errors: SINGULAR, BUDGET, HIP, STATE. */
gdsw_status gdsw_factor(gdsw_handle h, void *stream);

/* Numeric re-setup with new values on the same pattern (Sec. V-A: the
 * numerical phase repeated for a new matrix of the same structure).
 *   val: host FP64 array of the nnz values in the CSR order given to
 *        gdsw_analyze (copied during the call).
 * Keeps the symbolic analysis, every device map and buffer (the factors,
 * Phi, A_0^{-1} and the Krylov vectors stay at the same device addresses, so
 * captured graphs remain valid), the launch configurations chosen by
 * gdsw_autotune / gdsw_set_launch and the captured CG graphs; recomputes the
 * local factors, the extension Phi_I, A_0 and its inverse from the new
 * values.  The maps and scratch of the numerical setup stay resident from the
 * first call on (reported in device_bytes), so later calls upload and
 * allocate nothing.  A handle that is not factored is factored afresh.
 * Synchronises `stream`.  Errors: INVALID_ARG (non-finite value), SINGULAR
 * (the handle is then left unfactored), BUDGET, HIP. */
gdsw_status gdsw_refactor(gdsw_handle h, const double *val, void *stream);

/* gdsw_analyze followed by gdsw_factor. */
gdsw_status gdsw_setup(const gdsw_csr *A, const int32_t *part, int32_t n_parts,
                       int32_t dpn, const double *Z, int32_t n_null,
                       const gdsw_options *opt, void *stream, gdsw_handle *out);

/* Phase (c): z = M^{-1} r, eq. (1).  r_dev, z_dev: FP64 device vectors of
 * length n (distinct).  Queued on `stream`, no synchronisation. */
gdsw_status gdsw_apply(gdsw_handle h, const double *r_dev, double *z_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * z = M^{-1} r as gdsw_apply, bit for bit, with the apply's scratch (the
 * local results, the coarse restriction partials, r_0 and z_0, the blocked
 * coarse prolongation, the sweep iterates of subdomains too large for LDS,
 * the struct products of the supernodal solves) taken from a static device array of GDSW_STATIC_SCRATCH_BYTES per GPU
 * instead of the handle's own buffers.  Allocates nothing (no hipMalloc or
 * hipFree, no allocating library call); the array is held by every GPU the
 * library runs on until the process ends.  The current device must be the
 * one the handle was factored on.  Every call on one GPU, from any handle,
 * shares that GPU's array and leaves the last call's contents in it: calls
 * that overlap on one GPU (queued on different streams, or from different
 * threads) race and give wrong results; calls queued one after another on
 * one stream are safe.  r_dev, z_dev: FP64 device vectors of length n
 * (distinct), caller-owned.  Queued on `stream`, no synchronisation.
 * Errors: STATE (not factored), INVALID_ARG (bad pointers, other device),
 * BUDGET (the handle needs more scratch than the array holds; the message
 * gives both sizes), HIP. */
#define GDSW_STATIC_SCRATCH_BYTES 67108864
gdsw_status gdsw_apply_static(gdsw_handle h, const double *r_dev, double *z_dev, void *stream);

/* Parts of eq. (1) alone: which = 1 one-level sum only, 2 coarse term only,
 * 3 both (same as gdsw_apply); 4 = only the batched local solves
 * A_i^{-1} R_i r, kept in the handle's local buffer (z_dev unused, may be
 * NULL) -- used to time the local-solve kernel by itself. */
gdsw_status gdsw_apply_part(gdsw_handle h, const double *r_dev, double *z_dev,
                            int32_t which, void *stream);

/* y = A x with the matrix given to gdsw_analyze (FP64 device vectors). */
gdsw_status gdsw_spmv(gdsw_handle h, const double *x_dev, double *y_dev, void *stream);

/* Preconditioned Krylov solve of A x = b (Sec. VII), x0 = 0.
 *   krylov : GDSW_KRYLOV_CG, GDSW_KRYLOV_GMRES (right preconditioned,
 *            classical Gram-Schmidt applied twice: three reductions per
 *            iteration) or GDSW_KRYLOV_GMRES_SR (the single-reduce GMRES of
 *            the paper's experiments, Sec. VII: the same iterates in exact
 *            arithmetic, one reduction per iteration; the second projection
 *            pass and the normalisation of each basis vector are delayed to
 *            the next iteration, so convergence is seen one iteration later
 *            and one extra preconditioned product is formed).
 *            The GMRES variants need a handle with one problem.
 *   restart: GMRES restart length (paper: 30, at most 64); ignored by CG.
 *   rtol   : stop when ||r_k||_2 <= rtol ||b||_2.
 *   maxit  : iteration cap.  If fixed_iters > 0 exactly that many iterations
 *            are run whatever the residual (used to compare iterates).
 *   b_dev, x_dev: FP64 device vectors of length n; x_dev receives x.
 *   info   : optional, filled on return.
 * Synchronises `stream` to poll convergence.
 * Errors: NOT_CONVERGED (x holds the last iterate), BREAKDOWN. */
gdsw_status gdsw_solve(gdsw_handle h, const double *b_dev, double *x_dev,
                       int32_t krylov, int32_t restart, double rtol, int32_t maxit,
                       int32_t fixed_iters, gdsw_solve_info *info, void *stream);

/* ---- several independent problems in one handle ------------------------
 * A batch handle packs `count` independent problems (matrices of any size
 * and partition) as one block-diagonal system: their subdomains, interface
 * components and coarse blocks never couple, the coarse matrix is one dense
 * block per problem, and every kernel of the apply and the Krylov solve
 * covers all problems in one launch (many subdomains per launch, the
 * paper's reason for running several subdomains per GPU, Sec. VI).  Each
 * problem keeps its own Krylov scalars and stopping test, and its
 * reductions use row blocks of its own, so its results are the same alone
 * and in a batch.  Vectors of a batch handle are the concatenation of the
 * problems' vectors (length = sum of the n_k, problem k first at offset
 * sum_{j<k} n_j).
 *   A[count], part[count] ([n_k/dpn] each), n_parts[count]: per problem,
 *   Z: NULL (constants) or Z[count] column-major [n_k x n_null] blocks. */
gdsw_status gdsw_analyze_batch(int32_t count, const gdsw_csr *A, const int32_t *const *part,
                               const int32_t *n_parts, int32_t dpn, const double *const *Z,
                               int32_t n_null, const gdsw_options *opt, gdsw_handle *out);

/* CG on every problem of a (batch) handle; infos[count] receives one record
 * per problem (gdsw_solve on a batch handle reports the worst problem). */
gdsw_status gdsw_solve_batch(gdsw_handle h, const double *b_dev, double *x_dev, double rtol,
                             int32_t maxit, gdsw_solve_info *infos, void *stream);

/* ---- continuous batching over the problems ("slots") of a handle --------
 * gdsw_slots_begin binds caller-owned device vectors b_dev, x_dev (length
 *   sum n_k) and marks every slot idle.
 * gdsw_slot_start starts CG (x0 = 0) on slot k from the slot's rows of
 *   b_dev, which the caller has filled; other slots are not disturbed.
 * gdsw_slots_step advances every running slot by `iters` CG iterations in
 *   shared kernel launches, synchronises `stream` and writes state[k]:
 *   -1 idle, 0 running, 1 finished (result ready), 2 failed.
 * gdsw_slot_finish reads slot k's record (true residual of its rows
 *   recomputed), leaves its solution in its rows of x_dev and makes the
 *   slot idle.
 * Slots run concurrently; calls on one handle must not overlap. */
gdsw_status gdsw_slots_begin(gdsw_handle h, const double *b_dev, double *x_dev, double rtol,
                             int32_t maxit, void *stream);
gdsw_status gdsw_slot_start(gdsw_handle h, int32_t slot, void *stream);
gdsw_status gdsw_slots_step(gdsw_handle h, int32_t iters, int32_t *state, void *stream);
gdsw_status gdsw_slot_finish(gdsw_handle h, int32_t slot, gdsw_solve_info *info, void *stream);

/* Autotuner: times every launch configuration of the local-solve kernel
 * (ILU(0): register-resident sweeps with 512 or 1024 threads, streaming
 * sweeps with 256 or 512 threads; exact: band solves with 256, 512 or 1024
 * threads, one workgroup per subdomain or as persistent workgroups drawing
 * subdomains from a work counter), both coarse GEMV variants, and the whole
 * apply with the coarse part on the caller's stream after the local solves
 * or on a second stream beside them, on the handle's own factors, `reps`
 * launches each, and keeps the fastest for all later applies; also the
 * coarse part of the prolongation z += Phi z0 per dof (each dof reads its row
 * of Phi) or by blocks (each block of Phi times z0 streamed once on the
 * coarse chain, the per-dof pass then adds one value).  times_ms (optional,
 * host, 16 floats) receives the average milliseconds per launch (-1 for
 * configurations that do not fit): [0..7] local variants (ILU(0): 0..3,
 * exact: 0..5), [8..9] GEMV variants, [10..11] apply in one stream / two
 * streams, [12..13] apply with the prolongation per dof / by blocks,
 * [14..15] the local solves as one launch in size order / split into size
 * classes (subdomain sizes within a factor two, at most six classes,
 * each with its own tuned configuration, launched at once on streams of
 * their own; -1 when the sizes form one class).  Synchronises `stream`. */
gdsw_status gdsw_autotune(gdsw_handle h, int32_t reps, float *times_ms, void *stream);

/* Pins the launch configurations gdsw_autotune chooses from, for callers
 * that fix them themselves (and for tests of each configuration):
 *   local_variant: -1 = fixed rule, else an index of times_ms[0..3] above;
 *   gemv_variant : -1 = rule (workgroup per row from n0 >= 1024), 0 = one
 *                  wavefront per row, 1 = one workgroup per row;
 *   apply_streams: -1 = rule (two streams when there are fewer subdomains
 *                  than compute units), 1 or 2;
 *   prolong_variant: -1 = rule (by blocks when Phi holds at least 16
 *                  values per dof), 0 = per dof, 1 = by blocks (allocates
 *                  one vector of n doubles on first use).
 * The local variant is launched once on `stream` (on internal buffers) to
 * check that it fits the handle; one that does not (LDS, registers) gives
 * GDSW_ERR_INVALID_ARG and nothing changes.  The local-solve and stream
 * configurations compute each value in the same order (results do not
 * depend on them, and the two prolongation forms add each dof's products
 * in the same order); the two GEMV variants sum a row of A_0^{-1} in
 * different orders and agree to rounding. */
gdsw_status gdsw_set_launch(gdsw_handle h, int32_t local_variant, int32_t gemv_variant,
                            int32_t apply_streams, int32_t prolong_variant, void *stream);

/* Pins the other choice gdsw_autotune makes for the local solves: split = 0
 * runs them as one launch in size order (the default), split = 1 as one
 * launch per size class (subdomain sizes within a factor two, at most six
 * classes, the largest first), all at once on streams of their own, each
 * class with its tuned configuration (or the handle's).  Each subdomain's
 * solve is the same computation either way (the results do not change).
 * A handle whose subdomain sizes form one class ignores split = 1 and
 * reports one class in gdsw_info.local_classes.  Errors: STATE (not
 * factored), INVALID_ARG. */
gdsw_status gdsw_set_size_classes(gdsw_handle h, int32_t split);

/* Timing of the local solves where they run (Sec. VII times the local-solver
 * phase of the apply on its own).  With enable != 0 every later apply of the
 * handle, those inside the solvers included, records a pair of HIP events on
 * its stream just before and just after the local-solve launch, for up to
 * GDSW_PROFILE_MAX applies (later ones are not recorded), except while the
 * stream is being captured into a graph; enable != 0 also clears earlier
 * records, enable == 0 stops recording and keeps them.  Creates the events on
 * first use. */
#define GDSW_PROFILE_MAX 1024
gdsw_status gdsw_profile_local(gdsw_handle h, int32_t enable);

/* Waits for the recorded event pairs and writes the elapsed milliseconds of
 * the first min(count recorded, max) of them to ms (host, max floats);
 * *count receives the number recorded. */
gdsw_status gdsw_profile_read(gdsw_handle h, float *ms, int32_t max, int32_t *count);

/* Dof offsets of the Krylov problems of a handle, offsets[slots * n_problems
 * + 1] (host): problem p in slot k is entry k * n_problems + p, its rows
 * k n + (offsets of p). */
gdsw_status gdsw_problem_offsets(gdsw_handle h, int64_t *offsets);

gdsw_status gdsw_get_info(gdsw_handle h, gdsw_info *info);

/* Number of elements of a GDSW_MAP_* array, and a copy of it into host
 * memory of at least that many elements of the documented type. */
gdsw_status gdsw_map_size(gdsw_handle h, int32_t map, int64_t *count);
gdsw_status gdsw_copy_map(gdsw_handle h, int32_t map, void *host_out);

/* Releases all host and device memory of the handle (NULL is accepted). */
gdsw_status gdsw_destroy(gdsw_handle h);

const char *gdsw_status_string(gdsw_status s);
const char *gdsw_last_error(gdsw_handle h);

#ifdef __cplusplus
}
#endif
#endif /* GDSW_H */
