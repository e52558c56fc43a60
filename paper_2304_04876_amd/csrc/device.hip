// Device side of a GDSW handle: upload of the symbolic maps, the numerical
// setup (phase (b)), the preconditioner apply and the Krylov solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "gdsw_impl.hpp"
#include "kernels_apply.hpp"
#include "kernels_krylov.hpp"
#include "kernels_nd.hpp"
#include "kernels_setup.hpp"

// Scratch of the allocation-free apply (gdsw_apply_static): the local
// results, the coarse restriction partials, r_0, z_0 and its repetitions,
// the coarse part of the prolongation, the sweep iterates of large
// subdomains and the struct products of the supernodal solves, carved from
// this array instead of the handle's buffers.  Each
// GPU the library runs on holds its own copy until the process ends; host
// code uses the address hipGetSymbolAddress returns for the current device,
// never the array's name.
static __device__ __align__(256) unsigned char scratch[GDSW_STATIC_SCRATCH_BYTES];

#include <mutex>

namespace gdsw {

struct DevError {
    gdsw_status st;
    std::string msg;
};

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            throw DevError{GDSW_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

static inline int nblocks(int64_t n, int nt, int64_t cap = 1 << 20) {
    int64_t b = (n + nt - 1) / nt;
    if (b < 1) b = 1;
    return int(std::min(b, cap));
}

static size_t prec_size(int p) {
    switch (p) {
        case GDSW_FP64: return 8;
        case GDSW_FP32: return 4;
        default: return 2;
    }
}

constexpr int QUEUE_HALF = 4096;   // work counters per band-solve kind (one per slot)

// Device address of `scratch` on GPU `dev` (which must be the current
// device), looked up once per device and kept.
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES] = {};

static gdsw_status static_scratch(int dev, void **out, std::string *err) {
    if (dev < 0 || dev >= MAX_DEVICES) {
        *err = "device index out of range for the static scratch table";
        return GDSW_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return GDSW_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    if (out) *out = g_scratch_ptr[dev];
    return GDSW_OK;
}

struct Device {
    std::vector<void *> allocs;
    int64_t bytes = 0;
    int64_t budget = 0;

    void *raw_alloc(size_t sz) {
        if (sz == 0) sz = 16;
        if (budget > 0 && bytes + int64_t(sz) > budget)
            throw DevError{GDSW_ERR_BUDGET, "device memory budget exceeded"};
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, sz);
        if (e != hipSuccess) throw DevError{GDSW_ERR_BUDGET, std::string("hipMalloc: ") + hipGetErrorString(e)};
        allocs.push_back(p);
        bytes += int64_t(sz);
        return p;
    }
    void release(void *p, size_t sz) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) {
            allocs.erase(it);
            (void)hipFree(p);
            bytes -= int64_t(sz == 0 ? 16 : sz);
        }
    }
    template <typename T>
    T *alloc(int64_t count) { return static_cast<T *>(raw_alloc(sizeof(T) * size_t(std::max<int64_t>(count, 1)))); }
    template <typename T>
    T *upload(const std::vector<T> &v, hipStream_t s) {
        T *p = alloc<T>(int64_t(v.size()));
        if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
        return p;
    }
    // Buffers of the numerical setup alone: uploaded index maps of the
    // analysis (which do not depend on the matrix values) and scratch.  The
    // first factorisation frees them when it is done; from the first numeric
    // re-setup on (gdsw_refactor) they stay resident, keyed by the host
    // vector they hold or by a scratch tag, so that later re-setups neither
    // upload maps nor allocate.
    bool keep_setup = false;
    struct Held {
        const void *key;
        void *p;
        size_t sz;
    };
    std::vector<Held> held;
    void *held_find(const void *key, size_t sz) const {
        for (const Held &x : held)
            if (x.key == key) {
                if (x.sz != std::max<size_t>(sz, 16)) throw DevError{GDSW_ERR_INTERNAL, "setup buffer size changed"};
                return x.p;
            }
        return nullptr;
    }
    template <typename T>
    T *setup_upload(const std::vector<T> &v, hipStream_t s) {
        const size_t sz = sizeof(T) * std::max<size_t>(v.size(), 1);
        if (keep_setup)
            if (void *p = held_find(&v, sz)) return static_cast<T *>(p);
        T *p = upload(v, s);
        if (keep_setup) held.push_back({&v, p, std::max<size_t>(sz, 16)});
        return p;
    }
    template <typename T>
    T *setup_scratch(int tag, int64_t count) {
        const void *key = reinterpret_cast<const void *>(uintptr_t(tag));
        const size_t sz = sizeof(T) * size_t(std::max<int64_t>(count, 1));
        if (keep_setup)
            if (void *p = held_find(key, sz)) return static_cast<T *>(p);
        T *p = static_cast<T *>(raw_alloc(sz));
        if (keep_setup) held.push_back({key, p, std::max<size_t>(sz, 16)});
        return p;
    }
    void setup_release(void *p, size_t sz) {
        if (!keep_setup) release(p, sz);
    }
    // the coarse part of an apply runs on `side` beside the local solves
    // (fork/join with two events); created with the default priority
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int apply_streams = -1;   // -1: rule (two streams when np < compute units), 1 or 2: tuned
    int n_cu = 256;
    // captured CG chunks (GDSW_FLAG_GRAPHS): key (x, iterations)
    hipStream_t cap = nullptr;
    struct CgGraph {
        const double *x;
        int iters, par;
        hipGraphExec_t exec;
    };
    std::vector<CgGraph> cg_graphs;
    // timing of the local solves inside applies (gdsw_profile_local): event
    // pair i brackets the local-solve launch of the i-th recorded apply
    bool prof_on = false;
    int prof_n = 0;
    std::vector<hipEvent_t> prof_ev;

    ~Device() {
        for (hipEvent_t e : prof_ev) (void)hipEventDestroy(e);
        for (auto &g : cg_graphs) (void)hipGraphExecDestroy(g.exec);
        if (cap) (void)hipStreamDestroy(cap);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_cfork) (void)hipEventDestroy(ev_cfork);
        for (int k = 0; k < MAX_CLASSES - 1; ++k) {
            if (ev_cjoin[k]) (void)hipEventDestroy(ev_cjoin[k]);
            if (cstream[k]) (void)hipStreamDestroy(cstream[k]);
        }
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
        for (void *p : allocs) (void)hipFree(p);
    }

    // ---- matrix ----
    int32_t *rowptr = nullptr, *col = nullptr, *arow = nullptr;
    double *val = nullptr;
    int64_t *adiag = nullptr;
    double *dscale = nullptr;   // diagonal scaling of reduced-precision factors (or null)
    // ---- restriction / prolongation ----
    int32_t *ov_idx = nullptr;
    int64_t *ov_ptr = nullptr;
    int32_t *t_ptr = nullptr;
    Sell sell{};          // A for the SpMV
    int32_t *t_pos = nullptr;
    double *zloc = nullptr;
    // ---- local factors ----
    void *band = nullptr;   // exact: band in local precision
    int64_t *band_off = nullptr;
    int32_t *bw = nullptr;
    void *Lv = nullptr, *Uv = nullptr, *dinv = nullptr;   // ILU(0): sweep layout
    uint16_t *Lc = nullptr, *Uc = nullptr;
    uint32_t *Cp = nullptr;   // the columns packed by row (register-resident sweeps only)
    int64_t *ell_off = nullptr;
    // ---- coarse ----
    int64_t *blk_row_ptr = nullptr, *blk_col_ptr = nullptr, *blk_val_off = nullptr;
    int32_t *blk_rows = nullptr;
    double *phi = nullptr;    // FP64 coarse-basis values
    float *phi32 = nullptr;   // FP32 copy when basis_prec == FP32
    int64_t *red_ptr = nullptr;
    int32_t *red_idx = nullptr;
    int64_t *blk_poff = nullptr;   // first restriction partial of every block
    int32_t *tile_blk = nullptr, *tile_l0 = nullptr, *tile_l1 = nullptr;   // restriction tiles of the big blocks
    int64_t *tile_poff = nullptr;
    int32_t *wk_tile = nullptr, *wk_s0 = nullptr;   // restriction work items: (tile, first column)
    int ntiles = 0, nwork = 0;
    int32_t *dof_blk = nullptr, *dof_lr = nullptr;
    double *partial = nullptr, *r0 = nullptr, *z0 = nullptr;
    // z0 repeated in the column order of the coarse basis blocks, and the
    // positions of each coarse column there
    double *zg = nullptr;
    int64_t *cpos_ptr = nullptr;
    int32_t *cpos = nullptr;
    double *A0 = nullptr;     // assembled coarse matrix
    double *A0inv = nullptr;  // its inverse (dense blocks, one per problem)
    int32_t *cprob = nullptr, *prob_c0 = nullptr;
    int64_t *a0_off = nullptr;
    // ---- Krylov ----
    double *kr = nullptr, *kz = nullptr, *kp = nullptr, *kq = nullptr, *kt = nullptr, *kpart = nullptr;
    double *kpart2 = nullptr;   // second partial sums (r.r beside r.z)
    double *kp2 = nullptr;      // the other CG direction buffer (p alternates between kp and kp2)
    int cg_par = 0;             // which of the two holds the current direction
    KState *kst = nullptr;          // one per problem
    int *kdone = nullptr;           // done flags mirrored per problem (skip mask of the apply)
    int *kmask = nullptr;           // one-problem-active mask (slot start)
    int32_t *kb_prob = nullptr, *kb_row0 = nullptr, *kb_row1 = nullptr, *pb_ptr = nullptr;
    std::vector<int32_t> h_pb_ptr;  // host copy: first row block of every problem
    int nkb = 0;
    int32_t *sub_prob = nullptr, *blk_prob = nullptr;
    int64_t *prob_ptr = nullptr;
    // slots (continuous batching)
    double *slot_x = nullptr;
    const double *slot_b = nullptr;
    std::vector<KState> h_state;
    int64_t phi_entries = 0;
    int64_t local_entries = 0;
    int KLp = 1, KUp = 1;   // slot counts of the sweep layout
    int max_n0 = 0;         // largest coarse block
    int nb_big = 0;         // leading coarse-basis blocks restricted by a workgroup each
    int max_k_big = 0;      // most columns of a big block
    int band_kinds = 0;     // band solve instances the subdomains need (bit 0 substitution, bit 1 inverse)
    bool split_rule = false;   // prolongation's coarse part by blocks under the fixed rule
    int prolong_split = -1;    // -1: rule, 0: per dof, 1: by blocks (k_coarse_prolong into zc)
    double *zc = nullptr;      // coarse part of the prolongation, by blocks
    size_t max_lds = 64 * 1024;   // dynamic LDS a workgroup may use on this device
    double *gm_V = nullptr, *gm_part = nullptr;   // GMRES basis and partial sums
    int gm_m = 0;
    GState *gm_st = nullptr;
    void *sweep_buf = nullptr;    // iterates of subdomains too large for LDS
    size_t sweep_bytes = 0;       // (one slot)
    int64_t n_partial = 0;        // coarse restriction partials (one slot)
    int device = 0;               // the GPU the handle was factored on
    // right-hand-side slots: ns slots of every problem; the Krylov problems
    // are the nvp = ns * nprob (slot, problem) pairs over nv = ns * n rows
    int ns = 1, nvp = 1;
    int64_t nv = 0;
    Slots slots{};
    int32_t *sub_order = nullptr;   // local-solve launch order (decreasing size), or null
    int *queue = nullptr;           // work counters of the persistent band solves (QUEUE_HALF per kind)
    // nested-dissection supernodal factor (exact local solver): subdomains
    // with it and with a band (largest of each)
    bool nd = false;
    int nd_max_ni = 0, band_max_ni = 0;
    void *ndL = nullptr;                                   // panels in the local precision
    int32_t *nd_iperm = nullptr, *nd_first = nullptr, *nd_ncol = nullptr, *nd_nrow = nullptr;
    int64_t *nd_voff = nullptr, *nd_st_ptr = nullptr, *nd_rc_ptr = nullptr, *nd_lv_base = nullptr;
    int64_t *nd_sn_ptr = nullptr;
    int32_t *nd_st_row = nullptr, *nd_st_sn = nullptr, *nd_row_sn = nullptr, *nd_lv_ptr = nullptr;
    int32_t *nd_rc_w = nullptr, *nd_ch_row = nullptr;
    int64_t *nd_ch_base = nullptr;
    int4 *nd_lv_info = nullptr;
    // the solve's struct products (one value per struct entry and slot,
    // accumulator precision, sized for FP64)
    double *nd_w = nullptr;
    int64_t nd_nst = 0;
    // size classes of the local solves: consecutive ranges of the launch
    // order whose sizes lie within a factor two of the class's largest; each
    // is launched with LDS and rows per thread for its own largest
    // subdomain, in the launch configuration tuned for it (-1: the handle's)
    struct SizeClass {
        int begin, end, max_ni, variant, idx;
    };
    std::vector<SizeClass> cls;                 // the classes in use
    std::vector<SizeClass> cls_one, cls_split;  // one class; split by size (autotuned choice)
    // classes after the first run on their own streams beside it (fork and
    // join by events), created with the default priority
    static constexpr int MAX_CLASSES = 6;
    hipStream_t cstream[MAX_CLASSES - 1] = {};
    hipEvent_t ev_cfork = nullptr, ev_cjoin[MAX_CLASSES - 1] = {};
    int local_variant = -1;       // launch configuration of the local solves (-1: fixed rule)
    int gemv_variant = -1;        // coarse GEMV: 0 wavefront per row, 1 workgroup per row
};

// Scratch tags of the numerical setup (Device::setup_scratch).
enum SetupTag {
    ST_STATUS = 1, ST_LVAL, ST_FI_A, ST_FI_V, ST_BAND64, ST_BP_LOCAL, ST_BP_INT, ST_E, ST_IBAND, ST_T2, ST_T1,
    ST_GJ_P, ST_GJ_W, ST_SUB_BLK, ST_ND64
};

// Values of A in the sliced ELL layout of the Krylov SpMV (slices of SELL_C
// rows, slot-major, padded to the slice's longest row with zeros).
static std::vector<double> sell_values(const Symbolic &S, std::vector<int64_t> *off_out = nullptr,
                                       std::vector<int32_t> *wid_out = nullptr) {
    const int64_t nsl = (S.n + SELL_C - 1) / SELL_C;
    std::vector<int64_t> off(nsl + 1, 0);
    std::vector<int32_t> wid(nsl, 0);
    for (int64_t sl = 0; sl < nsl; ++sl) {
        int32_t w = 0;
        for (int64_t i = sl * SELL_C; i < std::min<int64_t>(S.n, (sl + 1) * SELL_C); ++i)
            w = std::max<int32_t>(w, int32_t(S.rowptr[i + 1] - S.rowptr[i]));
        wid[sl] = w;
        off[sl + 1] = off[sl] + int64_t(w) * SELL_C;
    }
    std::vector<double> sv(off[nsl], 0.0);
    for (int64_t i = 0; i < S.n; ++i) {
        const int64_t base = off[i / SELL_C] + i % SELL_C;
        int j = 0;
        for (int64_t p = S.rowptr[i]; p < S.rowptr[i + 1]; ++p, ++j) sv[base + int64_t(j) * SELL_C] = S.val[p];
    }
    if (off_out) *off_out = std::move(off);
    if (wid_out) *wid_out = std::move(wid);
    return sv;
}

// ---------------------------------------------------------------------------
static void upload_all(gdsw_handle_s *h, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    std::vector<int32_t> rp32(S.n + 1), arow(S.nnz);
    for (int64_t i = 0; i <= S.n; ++i) rp32[i] = int32_t(S.rowptr[i]);
    std::vector<int64_t> adiag(S.n);
    for (int64_t i = 0; i < S.n; ++i)
        for (int64_t p = S.rowptr[i]; p < S.rowptr[i + 1]; ++p) {
            arow[p] = int32_t(i);
            if (S.col[p] == i) adiag[i] = p;
        }
    D.rowptr = D.upload(rp32, s);
    D.col = D.upload(S.col, s);
    D.val = D.upload(S.val, s);
    D.arow = D.upload(arow, s);
    D.adiag = D.upload(adiag, s);
    D.ov_idx = D.upload(S.ov_idx, s);
    D.ov_ptr = D.upload(S.ov_ptr, s);
    {
        std::vector<int32_t> tp(S.t_ptr.begin(), S.t_ptr.end());
        D.t_ptr = D.upload(tp, s);
        // sliced ELL copy of A
        std::vector<int64_t> off;
        std::vector<int32_t> wid;
        std::vector<double> sv = sell_values(S, &off, &wid);
        const int64_t nsl = int64_t(wid.size());
        std::vector<int32_t> sc(off[nsl], 0);
        for (int64_t i = 0; i < S.n; ++i) {
            const int64_t base = off[i / SELL_C] + i % SELL_C;
            int j = 0;
            for (int64_t p = S.rowptr[i]; p < S.rowptr[i + 1]; ++p, ++j) sc[base + int64_t(j) * SELL_C] = S.col[p];
            for (; j < wid[i / SELL_C]; ++j) sc[base + int64_t(j) * SELL_C] = int32_t(i);
        }
        D.sell.off = D.upload(off, s);
        D.sell.width = D.upload(wid, s);
        D.sell.val = D.upload(sv, s);
        // 16-bit column offsets when every entry lies within 32767 of its row
        bool near = true;
        for (int64_t i = 0; i < S.n && near; ++i)
            for (int64_t p = S.rowptr[i]; p < S.rowptr[i + 1]; ++p)
                if (std::abs(int64_t(S.col[p]) - i) > 32767) {
                    near = false;
                    break;
                }
        std::vector<int16_t> sd;
        if (near) {
            sd.resize(sc.size());
            for (int64_t sl = 0; sl < nsl; ++sl)
                for (int64_t j = 0; j < int64_t(wid[sl]) * SELL_C; ++j) {
                    const int64_t e = off[sl] + j, i = sl * SELL_C + j % SELL_C;
                    sd[size_t(e)] = int16_t(i < S.n ? sc[size_t(e)] - i : 0);
                }
            D.sell.dcol = D.upload(sd, s);
        } else {
            D.sell.col = D.upload(sc, s);
        }
        HIPCHK(hipStreamSynchronize(s));
    }
    D.t_pos = D.upload(S.t_pos, s);
    D.ns = std::max(1, S.opt.slots);
    D.nvp = D.ns * S.nprob;
    D.nv = int64_t(D.ns) * S.n;
    if (D.nv >= (int64_t(1) << 31)) throw DevError{GDSW_ERR_INVALID_ARG, "slots * n must stay below 2^31"};
    D.slots.ns = D.ns;
    D.slots.n = S.n;
    D.slots.zl = S.ov_ptr[S.np];
    D.zloc = D.alloc<double>(D.ns * S.ov_ptr[S.np]);
    const int64_t n = D.nv;
    D.kr = D.alloc<double>(n);
    D.kz = D.alloc<double>(n);
    D.kp = D.alloc<double>(n);
    D.kp2 = D.alloc<double>(n);
    D.kq = D.alloc<double>(n);
    D.kt = D.alloc<double>(n);
    // Krylov row blocks: KROWS rows each, never across problems or slots;
    // Krylov problem v = k nprob + p is problem p in slot k (rows k n + ...)
    {
        std::vector<int32_t> bp, b0, b1;
        D.h_pb_ptr.assign(D.nvp + 1, 0);
        for (int v = 0; v < D.nvp; ++v) {
            const int k = v / S.nprob, p = v % S.nprob;
            const int64_t sh = int64_t(k) * S.n;
            for (int64_t r = S.prob_ptr[p]; r < S.prob_ptr[p + 1]; r += KROWS) {
                bp.push_back(v);
                b0.push_back(int32_t(sh + r));
                b1.push_back(int32_t(sh + std::min<int64_t>(r + KROWS, S.prob_ptr[p + 1])));
            }
            D.h_pb_ptr[v + 1] = int32_t(bp.size());
        }
        D.nkb = int(bp.size());
        D.kb_prob = D.upload(bp, s);
        D.kb_row0 = D.upload(b0, s);
        D.kb_row1 = D.upload(b1, s);
        D.pb_ptr = D.upload(D.h_pb_ptr, s);
        HIPCHK(hipStreamSynchronize(s));
    }
    D.kpart = D.alloc<double>(std::max(D.nkb, 1));
    D.kpart2 = D.alloc<double>(std::max(D.nkb, 1));
    D.kst = D.alloc<KState>(D.nvp);
    D.kdone = D.alloc<int>(D.nvp);
    D.kmask = D.alloc<int>(D.nvp);
    D.sub_prob = D.upload(S.sub_prob, s);
    D.prob_ptr = D.upload(S.prob_ptr, s);
    {
        // the local solves start with the largest subdomains (a stable sort
        // by decreasing size; none when all have one size)
        std::vector<int32_t> ord(S.np);
        for (int i = 0; i < S.np; ++i) ord[i] = i;
        auto sz = [&](int i) { return S.ov_ptr[i + 1] - S.ov_ptr[i]; };
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return sz(a) > sz(b); });
        bool uniform = true;
        for (int i = 1; i < S.np && uniform; ++i) uniform = sz(i) == sz(0);
        if (!uniform) D.sub_order = D.upload(ord, s);
        // size classes: consecutive ranges of that order whose sizes lie
        // within a factor two of the class's largest (at most MAX_CLASSES,
        // the last takes the rest), each launched with LDS and rows per
        // thread for its own largest subdomain and, from the second on, on
        // a stream of its own beside the first, so that the smaller
        // subdomains run more workgroups per compute unit next to the large
        // ones.  Whether this beats one launch in size order depends on the
        // local solver (256-problem diffusion batch: supernodal solves 888
        // -> 1,037 solves/s, with classes within a factor four 967; band
        // solves 877 -> 830), so the autotuner times both.  (Launched one
        // after another on one stream, classes were slower still: 688
        // against 827 for the band.)
        D.cls_split.clear();
        int b = 0;
        while (b < S.np) {
            const int64_t top = std::max<int64_t>(sz(ord[b]), 1);
            int e = b + 1;
            if (int(D.cls_split.size()) == Device::MAX_CLASSES - 1) e = S.np;
            else
                while (e < S.np && 2 * sz(ord[e]) > top) ++e;
            D.cls_split.push_back({b, e, int(top), -1, int(D.cls_split.size())});
            b = e;
        }
        D.cls_one.assign(1, {0, S.np, int(std::max<int64_t>(S.max_ni, 1)), -1, 0});
        for (size_t k = 1; k < D.cls_split.size(); ++k) {
            if (!D.cstream[k - 1]) HIPCHK(hipStreamCreateWithFlags(&D.cstream[k - 1], hipStreamNonBlocking));
            if (!D.ev_cjoin[k - 1]) HIPCHK(hipEventCreateWithFlags(&D.ev_cjoin[k - 1], hipEventDisableTiming));
        }
        if (D.cls_split.size() > 1 && !D.ev_cfork)
            HIPCHK(hipEventCreateWithFlags(&D.ev_cfork, hipEventDisableTiming));
        // one class until the autotuner finds the split faster
        D.cls = D.cls_one;
        HIPCHK(hipStreamSynchronize(s));
    }
    {
        std::vector<int32_t> bprob(std::max<int32_t>(S.blk.nb, 1), 0);
        for (int g = 0; g < S.blk.nb; ++g)
            bprob[g] = S.blk.kind[g] == 0 ? S.sub_prob[S.blk.owner[g]]
                                          : int32_t(std::upper_bound(S.prob_ptr.begin(), S.prob_ptr.end(),
                                                                     int64_t(S.comp_nodes[S.comp_ptr[S.blk.owner[g]]]) * S.dpn) -
                                                    S.prob_ptr.begin() - 1);
        D.blk_prob = D.upload(bprob, s);
        HIPCHK(hipStreamSynchronize(s));
    }
    // the sync below makes the host vectors above safe to release
    HIPCHK(hipStreamSynchronize(s));
}

template <typename VT>
static void pack_ilu(gdsw_handle_s *h, const int64_t *d_lrowptr, const int32_t *d_lcol, const int32_t *d_ldiag,
                     const double *d_lval, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    // slot counts: 3 + 3 (ILU(0) of the 7-point stencil) or 6 + 6 (ILU(1))
    // padded for the register-resident sweeps, else the exact counts for the
    // streaming sweeps
    const bool small = S.KL <= ILU_KL && S.KU <= ILU_KU;
    const bool mid = !small && S.KL <= ILU_KL2 && S.KU <= ILU_KU2;
    const int KL = small ? ILU_KL : mid ? ILU_KL2 : std::max(S.KL, 1);
    const int KU = small ? ILU_KU : mid ? ILU_KU2 : std::max(S.KU, 1);
    if (!D.Lv) {   // (a numeric re-setup writes into the same buffers)
        D.KLp = KL;
        D.KUp = KU;
        // (the 6 + 6 layout carries ILU_PAD_ROWS zeroed rows past the last
        // slot and the last packed row, for the phased sweeps' unclamped reads)
        const int64_t pad = mid ? ILU_PAD_ROWS : 0;
        const int cw = (KL + KU + 1) / 2;
        D.Lv = D.alloc<VT>(int64_t(KL) * S.ell_rows + pad);
        D.Uv = D.alloc<VT>(int64_t(KU) * S.ell_rows + pad);
        D.dinv = D.alloc<VT>(S.ell_rows);
        D.Lc = D.alloc<uint16_t>(int64_t(KL) * S.ell_rows);
        D.Uc = D.alloc<uint16_t>(int64_t(KU) * S.ell_rows);
        if (small || mid) D.Cp = D.alloc<uint32_t>(int64_t(cw) * (S.ell_rows + pad));
        if (mid) {
            HIPCHK(hipMemsetAsync(D.Lv, 0, sizeof(VT) * size_t(int64_t(KL) * S.ell_rows + pad), s));
            HIPCHK(hipMemsetAsync(D.Uv, 0, sizeof(VT) * size_t(int64_t(KU) * S.ell_rows + pad), s));
            HIPCHK(hipMemsetAsync(D.Cp, 0, sizeof(uint32_t) * size_t(int64_t(cw) * (S.ell_rows + pad)), s));
        }
    }
    int64_t maxpad = 0;
    for (int i = 0; i < S.np; ++i) maxpad = std::max(maxpad, S.ell_off[i + 1] - S.ell_off[i]);
    dim3 grid(nblocks(maxpad, 256), S.np);
    hipLaunchKernelGGL(k_ilu_pack<VT>, grid, dim3(256), 0, s, D.ov_ptr, D.ell_off, d_lrowptr, d_lcol, d_ldiag,
                       d_lval, S.ell_rows, KL, KU, (VT *)D.Lv, D.Lc, (VT *)D.Uv, D.Uc, (VT *)D.dinv, D.Cp,
                       mid ? S.ell_rows + ILU_PAD_ROWS : int64_t(0));
    HIPCHK(hipGetLastError());
    D.local_entries = int64_t(KL + KU + 1) * S.ell_rows;
}

static void check_status(Device &D, int *d_status, int count, hipStream_t s, const char *what) {
    std::vector<int> st(count);
    HIPCHK(hipMemcpyAsync(st.data(), d_status, sizeof(int) * count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i)
        if (st[i]) throw DevError{GDSW_ERR_SINGULAR, std::string(what) + ": non-positive or zero pivot in part " +
                                                         std::to_string(i) + " at row " + std::to_string(st[i] - 1)};
}


// Replaces the 64x64 diagonal blocks of the band factors of every subdomain
// whose band holds whole triangles by their inverses (k_band_invert_diag);
// rows_h: host row offsets of the subdomains, bw_h: host bandwidths.
// (per subdomain: band_inverted(b)); returns which solve instances the
// subdomains need: bit 0 the substitution one, bit 1 the inverse one.
static int invert_diagonal_blocks(Device &D, double *band, const int64_t *off, const int32_t *bw, const int64_t *rptr,
                                  const std::vector<int64_t> &rows_h, const std::vector<int32_t> &bw_h, int np,
                                  int tag, hipStream_t s, const std::vector<int64_t> *off_h = nullptr) {
    std::vector<int64_t> bp(size_t(np) + 1, 0);
    int kinds = 0;
    for (int i = 0; i < np; ++i) {
        // (subdomains without a band: none)
        const int64_t n = (off_h && (*off_h)[i + 1] == (*off_h)[i]) ? 0 : rows_h[i + 1] - rows_h[i];
        const bool inv = band_inverted(bw_h[i]);
        if (n > 0) kinds |= inv ? 2 : 1;
        bp[i + 1] = bp[i] + (inv ? (n + BS_NB - 1) / BS_NB : 0);
    }
    if (bp[np] == 0) return kinds;
    const size_t lds = sizeof(double) * 2 * BS_NB * (BS_NB + 1);
    if (lds > D.max_lds) throw DevError{GDSW_ERR_INTERNAL, "LDS too small for the diagonal-block inverses"};
    int64_t *d_bp = D.setup_scratch<int64_t>(tag, int64_t(bp.size()));
    HIPCHK(hipMemcpyAsync(d_bp, bp.data(), sizeof(int64_t) * bp.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_band_invert_diag, dim3(unsigned(bp[np])), dim3(64), lds, s, band, off, bw, rptr, d_bp, np);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    D.setup_release(d_bp, sizeof(int64_t) * bp.size());
    return kinds;
}

// Local factors (ILU(k) in the sweep layout, or band Cholesky factors with
// inverted diagonal blocks) from the current values of A.  Allocates the
// factor buffers on the first call; a numeric re-setup overwrites them.
// Nested-dissection supernodal factor: the structure maps uploaded once,
// A_i's lower entries scattered into FP64 panels, the left-looking
// supernodal Cholesky, the diagonal blocks inverted, then the cast to the
// local precision.
static void factor_nd(gdsw_handle_s *h, int *d_status, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const NDSym &N = S.nd;
    const int prec = S.opt.local_prec;
    const int64_t nv = N.voff[N.nsn];
    if (!D.nd_iperm) {
        std::vector<int32_t> iperm(N.perm.size());
        for (int i = 0; i < S.np; ++i)
            for (int64_t p = S.ov_ptr[i]; p < S.ov_ptr[i + 1]; ++p) iperm[S.ov_ptr[i] + N.perm[p]] = int32_t(p - S.ov_ptr[i]);
        D.nd_iperm = D.upload(iperm, s);
        D.nd_first = D.upload(N.first, s);
        D.nd_ncol = D.upload(N.ncol, s);
        D.nd_nrow = D.upload(N.nrow, s);
        D.nd_voff = D.upload(N.voff, s);
        D.nd_sn_ptr = D.upload(N.sn_ptr, s);
        D.nd_st_ptr = D.upload(N.st_ptr, s);
        D.nd_st_row = D.upload(N.st_row, s);
        D.nd_st_sn = D.upload(N.st_sn, s);
        D.nd_row_sn = D.upload(N.row_sn, s);
        D.nd_rc_ptr = D.upload(N.rc_ptr, s);
        D.nd_rc_w = D.upload(N.rc_w, s);
        D.nd_lv_base = D.upload(N.lv_base, s);
        D.nd_lv_ptr = D.upload(N.lv_ptr, s);
        std::vector<int4> info(N.lv_info.size() / 4);
        for (size_t q = 0; q < info.size(); ++q)
            info[q] = make_int4(N.lv_info[4 * q], N.lv_info[4 * q + 1], N.lv_info[4 * q + 2], N.lv_info[4 * q + 3]);
        D.nd_lv_info = D.upload(info, s);
        D.nd_ch_base = D.upload(N.ch_base, s);
        D.nd_ch_row = D.upload(N.ch_row, s);
        D.nd_nst = N.st_ptr[N.nsn];
        D.nd_w = D.alloc<double>(std::max<int64_t>(1, int64_t(D.ns) * D.nd_nst));
        HIPCHK(hipStreamSynchronize(s));   // (the packed host copies go out of scope)
    }
    // factorization in FP64 panels (setup scratch), then the solve layout
    // in the storage precision
    double *P64 = D.setup_scratch<double>(ST_ND64, nv);
    hipLaunchKernelGGL(k_fill, dim3(nblocks(nv, 256, 65536)), dim3(256), 0, s, P64, 0.0, nv);
    int64_t *d_src = D.setup_upload(N.asm_src, s);
    int64_t *d_dst = D.setup_upload(N.asm_dst, s);
    const int64_t ne = int64_t(N.asm_src.size());
    hipLaunchKernelGGL(k_gather_vals, dim3(nblocks(ne, 256, 65536)), dim3(256), 0, s, D.val, d_src, d_dst, P64, ne,
                       D.dscale, D.arow, D.col);
    int64_t *d_up_ptr = D.setup_upload(N.up_ptr, s);
    int32_t *d_up_k = D.setup_upload(N.up_k, s);
    int32_t *d_up_s0 = D.setup_upload(N.up_s0, s);
    int32_t *d_up_n1 = D.setup_upload(N.up_n1, s);
    int64_t *d_up_rel = D.setup_upload(N.up_rel, s);
    int32_t *d_rel = D.setup_upload(N.rel, s);
    hipLaunchKernelGGL(k_nd_factor<256>, dim3(S.np), dim3(256), 0, s, P64, D.nd_sn_ptr, D.nd_first, D.nd_ncol,
                       D.nd_nrow, D.nd_voff, D.nd_st_ptr, d_up_ptr, d_up_k, d_up_s0, d_up_n1, d_up_rel, d_rel,
                       d_status);
    HIPCHK(hipGetLastError());
    check_status(D, d_status, S.np, s, "supernodal Cholesky");
    const size_t lds = sizeof(double) * size_t(std::max(N.max_ncol, 1));
    if (lds > D.max_lds) throw DevError{GDSW_ERR_INVALID_ARG, "a supernode is too wide for LDS"};
    hipLaunchKernelGGL(k_nd_invert<256>, dim3(S.np), dim3(256), lds, s, P64, D.nd_sn_ptr, D.nd_ncol, D.nd_nrow,
                       D.nd_voff);
    HIPCHK(hipGetLastError());
    if (!D.ndL) D.ndL = D.raw_alloc(prec_size(prec) * size_t(std::max<int64_t>(nv, 1)));
    const dim3 gs(unsigned(N.nsn));
    if (prec == GDSW_FP64)
        hipLaunchKernelGGL(k_nd_split<double>, gs, dim3(256), 0, s, P64, (double *)D.ndL, D.nd_ncol, D.nd_nrow, D.nd_voff);
    else if (prec == GDSW_FP32)
        hipLaunchKernelGGL(k_nd_split<float>, gs, dim3(256), 0, s, P64, (float *)D.ndL, D.nd_ncol, D.nd_nrow, D.nd_voff);
    else if (prec == GDSW_BF16)
        hipLaunchKernelGGL(k_nd_split<bf16>, gs, dim3(256), 0, s, P64, (bf16 *)D.ndL, D.nd_ncol, D.nd_nrow, D.nd_voff);
    else
        hipLaunchKernelGGL(k_nd_split<fp16>, gs, dim3(256), 0, s, P64, (fp16 *)D.ndL, D.nd_ncol, D.nd_nrow, D.nd_voff);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    D.setup_release(P64, sizeof(double) * size_t(nv));
    D.setup_release(d_src, sizeof(int64_t) * N.asm_src.size());
    D.setup_release(d_dst, sizeof(int64_t) * N.asm_dst.size());
    D.setup_release(d_up_ptr, sizeof(int64_t) * N.up_ptr.size());
    D.setup_release(d_up_k, sizeof(int32_t) * N.up_k.size());
    D.setup_release(d_up_s0, sizeof(int32_t) * N.up_s0.size());
    D.setup_release(d_up_n1, sizeof(int32_t) * N.up_n1.size());
    D.setup_release(d_up_rel, sizeof(int64_t) * N.up_rel.size());
    D.setup_release(d_rel, sizeof(int32_t) * N.rel.size());
    D.nd = true;
    D.local_entries += nv;
}

static void factor_band(gdsw_handle_s *h, int *d_status, hipStream_t s);

static void factor_local(gdsw_handle_s *h, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const int prec = S.opt.local_prec;
    const bool scaled = prec != GDSW_FP64;
    if (scaled) {
        if (!D.dscale) D.dscale = D.alloc<double>(S.n);
        hipLaunchKernelGGL(k_diag_scale, dim3(nblocks(S.n, 256)), dim3(256), 0, s, D.val, D.adiag, D.dscale, S.n);
    }
    int *d_status = D.setup_scratch<int>(ST_STATUS, S.np);
    HIPCHK(hipMemsetAsync(d_status, 0, sizeof(int) * S.np, s));
    if (S.opt.local == GDSW_LOCAL_ILU0) {
        int64_t *d_lrowptr = D.setup_upload(S.lrowptr, s);
        int32_t *d_lcol = D.setup_upload(S.lcol, s);
        int64_t *d_lgpos = D.setup_upload(S.lgpos, s);
        int32_t *d_ldiag = D.setup_upload(S.ldiag, s);
        int64_t *d_lvl_base = D.setup_upload(S.lvl_base, s);
        int32_t *d_lvl_ptr = D.setup_upload(S.lvl_ptr, s);
        int32_t *d_lvl_rows = D.setup_upload(S.lvl_rows, s);
        if (!D.ell_off) D.ell_off = D.upload(S.ell_off, s);
        const int64_t ne = int64_t(S.lcol.size());
        double *d_lval = D.setup_scratch<double>(ST_LVAL, ne);
        hipLaunchKernelGGL(k_gather_vals, dim3(nblocks(ne, 256, 65536)), dim3(256), 0, s, D.val, d_lgpos,
                           (const int64_t *)nullptr, d_lval, ne, D.dscale, D.arow, D.col);
        if (S.opt.ilu_factor_sweeps > 0) {
            // FastILU: sweeps over the factor entries from the start l = a/a_jj, u = a
            double *d_a = D.setup_scratch<double>(ST_FI_A, ne), *d_v = D.setup_scratch<double>(ST_FI_V, ne);
            int64_t *d_fptr = D.setup_upload(S.fi_ptr, s);
            int32_t *d_pairs = D.setup_upload(S.fi_pairs, s);
            int32_t *d_dpos = D.setup_upload(S.fi_dpos, s);
            HIPCHK(hipMemcpyAsync(d_a, d_lval, sizeof(double) * size_t(ne), hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_fastilu_start, dim3(nblocks(ne, 256)), dim3(256), 0, s, d_a, d_dpos, d_lval, ne);
            double *cur = d_lval, *nxt = d_v;
            for (int k = 0; k < S.opt.ilu_factor_sweeps; ++k) {
                hipLaunchKernelGGL(k_fastilu_sweep, dim3(nblocks(ne, 256)), dim3(256), 0, s, d_a, d_fptr, d_pairs,
                                   d_dpos, cur, nxt, ne);
                std::swap(cur, nxt);
            }
            if (cur != d_lval)
                HIPCHK(hipMemcpyAsync(d_lval, cur, sizeof(double) * size_t(ne), hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_ilu_pivot_check, dim3(S.np), dim3(256), 0, s, D.ov_ptr, d_lrowptr, d_ldiag, d_lval,
                               d_status);
            HIPCHK(hipGetLastError());
            check_status(D, d_status, S.np, s, "FastILU");
            D.setup_release(d_a, sizeof(double) * ne);
            D.setup_release(d_v, sizeof(double) * ne);
            D.setup_release(d_fptr, sizeof(int64_t) * S.fi_ptr.size());
            D.setup_release(d_pairs, sizeof(int32_t) * S.fi_pairs.size());
            D.setup_release(d_dpos, sizeof(int32_t) * S.fi_dpos.size());
        } else {
            hipLaunchKernelGGL(k_ilu0_factor, dim3(S.np), dim3(256), 0, s, D.ov_ptr, d_lrowptr, d_lcol, d_ldiag,
                               d_lvl_base, d_lvl_ptr, d_lvl_rows, d_lval, d_status);
            HIPCHK(hipGetLastError());
            check_status(D, d_status, S.np, s, "ILU");
        }
        switch (prec) {
            case GDSW_FP64: pack_ilu<double>(h, d_lrowptr, d_lcol, d_ldiag, d_lval, s); break;
            case GDSW_FP32: pack_ilu<float>(h, d_lrowptr, d_lcol, d_ldiag, d_lval, s); break;
            case GDSW_BF16: pack_ilu<bf16>(h, d_lrowptr, d_lcol, d_ldiag, d_lval, s); break;
            default: pack_ilu<fp16>(h, d_lrowptr, d_lcol, d_ldiag, d_lval, s); break;
        }
        // subdomains whose three sweep vectors do not fit in LDS (and that the
        // register-resident kernel does not cover) keep them in global memory
        {
            const size_t asz = prec == GDSW_FP64 ? 8 : 4;
            if (3 * asz * size_t(S.max_ni) > D.max_lds && !D.sweep_buf) {
                D.sweep_bytes = 3 * asz * size_t(S.ov_ptr[S.np]);
                D.sweep_buf = D.raw_alloc(D.sweep_bytes * size_t(D.ns));
            }
        }
        HIPCHK(hipStreamSynchronize(s));
        D.setup_release(d_lval, sizeof(double) * ne);
        D.setup_release(d_lrowptr, sizeof(int64_t) * S.lrowptr.size());
        D.setup_release(d_lcol, sizeof(int32_t) * S.lcol.size());
        D.setup_release(d_lgpos, sizeof(int64_t) * S.lgpos.size());
        D.setup_release(d_ldiag, sizeof(int32_t) * S.ldiag.size());
        D.setup_release(d_lvl_base, sizeof(int64_t) * S.lvl_base.size());
        D.setup_release(d_lvl_ptr, sizeof(int32_t) * S.lvl_ptr.size());
        D.setup_release(d_lvl_rows, sizeof(int32_t) * S.lvl_rows.size());
    } else {
        // supernodal subdomains, then the banded ones (either set may be empty)
        D.nd_max_ni = D.band_max_ni = 0;
        for (int i = 0; i < S.np; ++i) {
            const int ni = int(S.ov_ptr[i + 1] - S.ov_ptr[i]);
            if (S.nd_mask[i]) D.nd_max_ni = std::max(D.nd_max_ni, ni);
            else D.band_max_ni = std::max(D.band_max_ni, ni);
        }
        D.local_entries = 0;
        if (S.nd.nsn > 0) factor_nd(h, d_status, s);
        if (S.band_off[S.np] > 0) factor_band(h, d_status, s);
    }
    HIPCHK(hipStreamSynchronize(s));
    D.setup_release(d_status, sizeof(int) * S.np);
}

// Band Cholesky factors of the subdomains with a band (natural order), with
// inverted diagonal blocks, in the local precision.
static void factor_band(gdsw_handle_s *h, int *d_status, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const int prec = S.opt.local_prec;
    {
        const int64_t nb = S.band_off[S.np];
        // FP64 factors are the band itself; reduced precision casts a
        // scratch FP64 band into it
        double *band64 = prec == GDSW_FP64 ? static_cast<double *>(D.band) : D.setup_scratch<double>(ST_BAND64, nb);
        if (!band64) band64 = static_cast<double *>(D.band = D.alloc<double>(nb));
        HIPCHK(hipMemsetAsync(band64, 0, sizeof(double) * size_t(nb), s));
        int64_t *d_src = D.setup_upload(S.bscat_src, s);
        int64_t *d_dst = D.setup_upload(S.bscat_dst, s);
        const int64_t ne = int64_t(S.bscat_src.size());
        hipLaunchKernelGGL(k_gather_vals, dim3(nblocks(ne, 256, 65536)), dim3(256), 0, s, D.val, d_src, d_dst,
                           band64, ne, D.dscale, D.arow, D.col);
        if (!D.band_off) D.band_off = D.upload(S.band_off, s);
        if (!D.bw) D.bw = D.upload(S.bw, s);
        if (!D.queue) D.queue = D.alloc<int>(2 * QUEUE_HALF);
        const size_t lds = sizeof(double) * (CH_NB * CH_LD + CH_NB + size_t(std::max(S.max_bw, 1)) * CH_LD);
        if (lds > D.max_lds)
            throw DevError{GDSW_ERR_INVALID_ARG, "local bandwidth too large for the banded Cholesky"};
        hipLaunchKernelGGL(k_band_chol<256>, dim3(S.np), dim3(256), lds, s, band64, D.band_off, D.bw, D.ov_ptr,
                           d_status);
        HIPCHK(hipGetLastError());
        check_status(D, d_status, S.np, s, "banded Cholesky");
        D.band_kinds = invert_diagonal_blocks(D, band64, D.band_off, D.bw, D.ov_ptr, S.ov_ptr, S.bw, S.np,
                                              ST_BP_LOCAL, s, &S.band_off);
        D.setup_release(d_src, sizeof(int64_t) * S.bscat_src.size());
        D.setup_release(d_dst, sizeof(int64_t) * S.bscat_dst.size());
        if (prec != GDSW_FP64) {
            if (!D.band) D.band = D.raw_alloc(prec_size(prec) * size_t(nb));
            void *bl = D.band;
            const int gb = nblocks(nb, 256, 65536);
            if (prec == GDSW_FP32) hipLaunchKernelGGL(k_cast<float>, dim3(gb), dim3(256), 0, s, band64, (float *)bl, nb);
            else if (prec == GDSW_BF16) hipLaunchKernelGGL(k_cast<bf16>, dim3(gb), dim3(256), 0, s, band64, (bf16 *)bl, nb);
            else hipLaunchKernelGGL(k_cast<fp16>, dim3(gb), dim3(256), 0, s, band64, (fp16 *)bl, nb);
            HIPCHK(hipStreamSynchronize(s));
            D.setup_release(band64, sizeof(double) * size_t(nb));
        }
        D.local_entries += nb;
    }
}

// Layout of the coarse part, built once per handle: block maps, restriction
// tiles and work items, reduction lists, the coarse vectors, and the buffers
// of Phi and A_0; the interface blocks of Phi (orthonormal null-space bases,
// independent of the matrix values) are copied in here.
static void coarse_layout(gdsw_handle_s *h, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const PhiBlocks &B = S.blk;
    if (S.opt.coarse == GDSW_COARSE_NONE || S.n0 == 0 || B.nb == 0) return;
    const int n0 = S.n0;
    D.blk_row_ptr = D.upload(B.row_ptr, s);
    // interior blocks come first; they (and any block of many rows) take a
    // workgroup each in the restriction
    D.nb_big = 0;
    while (D.nb_big < B.nb && (B.kind[D.nb_big] == 0 || B.row_ptr[D.nb_big + 1] - B.row_ptr[D.nb_big] >= 512))
        ++D.nb_big;
    for (int g = 0; g < D.nb_big; ++g)
        D.max_k_big = std::max(D.max_k_big, int(B.col_ptr[g + 1] - B.col_ptr[g]));
    // many columns per row of Phi (elasticity: ~90): the per-dof form reads
    // them with scattered loads, the block form streams each block once
    D.split_rule = B.val_off[size_t(B.nb)] >= 16 * S.n && sizeof(double) * size_t(D.max_k_big) <= D.max_lds;
    if (D.split_rule) D.zc = D.alloc<double>(D.ns * S.n);
    D.blk_col_ptr = D.upload(B.col_ptr, s);
    D.blk_val_off = D.upload(B.val_off, s);
    D.blk_rows = D.upload(B.rows, s);
    // restriction partials: block g has ntile(g) tiles of k(g) partials each
    // (one tile unless it is a big block of more than RT_ROWS rows); the
    // reduction of column c adds them by ascending block, then tile
    {
        std::vector<int64_t> poff(size_t(B.nb) + 1, 0);
        std::vector<int32_t> ntile(size_t(B.nb), 1), tb, tl0, tl1;
        std::vector<int64_t> tpo;
        for (int g = 0; g < B.nb; ++g) {
            const int64_t nr = B.row_ptr[g + 1] - B.row_ptr[g];
            const int64_t k = B.col_ptr[g + 1] - B.col_ptr[g];
            if (g < D.nb_big) {
                const int64_t nt = std::max<int64_t>(1, (nr + RT_ROWS - 1) / RT_ROWS);
                const int64_t per = (nr + nt - 1) / nt;
                ntile[g] = int32_t(nt);
                for (int64_t t = 0; t < nt; ++t) {
                    tb.push_back(g);
                    tl0.push_back(int32_t(std::min(nr, t * per)));
                    tl1.push_back(int32_t(std::min(nr, (t + 1) * per)));
                    tpo.push_back(poff[g] + t * k);
                }
            }
            poff[g + 1] = poff[g] + int64_t(ntile[g]) * k;
        }
        if (poff[B.nb] >= (int64_t(1) << 31)) throw DevError{GDSW_ERR_INTERNAL, "too many restriction partials"};
        std::vector<int32_t> qblk(B.cols.size());
        for (int g = 0; g < B.nb; ++g)
            for (int64_t q = B.col_ptr[g]; q < B.col_ptr[g + 1]; ++q) qblk[size_t(q)] = g;
        std::vector<int64_t> rptr(size_t(n0) + 1, 0);
        std::vector<int32_t> ridx;
        ridx.reserve(size_t(poff[B.nb]));
        for (int c = 0; c < n0; ++c) {
            for (int64_t e = S.red_ptr[c]; e < S.red_ptr[c + 1]; ++e) {
                const int64_t q = S.red_idx[size_t(e)];
                const int g = qblk[size_t(q)];
                const int64_t k = B.col_ptr[g + 1] - B.col_ptr[g], sidx = q - B.col_ptr[g];
                for (int t = 0; t < ntile[g]; ++t) ridx.push_back(int32_t(poff[g] + t * k + sidx));
            }
            rptr[c + 1] = int64_t(ridx.size());
        }
        D.red_ptr = D.upload(rptr, s);
        D.red_idx = D.upload(ridx, s);
        D.blk_poff = D.upload(poff, s);
        D.ntiles = int(tb.size());
        std::vector<int32_t> wt, ws;
        for (int t = 0; t < D.ntiles; ++t) {
            const int g = tb[size_t(t)];
            const int64_t k = B.col_ptr[g + 1] - B.col_ptr[g];
            for (int64_t c = 0; c < std::max<int64_t>(k, 1); c += RT_CK) {
                wt.push_back(t);
                ws.push_back(int32_t(c));
            }
        }
        D.nwork = int(wt.size());
        D.wk_tile = D.upload(wt, s);
        D.wk_s0 = D.upload(ws, s);
        D.tile_blk = D.upload(tb, s);
        D.tile_l0 = D.upload(tl0, s);
        D.tile_l1 = D.upload(tl1, s);
        D.tile_poff = D.upload(tpo, s);
        D.partial = D.alloc<double>(D.ns * poff[B.nb]);
        D.n_partial = poff[B.nb];
        D.slots.part = poff[B.nb];
        HIPCHK(hipStreamSynchronize(s));   // the host vectors above go out of scope
    }
    D.dof_blk = D.upload(S.dof_blk, s);
    D.dof_lr = D.upload(S.dof_lr, s);
    D.r0 = D.alloc<double>(D.ns * n0);
    D.z0 = D.alloc<double>(D.ns * n0);
    D.zg = D.alloc<double>(D.ns * int64_t(B.cols.size()));
    D.slots.n0 = n0;
    D.slots.cols = int64_t(B.cols.size());
    D.cpos_ptr = D.upload(S.red_ptr, s);
    D.cpos = D.upload(S.red_idx, s);
    const int64_t nphi = B.val_off[B.nb];
    D.phi = D.alloc<double>(nphi);
    D.phi_entries = nphi;
    // interface blocks: the orthonormal bases from the analysis
    for (int g = 0; g < B.nb; ++g)
        if (B.kind[g] != 0) {
            const int c = B.owner[g];
            HIPCHK(hipMemcpyAsync(D.phi + B.val_off[g], S.phig.data() + S.phig_off[c],
                                  sizeof(double) * size_t(S.phig_off[c + 1] - S.phig_off[c]),
                                  hipMemcpyHostToDevice, s));
        }
    D.A0 = D.alloc<double>(S.a0_off[S.nprob]);
    D.A0inv = D.alloc<double>(S.a0_off[S.nprob]);
    D.cprob = D.upload(S.cprob, s);
    D.prob_c0 = D.upload(S.prob_c0, s);
    for (int k = 0; k < S.nprob; ++k) D.max_n0 = std::max(D.max_n0, S.prob_c0[k + 1] - S.prob_c0[k]);
    D.a0_off = D.upload(S.a0_off, s);
    if (S.opt.basis_prec == GDSW_FP32) D.phi32 = D.alloc<float>(nphi);
    HIPCHK(hipStreamSynchronize(s));
}

// Numerical part of the coarse space from the current values of A: the
// extension Phi_I = -A_II^{-1} A_IG Phi_G (eq. (2)), A_0 = Phi^T A Phi and its
// inverse, written into the buffers of coarse_layout.
static void coarse_numeric(gdsw_handle_s *h, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const PhiBlocks &B = S.blk;
    if (S.opt.coarse == GDSW_COARSE_NONE || S.n0 == 0 || B.nb == 0) return;
    const int64_t nphi = B.val_off[B.nb];
    int32_t *d_sub_blk = nullptr;
    {
        std::vector<int32_t> sub_blk(S.np, -1);
        for (int g = 0; g < B.nb; ++g)
            if (B.kind[g] == 0) sub_blk[B.owner[g]] = g;
        d_sub_blk = D.setup_scratch<int32_t>(ST_SUB_BLK, S.np);
        HIPCHK(hipMemcpyAsync(d_sub_blk, sub_blk.data(), sizeof(int32_t) * size_t(S.np), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    double *d_phig = D.setup_upload(S.phig, s);
    int64_t *d_phig_off = D.setup_upload(S.phig_off, s);
    int32_t *d_comp_rank = D.setup_upload(S.comp_rank, s);
    int64_t *d_int_ptr = D.setup_upload(S.int_ptr, s);
    int64_t *d_scol_ptr = D.setup_upload(S.scol_ptr, s);
    int64_t *d_ext_off = D.setup_upload(S.ext_off, s);
    // ---- extension: E_i = A_{I_i G} Phi_G, A_{I_i I_i} = L L^T, Phi_I = -A_II^{-1} E_i
    const int64_t nint = S.int_ptr[S.np];
    const int64_t next = S.ext_off[S.np];
    double *E = D.setup_scratch<double>(ST_E, next);
    HIPCHK(hipMemsetAsync(E, 0, sizeof(double) * size_t(std::max<int64_t>(next, 1)), s));
    {
        int64_t *a = D.setup_upload(S.cpl_ptr, s);
        int64_t *b = D.setup_upload(S.cpl_apos, s);
        int64_t *c = D.setup_upload(S.cpl_phi, s);
        int32_t *d = D.setup_upload(S.cpl_stride, s);
        int32_t *e = D.setup_upload(S.cpl_rank, s);
        int32_t *f = D.setup_upload(S.cpl_slot, s);
        int32_t *fm = D.setup_upload(S.cpl_slotmap, s);
        hipLaunchKernelGGL(k_ext_rhs, dim3(nblocks(nint, 256)), dim3(256), 0, s, D.val, d_int_ptr, S.np, d_ext_off,
                           a, b, c, d, e, f, fm, d_phig, E, nint);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        D.setup_release(a, 8 * S.cpl_ptr.size());
        D.setup_release(b, 8 * S.cpl_apos.size());
        D.setup_release(c, 8 * S.cpl_phi.size());
        D.setup_release(d, 4 * S.cpl_stride.size());
        D.setup_release(e, 4 * S.cpl_rank.size());
        D.setup_release(f, 4 * S.cpl_slot.size());
        D.setup_release(fm, 4 * S.cpl_slotmap.size());
    }
    int *d_status = D.setup_scratch<int>(ST_STATUS, std::max(S.np, 1));
    HIPCHK(hipMemsetAsync(d_status, 0, sizeof(int) * S.np, s));
    {
        const int64_t nb = S.iband_off[S.np];
        double *iband = D.setup_scratch<double>(ST_IBAND, nb);
        HIPCHK(hipMemsetAsync(iband, 0, sizeof(double) * size_t(std::max<int64_t>(nb, 1)), s));
        int64_t *d_src = D.setup_upload(S.ibscat_src, s);
        int64_t *d_dst = D.setup_upload(S.ibscat_dst, s);
        int64_t *d_ioff = D.setup_upload(S.iband_off, s);
        int32_t *d_ibw = D.setup_upload(S.ibw, s);
        const int64_t ne = int64_t(S.ibscat_src.size());
        hipLaunchKernelGGL(k_gather_vals, dim3(nblocks(ne, 256, 65536)), dim3(256), 0, s, D.val, d_src, d_dst, iband,
                           ne, (const double *)nullptr, D.arow, D.col);
        const size_t lds = sizeof(double) * (CH_NB * CH_LD + CH_NB + size_t(std::max(S.max_ibw, 1)) * CH_LD);
        if (lds > D.max_lds) throw DevError{GDSW_ERR_INVALID_ARG, "interior bandwidth too large"};
        hipLaunchKernelGGL(k_band_chol<256>, dim3(S.np), dim3(256), lds, s, iband, d_ioff, d_ibw, d_int_ptr, d_status);
        HIPCHK(hipGetLastError());
        check_status(D, d_status, S.np, s, "interior Cholesky");
        const int ikinds = invert_diagonal_blocks(D, iband, d_ioff, d_ibw, d_int_ptr, S.int_ptr, S.ibw, S.np,
                                                  ST_BP_INT, s);
        const size_t lds2 = sizeof(double) * (size_t(std::max(S.max_nii, 1)) + BS_NB * BS_LD);
        if (lds2 > D.max_lds) throw DevError{GDSW_ERR_INVALID_ARG, "interior block too large for LDS"};
        if (ikinds & 2)
            hipLaunchKernelGGL((k_ext_solve<512, true>), dim3(S.np), dim3(512), lds2, s, iband, d_ioff, d_ibw,
                               d_int_ptr, d_scol_ptr, d_ext_off, E, d_sub_blk, D.blk_val_off, D.phi);
        if (ikinds & 1)
            hipLaunchKernelGGL((k_ext_solve<512, false>), dim3(S.np), dim3(512), lds2, s, iband, d_ioff, d_ibw,
                               d_int_ptr, d_scol_ptr, d_ext_off, E, d_sub_blk, D.blk_val_off, D.phi);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        D.setup_release(iband, sizeof(double) * size_t(nb));
        D.setup_release(d_src, 8 * S.ibscat_src.size());
        D.setup_release(d_dst, 8 * S.ibscat_dst.size());
        D.setup_release(d_ioff, 8 * S.iband_off.size());
        D.setup_release(d_ibw, 4 * S.ibw.size());
    }
    // ---- A_0 = Phi_G^T A_GG Phi_G + sum_i E_i^T Phi_{I_i}
    // A_0 is block diagonal over the independent problems: one dense block each
    const int64_t na0 = S.a0_off[S.nprob];
    double *A0raw = D.A0inv;   // assembled here, then inverted in place below
    HIPCHK(hipMemsetAsync(A0raw, 0, sizeof(double) * size_t(na0), s));
    {
        const int npairs = int(S.pair_c.size());
        if (npairs) {
            int32_t *pc = D.setup_upload(S.pair_c, s);
            int32_t *pd = D.setup_upload(S.pair_d, s);
            int64_t *po = D.setup_upload(S.pair_off, s);
            int64_t *pe = D.setup_upload(S.pair_eptr, s);
            int64_t *pa = D.setup_upload(S.pair_apos, s);
            int32_t *plc = D.setup_upload(S.pair_lr_c, s);
            int32_t *pld = D.setup_upload(S.pair_lr_d, s);
            const int64_t total = S.pair_off[npairs];
            double *T2 = D.setup_scratch<double>(ST_T2, total);
            hipLaunchKernelGGL(k_t2, dim3(nblocks(total, 256)), dim3(256), 0, s, D.val, npairs, pc, pd, po, pe, pa,
                               plc, pld, d_comp_rank, d_phig_off, d_phig, T2, total);
            int64_t *st2 = D.setup_upload(S.a0seg2_tgt, s);
            int64_t *sp2 = D.setup_upload(S.a0seg2_ptr, s);
            int64_t *ss2 = D.setup_upload(S.a0seg2_src, s);
            const int64_t nseg2 = int64_t(S.a0seg2_tgt.size());
            hipLaunchKernelGGL(k_a0_segments, dim3(nblocks(nseg2, 256)), dim3(256), 0, s, st2, sp2, ss2, T2, A0raw,
                               nseg2);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(s));
            D.setup_release(T2, 8 * size_t(total));
            D.setup_release(st2, 8 * S.a0seg2_tgt.size()); D.setup_release(sp2, 8 * S.a0seg2_ptr.size());
            D.setup_release(ss2, 8 * S.a0seg2_src.size());
            D.setup_release(pc, 4 * S.pair_c.size()); D.setup_release(pd, 4 * S.pair_d.size());
            D.setup_release(po, 8 * S.pair_off.size()); D.setup_release(pe, 8 * S.pair_eptr.size());
            D.setup_release(pa, 8 * S.pair_apos.size()); D.setup_release(plc, 4 * S.pair_lr_c.size());
            D.setup_release(pld, 4 * S.pair_lr_d.size());
        }
        const int64_t nt1 = S.t1_off[S.np];
        if (nt1) {
            double *T1 = D.setup_scratch<double>(ST_T1, nt1);
            int64_t *d_t1off = D.setup_upload(S.t1_off, s);
            int kmax = 0;
            for (int i = 0; i < S.np; ++i) kmax = std::max<int>(kmax, int(S.scol_ptr[i + 1] - S.scol_ptr[i]));
            dim3 grid(nblocks(int64_t(kmax) * kmax, 256), S.np);
            hipLaunchKernelGGL(k_t1, grid, dim3(256), 0, s, d_int_ptr, d_scol_ptr, d_ext_off, E, d_sub_blk,
                               D.blk_val_off, D.phi, d_t1off, T1);
            int64_t *st = D.setup_upload(S.a0seg_tgt, s);
            int64_t *sp = D.setup_upload(S.a0seg_ptr, s);
            int64_t *ss = D.setup_upload(S.a0seg_src, s);
            const int64_t nseg = int64_t(S.a0seg_tgt.size());
            hipLaunchKernelGGL(k_a0_segments, dim3(nblocks(nseg, 256)), dim3(256), 0, s, st, sp, ss, T1, A0raw, nseg);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(s));
            D.setup_release(T1, 8 * nt1); D.setup_release(d_t1off, 8 * S.t1_off.size());
            D.setup_release(st, 8 * S.a0seg_tgt.size()); D.setup_release(sp, 8 * S.a0seg_ptr.size());
            D.setup_release(ss, 8 * S.a0seg_src.size());
        }
    }
    for (int k = 0; k < S.nprob; ++k) {
        const int nk = S.prob_c0[k + 1] - S.prob_c0[k];
        if (nk == 0) continue;
        hipLaunchKernelGGL(k_symmetrize, dim3(nblocks(int64_t(nk) * nk, 256)), dim3(256), 0, s, A0raw + S.a0_off[k],
                           D.A0 + S.a0_off[k], nk);
    }
    // ---- A_0^{-1} by blocked Gauss-Jordan sweeps, block by block, on a copy
    hipLaunchKernelGGL(k_copy, dim3(nblocks(na0, 256, 65536)), dim3(256), 0, s, D.A0, D.A0inv, na0);
    {
        int nmax = 0;
        for (int k = 0; k < S.nprob; ++k) nmax = std::max(nmax, S.prob_c0[k + 1] - S.prob_c0[k]);
        double *P = D.setup_scratch<double>(ST_GJ_P, GJ_NB * GJ_NB);
        double *W = D.setup_scratch<double>(ST_GJ_W, int64_t(nmax) * GJ_NB);
        HIPCHK(hipMemsetAsync(d_status, 0, sizeof(int) * S.np, s));
        for (int k = 0; k < S.nprob; ++k) {
            const int nk = S.prob_c0[k + 1] - S.prob_c0[k];
            double *Ak = D.A0inv + S.a0_off[k];
            const dim3 tiles((nk + 63) / 64, (nk + 63) / 64);
            for (int k0 = 0; k0 < nk; k0 += GJ_NB) {
                const int kb = std::min(GJ_NB, nk - k0);
                hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, Ak, nk, k0, kb, P, d_status + (k % S.np));
                hipLaunchKernelGGL(k_gj_panel, dim3(nblocks(nk, 256)), dim3(256), 0, s, Ak, nk, k0, kb, P, W);
                hipLaunchKernelGGL(k_gj_update, tiles, dim3(256), 0, s, Ak, nk, k0, kb, W);
                hipLaunchKernelGGL(k_gj_fix, dim3(nblocks(nk, 256)), dim3(256), 0, s, Ak, nk, k0, kb, W, P);
            }
        }
        hipLaunchKernelGGL(k_negate, dim3(nblocks(na0, 256, 65536)), dim3(256), 0, s, D.A0inv, na0);
        HIPCHK(hipGetLastError());
        check_status(D, d_status, std::min(S.np, S.nprob), s, "coarse matrix inverse");
        D.setup_release(P, 8 * GJ_NB * GJ_NB);
        D.setup_release(W, 8 * size_t(nmax) * GJ_NB);
    }
    if (D.phi32) {
        hipLaunchKernelGGL(k_cast<float>, dim3(nblocks(nphi, 256, 65536)), dim3(256), 0, s, D.phi, D.phi32, nphi);
    }
    HIPCHK(hipStreamSynchronize(s));
    D.setup_release(E, 8 * std::max<int64_t>(next, 1));
    D.setup_release(d_phig, 8 * S.phig.size());
    D.setup_release(d_phig_off, 8 * S.phig_off.size());
    D.setup_release(d_comp_rank, 4 * S.comp_rank.size());
    D.setup_release(d_sub_blk, 4 * size_t(S.np));
    D.setup_release(d_int_ptr, 8 * S.int_ptr.size());
    D.setup_release(d_scol_ptr, 8 * S.scol_ptr.size());
    D.setup_release(d_ext_off, 8 * S.ext_off.size());
    D.setup_release(d_status, 4 * std::max(S.np, 1));
}

gdsw_status factor(gdsw_handle_s *h, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto t0 = std::chrono::steady_clock::now();
    try {
        destroy_device(h);
        h->dev = new Device();
        h->dev->budget = h->sym.opt.hbm_budget_bytes;
        {
            int dev = 0, lds = 0;
            HIPCHK(hipGetDevice(&dev));
            h->dev->device = dev;
            // the allocation-free apply's scratch on this GPU
            if (gdsw_status st = static_scratch(dev, nullptr, &h->err); st != GDSW_OK)
                throw DevError{st, h->err};
            HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            h->dev->max_lds = size_t(lds);
            int cus = 0;
            HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            h->dev->n_cu = cus;
            HIPCHK(hipStreamCreateWithFlags(&h->dev->side, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&h->dev->ev_fork, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&h->dev->ev_join, hipEventDisableTiming));
        }
        upload_all(h, s);
        factor_local(h, s);
        coarse_layout(h, s);
        coarse_numeric(h, s);
        HIPCHK(hipStreamSynchronize(s));
    } catch (const DevError &e) {
        h->err = e.msg;
        destroy_device(h);
        return e.st;
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed";
        destroy_device(h);
        return GDSW_ERR_BUDGET;
    }
    h->factored = true;
    h->t_factor = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return GDSW_OK;
}

// Numeric re-setup (Sec. V-A: the numerical phase repeated on new values of
// the same pattern).  The symbolic analysis, every device map, the buffers
// of the factors, Phi, A_0^{-1} and the Krylov vectors (same addresses, so
// captured graphs stay valid), the tuned launch configurations and the
// captured CG graphs are kept; only the values of A (CSR and sliced ELL
// copies), the local factors, the extension Phi_I, A_0 and its inverse are
// recomputed.  The setup's own maps and scratch stay resident from the first
// re-setup on, so later ones upload and allocate nothing.  On an error the
// handle is left unfactored (a later refactor or factor starts afresh).
gdsw_status refactor(gdsw_handle_s *h, const double *val, void *stream) {
    if (!val) return GDSW_ERR_INVALID_ARG;
    for (int64_t p = 0; p < h->sym.nnz; ++p)
        if (!std::isfinite(val[p])) {
            h->err = "non-finite matrix value";
            return GDSW_ERR_INVALID_ARG;
        }
    h->sym.val.assign(val, val + h->sym.nnz);
    if (!h->factored || !h->dev) return factor(h, stream);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto t0 = std::chrono::steady_clock::now();
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    try {
        D.keep_setup = true;
        HIPCHK(hipMemcpyAsync(D.val, S.val.data(), sizeof(double) * size_t(S.nnz), hipMemcpyHostToDevice, s));
        {
            const std::vector<double> sv = sell_values(S);
            HIPCHK(hipMemcpyAsync(const_cast<double *>(D.sell.val), sv.data(), sizeof(double) * sv.size(),
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));   // sv goes out of scope
        }
        factor_local(h, s);
        coarse_numeric(h, s);
        HIPCHK(hipStreamSynchronize(s));
    } catch (const DevError &e) {
        h->err = e.msg;
        h->factored = false;
        return e.st;
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed";
        h->factored = false;
        return GDSW_ERR_BUDGET;
    }
    h->t_refactor = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return GDSW_OK;
}

// ---------------------------------------------------------------------------
// Launch configurations of the local-solve kernels.  ILU(0): 0 = registers,
// 512 threads; 1 = registers, 1024 threads; 2 = streaming, 256 threads;
// 3 = streaming, 512 threads.  Exact: 0 = 256 threads, 1 = 512, 2 = 1024,
// one workgroup per subdomain; 3, 4, 5 = the same as persistent workgroups
// (as many as fit the compute units at once) drawing subdomains from a work
// counter.  -1 picks by a fixed rule; gdsw_autotune times the candidates.
constexpr int N_ILU_VARIANTS = 4, N_BAND_VARIANTS = 6;

// One size class c of the local solves: workgroup b takes subdomain
// sub_order[c.begin + b] (or b itself without an order), with LDS and rows
// per thread for the class's largest subdomain.
static Skip class_skip(const Device &D, const Skip &sk, const Device::SizeClass &c) {
    Skip k = sk;
    k.order = D.sub_order ? D.sub_order + c.begin : nullptr;
    return k;
}

// The phased register-resident sweeps (ILU(k) with fill, 6 + 6 slots),
// one right-hand-side slot; rows per thread that keep the L (then U)
// entries in registers without spilling at this workgroup size.
template <typename VT, int NT>
static bool launch_ilu_phased(const Symbolic &S, Device &D, const double *r, const Skip &sk, hipStream_t s,
                              const Device::SizeClass &c) {
    if (D.ns > 1) return false;
    constexpr bool f64 = std::is_same<VT, double>::value;
    const int need = (c.max_ni + NT - 1) / NT;
    const int nb = c.end - c.begin;
    const Skip kc = class_skip(D, sk, c);
    using AT = typename AccOf<VT>::type;
#define GDSW_ILU_CASE(RR)                                                                                    \
    if (need <= RR) {                                                                                        \
        const size_t lds = (2 * sizeof(AT) + (f64 ? 0 : sizeof(double))) * NT * RR;                          \
        if (lds > D.max_lds) return false;                                                                   \
        hipLaunchKernelGGL((k_ilu_jacobi_phased<NT, RR, ILU_KL2, ILU_KU2, VT>), dim3(nb), dim3(NT), lds, s,  \
                           r, D.ov_idx, D.ov_ptr, D.ell_off, S.ell_rows, (const VT *)D.Lv, (const VT *)D.Uv,  \
                           D.Cp, S.ell_rows + ILU_PAD_ROWS, (const VT *)D.dinv, D.dscale, S.opt.jacobi_sweeps,  \
                           D.zloc, kc);                                                                       \
        return true;                                                                                         \
    }
    GDSW_ILU_CASE(2)
    GDSW_ILU_CASE(4)
    if constexpr (!(f64 && NT == 1024)) {
        GDSW_ILU_CASE(6)
        GDSW_ILU_CASE(8)
    }
    if constexpr (NT == 512) { GDSW_ILU_CASE(11) }
#undef GDSW_ILU_CASE
    return false;
}

// ILU(k) factors with more slots than the register-resident kernels take:
// the first 6 slots of each row held in registers (4 with FP64 entries for
// more than 4,096 rows a workgroup, the register budget), the rest streamed
// (512 threads with up to 11 rows each, or 1024 with up to 6, 4 for FP64)
template <typename VT, int NT>
static bool launch_ilu_hold(const Symbolic &S, Device &D, const double *r, const Skip &sk, hipStream_t s,
                            const Device::SizeClass &c) {
    if constexpr (NT != 512 && NT != 1024) {
        return false;
    } else {
        if (S.opt.jacobi_sweeps < 2 || !D.Lc || !D.Uc || D.KLp < 2 || D.KUp < 2) return false;
        using AT = typename AccOf<VT>::type;
        constexpr bool f64 = std::is_same<VT, double>::value;
        const size_t lds = 3 * sizeof(AT) * size_t(std::max(c.max_ni, 1));
        if (lds > D.max_lds) return false;
        const int need = (c.max_ni + NT - 1) / NT;
        const int nb = c.end - c.begin;
        const Skip kc = class_skip(D, sk, c);
#define GDSW_ILU_HOLD(RR)                                                                                     \
        if (need <= RR) {                                                                                     \
            hipLaunchKernelGGL((k_ilu_jacobi_hold<NT, RR, (f64 && RR * NT > 4096) ? 4 : 6, VT>), dim3(nb, D.ns), \
                               dim3(NT), lds, s, r,                                                           \
                               D.ov_idx, D.ov_ptr, D.ell_off, S.ell_rows, D.KLp, D.KUp, (const VT *)D.Lv,     \
                               D.Lc, (const VT *)D.Uv, D.Uc, (const VT *)D.dinv, D.dscale,                    \
                               S.opt.jacobi_sweeps, D.zloc, c.max_ni, kc);                                    \
            return true;                                                                                      \
        }
        if constexpr (NT == 512) {
            GDSW_ILU_HOLD(4)
            GDSW_ILU_HOLD(8)
            GDSW_ILU_HOLD(11)
        } else {
            GDSW_ILU_HOLD(2)
            GDSW_ILU_HOLD(4)
            if constexpr (!f64) { GDSW_ILU_HOLD(6) }   // (FP64 at 6 rows a thread spills)
        }
#undef GDSW_ILU_HOLD
        return false;
    }
}

template <typename VT, int NT>
static bool launch_ilu_regs(const Symbolic &S, Device &D, const double *r, const Skip &sk, hipStream_t s,
                            const Device::SizeClass &c) {
    // more slots than the phased kernel holds: the first ones held
    if (D.KLp > ILU_KL2 || D.KUp > ILU_KU2) return launch_ilu_hold<VT, NT>(S, D, r, sk, s, c);
    // (one sweep per triangle needs no factor entries: the streaming kernel)
    if (!D.Cp || S.opt.jacobi_sweeps < 2) return false;
    if (D.KLp == ILU_KL2 && D.KUp == ILU_KU2) return launch_ilu_phased<VT, NT>(S, D, r, sk, s, c);
    if (D.KLp != ILU_KL || D.KUp != ILU_KU) return false;
    constexpr bool f64 = std::is_same<VT, double>::value;
    const int need = (c.max_ni + NT - 1) / NT;
    const int nb = c.end - c.begin;
    const Skip kc = class_skip(D, sk, c);
    using AT = typename AccOf<VT>::type;
    // with several right-hand-side slots, one workgroup takes every slot of
    // its subdomain with the factor entries loaded once
#define GDSW_ILU_CASE(RR)                                                                                    \
    if (need <= RR) {                                                                                        \
        const size_t lds = (3 * sizeof(AT) + (f64 ? 0 : sizeof(double))) * NT * RR;                          \
        if (lds > D.max_lds) return false;                                                                   \
        if (D.ns > 1)                                                                                        \
            hipLaunchKernelGGL((k_ilu_jacobi<NT, RR, ILU_KL, ILU_KU, VT, true>), dim3(nb), dim3(NT), lds,    \
                               s, r, D.ov_idx, D.ov_ptr, D.ell_off, S.ell_rows, (const VT *)D.Lv,            \
                               (const VT *)D.Uv, D.Cp, (const VT *)D.dinv, D.dscale, S.opt.jacobi_sweeps,    \
                               D.zloc, kc);                                                                  \
        else                                                                                                 \
            hipLaunchKernelGGL((k_ilu_jacobi<NT, RR, ILU_KL, ILU_KU, VT, false>), dim3(nb), dim3(NT), lds,   \
                               s, r, D.ov_idx, D.ov_ptr, D.ell_off, S.ell_rows, (const VT *)D.Lv,            \
                               (const VT *)D.Uv, D.Cp, (const VT *)D.dinv, D.dscale, S.opt.jacobi_sweeps,    \
                               D.zloc, kc);                                                                  \
        return true;                                                                                         \
    }
    // the row counts per thread whose factor entries stay in registers
    // without spilling at this workgroup size
    GDSW_ILU_CASE(2)
    GDSW_ILU_CASE(4)
    if constexpr (!(f64 && NT == 1024)) {
        GDSW_ILU_CASE(6)
        GDSW_ILU_CASE(8)
    }
    if constexpr (NT == 512) { GDSW_ILU_CASE(11) }
#undef GDSW_ILU_CASE
    return false;
}

template <typename VT, int NT>
static bool launch_ilu_stream(const Symbolic &S, Device &D, const double *r, const Skip &sk, hipStream_t s,
                              const Device::SizeClass &c) {
    using AT = typename AccOf<VT>::type;
    size_t lds = 3 * sizeof(AT) * size_t(c.max_ni);
    void *gbuf = nullptr;
    if (lds > D.max_lds) {
        if (!D.sweep_buf) return false;
        gbuf = D.sweep_buf;
        lds = 0;
    }
    hipLaunchKernelGGL((k_ilu_jacobi_generic<NT, VT>), dim3(c.end - c.begin, D.ns), dim3(NT), lds, s, r, D.ov_idx,
                       D.ov_ptr, D.ell_off, S.ell_rows, D.KLp, D.KUp, (const VT *)D.Lv, D.Lc, (const VT *)D.Uv, D.Uc,
                       (const VT *)D.dinv, D.dscale, S.opt.jacobi_sweeps, D.zloc, c.max_ni, gbuf,
                       class_skip(D, sk, c));
    return true;
}

template <typename VT, int NT>
static bool launch_band(const Symbolic &S, Device &D, const double *r, const Skip &sk, hipStream_t s,
                        const Device::SizeClass &c, bool persistent) {
    using AT = typename AccOf<VT>::type;
    const size_t lds = sizeof(AT) * (size_t(c.max_ni) + BS_NB * BS_LD);
    if (lds > D.max_lds) return false;
    const Skip kc = class_skip(D, sk, c);
    const int nb = c.end - c.begin;
    if (persistent) {
        // as many workgroups as are resident at once: 2048 threads and the
        // LDS of a compute unit
        const int per_cu = std::max<int>(1, std::min<int>(2048 / NT, int(D.max_lds / lds)));
        const int g = std::max(1, std::min(nb, per_cu * D.n_cu));
        for (int kind = 0; kind < 2; ++kind) {
            const bool inv = kind == 0;
            if (!(D.band_kinds & (inv ? 2 : 1))) continue;
            // (one counter per slot and size class: the classes may run at once)
            if ((c.idx + 1) * D.ns > QUEUE_HALF) return false;
            int *q = D.queue + (inv ? 0 : QUEUE_HALF) + c.idx * D.ns;
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, q, 0, D.ns);
            if (inv)
                hipLaunchKernelGGL((k_band_apply_pers<NT, VT, true>), dim3(g, D.ns), dim3(NT), lds, s, r, D.ov_idx,
                                   D.ov_ptr, (const VT *)D.band, D.band_off, D.bw, D.dscale, D.zloc, c.max_ni, kc, q,
                                   nb);
            else
                hipLaunchKernelGGL((k_band_apply_pers<NT, VT, false>), dim3(g, D.ns), dim3(NT), lds, s, r, D.ov_idx,
                                   D.ov_ptr, (const VT *)D.band, D.band_off, D.bw, D.dscale, D.zloc, c.max_ni, kc, q,
                                   nb);
        }
        return true;
    }
    if (D.band_kinds & 2)
        hipLaunchKernelGGL((k_band_apply<NT, VT, true>), dim3(nb, D.ns), dim3(NT), lds, s, r, D.ov_idx, D.ov_ptr,
                           (const VT *)D.band, D.band_off, D.bw, D.dscale, D.zloc, c.max_ni, kc);
    if (D.band_kinds & 1)
        hipLaunchKernelGGL((k_band_apply<NT, VT, false>), dim3(nb, D.ns), dim3(NT), lds, s, r, D.ov_idx, D.ov_ptr,
                           (const VT *)D.band, D.band_off, D.bw, D.dscale, D.zloc, c.max_ni, kc);
    return true;
}

template <typename VT, int NT>
static bool launch_nd(const Symbolic &S, Device &D, const double *r, const Skip &sk, hipStream_t s,
                      const Device::SizeClass &c) {
    using AT = typename AccOf<VT>::type;
    const size_t lds = nd_lds_bytes(c.max_ni, S.nd.max_t, S.nd.max_sn, sizeof(AT));
    if (lds > D.max_lds) return false;
    hipLaunchKernelGGL((k_nd_apply<NT, VT>), dim3(c.end - c.begin, D.ns), dim3(NT), lds, s, r, D.ov_idx, D.ov_ptr,
                       D.nd_iperm, (const VT *)D.ndL, D.nd_sn_ptr, D.nd_first, D.nd_ncol, D.nd_nrow, D.nd_voff,
                       D.nd_st_ptr, D.nd_st_row, D.nd_st_sn, D.nd_row_sn, D.nd_rc_ptr, D.nd_rc_w, D.nd_lv_base,
                       D.nd_lv_ptr, D.nd_lv_info, D.nd_ch_base, D.nd_ch_row, D.dscale, D.zloc,
                       reinterpret_cast<AT *>(D.nd_w), D.nd_nst, c.max_ni, S.nd.max_t, S.nd.max_sn,
                       class_skip(D, sk, c));
    return true;
}

template <typename VT>
static bool launch_band_variant(const Symbolic &S, Device &D, int v, const double *r, const Skip &sk,
                                hipStream_t s, const Device::SizeClass &c) {
    switch (v) {
        case 0: return launch_band<VT, 256>(S, D, r, sk, s, c, false);
        case 1: return launch_band<VT, 512>(S, D, r, sk, s, c, false);
        case 2: return launch_band<VT, 1024>(S, D, r, sk, s, c, false);
        case 3: return launch_band<VT, 256>(S, D, r, sk, s, c, true);
        case 4: return launch_band<VT, 512>(S, D, r, sk, s, c, true);
        default: return launch_band<VT, 1024>(S, D, r, sk, s, c, true);
    }
}

template <typename VT>
static bool launch_local_variant(const Symbolic &S, Device &D, int v, const double *r, const Skip &sk,
                                 hipStream_t s, const Device::SizeClass &c) {
    if (S.opt.local == GDSW_LOCAL_EXACT) {
        // the banded subdomains in configuration v, the supernodal ones with
        // 256, 512 or 1024 threads (v mod 3); each kernel leaves the other
        // kind's subdomains alone
        bool ok = true;
        if (D.band_kinds) {
            Device::SizeClass cb = c;
            cb.max_ni = std::min(c.max_ni, std::max(D.band_max_ni, 1));
            ok = launch_band_variant<VT>(S, D, v, r, sk, s, cb);
        }
        if (ok && D.nd) {
            Device::SizeClass cn = c;
            cn.max_ni = std::min(c.max_ni, std::max(D.nd_max_ni, 1));
            switch (v % 3) {
                case 0: ok = launch_nd<VT, 256>(S, D, r, sk, s, cn); break;
                case 1: ok = launch_nd<VT, 512>(S, D, r, sk, s, cn); break;
                default: ok = launch_nd<VT, 1024>(S, D, r, sk, s, cn); break;
            }
        }
        return ok;
    }
    if (S.opt.local == GDSW_LOCAL_ILU0) {
        switch (v) {
            case 0: return launch_ilu_regs<VT, 512>(S, D, r, sk, s, c);
            case 1: return launch_ilu_regs<VT, 1024>(S, D, r, sk, s, c);
            case 2: return launch_ilu_stream<VT, 256>(S, D, r, sk, s, c);
            default: return launch_ilu_stream<VT, 512>(S, D, r, sk, s, c);
        }
    }
    return false;
}

// Every size class in the configuration tuned for it, else the handle's
// (gdsw_set_launch / gdsw_autotune), else the fixed rule: register-resident
// sweeps when they fit (FP64: 512 threads, reduced precision: 1024), else
// streaming; band solves with 512 threads.
template <typename VT>
static void launch_local_class(const Symbolic &S, Device &D, const double *r, const Skip &sk, hipStream_t s,
                               const Device::SizeClass &c) {
    if (c.variant >= 0 && launch_local_variant<VT>(S, D, c.variant, r, sk, s, c)) return;
    if (D.local_variant >= 0 && launch_local_variant<VT>(S, D, D.local_variant, r, sk, s, c)) return;
    static const int ilu_order_f64[N_ILU_VARIANTS] = {0, 1, 2, 3}, ilu_order_lo[N_ILU_VARIANTS] = {1, 0, 2, 3},
                     band_order[N_BAND_VARIANTS] = {1, 0, 2, 4, 3, 5};
    const bool ilu = S.opt.local == GDSW_LOCAL_ILU0;
    const int *order = ilu ? (std::is_same<VT, double>::value ? ilu_order_f64 : ilu_order_lo) : band_order;
    const int nv = ilu ? N_ILU_VARIANTS : N_BAND_VARIANTS;
    for (int q = 0; q < nv; ++q)
        if (launch_local_variant<VT>(S, D, order[q], r, sk, s, c)) return;
    throw DevError{GDSW_ERR_INVALID_ARG, "no local-solve kernel fits this subdomain size"};
}

template <typename VT>
static void launch_local(const Symbolic &S, Device &D, const double *r, const Skip &sk, hipStream_t s) {
    if (D.cls.size() == 1) {
        launch_local_class<VT>(S, D, r, sk, s, D.cls[0]);
        return;
    }
    // the first (largest) class on `s`, queued first so that its long
    // workgroups take the compute units first, the others beside it, joined
    // back
    HIPCHK(hipEventRecord(D.ev_cfork, s));
    launch_local_class<VT>(S, D, r, sk, s, D.cls[0]);
    for (size_t k = 1; k < D.cls.size(); ++k) {
        HIPCHK(hipStreamWaitEvent(D.cstream[k - 1], D.ev_cfork, 0));
        launch_local_class<VT>(S, D, r, sk, D.cstream[k - 1], D.cls[k]);
        HIPCHK(hipEventRecord(D.ev_cjoin[k - 1], D.cstream[k - 1]));
    }
    for (size_t k = 1; k < D.cls.size(); ++k) HIPCHK(hipStreamWaitEvent(s, D.ev_cjoin[k - 1], 0));
}

// One launch configuration for every size class (false: it does not fit
// every class).
template <typename VT>
static bool launch_local_fits_all(const Symbolic &S, Device &D, int v, const double *r, const Skip &sk,
                                  hipStream_t s) {
    for (const Device::SizeClass &c : D.cls)
        if (!launch_local_variant<VT>(S, D, v, r, sk, s, c)) return false;
    return true;
}

// The prolongation kernels for the parts w (bit 0 one-level, bit 1 coarse)
// and the form of the coarse part (zc != nullptr: formed by blocks).
template <typename PT, int W, bool BLK>
static void launch_prolong_inst(const Symbolic &S, Device &D, const double *zc, double *z, const Skip &sk,
                                hipStream_t s, const double *dot_r) {
    const PT *phi = std::is_same<PT, float>::value ? (const PT *)D.phi32 : (const PT *)D.phi;
    if (dot_r)
        hipLaunchKernelGGL((k_prolong_dot<PT, W, BLK>), dim3(D.nkb), dim3(256), 0, s, D.t_ptr, D.t_pos, D.zloc,
                           D.dof_blk, D.dof_lr, D.blk_row_ptr, D.blk_col_ptr, D.blk_val_off, phi, D.zg, zc, z, sk,
                           D.kb_row0, D.kb_row1, dot_r, D.kpart);
    else
        hipLaunchKernelGGL((k_prolong<PT, W, BLK>), dim3(nblocks(S.n, 256), D.ns), dim3(256), 0, s, D.t_ptr, D.t_pos,
                           D.zloc, D.dof_blk, D.dof_lr, D.blk_row_ptr, D.blk_col_ptr, D.blk_val_off, phi, D.zg, zc,
                           z, S.n, sk);
}

template <typename PT>
static void launch_prolong(const Symbolic &S, Device &D, int w, const double *zc, double *z, const Skip &sk,
                           hipStream_t s, const double *dot_r) {
    if (w == 0)   // neither part (the coarse part of a handle without one): z = 0
        launch_prolong_inst<PT, 0, false>(S, D, nullptr, z, sk, s, dot_r);
    else if (w == 1)
        launch_prolong_inst<PT, 1, false>(S, D, nullptr, z, sk, s, dot_r);
    else if (w == 2 && zc)
        launch_prolong_inst<PT, 2, true>(S, D, zc, z, sk, s, dot_r);
    else if (w == 2)
        launch_prolong_inst<PT, 2, false>(S, D, nullptr, z, sk, s, dot_r);
    else if (zc)
        launch_prolong_inst<PT, 3, true>(S, D, zc, z, sk, s, dot_r);
    else
        launch_prolong_inst<PT, 3, false>(S, D, nullptr, z, sk, s, dot_r);
}

// z = M^{-1} r (which = 3), or one part of it; with dot_r the prolongation
// also writes the Krylov-block partials of dot_r . z into the partial buffer.
static void launch_apply(gdsw_handle_s *h, const double *r, double *z, int which, const Skip &sk_in, hipStream_t s,
                         const double *dot_r = nullptr) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    Skip sk = sk_in;
    sk.sl = D.slots;
    if (!sk.flag) sk.nprob = S.nprob;
    const bool local = (which & 1) || which == 4;
    const bool coarse = (which & 2) && D.A0inv != nullptr;
    // the coarse chain (restriction, reduction, GEMV) and the local solves
    // are independent: the chain may run on the side stream beside them,
    // which pays when the local solves leave compute units idle
    const bool two = D.apply_streams == 2 || (D.apply_streams < 0 && S.np < D.n_cu);
    const bool fork = local && coarse && two && D.side != nullptr;
    const bool split = coarse && D.zc != nullptr && (D.prolong_split == 1 || (D.prolong_split < 0 && D.split_rule));
    const double *zc = split ? D.zc : nullptr;
    hipStream_t sc = s;
    if (fork) {
        HIPCHK(hipEventRecord(D.ev_fork, s));
        HIPCHK(hipStreamWaitEvent(D.side, D.ev_fork, 0));
        sc = D.side;
    }
    if (coarse) {
        const PhiBlocks &B = S.blk;
        // blocks with many rows (subdomain interiors) first, then the small ones
        const int nbig = D.nb_big, nsmall = B.nb - nbig;
        const int nsw = (nsmall + RT_NT / 64 - 1) / (RT_NT / 64);
        const int nwg = D.nwork + nsw;
        if (nwg > 0) {
            if (D.phi32)
                hipLaunchKernelGGL(k_coarse_restrict<float>, dim3(nwg, D.ns), dim3(RT_NT), 0, sc, r, D.blk_row_ptr,
                                   D.blk_rows, D.blk_col_ptr, D.blk_val_off, (const float *)D.phi32, D.tile_blk,
                                   D.tile_l0, D.tile_l1, D.tile_poff, D.wk_tile, D.wk_s0, D.blk_poff, D.partial,
                                   D.nwork, nbig, B.nb, sk);
            else
                hipLaunchKernelGGL(k_coarse_restrict<double>, dim3(nwg, D.ns), dim3(RT_NT), 0, sc, r, D.blk_row_ptr,
                                   D.blk_rows, D.blk_col_ptr, D.blk_val_off, (const double *)D.phi, D.tile_blk,
                                   D.tile_l0, D.tile_l1, D.tile_poff, D.wk_tile, D.wk_s0, D.blk_poff, D.partial,
                                   D.nwork, nbig, B.nb, sk);
        }
        hipLaunchKernelGGL(k_coarse_reduce, dim3((S.n0 + 3) / 4, D.ns), dim3(256), 0, sc, D.red_ptr, D.red_idx,
                           D.partial, D.r0, S.n0, sk);
        if (D.gemv_variant == 1 || (D.gemv_variant < 0 && D.max_n0 >= 1024))
            hipLaunchKernelGGL(k_block_gemv_wg, dim3((S.n0 + GW_R - 1) / GW_R, D.ns), dim3(256), 0, sc, D.A0inv, D.a0_off, D.prob_c0, D.cprob,
                               D.r0, D.z0, D.cpos_ptr, D.cpos, D.zg, S.n0, sk);
        else
            hipLaunchKernelGGL(k_block_gemv, dim3((S.n0 + 3) / 4, D.ns), dim3(256), 0, sc, D.A0inv, D.a0_off, D.prob_c0,
                               D.cprob, D.r0, D.z0, D.cpos_ptr, D.cpos, D.zg, S.n0, sk);
        const int nwp = D.ntiles * RT_RPT + nsw;
        if (split && nwp > 0) {
            const size_t lds = sizeof(double) * size_t(std::max(1, D.max_k_big));
            if (D.phi32)
                hipLaunchKernelGGL(k_coarse_prolong<float>, dim3(nwp, D.ns), dim3(RT_NT), lds, sc, D.blk_row_ptr,
                                   D.blk_rows, D.blk_col_ptr, D.blk_val_off, (const float *)D.phi32,
                                   D.tile_blk, D.tile_l0, D.tile_l1, D.zg, D.zc, D.ntiles, nbig, B.nb, sk);
            else
                hipLaunchKernelGGL(k_coarse_prolong<double>, dim3(nwp, D.ns), dim3(RT_NT), lds, sc, D.blk_row_ptr,
                                   D.blk_rows, D.blk_col_ptr, D.blk_val_off, (const double *)D.phi,
                                   D.tile_blk, D.tile_l0, D.tile_l1, D.zg, D.zc, D.ntiles, nbig, B.nb, sk);
        }
    }
    if (local) {
        // optional timing of the local solves where they run
        bool prof = D.prof_on && D.prof_n < GDSW_PROFILE_MAX;
        if (prof) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            HIPCHK(hipStreamIsCapturing(s, &cs));
            prof = cs == hipStreamCaptureStatusNone;
        }
        if (prof) HIPCHK(hipEventRecord(D.prof_ev[size_t(2 * D.prof_n)], s));
        switch (S.opt.local_prec) {
            case GDSW_FP64: launch_local<double>(S, D, r, sk, s); break;
            case GDSW_FP32: launch_local<float>(S, D, r, sk, s); break;
            case GDSW_BF16: launch_local<bf16>(S, D, r, sk, s); break;
            default: launch_local<fp16>(S, D, r, sk, s); break;
        }
        if (prof) {
            HIPCHK(hipEventRecord(D.prof_ev[size_t(2 * D.prof_n + 1)], s));
            ++D.prof_n;
        }
    }
    if (fork) {
        HIPCHK(hipEventRecord(D.ev_join, D.side));
        HIPCHK(hipStreamWaitEvent(s, D.ev_join, 0));
    }
    if (which == 4) {   // the local solves alone (results stay in zloc)
        HIPCHK(hipGetLastError());
        return;
    }
    const int w = (which & 1) | (coarse ? 2 : 0);
    if (D.phi32)
        launch_prolong<float>(S, D, w, zc, z, sk, s, dot_r);
    else
        launch_prolong<double>(S, D, w, zc, z, sk, s, dot_r);
    HIPCHK(hipGetLastError());
}

gdsw_status apply(gdsw_handle_s *h, const double *r, double *z, int which, void *stream) {
    if (!h->factored || !h->dev) {
        h->err = "apply before factor";
        return GDSW_ERR_STATE;
    }
    if (!r || (which != 4 && (!z || r == z)) || which < 1 || which > 4) {
        h->err = "apply: bad arguments";
        return GDSW_ERR_INVALID_ARG;
    }
    try {
        launch_apply(h, r, z, which, Skip(), static_cast<hipStream_t>(stream));
    } catch (const DevError &e) {
        h->err = e.msg;
        return e.st;
    }
    return GDSW_OK;
}

// The apply of eq. (1) with its scratch taken from the static array: the
// handle's buffers of the local results, the coarse partials, r_0, z_0 (and
// its repetitions), the blocked coarse prolongation and the sweep iterates
// are swapped for consecutive 256-byte aligned pieces of `scratch` for the
// duration of the launches (kernel arguments are copied at launch), then
// restored.  Every piece is fully written before it is read within one
// apply, so nothing needs clearing.
gdsw_status apply_static(gdsw_handle_s *h, const double *r, double *z, void *stream) {
    if (!h->factored || !h->dev) {
        h->err = "apply before factor";
        return GDSW_ERR_STATE;
    }
    if (!r || !z || r == z) {
        h->err = "apply_static: bad arguments";
        return GDSW_ERR_INVALID_ARG;
    }
    Device &D = *h->dev;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != D.device) {
        h->err = "apply_static: the current device is not the one the handle was factored on";
        return GDSW_ERR_INVALID_ARG;
    }
    void *base = nullptr;
    if (gdsw_status st = static_scratch(cur, &base, &h->err); st != GDSW_OK) return st;
    const bool split_used = D.zc != nullptr;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return at;
    };
    const Symbolic &S = h->sym;
    const size_t ns = size_t(D.ns);   // every right-hand-side slot
    const size_t o_zloc = take(ns * sizeof(double) * size_t(S.ov_ptr[S.np]));
    const size_t o_part = take(ns * sizeof(double) * size_t(D.n_partial));
    const size_t o_r0 = take(ns * sizeof(double) * size_t(S.n0));
    const size_t o_z0 = take(ns * sizeof(double) * size_t(S.n0));
    const size_t o_zg = take(ns * sizeof(double) * S.blk.cols.size());
    const size_t o_zc = split_used ? take(ns * sizeof(double) * size_t(S.n)) : 0;
    const size_t o_sw = D.sweep_buf ? take(ns * D.sweep_bytes) : 0;
    const size_t o_ndw = D.nd_w ? take(ns * sizeof(double) * size_t(D.nd_nst)) : 0;
    if (off > GDSW_STATIC_SCRATCH_BYTES) {
        h->err = "apply_static: this handle needs " + std::to_string(off) + " bytes of scratch, more than the " +
                 std::to_string(size_t(GDSW_STATIC_SCRATCH_BYTES)) + " of the static array";
        return GDSW_ERR_BUDGET;
    }
    unsigned char *b = static_cast<unsigned char *>(base);
    struct Swap {
        Device &D;
        double *zloc, *partial, *r0, *z0, *zg, *zc;
        void *sweep;
        double *ndw;
        ~Swap() {
            D.zloc = zloc, D.partial = partial, D.r0 = r0, D.z0 = z0, D.zg = zg, D.zc = zc;
            D.sweep_buf = sweep;
            D.nd_w = ndw;
        }
    } keep{D, D.zloc, D.partial, D.r0, D.z0, D.zg, D.zc, D.sweep_buf, D.nd_w};
    D.zloc = reinterpret_cast<double *>(b + o_zloc);
    D.partial = reinterpret_cast<double *>(b + o_part);
    D.r0 = reinterpret_cast<double *>(b + o_r0);
    D.z0 = reinterpret_cast<double *>(b + o_z0);
    D.zg = reinterpret_cast<double *>(b + o_zg);
    if (split_used) D.zc = reinterpret_cast<double *>(b + o_zc);
    if (D.sweep_buf) D.sweep_buf = b + o_sw;
    if (D.nd_w) D.nd_w = reinterpret_cast<double *>(b + o_ndw);
    try {
        launch_apply(h, r, z, 3, Skip(), static_cast<hipStream_t>(stream));
    } catch (const DevError &e) {
        h->err = e.msg;
        return e.st;
    }
    return GDSW_OK;
}

gdsw_status spmv(gdsw_handle_s *h, const double *x, double *y, void *stream) {
    if (!h->dev) {
        h->err = "spmv before factor";
        return GDSW_ERR_STATE;
    }
    if (!x || !y || x == y) return GDSW_ERR_INVALID_ARG;
    const int n = int(h->dev->nv), pn = int(h->sym.n);   // every right-hand-side slot
    if (h->dev->sell.dcol)
        hipLaunchKernelGGL(k_spmv<true>, dim3(nblocks(n, KNT)), dim3(KNT), 0, static_cast<hipStream_t>(stream), h->dev->sell,
                           x, y, n, pn);
    else
        hipLaunchKernelGGL(k_spmv<false>, dim3(nblocks(n, KNT)), dim3(KNT), 0, static_cast<hipStream_t>(stream), h->dev->sell,
                           x, y, n, pn);
    return hipGetLastError() == hipSuccess ? GDSW_OK : GDSW_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Preconditioned CG from x0 = 0 (the oracle's order of operations):
//   r = b, z = M r, p = z, rho = r.z;
//   repeat: q = A p, alpha = rho / p.q, x += alpha p, r -= alpha q, stop if
//           ||r|| <= rtol ||b||; z = M r, beta = r.z / rho, p = z + beta p.
// Iterations are queued in chunks; the host reads the device state once per
// chunk, kernels after convergence return immediately.
static Skip make_skip(const Symbolic &S, const Device &D, const int *flag) {
    Skip sk;
    sk.flag = flag;
    sk.sub_prob = D.sub_prob;
    sk.blk_prob = D.blk_prob;
    sk.cprob = D.cprob;
    sk.prob_ptr = D.prob_ptr;
    sk.nprob = S.nprob;
    return sk;
}

// One CG iteration of every running problem (the oracle's order):
//   q = A p, alpha = rho / p.q, x += alpha p, r -= alpha q, stop if
//   ||r|| <= rtol ||b||; z = M r, beta = r.z / rho, p = z + beta p.
static void queue_cg_iteration(gdsw_handle_s *h, double *x, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const KBlk all{D.kb_prob, D.kb_row0, D.kb_row1, 0};
    const int nkb = D.nkb, np = D.nvp;
    double *pold = D.cg_par ? D.kp2 : D.kp, *pnew = D.cg_par ? D.kp : D.kp2;
    // p = z + beta p fused into the product with A (with several
    // right-hand-side slots, each matrix entry is loaded once for them)
    if (D.ns > 1) {
        const int nkb1 = nkb / D.ns;
        if (D.sell.dcol)
            hipLaunchKernelGGL(k_cg_spmv_dot_p_ms<true>, dim3(nkb1), dim3(KNT), 0, s, D.sell, (const double *)D.kz,
                               (const double *)pold, pnew, D.kq, D.kpart, D.kst, all, int(S.n), D.ns, nkb1);
        else
            hipLaunchKernelGGL(k_cg_spmv_dot_p_ms<false>, dim3(nkb1), dim3(KNT), 0, s, D.sell, (const double *)D.kz,
                               (const double *)pold, pnew, D.kq, D.kpart, D.kst, all, int(S.n), D.ns, nkb1);
    } else if (D.sell.dcol) {
        hipLaunchKernelGGL(k_cg_spmv_dot_p<true>, dim3(nkb), dim3(KNT), 0, s, D.sell, (const double *)D.kz,
                           (const double *)pold, pnew, D.kq, D.kpart, D.kst, all, int(S.n));
    } else {
        hipLaunchKernelGGL(k_cg_spmv_dot_p<false>, dim3(nkb), dim3(KNT), 0, s, D.sell, (const double *)D.kz,
                           (const double *)pold, pnew, D.kq, D.kpart, D.kst, all, int(S.n));
    }
    hipLaunchKernelGGL(k_cg_finish, dim3(np), dim3(KFIN_NT), 0, s, D.kpart, D.pb_ptr, D.kst, D.kdone, int(KF_ALPHA), 0,
                       (const double *)nullptr);
    hipLaunchKernelGGL(k_cg_update_xr, dim3(nkb), dim3(KNT), 0, s, x, D.kr, pnew, D.kq, D.kpart2, D.kst, all);
    launch_apply(h, D.kr, D.kz, 3, make_skip(S, D, D.kdone), s, D.kr);   // also the partials of r.z
    // stop test on ||r||^2 (partials from the update), then beta from r.z
    hipLaunchKernelGGL(k_cg_finish, dim3(np), dim3(KFIN_NT), 0, s, D.kpart, D.pb_ptr, D.kst, D.kdone, int(KF_RR_BETA), 0,
                       D.kpart2);
    D.cg_par ^= 1;
}

// `iters` CG iterations: queued kernel by kernel, or with GDSW_FLAG_GRAPHS as
// one captured graph per (x, iters), captured on a private stream on first
// use and replayed on s.
static void queue_cg_chunk(gdsw_handle_s *h, double *x, int iters, hipStream_t s) {
    Device &D = *h->dev;
    if (!(h->sym.opt.flags & GDSW_FLAG_GRAPHS)) {
        for (int k = 0; k < iters; ++k) queue_cg_iteration(h, x, s);
        return;
    }
    hipGraphExec_t exec = nullptr;
    const int par = D.cg_par;   // the direction buffers alternate: a graph is tied to its start parity
    for (auto &g : D.cg_graphs)
        if (g.x == x && g.iters == iters && g.par == par) exec = g.exec;
    if (!exec) {
        if (!D.cap) HIPCHK(hipStreamCreateWithFlags(&D.cap, hipStreamNonBlocking));
        if (D.cg_graphs.size() >= 16) {
            HIPCHK(hipStreamSynchronize(s));
            for (auto &g : D.cg_graphs) (void)hipGraphExecDestroy(g.exec);
            D.cg_graphs.clear();
        }
        HIPCHK(hipStreamBeginCapture(D.cap, hipStreamCaptureModeThreadLocal));
        hipGraph_t graph = nullptr;
        try {
            for (int k = 0; k < iters; ++k) queue_cg_iteration(h, x, D.cap);
        } catch (...) {
            D.cg_par = par;
            (void)hipStreamEndCapture(D.cap, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        HIPCHK(hipStreamEndCapture(D.cap, &graph));
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(e);
        D.cg_graphs.push_back({x, iters, par, exec});
    }
    D.cg_par = par ^ (iters & 1);
    HIPCHK(hipGraphLaunch(exec, s));
}

// Starts CG (x0 = 0) for problem k alone, or for all problems (k < 0).
static void queue_cg_start(gdsw_handle_s *h, const double *b, double *x, int k, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const int base = k < 0 ? 0 : D.h_pb_ptr[k];
    const int nb = k < 0 ? D.nkb : D.h_pb_ptr[k + 1] - D.h_pb_ptr[k];
    const int pbase = k < 0 ? 0 : k, pn = k < 0 ? D.nvp : 1;
    const KBlk kb{D.kb_prob, D.kb_row0, D.kb_row1, base};
    hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(KNT), 0, s, x, D.kr, b, kb);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(KNT), 0, s, b, b, D.kpart, D.kst, 0, kb);
    hipLaunchKernelGGL(k_cg_finish, dim3(pn), dim3(KFIN_NT), 0, s, D.kpart, D.pb_ptr, D.kst, D.kdone, int(KF_BB), pbase,
                       (const double *)nullptr);
    launch_apply(h, D.kr, D.kz, 3, make_skip(S, D, k < 0 ? D.kdone : D.kmask), s);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(KNT), 0, s, D.kr, D.kz, D.kpart, D.kst, 0, kb);
    hipLaunchKernelGGL(k_cg_finish, dim3(pn), dim3(KFIN_NT), 0, s, D.kpart, D.pb_ptr, D.kst, D.kdone, int(KF_RHO), pbase,
                       (const double *)nullptr);
    // p_old = z with beta = 0: the first product takes p = z
    hipLaunchKernelGGL(k_cg_start_p, dim3((nb + UPB - 1) / UPB), dim3(KNT), 0, s, D.cg_par ? D.kp2 : D.kp, D.kz,
                       kb, nb);
}

// ||b - A x|| / ||b|| of problem k (all problems: k < 0) into state.red
static void queue_true_residual(gdsw_handle_s *h, const double *b, const double *x, int k, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const int n = int(D.nv);
    const int base = k < 0 ? 0 : D.h_pb_ptr[k];
    const int nb = k < 0 ? D.nkb : D.h_pb_ptr[k + 1] - D.h_pb_ptr[k];
    const KBlk kb{D.kb_prob, D.kb_row0, D.kb_row1, base};
    if (D.sell.dcol)
        hipLaunchKernelGGL(k_spmv<true>, dim3(nblocks(n, KNT)), dim3(KNT), 0, s, D.sell, x, D.kt, n, int(S.n));
    else
        hipLaunchKernelGGL(k_spmv<false>, dim3(nblocks(n, KNT)), dim3(KNT), 0, s, D.sell, x, D.kt, n, int(S.n));
    hipLaunchKernelGGL(k_residual, dim3(nblocks(n, 256)), dim3(256), 0, s, b, D.kt, n);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(KNT), 0, s, D.kt, D.kt, D.kpart, D.kst, 0, kb);
    hipLaunchKernelGGL(k_cg_finish, dim3(k < 0 ? D.nvp : 1), dim3(KFIN_NT), 0, s, D.kpart, D.pb_ptr, D.kst,
                       (int *)nullptr, int(KF_RED), k < 0 ? 0 : k, (const double *)nullptr);
}

static void fill_info(const KState &f, gdsw_solve_info *info) {
    info->iterations = f.iters;
    info->converged = f.status == KS_CONVERGED;
    info->rel_res_recursive = f.bb > 0 ? std::sqrt(f.rr / f.bb) : 0.0;
    info->rel_res_true = f.bb > 0 ? std::sqrt(f.red / f.bb) : 0.0;
}

// Preconditioned CG from x0 = 0 for every problem of the handle.
// Iterations are queued in chunks; the host reads the device states once
// per chunk, kernels of finished problems return immediately.
static gdsw_status solve_cg(gdsw_handle_s *h, const double *b, double *x, double rtol, int maxit, int fixed,
                            gdsw_solve_info *infos, int ninfo, hipStream_t s) {
    Device &D = *h->dev;
    const int np = D.nvp;   // every (slot, problem) pair
    std::vector<KState> hs(np);
    for (auto &k : hs) {
        k = KState{};
        k.rtol2 = rtol * rtol;
        k.fixed = fixed;
        k.maxit = maxit;
    }
    std::vector<int> zeros(np, 0);
    HIPCHK(hipMemcpyAsync(D.kst, hs.data(), sizeof(KState) * np, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(D.kdone, zeros.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
    queue_cg_start(h, b, x, -1, s);
    const int limit = fixed > 0 ? fixed : maxit;
    const bool graphs = (h->sym.opt.flags & GDSW_FLAG_GRAPHS) != 0;
    // residual of every problem at the previous host check
    std::vector<double> rr_prev(np, -1.0);
    std::vector<int> it_prev(np, 0);
    int queued = 0, chunk = 4;
    while (queued < limit) {
        const int c = std::min(chunk, limit - queued);
        if (graphs) {
            // as captured chunks of 32, 16, ..., 1 iterations (few distinct graphs)
            for (int p = 32; p >= 1; p >>= 1)   // (c <= 32)
                if (c & p) queue_cg_chunk(h, x, p, s);
        } else {
            queue_cg_chunk(h, x, c, s);
        }
        queued += c;
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hs.data(), D.kst, sizeof(KState) * np, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bool all = true;
        for (auto &k : hs) all = all && k.done;
        if (all) break;
        // The next chunk: the iterations the slowest running problem needs at
        // the residual reduction per iteration it showed since the last check
        // (plus one), so that few iterations are queued after convergence;
        // doubling when there is no estimate (first check, no reduction, or
        // a fixed iteration count).  Only how many iterations are queued
        // between two checks changes, never an iterate.
        int est = 0;
        bool ok = fixed <= 0;
        for (int k = 0; k < np && ok; ++k) {
            const KState &f = hs[k];
            if (f.done) continue;
            if (rr_prev[k] > 0.0 && f.iters > it_prev[k] && f.rr > 0.0 && f.bb > 0.0 && f.rr < rr_prev[k]) {
                const double q = std::log(f.rr / rr_prev[k]) / double(f.iters - it_prev[k]);   // < 0
                const double need = std::log(f.rtol2 * f.bb / f.rr) / q;
                est = std::max(est, need <= 0.0 ? 1 : int(std::ceil(need)));
            } else {
                ok = false;
            }
        }
        for (int k = 0; k < np; ++k) {
            rr_prev[k] = hs[k].rr;
            it_prev[k] = hs[k].iters;
        }
        chunk = ok && est > 0 ? std::min(est + 1, 32) : std::min(chunk * 2, 32);
    }
    queue_true_residual(h, b, x, -1, s);
    HIPCHK(hipMemcpyAsync(hs.data(), D.kst, sizeof(KState) * np, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    gdsw_status st = GDSW_OK;
    for (int k = 0; k < np; ++k) {
        if (hs[k].status == KS_BREAKDOWN) st = GDSW_ERR_BREAKDOWN;
        else if (fixed <= 0 && hs[k].status != KS_CONVERGED && st == GDSW_OK) st = GDSW_ERR_NOT_CONVERGED;
    }
    if (infos) {
        if (ninfo >= np) {
            for (int k = 0; k < np; ++k) fill_info(hs[k], infos + k);
        } else {
            // one summary: the slowest / worst problem
            gdsw_solve_info agg{};
            agg.converged = 1;
            for (int k = 0; k < np; ++k) {
                gdsw_solve_info one{};
                fill_info(hs[k], &one);
                agg.iterations = std::max(agg.iterations, one.iterations);
                agg.converged = agg.converged && one.converged;
                agg.rel_res_recursive = std::max(agg.rel_res_recursive, one.rel_res_recursive);
                agg.rel_res_true = std::max(agg.rel_res_true, one.rel_res_true);
            }
            *infos = agg;
        }
    }
    if (st == GDSW_ERR_BREAKDOWN) h->err = "CG breakdown";
    if (st == GDSW_ERR_NOT_CONVERGED) h->err = "CG did not converge";
    return st;
}

gdsw_status solve_gmres(gdsw_handle_s *h, const double *b, double *x, int restart, double rtol, int maxit,
                        int fixed, bool single_reduce, gdsw_solve_info *info, hipStream_t s);

gdsw_status solve(gdsw_handle_s *h, const double *b, double *x, int krylov, int restart, double rtol, int maxit,
                  int fixed_iters, gdsw_solve_info *info, int ninfo, void *stream) {
    if (!h->factored || !h->dev) {
        h->err = "solve before factor";
        return GDSW_ERR_STATE;
    }
    if (!b || !x || b == x || !(rtol >= 0.0) || maxit < 0 || fixed_iters < 0 ||
        (krylov != GDSW_KRYLOV_CG && krylov != GDSW_KRYLOV_GMRES && krylov != GDSW_KRYLOV_GMRES_SR)) {
        h->err = "solve: bad arguments";
        return GDSW_ERR_INVALID_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto t0 = std::chrono::steady_clock::now();
    gdsw_status st;
    try {
        if (krylov == GDSW_KRYLOV_CG) {
            st = solve_cg(h, b, x, rtol, maxit, fixed_iters, info, info ? ninfo : 0, s);
        } else {
            if (h->sym.nprob != 1 || h->dev->ns != 1) {
                h->err = "GMRES needs a handle with one problem and one right-hand-side slot";
                return GDSW_ERR_INVALID_ARG;
            }
            st = solve_gmres(h, b, x, restart, rtol, maxit, fixed_iters, krylov == GDSW_KRYLOV_GMRES_SR, info, s);
        }
    } catch (const DevError &e) {
        h->err = e.msg;
        return e.st;
    }
    if (info) {
        const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int k = 0; k < std::max(ninfo, 1); ++k) info[k].seconds = sec;
    }
    return st;
}

// Restarted GMRES(m), right preconditioned, x0 = 0 (the oracle's order):
// every cycle r = b - A x, V_0 = r / ||r||; step j: w = A M^{-1} V_j,
// orthogonalised against V_0..V_j twice, Givens rotations on the new
// Hessenberg column, stop when |g_{j+1}| <= rtol ||b||; at the end of the
// cycle x += M^{-1} (V y) with y the small least-squares solution.
// single_reduce: the same iteration with one reduction per step (the
// second projection pass and the normalisation delayed one step; the
// kernels k_sr_*); a cycle of m columns takes m + 1 steps, the last one
// without an operator application.
gdsw_status solve_gmres(gdsw_handle_s *h, const double *b, double *x, int restart, double rtol, int maxit,
                        int fixed, bool single_reduce, gdsw_solve_info *info, hipStream_t s) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const int64_t n = S.n;
    const int m = std::max(1, std::min(restart, GM_MAX));
    const int g = nblocks(n, KNT);
    if (!D.gm_V || D.gm_m < m) {
        if (D.gm_V) D.release(D.gm_V, sizeof(double) * size_t(D.gm_m + 1) * size_t(n));
        D.gm_V = D.alloc<double>(int64_t(m + 1) * n);
        D.gm_m = m;
    }
    if (!D.gm_st) D.gm_st = D.alloc<GState>(1);
    const int gr = std::min(GM_RED, g);
    if (!D.gm_part) D.gm_part = D.alloc<double>(std::max<int64_t>(int64_t(GM_RED) * (GM_MAX + 1),
                                                                 int64_t(SR_MAXB) * SR_NV));
    const KBlk all{D.kb_prob, D.kb_row0, D.kb_row1, 0};
    // ||b||^2
    KState ks{};
    HIPCHK(hipMemcpyAsync(D.kst, &ks, sizeof(KState), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_dot, dim3(D.nkb), dim3(KNT), 0, s, b, b, D.kpart, D.kst, 0, all);
    hipLaunchKernelGGL(k_cg_finish, dim3(1), dim3(KFIN_NT), 0, s, D.kpart, D.pb_ptr, D.kst, (int *)nullptr, int(KF_BB), 0,
                       (const double *)nullptr);
    HIPCHK(hipMemcpyAsync(&ks, D.kst, sizeof(KState), hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n, 256, 65536)), dim3(256), 0, s, x, 0.0, n);
    HIPCHK(hipStreamSynchronize(s));
    if (!(ks.bb > 0.0)) {
        if (info) { info->iterations = 0; info->converged = 1; info->rel_res_recursive = 0; info->rel_res_true = 0; }
        return std::isfinite(ks.bb) ? GDSW_OK : GDSW_ERR_INVALID_ARG;
    }
    GState* hs = new GState();
    hs->bb = ks.bb;
    hs->rtol2 = rtol * rtol;
    hs->m = m;
    hs->fixed = fixed;
    hs->maxit = maxit;
    HIPCHK(hipMemcpyAsync(D.gm_st, hs, sizeof(GState), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    GState *st = D.gm_st;
    double *V = D.gm_V;
    double *v = D.kz, *t = D.kp, *w = D.kq, *r = D.kr, *u = D.kt;
    Skip gsk;
    gsk.flag = &st->cycle_done;
    int guard = 0;
    const int64_t sr_chunks = (n + int64_t(KNT) * SR_R - 1) / (int64_t(KNT) * SR_R);
    const int sr_nb = int(std::min<int64_t>(sr_chunks, SR_MAXB));
    while (single_reduce) {
        // u = r = b - A x; step 0 forms ||r|| in its reduction
        hipLaunchKernelGGL(k_sr_cycle_start, dim3(1), dim3(1024), 0, s, st);
        if (D.sell.dcol)
            hipLaunchKernelGGL(k_spmv<true>, dim3(g), dim3(KNT), 0, s, D.sell, x, r, int(n), int(n));
        else
            hipLaunchKernelGGL(k_spmv<false>, dim3(g), dim3(KNT), 0, s, D.sell, x, r, int(n), int(n));
        hipLaunchKernelGGL(k_residual, dim3(nblocks(n, 256)), dim3(256), 0, s, b, r, int(n));
        int queued = 0, chunk = 4;
        while (true) {
            const int c = std::min(chunk, m + 1 - queued);
            for (int k = 0; k < c; ++k) {
                const int j = queued + k;
                const bool last = j == m;   // completes column m-1 only
                if (!last) {
                    launch_apply(h, r, t, 3, gsk, s);
                    if (D.sell.dcol)
                        hipLaunchKernelGGL(k_gm_spmv<true>, dim3(g), dim3(KNT), 0, s, D.sell, t, w, int(n), st);
                    else
                        hipLaunchKernelGGL(k_gm_spmv<false>, dim3(g), dim3(KNT), 0, s, D.sell, t, w, int(n), st);
                }
                hipLaunchKernelGGL(k_sr_reduce, dim3(sr_nb), dim3(KNT), 0, s, V, r, last ? nullptr : w, n, j,
                                   D.gm_part, st);
                hipLaunchKernelGGL(k_sr_finish, dim3(1), dim3(SR_FIN_NT), 0, s, D.gm_part, sr_nb, st, j);
                if (!last)
                    hipLaunchKernelGGL(k_sr_update, dim3(nblocks(n, 256)), dim3(256), 0, s, V, r, w, n, j, st);
            }
            queued += c;
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(hs, st, GSTATE_POLL, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (hs->cycle_done || queued > m) break;
            chunk = std::min(chunk * 2, 16);
        }
        if (hs->j > 0 && hs->status != KS_BREAKDOWN) {
            hipLaunchKernelGGL(k_gm_lsq, dim3(1), dim3(64), 0, s, st);
            hipLaunchKernelGGL(k_gm_combine, dim3(nblocks(n, 256, 65536)), dim3(256), 0, s, V, u, n, st);
            launch_apply(h, u, t, 3, Skip(), s);
            hipLaunchKernelGGL(k_add, dim3(nblocks(n, 256, 65536)), dim3(256), 0, s, x, t, n);
        }
        HIPCHK(hipMemcpyAsync(hs, st, GSTATE_POLL, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hs->done || hs->j == 0) break;
        if (++guard > maxit + 2) break;
    }
    while (!single_reduce) {
        // r = b - A x
        if (D.sell.dcol)
            hipLaunchKernelGGL(k_spmv<true>, dim3(g), dim3(KNT), 0, s, D.sell, x, r, int(n), int(n));
        else
            hipLaunchKernelGGL(k_spmv<false>, dim3(g), dim3(KNT), 0, s, D.sell, x, r, int(n), int(n));
        hipLaunchKernelGGL(k_residual, dim3(nblocks(n, 256)), dim3(256), 0, s, b, r, int(n));
        hipLaunchKernelGGL(k_gm_sqnorm, dim3(gr), dim3(KNT), 0, s, r, n, D.gm_part, st, 1);
        hipLaunchKernelGGL(k_gm_start_finish, dim3(1), dim3(KNT), 0, s, D.gm_part, gr, st);
        hipLaunchKernelGGL(k_gm_v0, dim3(nblocks(n, 256, 65536)), dim3(256), 0, s, V, r, n, st);
        int queued = 0, chunk = 4;
        while (true) {
            const int c = std::min(chunk, m - queued);
            for (int k = 0; k < c; ++k) {
                hipLaunchKernelGGL(k_gm_get, dim3(nblocks(n, 256, 65536)), dim3(256), 0, s, V, v, n, st);
                launch_apply(h, v, t, 3, gsk, s);
                if (D.sell.dcol)
                    hipLaunchKernelGGL(k_gm_spmv<true>, dim3(g), dim3(KNT), 0, s, D.sell, t, w, int(n), st);
                else
                    hipLaunchKernelGGL(k_gm_spmv<false>, dim3(g), dim3(KNT), 0, s, D.sell, t, w, int(n), st);
                for (int pass = 0; pass < 2; ++pass) {
                    hipLaunchKernelGGL(k_gm_dots, dim3(gr), dim3(KNT), 0, s, V, w, n, D.gm_part, st);
                    hipLaunchKernelGGL(k_gm_dots_finish, dim3(1), dim3(GM_FIN_NT), 0, s, D.gm_part, gr, st, pass);
                    hipLaunchKernelGGL(k_gm_subtract, dim3(nblocks(n, 256, 65536)), dim3(256), 0, s, V, w, n, st);
                }
                hipLaunchKernelGGL(k_gm_sqnorm, dim3(gr), dim3(KNT), 0, s, w, n, D.gm_part, st, 0);
                hipLaunchKernelGGL(k_gm_step_finish, dim3(1), dim3(KNT), 0, s, D.gm_part, gr, st);
                hipLaunchKernelGGL(k_gm_scale, dim3(nblocks(n, 256, 65536)), dim3(256), 0, s, V, w, n, st);
            }
            queued += c;
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(hs, st, GSTATE_POLL, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (hs->cycle_done || queued >= m) break;
            chunk = std::min(chunk * 2, 16);
        }
        if (hs->j > 0 && hs->status != KS_BREAKDOWN) {
            hipLaunchKernelGGL(k_gm_lsq, dim3(1), dim3(64), 0, s, st);
            hipLaunchKernelGGL(k_gm_combine, dim3(nblocks(n, 256, 65536)), dim3(256), 0, s, V, u, n, st);
            launch_apply(h, u, t, 3, Skip(), s);
            hipLaunchKernelGGL(k_add, dim3(nblocks(n, 256, 65536)), dim3(256), 0, s, x, t, n);
        }
        HIPCHK(hipMemcpyAsync(hs, st, GSTATE_POLL, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hs->done) break;
        if (++guard > maxit + 2) break;
    }
    const int status = hs->status, total = hs->total;
    const double g_last = hs->j > 0 ? std::fabs(hs->g[hs->j]) : hs->beta;
    delete hs;
    // true residual
    queue_true_residual(h, b, x, 0, s);
    HIPCHK(hipMemcpyAsync(&ks, D.kst, sizeof(KState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (info) {
        info->iterations = total;
        info->rel_res_recursive = g_last / std::sqrt(ks.bb);
        info->rel_res_true = std::sqrt(ks.red / ks.bb);
        info->converged = fixed > 0 ? info->rel_res_true <= rtol : status == KS_CONVERGED;
    }
    if (status == KS_BREAKDOWN) {
        h->err = "GMRES breakdown";
        return GDSW_ERR_BREAKDOWN;
    }
    if (fixed > 0) return GDSW_OK;
    if (status != KS_CONVERGED) {
        h->err = "GMRES did not converge";
        return GDSW_ERR_NOT_CONVERGED;
    }
    return GDSW_OK;
}

// ---------------------------------------------------------------------------
// Continuous batching over the problems of a handle: each problem is a slot
// that runs its own CG; slots start and finish independently while every
// running slot advances in the same kernel launches.
gdsw_status slots_begin(gdsw_handle_s *h, const double *b, double *x, double rtol, int maxit, void *stream) {
    if (!h->factored || !h->dev) {
        h->err = "slots before factor";
        return GDSW_ERR_STATE;
    }
    if (!b || !x || b == x || !(rtol >= 0.0) || maxit <= 0) {
        h->err = "slots_begin: bad arguments";
        return GDSW_ERR_INVALID_ARG;
    }
    Device &D = *h->dev;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int np = h->dev->nvp;   // every (slot, problem) pair
    D.slot_b = b;
    D.slot_x = x;
    D.h_state.assign(np, KState{});
    for (auto &k : D.h_state) {
        k.rtol2 = rtol * rtol;
        k.maxit = maxit;
        k.done = 1;
        k.status = KS_IDLE;
    }
    std::vector<int> ones(np, 1);
    try {
        HIPCHK(hipMemcpyAsync(D.kst, D.h_state.data(), sizeof(KState) * np, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(D.kdone, ones.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    } catch (const DevError &e) {
        h->err = e.msg;
        return e.st;
    }
    return GDSW_OK;
}

gdsw_status slot_start(gdsw_handle_s *h, int slot, void *stream) {
    if (!h->dev || !h->dev->slot_x) {
        h->err = "slot_start before slots_begin";
        return GDSW_ERR_STATE;
    }
    Device &D = *h->dev;
    const int np = h->dev->nvp;   // every (slot, problem) pair
    if (slot < 0 || slot >= np) return GDSW_ERR_INVALID_ARG;
    if (D.h_state[slot].status != KS_IDLE) {
        h->err = "slot is busy";
        return GDSW_ERR_STATE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    try {
        KState k = D.h_state[slot];
        k.done = 0;
        k.status = KS_RUNNING;
        k.iters = 0;
        k.beta = 0.0;   // the first product takes p = z
        D.h_state[slot] = k;
        // this slot alone is active in the start-up apply
        std::vector<int> mask(np, 1);
        mask[slot] = 0;
        const int zero = 0;
        HIPCHK(hipMemcpyAsync(D.kst + slot, &k, sizeof(KState), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(D.kdone + slot, &zero, sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(D.kmask, mask.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
        queue_cg_start(h, D.slot_b, D.slot_x, slot, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
    } catch (const DevError &e) {
        h->err = e.msg;
        return e.st;
    }
    return GDSW_OK;
}

gdsw_status slots_step(gdsw_handle_s *h, int iters, int32_t *state, void *stream) {
    if (!h->dev || !h->dev->slot_x) {
        h->err = "slots_step before slots_begin";
        return GDSW_ERR_STATE;
    }
    Device &D = *h->dev;
    const int np = h->dev->nvp;   // every (slot, problem) pair
    hipStream_t s = static_cast<hipStream_t>(stream);
    try {
        bool any = false;
        for (auto &k : D.h_state) any = any || (k.status == KS_RUNNING && !k.done);
        if (any && iters > 0) queue_cg_chunk(h, D.slot_x, iters, s);
        HIPCHK(hipGetLastError());
        std::vector<KState> dev(np);
        HIPCHK(hipMemcpyAsync(dev.data(), D.kst, sizeof(KState) * np, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int k = 0; k < np; ++k) {
            if (D.h_state[k].status == KS_IDLE) {
                if (state) state[k] = -1;
                continue;
            }
            D.h_state[k] = dev[k];
            if (state) state[k] = !dev[k].done ? 0 : (dev[k].status == KS_CONVERGED ? 1 : 2);
        }
    } catch (const DevError &e) {
        h->err = e.msg;
        return e.st;
    }
    return GDSW_OK;
}

gdsw_status slot_finish(gdsw_handle_s *h, int slot, gdsw_solve_info *info, void *stream) {
    if (!h->dev || !h->dev->slot_x) return GDSW_ERR_STATE;
    Device &D = *h->dev;
    if (slot < 0 || slot >= D.nvp) return GDSW_ERR_INVALID_ARG;
    if (D.h_state[slot].status == KS_IDLE || !D.h_state[slot].done) {
        h->err = "slot has no finished result";
        return GDSW_ERR_STATE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    try {
        queue_true_residual(h, D.slot_b, D.slot_x, slot, s);
        KState k{};
        HIPCHK(hipMemcpyAsync(&k, D.kst + slot, sizeof(KState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (info) {
            fill_info(k, info);
            info->seconds = 0.0;
        }
        const gdsw_status st = k.status == KS_CONVERGED ? GDSW_OK
                               : k.status == KS_BREAKDOWN ? GDSW_ERR_BREAKDOWN : GDSW_ERR_NOT_CONVERGED;
        KState idle = D.h_state[slot];
        idle.done = 1;
        idle.status = KS_IDLE;
        D.h_state[slot] = idle;
        const int one = 1;
        HIPCHK(hipMemcpyAsync(D.kst + slot, &idle, sizeof(KState), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(D.kdone + slot, &one, sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        return st;
    } catch (const DevError &e) {
        h->err = e.msg;
        return e.st;
    }
}

// ---------------------------------------------------------------------------
// Autotuner: times every launch configuration of the local-solve kernel and
// both coarse GEMV variants on the handle's own data and keeps the fastest.
template <typename VT>
static float time_local(gdsw_handle_s *h, int v, const Device::SizeClass &c, int reps, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    Skip none;
    none.sl = D.slots;
    if (!launch_local_variant<VT>(S, D, v, D.kr, none, s, c)) return -1.0f;
    HIPCHK(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) launch_local_variant<VT>(S, D, v, D.kr, none, s, c);
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return ms / reps;
}

gdsw_status autotune(gdsw_handle_s *h, int reps, float *times, void *stream) {
    if (!h->factored || !h->dev) {
        h->err = "autotune before factor";
        return GDSW_ERR_STATE;
    }
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        hipLaunchKernelGGL(k_fill, dim3(nblocks(D.nv, 256, 65536)), dim3(256), 0, s, D.kr, 1.0, D.nv);
        // every size class of the local solves on its own: the fastest
        // configuration per class (times[v]: the sum over the classes of one
        // launch, -1 where v does not fit a class); then the whole local
        // solve with the classes split by size (at once, on their streams)
        // against one class, the faster kept
        const int nv = S.opt.local == GDSW_LOCAL_ILU0 ? N_ILU_VARIANTS : N_BAND_VARIANTS;
        if (times)
            for (int v = 0; v < nv; ++v) times[v] = 0.0f;
        const bool split = D.cls_split.size() > 1;
        if (split) {
            D.cls = D.cls_split;
            for (Device::SizeClass &c : D.cls) {
                float best = -1.0f;
                int bv = -1;
                for (int v = 0; v < nv; ++v) {
                    float t;
                    switch (S.opt.local_prec) {
                        case GDSW_FP64: t = time_local<double>(h, v, c, reps, s, e0, e1); break;
                        case GDSW_FP32: t = time_local<float>(h, v, c, reps, s, e0, e1); break;
                        case GDSW_BF16: t = time_local<bf16>(h, v, c, reps, s, e0, e1); break;
                        default: t = time_local<fp16>(h, v, c, reps, s, e0, e1); break;
                    }
                    if (t > 0.0f && (best < 0.0f || t < best)) {
                        best = t;
                        bv = v;
                    }
                }
                c.variant = bv;
            }
            D.cls_split = D.cls;
            D.cls = D.cls_one;
        }
        for (size_t ci = 0; ci < D.cls.size(); ++ci) {
            Device::SizeClass &c = D.cls[ci];
            float best = -1.0f;
            int bv = -1;
            for (int v = 0; v < nv; ++v) {
                float t;
                switch (S.opt.local_prec) {
                    case GDSW_FP64: t = time_local<double>(h, v, c, reps, s, e0, e1); break;
                    case GDSW_FP32: t = time_local<float>(h, v, c, reps, s, e0, e1); break;
                    case GDSW_BF16: t = time_local<bf16>(h, v, c, reps, s, e0, e1); break;
                    default: t = time_local<fp16>(h, v, c, reps, s, e0, e1); break;
                }
                if (times) times[v] = (t < 0.0f || times[v] < 0.0f) ? -1.0f : times[v] + t;
                if (t > 0.0f && (best < 0.0f || t < best)) {
                    best = t;
                    bv = v;
                }
            }
            c.variant = bv;
        }
        D.cls_one = D.cls;
        if (split) {
            float tl[2];
            for (int k = 0; k < 2; ++k) {
                D.cls = k == 0 ? D.cls_one : D.cls_split;
                Skip none;
                none.sl = D.slots;
                switch (S.opt.local_prec) {
                    case GDSW_FP64: launch_local<double>(S, D, D.kr, none, s); break;
                    case GDSW_FP32: launch_local<float>(S, D, D.kr, none, s); break;
                    case GDSW_BF16: launch_local<bf16>(S, D, D.kr, none, s); break;
                    default: launch_local<fp16>(S, D, D.kr, none, s); break;
                }
                HIPCHK(hipEventRecord(e0, s));
                for (int q = 0; q < reps; ++q) switch (S.opt.local_prec) {
                        case GDSW_FP64: launch_local<double>(S, D, D.kr, none, s); break;
                        case GDSW_FP32: launch_local<float>(S, D, D.kr, none, s); break;
                        case GDSW_BF16: launch_local<bf16>(S, D, D.kr, none, s); break;
                        default: launch_local<fp16>(S, D, D.kr, none, s); break;
                    }
                HIPCHK(hipEventRecord(e1, s));
                HIPCHK(hipEventSynchronize(e1));
                HIPCHK(hipEventElapsedTime(&tl[k], e0, e1));
            }
            D.cls = tl[1] < tl[0] ? D.cls_split : D.cls_one;
            if (times) times[14] = tl[0] / reps, times[15] = tl[1] / reps;
        }
        // reported: the configuration of the largest subdomains
        D.local_variant = D.cls.empty() ? -1 : D.cls[0].variant;
        if (D.A0inv) {
            float tg[2];
            for (int v = 0; v < 2; ++v) {
                D.gemv_variant = v;
                launch_apply(h, D.kr, D.kz, 2, Skip(), s);
                HIPCHK(hipEventRecord(e0, s));
                for (int k = 0; k < reps; ++k) launch_apply(h, D.kr, D.kz, 2, Skip(), s);
                HIPCHK(hipEventRecord(e1, s));
                HIPCHK(hipEventSynchronize(e1));
                HIPCHK(hipEventElapsedTime(&tg[v], e0, e1));
                if (times) times[8 + v] = tg[v] / reps;
            }
            D.gemv_variant = tg[1] < tg[0] ? 1 : 0;
            float ta[2];
            for (int v = 0; v < 2; ++v) {
                D.apply_streams = v + 1;
                launch_apply(h, D.kr, D.kz, 3, Skip(), s);
                HIPCHK(hipEventRecord(e0, s));
                for (int k = 0; k < reps; ++k) launch_apply(h, D.kr, D.kz, 3, Skip(), s);
                HIPCHK(hipEventRecord(e1, s));
                HIPCHK(hipEventSynchronize(e1));
                HIPCHK(hipEventElapsedTime(&ta[v], e0, e1));
                if (times) times[10 + v] = ta[v] / reps;
            }
            D.apply_streams = ta[1] < ta[0] ? 2 : 1;
            // coarse part of the prolongation per dof or by blocks
            const size_t lds = sizeof(double) * size_t(D.max_k_big);
            if (lds <= D.max_lds) {
                if (!D.zc) D.zc = D.alloc<double>(D.ns * S.n);
                float tp[2];
                for (int v = 0; v < 2; ++v) {
                    D.prolong_split = v;
                    launch_apply(h, D.kr, D.kz, 3, Skip(), s);
                    HIPCHK(hipEventRecord(e0, s));
                    for (int k = 0; k < reps; ++k) launch_apply(h, D.kr, D.kz, 3, Skip(), s);
                    HIPCHK(hipEventRecord(e1, s));
                    HIPCHK(hipEventSynchronize(e1));
                    HIPCHK(hipEventElapsedTime(&tp[v], e0, e1));
                    if (times) times[12 + v] = tp[v] / reps;
                }
                D.prolong_split = tp[1] < tp[0] ? 1 : 0;
            }
        }
        HIPCHK(hipEventDestroy(e0));
        HIPCHK(hipEventDestroy(e1));
    } catch (const DevError &e) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        h->err = e.msg;
        return e.st;
    }
    return GDSW_OK;
}

gdsw_status profile_local(gdsw_handle_s *h, int enable) {
    if (!h->factored || !h->dev) {
        h->err = "profile_local before factor";
        return GDSW_ERR_STATE;
    }
    Device &D = *h->dev;
    try {
        if (enable && D.prof_ev.empty()) {
            D.prof_ev.assign(size_t(2 * GDSW_PROFILE_MAX), nullptr);
            for (hipEvent_t &e : D.prof_ev) HIPCHK(hipEventCreate(&e));
        }
    } catch (const DevError &e) {
        for (hipEvent_t &ev : D.prof_ev)
            if (ev) (void)hipEventDestroy(ev);
        D.prof_ev.clear();
        h->err = e.msg;
        return e.st;
    }
    if (enable) D.prof_n = 0;
    D.prof_on = enable != 0;
    return GDSW_OK;
}

gdsw_status profile_read(gdsw_handle_s *h, float *ms, int max, int *count) {
    if (!h->factored || !h->dev) {
        h->err = "profile_read before factor";
        return GDSW_ERR_STATE;
    }
    Device &D = *h->dev;
    *count = D.prof_n;
    try {
        for (int i = 0; i < std::min(max, D.prof_n); ++i) {
            HIPCHK(hipEventSynchronize(D.prof_ev[size_t(2 * i + 1)]));
            HIPCHK(hipEventElapsedTime(&ms[i], D.prof_ev[size_t(2 * i)], D.prof_ev[size_t(2 * i + 1)]));
        }
    } catch (const DevError &e) {
        h->err = e.msg;
        return e.st;
    }
    return GDSW_OK;
}

gdsw_status set_launch(gdsw_handle_s *h, int local_variant, int gemv_variant, int apply_streams,
                       int prolong_variant, void *stream) {
    if (!h->factored || !h->dev) {
        h->err = "set_launch before factor";
        return GDSW_ERR_STATE;
    }
    Symbolic &S = h->sym;
    Device &D = *h->dev;
    const int nv = S.opt.local == GDSW_LOCAL_ILU0 ? N_ILU_VARIANTS : N_BAND_VARIANTS;
    if (local_variant < -1 || local_variant >= nv || gemv_variant < -1 || gemv_variant > 1 || apply_streams < -1 ||
        apply_streams == 0 || apply_streams > 2 || prolong_variant < -1 || prolong_variant > 1) {
        h->err = "set_launch: configuration out of range";
        return GDSW_ERR_INVALID_ARG;
    }
    if (prolong_variant == 1 && sizeof(double) * size_t(D.max_k_big) > D.max_lds) {
        h->err = "set_launch: the block prolongation does not fit this handle";
        return GDSW_ERR_INVALID_ARG;
    }
    if (local_variant >= 0) {
        hipStream_t s = static_cast<hipStream_t>(stream);
        bool fits = false;
        try {
            hipLaunchKernelGGL(k_fill, dim3(nblocks(D.nv, 256, 65536)), dim3(256), 0, s, D.kr, 1.0, D.nv);
            Skip none;
            none.sl = D.slots;
            switch (S.opt.local_prec) {
                case GDSW_FP64: fits = launch_local_fits_all<double>(S, D, local_variant, D.kr, none, s); break;
                case GDSW_FP32: fits = launch_local_fits_all<float>(S, D, local_variant, D.kr, none, s); break;
                case GDSW_BF16: fits = launch_local_fits_all<bf16>(S, D, local_variant, D.kr, none, s); break;
                default: fits = launch_local_fits_all<fp16>(S, D, local_variant, D.kr, none, s); break;
            }
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(s));
        } catch (const DevError &e) {
            h->err = e.msg;
            return e.st;
        }
        if (!fits) {
            h->err = "set_launch: the local-solve configuration does not fit this handle";
            return GDSW_ERR_INVALID_ARG;
        }
    }
    if (prolong_variant == 1 && !D.zc && D.A0inv) {
        try {
            D.zc = D.alloc<double>(D.ns * S.n);
        } catch (const DevError &e) {
            h->err = e.msg;
            return e.st;
        }
    }
    D.local_variant = local_variant;
    // one configuration for every class, in both class layouts
    for (auto *v : {&D.cls, &D.cls_one, &D.cls_split})
        for (Device::SizeClass &c : *v) c.variant = -1;
    D.gemv_variant = gemv_variant;
    D.apply_streams = apply_streams;
    D.prolong_split = prolong_variant;
    return GDSW_OK;
}

gdsw_status set_size_classes(gdsw_handle_s *h, int split) {
    if (!h->factored || !h->dev) {
        h->err = "set_size_classes before factor";
        return GDSW_ERR_STATE;
    }
    Device &D = *h->dev;
    D.cls = split && D.cls_split.size() > 1 ? D.cls_split : D.cls_one;
    return GDSW_OK;
}

int tuned_variant(const gdsw_handle_s *h, int which) {
    if (!h->dev) return -1;
    return which == 0 ? h->dev->local_variant
         : which == 1 ? h->dev->gemv_variant
         : which == 2 ? h->dev->apply_streams
         : which == 3 ? h->dev->prolong_split
                      : int(h->dev->cls.size());
}

void destroy_device(gdsw_handle_s *h) {
    delete h->dev;
    h->dev = nullptr;
    h->factored = false;
}

int64_t device_bytes(const gdsw_handle_s *h) { return h->dev ? h->dev->bytes : 0; }

// Device bytes held per right-hand-side slot (the six Krylov vectors, the
// local results, the coarse partials, r_0, z_0 and its repetitions, the
// blocked coarse prolongation, the sweep iterates, the Krylov row-block
// tables, partial sums and states of the slot's problems); the rest of
// device_bytes is the operator itself, held once.
int64_t slot_bytes(const gdsw_handle_s *h) {
    if (!h->dev) return 0;
    const Device &D = *h->dev;
    const Symbolic &S = h->sym;
    const int64_t cols = D.zg ? D.slots.cols : 0, n0 = D.z0 ? S.n0 : 0, nkb = D.nkb / D.ns;
    return int64_t(sizeof(double)) * (6 * S.n + S.ov_ptr[S.np] + D.n_partial + 2 * n0 + cols + (D.zc ? S.n : 0) +
                                      2 * nkb) +
           int64_t(D.sweep_bytes) + int64_t(sizeof(double)) * (D.nd_w ? D.nd_nst : 0) +
           int64_t(sizeof(int32_t)) * (3 * nkb + S.nprob) +
           int64_t(sizeof(KState) + 2 * sizeof(int)) * S.nprob;
}

gdsw_status copy_device_map(gdsw_handle_s *h, int map, void *out) {
    if (!h->factored || !h->dev) return GDSW_ERR_STATE;
    Device &D = *h->dev;
    Symbolic &S = h->sym;
    try {
        if (map == GDSW_MAP_A0) {
            if (!D.A0) return GDSW_ERR_STATE;
            HIPCHK(hipMemcpy(out, D.A0, sizeof(double) * size_t(S.a0_off[S.nprob]), hipMemcpyDeviceToHost));
            return GDSW_OK;
        }
        if (map == GDSW_MAP_PHI_VAL) {
            // values in the row order of the CSR view (rows ascending, block columns ascending)
            const PhiBlocks &B = S.blk;
            std::vector<double> vals(D.phi_entries);
            if (D.phi_entries)
                HIPCHK(hipMemcpy(vals.data(), D.phi, sizeof(double) * size_t(D.phi_entries), hipMemcpyDeviceToHost));
            double *o = static_cast<double *>(out);
            int64_t q = 0;
            for (int64_t d = 0; d < S.n; ++d) {
                const int g = S.dof_blk[d];
                if (g < 0) continue;
                const int64_t nr = B.row_ptr[g + 1] - B.row_ptr[g];
                for (int64_t c = B.col_ptr[g]; c < B.col_ptr[g + 1]; ++c)
                    o[q++] = vals[B.val_off[g] + (c - B.col_ptr[g]) * nr + S.dof_lr[d]];
            }
            return GDSW_OK;
        }
    } catch (const DevError &e) {
        h->err = e.msg;
        return e.st;
    }
    return GDSW_ERR_INVALID_ARG;
}

}  // namespace gdsw
