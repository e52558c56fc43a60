// C ABI entry points (include/gdsw.h): argument checks, error strings and
// dispatch to the host analysis (symbolic.cpp) and the device phases
// (device.hip).
#include <algorithm>
#include <cstring>
#include <new>

#include "gdsw_impl.hpp"

template <typename T>
static void copy_vec(const std::vector<T> &v, void *out) {
    if (!v.empty()) std::memcpy(out, v.data(), sizeof(T) * v.size());
}

extern "C" {

void gdsw_default_options(gdsw_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->overlap = 1;
    opt->coarse = GDSW_COARSE_GDSW;
    opt->local = GDSW_LOCAL_EXACT;
    opt->jacobi_sweeps = 5;
    opt->local_prec = GDSW_FP64;
    opt->basis_prec = GDSW_FP64;
    opt->hbm_budget_bytes = 0;
    opt->flags = 0;
    opt->slots = 1;
    opt->exact_order = GDSW_ORDER_NATURAL;
}

gdsw_status gdsw_analyze(const gdsw_csr *A, const int32_t *part, int32_t n_parts, int32_t dpn, const double *Z,
                         int32_t n_null, const gdsw_options *opt, gdsw_handle *out) {
    if (!out) return GDSW_ERR_INVALID_ARG;
    *out = nullptr;
    gdsw_handle_s *h = new (std::nothrow) gdsw_handle_s();
    if (!h) return GDSW_ERR_BUDGET;
    gdsw_status st = gdsw::analyze(h, A, part, n_parts, dpn, Z, n_null, opt);
    *out = h;   // returned even on error so that gdsw_last_error can be read
    return st;
}

gdsw_status gdsw_analyze_sharing(const gdsw_csr *A, const int32_t *part, int32_t n_parts, int32_t dpn,
                                 const double *Z, int32_t n_null, const int64_t *share_ptr,
                                 const int32_t *share_sub, const gdsw_options *opt, gdsw_handle *out) {
    if (!out) return GDSW_ERR_INVALID_ARG;
    *out = nullptr;
    if (!share_ptr || !share_sub) return GDSW_ERR_INVALID_ARG;
    gdsw_handle_s *h = new (std::nothrow) gdsw_handle_s();
    if (!h) return GDSW_ERR_BUDGET;
    gdsw_status st = gdsw::analyze(h, A, part, n_parts, dpn, Z, n_null, opt, share_ptr, share_sub);
    *out = h;
    return st;
}

gdsw_status gdsw_analyze_batch(int32_t count, const gdsw_csr *A, const int32_t *const *part, const int32_t *n_parts,
                               int32_t dpn, const double *const *Z, int32_t n_null, const gdsw_options *opt,
                               gdsw_handle *out) {
    if (!out) return GDSW_ERR_INVALID_ARG;
    *out = nullptr;
    gdsw_handle_s *h = new (std::nothrow) gdsw_handle_s();
    if (!h) return GDSW_ERR_BUDGET;
    gdsw_status st = gdsw::analyze_batch(h, count, A, part, n_parts, dpn, Z, n_null, opt);
    *out = h;
    return st;
}

gdsw_status gdsw_solve_batch(gdsw_handle h, const double *b_dev, double *x_dev, double rtol, int32_t maxit,
                             gdsw_solve_info *infos, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::solve(h, b_dev, x_dev, GDSW_KRYLOV_CG, 0, rtol, maxit, 0, infos,
                       std::max(1, h->sym.opt.slots) * h->sym.nprob, stream);
}

gdsw_status gdsw_slots_begin(gdsw_handle h, const double *b_dev, double *x_dev, double rtol, int32_t maxit,
                             void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::slots_begin(h, b_dev, x_dev, rtol, maxit, stream);
}

gdsw_status gdsw_slot_start(gdsw_handle h, int32_t slot, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::slot_start(h, slot, stream);
}

gdsw_status gdsw_slots_step(gdsw_handle h, int32_t iters, int32_t *state, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::slots_step(h, iters, state, stream);
}

gdsw_status gdsw_slot_finish(gdsw_handle h, int32_t slot, gdsw_solve_info *info, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::slot_finish(h, slot, info, stream);
}

gdsw_status gdsw_autotune(gdsw_handle h, int32_t reps, float *times_ms, void *stream) {
    if (!h || reps <= 0) return GDSW_ERR_INVALID_ARG;
    return gdsw::autotune(h, reps, times_ms, stream);
}

gdsw_status gdsw_set_launch(gdsw_handle h, int32_t local_variant, int32_t gemv_variant, int32_t apply_streams,
                            int32_t prolong_variant, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::set_launch(h, local_variant, gemv_variant, apply_streams, prolong_variant, stream);
}

gdsw_status gdsw_set_size_classes(gdsw_handle h, int32_t split) {
    if (!h || split < 0 || split > 1) return GDSW_ERR_INVALID_ARG;
    return gdsw::set_size_classes(h, split);
}

gdsw_status gdsw_profile_local(gdsw_handle h, int32_t enable) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::profile_local(h, enable);
}

gdsw_status gdsw_profile_read(gdsw_handle h, float *ms, int32_t max, int32_t *count) {
    if (!h || !count || max < 0 || (max > 0 && !ms)) return GDSW_ERR_INVALID_ARG;
    return gdsw::profile_read(h, ms, max, count);
}

gdsw_status gdsw_problem_offsets(gdsw_handle h, int64_t *offsets) {
    if (!h || !offsets) return GDSW_ERR_INVALID_ARG;
    if (!h->analyzed) return GDSW_ERR_STATE;
    const gdsw::Symbolic &S = h->sym;
    const int ns = std::max(1, S.opt.slots);
    for (int k = 0; k < ns; ++k)
        for (int p = 0; p < S.nprob; ++p) offsets[k * S.nprob + p] = int64_t(k) * S.n + S.prob_ptr[p];
    offsets[ns * S.nprob] = int64_t(ns) * S.n;
    return GDSW_OK;
}

gdsw_status gdsw_factor(gdsw_handle h, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    if (!h->analyzed) {
        h->err = "factor before a successful analysis";
        return GDSW_ERR_STATE;
    }
    return gdsw::factor(h, stream);
}

gdsw_status gdsw_refactor(gdsw_handle h, const double *val, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    if (!h->analyzed) return GDSW_ERR_STATE;
    return gdsw::refactor(h, val, stream);
}

gdsw_status gdsw_setup(const gdsw_csr *A, const int32_t *part, int32_t n_parts, int32_t dpn, const double *Z,
                       int32_t n_null, const gdsw_options *opt, void *stream, gdsw_handle *out) {
    gdsw_status st = gdsw_analyze(A, part, n_parts, dpn, Z, n_null, opt, out);
    if (st != GDSW_OK) return st;
    return gdsw_factor(*out, stream);
}

gdsw_status gdsw_apply(gdsw_handle h, const double *r_dev, double *z_dev, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::apply(h, r_dev, z_dev, 3, stream);
}

gdsw_status gdsw_apply_static(gdsw_handle h, const double *r_dev, double *z_dev, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::apply_static(h, r_dev, z_dev, stream);
}

gdsw_status gdsw_apply_part(gdsw_handle h, const double *r_dev, double *z_dev, int32_t which, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::apply(h, r_dev, z_dev, which, stream);
}

gdsw_status gdsw_spmv(gdsw_handle h, const double *x_dev, double *y_dev, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::spmv(h, x_dev, y_dev, stream);
}

gdsw_status gdsw_solve(gdsw_handle h, const double *b_dev, double *x_dev, int32_t krylov, int32_t restart,
                       double rtol, int32_t maxit, int32_t fixed_iters, gdsw_solve_info *info, void *stream) {
    if (!h) return GDSW_ERR_INVALID_ARG;
    return gdsw::solve(h, b_dev, x_dev, krylov, restart, rtol, maxit, fixed_iters, info, 1, stream);
}

gdsw_status gdsw_get_info(gdsw_handle h, gdsw_info *info) {
    if (!h || !info) return GDSW_ERR_INVALID_ARG;
    const gdsw::Symbolic &S = h->sym;
    std::memset(info, 0, sizeof(*info));
    info->n = S.n;
    info->n_nodes = S.nn;
    info->dpn = S.dpn;
    info->n_parts = S.np;
    info->sum_overlap_dofs = S.ov_ptr.empty() ? 0 : S.ov_ptr.back();
    info->n_gamma_nodes = S.n_gamma_nodes;
    info->n_components = S.nc;
    info->n0 = S.n0;
    info->phi_entries = S.blk.val_off.empty() ? 0 : S.blk.val_off.back();
    info->local_factor_entries = 0;
    if (S.opt.local == GDSW_LOCAL_EXACT)
        info->local_factor_entries =
            (S.nd.voff.empty() ? 0 : S.nd.voff.back()) + (S.band_off.empty() ? 0 : S.band_off.back());
    else
        info->local_factor_entries = S.lcol.size();
    info->device_bytes = gdsw::device_bytes(h);
    info->max_local_rows = S.max_ni;
    info->max_bandwidth = S.max_bw;
    info->t_analyze = S.t_analyze;
    info->t_factor = h->t_factor;
    info->n_problems = S.nprob;
    info->local_variant = gdsw::tuned_variant(h, 0);
    info->gemv_variant = gdsw::tuned_variant(h, 1);
    info->apply_streams = gdsw::tuned_variant(h, 2);
    info->prolong_variant = gdsw::tuned_variant(h, 3);
    info->t_refactor = h->t_refactor;
    info->slots = std::max(1, S.opt.slots);
    info->slot_bytes = gdsw::slot_bytes(h);
    info->exact_order = S.opt.exact_order;
    info->local_classes = h->dev ? gdsw::tuned_variant(h, 4) : 1;
    info->nd_subdomains = 0;
    for (uint8_t m : S.nd_mask) info->nd_subdomains += m;
    {
        const int64_t vb = S.opt.local_prec == GDSW_FP64 ? 8 : S.opt.local_prec == GDSW_FP32 ? 4 : 2;
        const int64_t nloc = S.ov_ptr.empty() ? 0 : S.ov_ptr.back();
        int64_t b = nloc * 20;   // restriction index, gathered r, local result
        if (S.opt.local == GDSW_LOCAL_ILU0) {
            const int64_t off = int64_t(S.lcol.size()) - nloc;   // off-diagonal factor entries
            b += off * (vb + 2) + nloc * vb;
        } else {
            // the band twice (forward, backward); the panels' lower parts
            // twice, their gather lists and struct rows once
            b += 2 * vb * (S.band_off.empty() ? 0 : S.band_off.back());
            for (int64_t J = 0; J < S.nd.nsn; ++J) {
                const int64_t nJ = S.nd.ncol[J], ns = S.nd.nrow[J] - nJ;
                b += 2 * vb * (nJ * (nJ + 1) / 2 + nJ * ns);
            }
            // the gather entries, the struct rows and their supernodes, the
            // struct products written and read back, the inverse permutation
            const int64_t ab = S.opt.local_prec == GDSW_FP64 ? 8 : 4;
            b += 4 * int64_t(S.nd.rc_w.size()) + (8 + 2 * ab) * int64_t(S.nd.st_row.size());
            for (int i = 0; i < S.np; ++i)
                if (!S.nd_mask.empty() && S.nd_mask[i]) b += 4 * (S.ov_ptr[i + 1] - S.ov_ptr[i]);
        }
        info->local_solve_bytes = b;
    }
    return GDSW_OK;
}

static int64_t map_count(gdsw_handle h, int32_t map) {
    const gdsw::Symbolic &S = h->sym;
    switch (map) {
        case GDSW_MAP_OV_PTR: return int64_t(S.ov_ptr.size());
        case GDSW_MAP_OV_IDX: return int64_t(S.ov_idx.size());
        case GDSW_MAP_IS_GAMMA: return int64_t(S.is_gamma.size());
        case GDSW_MAP_COMP_OF_NODE: return int64_t(S.comp_of_node.size());
        case GDSW_MAP_COMP_RANK: return int64_t(S.comp_rank.size());
        case GDSW_MAP_PHI_ROWPTR: return S.n + 1;
        case GDSW_MAP_PHI_COL:
        case GDSW_MAP_PHI_VAL: return S.blk.val_off.empty() ? 0 : S.blk.val_off.back();
        case GDSW_MAP_A0: return S.a0_off.empty() ? 0 : S.a0_off.back();
        case GDSW_MAP_LOCAL_ROWPTR: return int64_t(S.lrowptr.size());
        case GDSW_MAP_LOCAL_COL: return int64_t(S.lcol.size());
        case GDSW_MAP_ND_PERM: return int64_t(S.nd.perm.size());
        case GDSW_MAP_ND_SN_PTR: return int64_t(S.nd.sn_ptr.size());
        case GDSW_MAP_ND_SN: return 4 * S.nd.nsn;
        case GDSW_MAP_ND_VOFF: return int64_t(S.nd.voff.size());
        case GDSW_MAP_ND_ST_PTR: return int64_t(S.nd.st_ptr.size());
        case GDSW_MAP_ND_ST_ROW: return int64_t(S.nd.st_row.size());
        case GDSW_MAP_ND_RC_PTR: return int64_t(S.nd.rc_ptr.size());
        case GDSW_MAP_ND_RC: return 2 * int64_t(S.nd.rc_sn.size());
        case GDSW_MAP_ND_LV_BASE: return int64_t(S.nd.lv_base.size());
        case GDSW_MAP_ND_LV_PTR: return int64_t(S.nd.lv_ptr.size());
        case GDSW_MAP_ND_LV_ROWS: return int64_t(S.nd.lv_rows.size());
        case GDSW_MAP_ND_UP_PTR: return int64_t(S.nd.up_ptr.size());
        case GDSW_MAP_ND_UP: return 4 * int64_t(S.nd.up_k.size());
        case GDSW_MAP_ND_REL: return int64_t(S.nd.rel.size());
        case GDSW_MAP_ND_ASM: return 2 * int64_t(S.nd.asm_src.size());
        case GDSW_MAP_ND_RC_W: return int64_t(S.nd.rc_w.size());
        case GDSW_MAP_ND_ST_SN: return int64_t(S.nd.st_sn.size());
        case GDSW_MAP_ND_LV_INFO: return int64_t(S.nd.lv_info.size());
        case GDSW_MAP_ND_CH_BASE: return int64_t(S.nd.ch_base.size());
        case GDSW_MAP_ND_CH_ROW: return int64_t(S.nd.ch_row.size());
        default: return -1;
    }
}

gdsw_status gdsw_map_size(gdsw_handle h, int32_t map, int64_t *count) {
    if (!h || !count) return GDSW_ERR_INVALID_ARG;
    int64_t c = map_count(h, map);
    if (c < 0) return GDSW_ERR_INVALID_ARG;
    *count = c;
    return GDSW_OK;
}

gdsw_status gdsw_copy_map(gdsw_handle h, int32_t map, void *out) {
    if (!h || !out) return GDSW_ERR_INVALID_ARG;
    const gdsw::Symbolic &S = h->sym;
    switch (map) {
        case GDSW_MAP_OV_PTR:
            std::memcpy(out, S.ov_ptr.data(), 8 * S.ov_ptr.size());
            return GDSW_OK;
        case GDSW_MAP_OV_IDX: {
            int64_t *o = static_cast<int64_t *>(out);
            for (size_t p = 0; p < S.ov_idx.size(); ++p) o[p] = S.ov_idx[p];
            return GDSW_OK;
        }
        case GDSW_MAP_IS_GAMMA:
            std::memcpy(out, S.is_gamma.data(), S.is_gamma.size());
            return GDSW_OK;
        case GDSW_MAP_COMP_OF_NODE:
            std::memcpy(out, S.comp_of_node.data(), 4 * S.comp_of_node.size());
            return GDSW_OK;
        case GDSW_MAP_COMP_RANK:
            std::memcpy(out, S.comp_rank.data(), 4 * S.comp_rank.size());
            return GDSW_OK;
        case GDSW_MAP_PHI_ROWPTR:
        case GDSW_MAP_PHI_COL: {
            // CSR view of Phi: rows ascending, each row's block columns ascending
            const gdsw::PhiBlocks &B = S.blk;
            int64_t *rp = map == GDSW_MAP_PHI_ROWPTR ? static_cast<int64_t *>(out) : nullptr;
            int32_t *cc = map == GDSW_MAP_PHI_COL ? static_cast<int32_t *>(out) : nullptr;
            int64_t q = 0;
            if (rp) rp[0] = 0;
            for (int64_t d = 0; d < S.n; ++d) {
                const int g = S.dof_blk.empty() ? -1 : S.dof_blk[d];
                if (g >= 0)
                    for (int64_t c = B.col_ptr[g]; c < B.col_ptr[g + 1]; ++c) {
                        if (cc) cc[q] = B.cols[c];
                        ++q;
                    }
                if (rp) rp[d + 1] = q;
            }
            return GDSW_OK;
        }
        case GDSW_MAP_PHI_VAL:
        case GDSW_MAP_A0:
            return gdsw::copy_device_map(h, map, out);
        case GDSW_MAP_LOCAL_ROWPTR:
            std::memcpy(out, S.lrowptr.data(), 8 * S.lrowptr.size());
            return GDSW_OK;
        case GDSW_MAP_LOCAL_COL:
            std::memcpy(out, S.lcol.data(), 4 * S.lcol.size());
            return GDSW_OK;
        case GDSW_MAP_ND_PERM: copy_vec(S.nd.perm, out); return GDSW_OK;
        case GDSW_MAP_ND_SN_PTR: copy_vec(S.nd.sn_ptr, out); return GDSW_OK;
        case GDSW_MAP_ND_SN: {
            int32_t *o = static_cast<int32_t *>(out);
            for (int64_t J = 0; J < S.nd.nsn; ++J) {
                o[4 * J] = S.nd.first[J];
                o[4 * J + 1] = S.nd.ncol[J];
                o[4 * J + 2] = S.nd.nrow[J];
                o[4 * J + 3] = S.nd.height[J];
            }
            return GDSW_OK;
        }
        case GDSW_MAP_ND_VOFF: copy_vec(S.nd.voff, out); return GDSW_OK;
        case GDSW_MAP_ND_ST_PTR: copy_vec(S.nd.st_ptr, out); return GDSW_OK;
        case GDSW_MAP_ND_ST_ROW: copy_vec(S.nd.st_row, out); return GDSW_OK;
        case GDSW_MAP_ND_RC_PTR: copy_vec(S.nd.rc_ptr, out); return GDSW_OK;
        case GDSW_MAP_ND_RC: {
            int32_t *o = static_cast<int32_t *>(out);
            for (size_t q = 0; q < S.nd.rc_sn.size(); ++q) {
                o[2 * q] = S.nd.rc_sn[q];
                o[2 * q + 1] = S.nd.rc_pos[q];
            }
            return GDSW_OK;
        }
        case GDSW_MAP_ND_LV_BASE: copy_vec(S.nd.lv_base, out); return GDSW_OK;
        case GDSW_MAP_ND_LV_PTR: copy_vec(S.nd.lv_ptr, out); return GDSW_OK;
        case GDSW_MAP_ND_LV_ROWS: copy_vec(S.nd.lv_rows, out); return GDSW_OK;
        case GDSW_MAP_ND_UP_PTR: copy_vec(S.nd.up_ptr, out); return GDSW_OK;
        case GDSW_MAP_ND_UP: {
            int64_t *o = static_cast<int64_t *>(out);
            for (size_t q = 0; q < S.nd.up_k.size(); ++q) {
                o[4 * q] = S.nd.up_k[q];
                o[4 * q + 1] = S.nd.up_s0[q];
                o[4 * q + 2] = S.nd.up_n1[q];
                o[4 * q + 3] = S.nd.up_rel[q];
            }
            return GDSW_OK;
        }
        case GDSW_MAP_ND_REL: copy_vec(S.nd.rel, out); return GDSW_OK;
        case GDSW_MAP_ND_RC_W: copy_vec(S.nd.rc_w, out); return GDSW_OK;
        case GDSW_MAP_ND_ST_SN: copy_vec(S.nd.st_sn, out); return GDSW_OK;
        case GDSW_MAP_ND_LV_INFO: copy_vec(S.nd.lv_info, out); return GDSW_OK;
        case GDSW_MAP_ND_CH_BASE: copy_vec(S.nd.ch_base, out); return GDSW_OK;
        case GDSW_MAP_ND_CH_ROW: copy_vec(S.nd.ch_row, out); return GDSW_OK;
        case GDSW_MAP_ND_ASM: {
            int64_t *o = static_cast<int64_t *>(out);
            for (size_t q = 0; q < S.nd.asm_src.size(); ++q) {
                o[2 * q] = S.nd.asm_src[q];
                o[2 * q + 1] = S.nd.asm_dst[q];
            }
            return GDSW_OK;
        }
        default:
            return GDSW_ERR_INVALID_ARG;
    }
}

gdsw_status gdsw_destroy(gdsw_handle h) {
    if (!h) return GDSW_OK;
    gdsw::destroy_device(h);
    delete h;
    return GDSW_OK;
}

const char *gdsw_status_string(gdsw_status s) {
    switch (s) {
        case GDSW_OK: return "ok";
        case GDSW_ERR_INVALID_ARG: return "invalid argument";
        case GDSW_ERR_SINGULAR: return "singular or indefinite pivot";
        case GDSW_ERR_BREAKDOWN: return "Krylov breakdown";
        case GDSW_ERR_NOT_CONVERGED: return "not converged";
        case GDSW_ERR_BUDGET: return "device memory budget exceeded";
        case GDSW_ERR_HIP: return "HIP runtime error";
        case GDSW_ERR_STATE: return "call out of order";
        case GDSW_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *gdsw_last_error(gdsw_handle h) {
    if (!h) return "null handle";
    return h->err.c_str();
}

}  // extern "C"
