// Host symbolic analysis of the GDSW preconditioner: phase (a) of the
// paper's three-phase solver structure (Sec. V-A, "Software Structure"):
// everything that depends only on the sparsity pattern, the partition and
// the null space, computed once on the CPU and uploaded by the numeric phase.
//
//  * node graph of the matrix pattern;
//  * overlapping subdomains Omega_i' (Sec. III: the nonoverlapping
//    subdomains grown by `overlap` layers; the experiments use an algebraic
//    overlap of one, Sec. VII) and the restriction maps R_i;
//  * interface Gamma and interior I of the nonoverlapping partition
//    (Sec. III, 2x2 block form): a node is on the interface when it has a
//    neighbour in a lower-numbered subdomain; this gives a one-node-thick
//    interface with A_II block diagonal, as the extension of eq. (2) needs;
//  * interface components (Sec. III item 1): nodes grouped by the set of
//    subdomains that meet them, split into connected pieces, ordered by their
//    smallest node; the pieces are disjoint so the partition of unity of
//    item 2 is the identity;
//  * interface basis Phi_G (Sec. III items 3-4): the null space restricted
//    to each component, orthonormalised by modified Gram-Schmidt with one
//    reorthogonalisation, dropping columns that vanish (relative 1e-10);
//  * local matrix patterns, band profiles (exact solver), level schedules
//    and padded sweep layout (ILU(0)), coarse-block maps and the assembly
//    lists of A_0 = Phi^T A Phi.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <functional>
#include <map>
#include <numeric>
#include <queue>
#include <stdexcept>
#include <string>
#include <vector>

#include "gdsw_impl.hpp"

namespace gdsw {
namespace {

struct Fail {
    gdsw_status st;
    std::string msg;
};

[[noreturn]] void fail(gdsw_status st, const std::string &m) { throw Fail{st, m}; }

template <class T>
void exclusive_scan_inplace(std::vector<T> &v) {
    T run = 0;
    for (auto &x : v) {
        T t = x;
        x = run;
        run += t;
    }
}

// ---------------------------------------------------------------------------
void validate_and_copy(Symbolic &s, const gdsw_csr *A, const int32_t *part, int32_t n_parts,
                       int32_t dpn, const double *Z, int32_t n_null, const gdsw_options *opt) {
    if (!A || !A->rowptr || !A->col || !A->val || !part) fail(GDSW_ERR_INVALID_ARG, "null argument");
    if (A->n <= 0 || A->n >= (int64_t(1) << 31)) fail(GDSW_ERR_INVALID_ARG, "n out of range");
    if (dpn <= 0 || A->n % dpn) fail(GDSW_ERR_INVALID_ARG, "n must be a multiple of dpn");
    if (n_parts <= 0) fail(GDSW_ERR_INVALID_ARG, "n_parts must be positive");
    gdsw_options o;
    if (opt) o = *opt; else gdsw_default_options(&o);
    if (o.overlap < 0 || o.overlap > 64) fail(GDSW_ERR_INVALID_ARG, "overlap out of range");
    if (o.coarse != GDSW_COARSE_NONE && o.coarse != GDSW_COARSE_GDSW && o.coarse != GDSW_COARSE_RGDSW)
        fail(GDSW_ERR_INVALID_ARG, "coarse");
    if (o.local != GDSW_LOCAL_EXACT && o.local != GDSW_LOCAL_ILU0) fail(GDSW_ERR_INVALID_ARG, "local");
    if (o.jacobi_sweeps < 1 || o.jacobi_sweeps > 1000) fail(GDSW_ERR_INVALID_ARG, "jacobi_sweeps");
    if (o.local_prec < GDSW_FP64 || o.local_prec > GDSW_FP16) fail(GDSW_ERR_INVALID_ARG, "local_prec");
    if (o.basis_prec != GDSW_FP64 && o.basis_prec != GDSW_FP32) fail(GDSW_ERR_INVALID_ARG, "basis_prec");
    if (o.flags & ~uint64_t(GDSW_FLAG_GRAPHS)) fail(GDSW_ERR_INVALID_ARG, "unknown flags");
    if (o.ilu_level < 0 || o.ilu_level > 8) fail(GDSW_ERR_INVALID_ARG, "ilu_level out of range");
    if (o.ilu_factor_sweeps < 0 || o.ilu_factor_sweeps > 100) fail(GDSW_ERR_INVALID_ARG, "ilu_factor_sweeps");
    if (o.slots == 0) o.slots = 1;
    if (o.slots < 0 || o.slots > 4096) fail(GDSW_ERR_INVALID_ARG, "slots out of range");
    if (o.exact_order != GDSW_ORDER_NATURAL && o.exact_order != GDSW_ORDER_ND && o.exact_order != GDSW_ORDER_AUTO)
        fail(GDSW_ERR_INVALID_ARG, "exact_order");
    if (o.local != GDSW_LOCAL_EXACT) o.exact_order = GDSW_ORDER_NATURAL;
    if (Z == nullptr && n_null > 1) fail(GDSW_ERR_INVALID_ARG, "Z == NULL needs n_null <= 1");
    if (Z != nullptr && (n_null <= 0 || n_null > 64)) fail(GDSW_ERR_INVALID_ARG, "n_null out of range");
    s.opt = o;
    s.n = A->n;
    s.dpn = dpn;
    s.nn = A->n / dpn;
    s.np = n_parts;
    if (A->rowptr[0] != 0) fail(GDSW_ERR_INVALID_ARG, "rowptr[0] != 0");
    for (int64_t i = 0; i < s.n; ++i)
        if (A->rowptr[i + 1] < A->rowptr[i]) fail(GDSW_ERR_INVALID_ARG, "rowptr not monotone");
    s.nnz = A->rowptr[s.n];
    if (s.nnz >= (int64_t(1) << 31)) fail(GDSW_ERR_INVALID_ARG, "nnz must be < 2^31");
    s.rowptr.assign(A->rowptr, A->rowptr + s.n + 1);
    s.col.assign(A->col, A->col + s.nnz);
    s.val.assign(A->val, A->val + s.nnz);
    for (int64_t i = 0; i < s.n; ++i) {
        bool diag = false;
        for (int64_t p = s.rowptr[i]; p < s.rowptr[i + 1]; ++p) {
            int32_t c = s.col[p];
            if (c < 0 || c >= s.n) fail(GDSW_ERR_INVALID_ARG, "column index out of range");
            if (p > s.rowptr[i] && c <= s.col[p - 1]) fail(GDSW_ERR_INVALID_ARG, "columns not sorted/unique");
            if (!std::isfinite(s.val[p])) fail(GDSW_ERR_INVALID_ARG, "non-finite matrix value");
            if (c == i) diag = true;
        }
        if (!diag) fail(GDSW_ERR_INVALID_ARG, "missing diagonal entry");
    }
    s.part.assign(part, part + s.nn);
    for (int32_t p : s.part)
        if (p < 0 || p >= n_parts) fail(GDSW_ERR_INVALID_ARG, "part out of range");
    s.n_null = Z ? n_null : 1;
    if (Z) {
        s.Z.assign(Z, Z + s.n * int64_t(n_null));
        for (double z : s.Z)
            if (!std::isfinite(z)) fail(GDSW_ERR_INVALID_ARG, "non-finite null-space value");
    } else {
        s.Z.assign(s.n, 1.0);
    }
    // the coarse assembly and the Cholesky local solver use symmetry of A
    if (o.coarse != GDSW_COARSE_NONE || o.local == GDSW_LOCAL_EXACT) {
        for (int64_t i = 0; i < s.n; ++i)
            for (int64_t p = s.rowptr[i]; p < s.rowptr[i + 1]; ++p) {
                int32_t j = s.col[p];
                const int32_t *b = s.col.data() + s.rowptr[j];
                const int32_t *e = s.col.data() + s.rowptr[j + 1];
                const int32_t *f = std::lower_bound(b, e, int32_t(i));
                if (f == e || *f != i) fail(GDSW_ERR_INVALID_ARG, "matrix pattern must be symmetric");
                const double vij = s.val[p], vji = s.val[f - s.col.data()];
                if (std::fabs(vij - vji) > 1e-12 * std::max(std::fabs(vij), std::fabs(vji)))
                    fail(GDSW_ERR_INVALID_ARG, "matrix must be symmetric");
            }
    }
}

// ---------------------------------------------------------------------------
// node graph: u ~ v (u != v) iff a stored entry couples a dof of u and a dof
// of v; symmetrised, sorted, without duplicates
void build_graph(Symbolic &s) {
    const int64_t nn = s.nn;
    const int dpn = s.dpn;
    std::vector<int64_t> dptr(nn + 1, 0);
    std::vector<int32_t> dadj;
    dadj.reserve(s.nnz / (dpn * dpn) + nn);
    std::vector<int32_t> mark(nn, -1);
    for (int64_t u = 0; u < nn; ++u) {
        size_t start = dadj.size();
        for (int k = 0; k < dpn; ++k) {
            int64_t r = u * dpn + k;
            for (int64_t p = s.rowptr[r]; p < s.rowptr[r + 1]; ++p) {
                int32_t v = s.col[p] / dpn;
                if (v != u && mark[v] != u) {
                    mark[v] = int32_t(u);
                    dadj.push_back(v);
                }
            }
        }
        std::sort(dadj.begin() + start, dadj.end());
        dptr[u + 1] = int64_t(dadj.size());
    }
    // transpose
    std::vector<int64_t> tptr(nn + 1, 0);
    for (int32_t v : dadj) tptr[v + 1]++;
    for (int64_t i = 0; i < nn; ++i) tptr[i + 1] += tptr[i];
    std::vector<int32_t> tadj(dadj.size());
    {
        std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
        for (int64_t u = 0; u < nn; ++u)
            for (int64_t p = dptr[u]; p < dptr[u + 1]; ++p) tadj[fill[dadj[p]]++] = int32_t(u);
    }
    // union of the sorted rows (transposed rows are generated in ascending u)
    s.gptr.assign(nn + 1, 0);
    s.gadj.clear();
    s.gadj.reserve(dadj.size() + 8);
    for (int64_t u = 0; u < nn; ++u) {
        int64_t a = dptr[u], ae = dptr[u + 1], b = tptr[u], be = tptr[u + 1];
        while (a < ae || b < be) {
            int32_t x;
            if (b >= be || (a < ae && dadj[a] < tadj[b])) x = dadj[a++];
            else if (a >= ae || tadj[b] < dadj[a]) x = tadj[b++];
            else { x = dadj[a++]; ++b; }
            s.gadj.push_back(x);
        }
        s.gptr[u + 1] = int64_t(s.gadj.size());
    }
}

// ---------------------------------------------------------------------------
// overlapping subdomains by breadth-first growth, restriction maps and their
// transpose
void build_overlap(Symbolic &s) {
    const int64_t nn = s.nn;
    const int np = s.np, dpn = s.dpn;
    std::vector<int64_t> pptr(np + 1, 0);
    for (int32_t p : s.part) pptr[p + 1]++;
    for (int i = 0; i < np; ++i) pptr[i + 1] += pptr[i];
    std::vector<int32_t> pnodes(nn);
    {
        std::vector<int64_t> fill(pptr.begin(), pptr.end() - 1);
        for (int64_t v = 0; v < nn; ++v) pnodes[fill[s.part[v]]++] = int32_t(v);
    }
    std::vector<std::vector<int32_t>> ov(np);
#pragma omp parallel
    {
        std::vector<int32_t> mark(nn, -1);
#pragma omp for schedule(dynamic)
        for (int i = 0; i < np; ++i) {
            std::vector<int32_t> set(pnodes.begin() + pptr[i], pnodes.begin() + pptr[i + 1]);
            for (int32_t v : set) mark[v] = i;
            size_t frontier_begin = 0;
            for (int layer = 0; layer < s.opt.overlap; ++layer) {
                size_t fe = set.size();
                for (size_t q = frontier_begin; q < fe; ++q) {
                    int32_t v = set[q];
                    for (int64_t p = s.gptr[v]; p < s.gptr[v + 1]; ++p) {
                        int32_t u = s.gadj[p];
                        if (mark[u] != i) {
                            mark[u] = i;
                            set.push_back(u);
                        }
                    }
                }
                frontier_begin = fe;
            }
            std::sort(set.begin(), set.end());
            for (int32_t v : set) mark[v] = -1;
            ov[i] = std::move(set);
        }
    }
    s.ov_ptr.assign(np + 1, 0);
    for (int i = 0; i < np; ++i) s.ov_ptr[i + 1] = s.ov_ptr[i] + int64_t(ov[i].size()) * dpn;
    if (s.ov_ptr[np] >= (int64_t(1) << 31)) fail(GDSW_ERR_INVALID_ARG, "sum of subdomain sizes too large");
    s.ov_idx.resize(s.ov_ptr[np]);
    s.max_ni = 0;
    for (int i = 0; i < np; ++i) {
        int64_t o = s.ov_ptr[i];
        for (int32_t v : ov[i])
            for (int k = 0; k < dpn; ++k) s.ov_idx[o++] = v * dpn + k;
        s.max_ni = std::max<int32_t>(s.max_ni, int32_t(s.ov_ptr[i + 1] - s.ov_ptr[i]));
    }
    // transpose: local rows of every dof in ascending subdomain order
    s.t_ptr.assign(s.n + 1, 0);
    for (int32_t d : s.ov_idx) s.t_ptr[d + 1]++;
    for (int64_t d = 0; d < s.n; ++d) s.t_ptr[d + 1] += s.t_ptr[d];
    s.t_pos.resize(s.ov_idx.size());
    std::vector<int64_t> fill(s.t_ptr.begin(), s.t_ptr.end() - 1);
    for (int64_t p = 0; p < int64_t(s.ov_idx.size()); ++p) s.t_pos[fill[s.ov_idx[p]]++] = int32_t(p);
}

// ---------------------------------------------------------------------------
// interface, its components and the interface basis.  The interface of the
// node partition: a node with a neighbour in a lower-numbered subdomain,
// its set the subdomains of those neighbours and its own; or, when the
// caller gives them, the sets of subdomains whose elements hold each node
// (the geometric interface of an element decomposition, Sec. III).
void build_interface(Symbolic &s) {
    const int64_t nn = s.nn;
    s.is_gamma.assign(nn, 0);
    std::vector<std::vector<int32_t>> S(nn);
    int64_t ng = 0;
    if (!s.share_ptr.empty()) {
        // sharing sets given (a decomposition into subdomains of elements):
        // a node shared by two or more subdomains is on the interface
        for (int64_t v = 0; v < nn; ++v) {
            std::vector<int32_t> set(s.share_sub.begin() + s.share_ptr[v], s.share_sub.begin() + s.share_ptr[v + 1]);
            std::sort(set.begin(), set.end());
            set.erase(std::unique(set.begin(), set.end()), set.end());
            if (!std::binary_search(set.begin(), set.end(), s.part[v]))
                fail(GDSW_ERR_INVALID_ARG, "sharing sets: node " + std::to_string(v) + " is not shared by its own subdomain");
            if (set.size() >= 2) {
                s.is_gamma[v] = 1;
                ++ng;
                S[v] = std::move(set);
            }
        }
        // the extension needs A_II block diagonal: an interior node's
        // neighbours are all shared by its subdomain
        for (int64_t v = 0; v < nn; ++v) {
            if (s.is_gamma[v]) continue;
            for (int64_t p = s.gptr[v]; p < s.gptr[v + 1]; ++p) {
                const int32_t u = s.gadj[p];
                const bool ok = s.is_gamma[u] ? std::binary_search(S[u].begin(), S[u].end(), s.part[v])
                                              : s.part[u] == s.part[v];
                if (!ok)
                    fail(GDSW_ERR_INVALID_ARG, "sharing sets: interior node " + std::to_string(v) +
                                                   " is coupled to node " + std::to_string(u) +
                                                   ", which its subdomain does not share");
            }
        }
    } else
        for (int64_t v = 0; v < nn; ++v) {
            int32_t pv = s.part[v];
            std::vector<int32_t> lower;
            for (int64_t p = s.gptr[v]; p < s.gptr[v + 1]; ++p) {
                int32_t pu = s.part[s.gadj[p]];
                if (pu < pv) lower.push_back(pu);
            }
            if (!lower.empty()) {
                s.is_gamma[v] = 1;
                ++ng;
                lower.push_back(pv);
                std::sort(lower.begin(), lower.end());
                lower.erase(std::unique(lower.begin(), lower.end()), lower.end());
                S[v] = std::move(lower);
            }
        }
    s.n_gamma_nodes = ng;
    // group by S
    std::map<std::vector<int32_t>, int32_t> gid;
    std::vector<int32_t> group(nn, -1);
    for (int64_t v = 0; v < nn; ++v)
        if (s.is_gamma[v]) {
            auto it = gid.find(S[v]);
            if (it == gid.end()) it = gid.emplace(S[v], int32_t(gid.size())).first;
            group[v] = it->second;
        }
    // connected pieces within each group; discovered in ascending seed order,
    // so the pieces are already ordered by their smallest node
    s.comp_of_node.assign(nn, -1);
    s.comp_ptr.assign(1, 0);
    s.comp_nodes.clear();
    std::vector<int32_t> stack;
    int32_t nc = 0;
    for (int64_t seed = 0; seed < nn; ++seed) {
        if (!s.is_gamma[seed] || s.comp_of_node[seed] >= 0) continue;
        size_t start = s.comp_nodes.size();
        stack.assign(1, int32_t(seed));
        s.comp_of_node[seed] = nc;
        while (!stack.empty()) {
            int32_t v = stack.back();
            stack.pop_back();
            s.comp_nodes.push_back(v);
            for (int64_t p = s.gptr[v]; p < s.gptr[v + 1]; ++p) {
                int32_t u = s.gadj[p];
                if (group[u] == group[v] && s.comp_of_node[u] < 0) {
                    s.comp_of_node[u] = nc;
                    stack.push_back(u);
                }
            }
        }
        std::sort(s.comp_nodes.begin() + start, s.comp_nodes.end());
        s.comp_ptr.push_back(int64_t(s.comp_nodes.size()));
        ++nc;
    }
    s.nc = nc;
    // interface basis
    const int dpn = s.dpn, nz = s.n_null;
    // Gram-Schmidt of the columns of a (m x nz) block given by value(r, j),
    // twice per column, dropping a column whose remainder is <= 1e-10 of its
    // norm; returns the kept orthonormal columns (column-major, m each)
    auto orthonormalise = [&](int64_t m, const std::function<double(int64_t, int)> &value, int &kept) {
        std::vector<double> Q;
        std::vector<double> v(m);
        kept = 0;
        for (int j = 0; j < nz; ++j) {
            double nb = 0.0;
            for (int64_t r = 0; r < m; ++r) {
                v[r] = value(r, j);
                nb += v[r] * v[r];
            }
            nb = std::sqrt(nb);
            if (nb == 0.0) continue;
            for (int pass = 0; pass < 2; ++pass)
                for (int q = 0; q < kept; ++q) {
                    const double *qc = Q.data() + int64_t(q) * m;
                    double d = 0.0;
                    for (int64_t r = 0; r < m; ++r) d += qc[r] * v[r];
                    for (int64_t r = 0; r < m; ++r) v[r] -= d * qc[r];
                }
            double nv = 0.0;
            for (int64_t r = 0; r < m; ++r) nv += v[r] * v[r];
            nv = std::sqrt(nv);
            if (nv <= 1e-10 * nb) continue;
            for (int64_t r = 0; r < m; ++r) Q.push_back(v[r] / nv);
            ++kept;
        }
        return Q;
    };
    auto zval = [&](int32_t c, int64_t r, int j) {   // Z at row r of component c's block
        int64_t node = s.comp_nodes[s.comp_ptr[c] + r / dpn];
        return s.Z[int64_t(j) * s.n + node * dpn + r % dpn];
    };
    s.comp_rank.assign(nc, 0);
    s.ccol_ptr.assign(nc + 1, 0);
    s.ccol.clear();
    s.col_comp.clear();
    s.phig_off.assign(nc + 1, 0);
    std::vector<std::vector<double>> blocks(nc);
    if (s.opt.coarse != GDSW_COARSE_RGDSW) {
        // GDSW: Z restricted to each component, orthonormalised
#pragma omp parallel for schedule(dynamic)
        for (int32_t c = 0; c < nc; ++c) {
            const int64_t m = (s.comp_ptr[c + 1] - s.comp_ptr[c]) * dpn;
            int kept = 0;
            blocks[c] = orthonormalise(m, [&](int64_t r, int j) { return zval(c, r, j); }, kept);
            s.comp_rank[c] = kept;
        }
        for (int32_t c = 0; c < nc; ++c) {
            for (int32_t j = 0; j < s.comp_rank[c]; ++j) {
                s.ccol.push_back(int32_t(s.col_comp.size()));
                s.col_comp.push_back(c);
            }
            s.ccol_ptr[c + 1] = int64_t(s.ccol.size());
        }
    } else {
        // reduced GDSW (coarse functions for the vertices only): component d
        // is an ancestor of c when S(c) is a proper subset of S(d); the
        // coarse nodes are the components without an ancestor; a coarse node
        // owns itself, any other component is owned by its coarse-node
        // ancestors and carries the weight 1 / (number of owners) in each of
        // their functions; a coarse node's functions are Z on its support,
        // weighted, orthonormalised over the support
        std::vector<const std::vector<int32_t> *> cset(nc);
        for (int32_t c = 0; c < nc; ++c) cset[c] = &S[s.comp_nodes[s.comp_ptr[c]]];
        std::vector<std::vector<int32_t>> comps_of_sub(s.np);
        for (int32_t c = 0; c < nc; ++c) comps_of_sub[(*cset[c])[0]].push_back(c);
        for (int32_t c = 0; c < nc; ++c)
            for (size_t t = 1; t < cset[c]->size(); ++t) comps_of_sub[(*cset[c])[t]].push_back(c);
        auto strict_subset = [&](int32_t a, int32_t b) {   // S(a) proper subset of S(b)
            const auto &x = *cset[a], &y = *cset[b];
            return x.size() < y.size() && std::includes(y.begin(), y.end(), x.begin(), x.end());
        };
        std::vector<char> is_coarse(nc, 1);
        for (int32_t c = 0; c < nc; ++c)
            for (int32_t d : comps_of_sub[(*cset[c])[0]])
                if (strict_subset(c, d)) { is_coarse[c] = 0; break; }
        std::vector<std::vector<int32_t>> owners(nc);
        for (int32_t c = 0; c < nc; ++c) {
            if (is_coarse[c]) { owners[c].push_back(c); continue; }
            for (int32_t d : comps_of_sub[(*cset[c])[0]])
                if (is_coarse[d] && strict_subset(c, d)) owners[c].push_back(d);
            std::sort(owners[c].begin(), owners[c].end());
        }
        std::vector<std::vector<int32_t>> support(nc);   // of each coarse node, ascending
        for (int32_t c = 0; c < nc; ++c)
            for (int32_t v : owners[c]) support[v].push_back(c);
        std::vector<int32_t> coarse_nodes;
        for (int32_t c = 0; c < nc; ++c)
            if (is_coarse[c]) coarse_nodes.push_back(c);
        const int32_t nv = int32_t(coarse_nodes.size());
        std::vector<std::vector<double>> vblocks(nv);
        std::vector<int> vrank(nv, 0);
        std::vector<std::vector<int64_t>> vrow0(nv);   // first support row of each supporting component
#pragma omp parallel for schedule(dynamic)
        for (int32_t t = 0; t < nv; ++t) {
            const int32_t v = coarse_nodes[t];
            const auto &sup = support[v];
            std::vector<int64_t> r0(sup.size() + 1, 0);
            for (size_t q = 0; q < sup.size(); ++q)
                r0[q + 1] = r0[q] + (s.comp_ptr[sup[q] + 1] - s.comp_ptr[sup[q]]) * dpn;
            const int64_t m = r0.back();
            auto value = [&](int64_t r, int j) {
                const size_t q = size_t(std::upper_bound(r0.begin(), r0.end(), r) - r0.begin()) - 1;
                const int32_t c = sup[q];
                return zval(c, r - r0[q], j) / double(owners[c].size());
            };
            int kept = 0;
            vblocks[t] = orthonormalise(m, value, kept);
            vrank[t] = kept;
            vrow0[t] = std::move(r0);
        }
        std::vector<int32_t> vcol0(nv + 1, 0), vidx(nc, -1);
        for (int32_t t = 0; t < nv; ++t) {
            vcol0[t + 1] = vcol0[t] + vrank[t];
            vidx[coarse_nodes[t]] = t;
            for (int j = 0; j < vrank[t]; ++j) s.col_comp.push_back(coarse_nodes[t]);
        }
        // per component: the columns of its owners (ascending) and their
        // values on its rows
        for (int32_t c = 0; c < nc; ++c) {
            const int64_t m = (s.comp_ptr[c + 1] - s.comp_ptr[c]) * dpn;
            for (int32_t v : owners[c]) {
                const int32_t t = vidx[v];
                const auto &sup = support[v];
                const size_t q = size_t(std::lower_bound(sup.begin(), sup.end(), c) - sup.begin());
                const int64_t off = vrow0[t][q], mv = vrow0[t].back();
                for (int j = 0; j < vrank[t]; ++j) {
                    s.ccol.push_back(vcol0[t] + j);
                    const double *src = vblocks[t].data() + int64_t(j) * mv + off;
                    blocks[c].insert(blocks[c].end(), src, src + m);
                }
                s.comp_rank[c] += vrank[t];
            }
            s.ccol_ptr[c + 1] = int64_t(s.ccol.size());
        }
    }
    for (int32_t c = 0; c < nc; ++c) s.phig_off[c + 1] = s.phig_off[c] + int64_t(blocks[c].size());
    s.n0 = (s.opt.coarse != GDSW_COARSE_NONE) ? int32_t(s.col_comp.size()) : 0;
    s.phig.resize(s.phig_off[nc]);
    for (int32_t c = 0; c < nc; ++c) std::copy(blocks[c].begin(), blocks[c].end(), s.phig.begin() + s.phig_off[c]);
}

// ---------------------------------------------------------------------------
// Level-of-fill pattern of ILU(p) of one local matrix (Sec. V-B, level-based
// incomplete LU): entries of A_i have level 0; eliminating pivot row k < l
// from row l reaches (l, j), j > k in row k, at level lev(l,k) + lev(k,j) + 1;
// the smallest such level counts and entries above p are dropped.  Row l is
// assembled with a min-heap of the pivots still to eliminate (ascending), so
// fill entries that become pivots themselves are eliminated in turn.
// On entry C/G/RL hold A_i's pattern row by row (columns ascending, G the
// position in A); on return the ILU(p) pattern, G = -1 on fill entries.
static void iluk_fill(int64_t ni, std::vector<int32_t> &C, std::vector<int64_t> &G, std::vector<int64_t> &RL,
                      int p) {
    std::vector<int32_t> nc, nlev;
    std::vector<int64_t> ng, nrl(ni, 0), start(ni + 1, 0);
    nc.reserve(C.size() * 2);
    nlev.reserve(C.size() * 2);
    ng.reserve(C.size() * 2);
    std::vector<int32_t> lev(ni, -1);      // -1: not in the current row
    std::vector<int64_t> gp(ni, -1);
    std::vector<int32_t> cols;
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> pivots;
    int64_t pos = 0;
    for (int64_t l = 0; l < ni; ++l) {
        cols.clear();
        for (int64_t q = 0; q < RL[l]; ++q, ++pos) {
            const int32_t c = C[pos];
            lev[c] = 0;
            gp[c] = G[pos];
            cols.push_back(c);
            if (c < l) pivots.push(c);
        }
        while (!pivots.empty()) {
            const int32_t k = pivots.top();
            pivots.pop();
            const int32_t lk = lev[k];
            for (int64_t e = start[k]; e < start[k + 1]; ++e) {
                const int32_t j = nc[e];
                if (j <= k) continue;
                const int32_t nl = lk + nlev[e] + 1;
                if (nl > p) continue;
                if (lev[j] < 0) {
                    lev[j] = nl;
                    gp[j] = -1;
                    cols.push_back(j);
                    if (j < l) pivots.push(j);
                } else if (nl < lev[j]) {
                    lev[j] = nl;
                }
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t c : cols) {
            nc.push_back(c);
            nlev.push_back(lev[c]);
            ng.push_back(gp[c]);
            lev[c] = -1;
        }
        nrl[l] = int64_t(cols.size());
        start[l + 1] = start[l] + nrl[l];
    }
    C.swap(nc);
    G.swap(ng);
    RL.swap(nrl);
}

// ---------------------------------------------------------------------------
// FastILU product lists (Sec. V-B, iterative variant of the incomplete
// factorisation): for every entry (l, j) of a local pattern, the pairs of
// positions (l, m), (m, j) with m < min(l, j) in ascending m, and for l > j
// the position of the pivot u_jj.  Positions index the concatenated local
// CSR values of all subdomains.
static void build_fastilu(Symbolic &s) {
    const int np = s.np;
    const int64_t ne = int64_t(s.lcol.size());
    if (ne >= (int64_t(1) << 31)) fail(GDSW_ERR_INVALID_ARG, "too many local entries for FastILU");
    s.fi_ptr.assign(ne + 1, 0);
    s.fi_dpos.assign(ne, -1);
    // position of (m, j) in local row m of subdomain i, or -1
    auto find = [&](int64_t o, int32_t m, int32_t j) -> int64_t {
        const int32_t *b = s.lcol.data() + s.lrowptr[o + m], *e = s.lcol.data() + s.lrowptr[o + m + 1];
        const int32_t *it = std::lower_bound(b, e, j);
        return (it != e && *it == j) ? int64_t(it - s.lcol.data()) : -1;
    };
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic)
        for (int i = 0; i < np; ++i) {
            const int64_t o = s.ov_ptr[i], ni = s.ov_ptr[i + 1] - o;
            for (int64_t l = 0; l < ni; ++l) {
                const int64_t rs = s.lrowptr[o + l], re = s.lrowptr[o + l + 1];
                for (int64_t e = rs; e < re; ++e) {
                    const int32_t j = s.lcol[e];
                    const int32_t lim = std::min<int32_t>(int32_t(l), j);
                    int64_t cnt = 0;
                    for (int64_t f = rs; f < re && s.lcol[f] < lim; ++f) {
                        const int64_t g = find(o, s.lcol[f], j);
                        if (g < 0) continue;
                        if (pass == 1) {
                            const int64_t q = s.fi_ptr[e] + cnt;
                            s.fi_pairs[2 * q] = int32_t(f);
                            s.fi_pairs[2 * q + 1] = int32_t(g);
                        }
                        ++cnt;
                    }
                    if (pass == 0) {
                        s.fi_ptr[e + 1] = cnt;
                        if (j < l) s.fi_dpos[e] = int32_t(s.lrowptr[o + j] + s.ldiag[o + j]);
                    }
                }
            }
        }
        if (pass == 0) {
            for (int64_t e = 0; e < ne; ++e) s.fi_ptr[e + 1] += s.fi_ptr[e];
            s.fi_pairs.resize(2 * s.fi_ptr[ne]);
        }
    }
}

// ---------------------------------------------------------------------------
// local matrices of the overlapping subdomains (CSR + band profile + ILU(k)
// level schedule) and of the interior blocks (band profile)
void build_local(Symbolic &s) {
    const int np = s.np;
    const int64_t nloc = s.ov_ptr[np];
    s.lrowptr.assign(nloc + 1, 0);
    s.ldiag.assign(nloc, 0);
    std::vector<std::vector<int32_t>> lc(np);
    std::vector<std::vector<int64_t>> lg(np);
    std::vector<std::vector<int64_t>> rowlen(np);
    s.bw.assign(np, 0);
    s.KL = 0;
    s.KU = 0;
    int32_t KL = 0, KU = 0;
#pragma omp parallel
    {
        std::vector<int32_t> g2l(s.n, -1);
        int32_t kl = 0, ku = 0;
#pragma omp for schedule(dynamic)
        for (int i = 0; i < np; ++i) {
            const int64_t o = s.ov_ptr[i], ni = s.ov_ptr[i + 1] - o;
            for (int64_t l = 0; l < ni; ++l) g2l[s.ov_idx[o + l]] = int32_t(l);
            auto &C = lc[i];
            auto &G = lg[i];
            auto &RL = rowlen[i];
            RL.assign(ni, 0);
            int32_t b = 0;
            for (int64_t l = 0; l < ni; ++l) {
                int32_t d = s.ov_idx[o + l];
                for (int64_t p = s.rowptr[d]; p < s.rowptr[d + 1]; ++p) {
                    int32_t q = g2l[s.col[p]];
                    if (q < 0) continue;
                    C.push_back(q);
                    G.push_back(p);
                    RL[l]++;
                    if (q < l) b = std::max<int32_t>(b, int32_t(l - q));
                }
            }
            if (s.opt.local == GDSW_LOCAL_ILU0 && s.opt.ilu_level > 0) iluk_fill(ni, C, G, RL, s.opt.ilu_level);
            for (int64_t l = 0, pos = 0; l < ni; ++l) {
                int32_t nl = 0, nu = 0;
                for (int64_t q = 0; q < RL[l]; ++q, ++pos) {
                    if (C[pos] < l) ++nl;
                    if (C[pos] > l) ++nu;
                }
                kl = std::max(kl, nl);
                ku = std::max(ku, nu);
            }
            s.bw[i] = b;
            for (int64_t l = 0; l < ni; ++l) g2l[s.ov_idx[o + l]] = -1;
        }
#pragma omp critical
        {
            KL = std::max(KL, kl);
            KU = std::max(KU, ku);
        }
    }
    s.KL = KL;
    s.KU = KU;
    for (int i = 0; i < np; ++i) {
        const int64_t o = s.ov_ptr[i];
        for (size_t l = 0; l < rowlen[i].size(); ++l) s.lrowptr[o + l + 1] = rowlen[i][l];
    }
    for (int64_t p = 0; p < nloc; ++p) s.lrowptr[p + 1] += s.lrowptr[p];
    s.lcol.resize(s.lrowptr[nloc]);
    s.lgpos.resize(s.lrowptr[nloc]);
    for (int i = 0; i < np; ++i) {
        int64_t base = s.lrowptr[s.ov_ptr[i]];
        std::copy(lc[i].begin(), lc[i].end(), s.lcol.begin() + base);
        std::copy(lg[i].begin(), lg[i].end(), s.lgpos.begin() + base);
        std::vector<int32_t>().swap(lc[i]);
        std::vector<int64_t>().swap(lg[i]);
    }
    // diagonal positions, level schedule of the ILU(0) rows, band scatter
    s.max_bw = 0;
    for (int i = 0; i < np; ++i) s.max_bw = std::max(s.max_bw, s.bw[i]);
    // (band profiles for the exact factor; the nested-dissection analysis
    // drops those of the subdomains that take the supernodal factor)
    const bool exact = s.opt.local == GDSW_LOCAL_EXACT;
    s.band_off.assign(np + 1, 0);
    for (int i = 0; i < np; ++i)
        s.band_off[i + 1] = s.band_off[i] + (exact ? (s.ov_ptr[i + 1] - s.ov_ptr[i]) * int64_t(s.bw[i] + 1) : 0);
    s.lvl_rows.assign(nloc, 0);
    std::vector<std::vector<int32_t>> lvptr(np);
    if (exact) {
        int64_t cnt = 0;
        for (int i = 0; i < np; ++i)
            for (int64_t p = s.ov_ptr[i]; p < s.ov_ptr[i + 1]; ++p)
                for (int64_t e = s.lrowptr[p]; e < s.lrowptr[p + 1]; ++e)
                    if (s.lcol[e] <= p - s.ov_ptr[i]) ++cnt;
        s.bscat_dst.resize(cnt);
        s.bscat_src.resize(cnt);
    }
    int64_t bpos = 0;
    for (int i = 0; i < np; ++i) {
        const int64_t o = s.ov_ptr[i], ni = s.ov_ptr[i + 1] - o;
        const int32_t b = s.bw[i];
        std::vector<int32_t> level(ni, 0);
        int32_t nlev = 0;
        for (int64_t l = 0; l < ni; ++l) {
            int32_t lv = 0;
            for (int64_t e = s.lrowptr[o + l]; e < s.lrowptr[o + l + 1]; ++e) {
                int32_t q = s.lcol[e];
                if (q < l) lv = std::max(lv, level[q] + 1);
                if (q == l) s.ldiag[o + l] = int32_t(e - s.lrowptr[o + l]);
                if (exact && q <= l) {
                    s.bscat_dst[bpos] = s.band_off[i] + l * int64_t(b + 1) + (q - l + b);
                    s.bscat_src[bpos] = s.lgpos[e];
                    ++bpos;
                }
            }
            level[l] = lv;
            nlev = std::max(nlev, lv + 1);
        }
        std::vector<int32_t> ptr(nlev + 1, 0);
        for (int64_t l = 0; l < ni; ++l) ptr[level[l] + 1]++;
        for (int32_t k = 0; k < nlev; ++k) ptr[k + 1] += ptr[k];
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t l = 0; l < ni; ++l) s.lvl_rows[o + fill[level[l]]++] = int32_t(l);
        lvptr[i] = std::move(ptr);
    }
    s.lvl_base.assign(np + 1, 0);
    for (int i = 0; i < np; ++i) s.lvl_base[i + 1] = s.lvl_base[i] + int64_t(lvptr[i].size());
    s.lvl_ptr.resize(s.lvl_base[np]);
    for (int i = 0; i < np; ++i) std::copy(lvptr[i].begin(), lvptr[i].end(), s.lvl_ptr.begin() + s.lvl_base[i]);
    // padded sweep layout: rows of subdomain i at ell_off[i] .. + roundup(n_i, 64)
    s.ell_off.assign(np + 1, 0);
    for (int i = 0; i < np; ++i) {
        int64_t ni = s.ov_ptr[i + 1] - s.ov_ptr[i];
        s.ell_off[i + 1] = s.ell_off[i] + ((ni + 63) / 64) * 64;
    }
    s.ell_rows = s.ell_off[np];
    if (s.opt.local == GDSW_LOCAL_ILU0 && s.opt.ilu_factor_sweeps > 0) build_fastilu(s);
}

// ---------------------------------------------------------------------------
// interior sets, the couplings A_{I_i, Gamma}, band profiles of A_{I_i I_i},
// coarse blocks of Phi, the coarse reduction and prolongation maps and the
// assembly lists of A_0
void build_coarse(Symbolic &s) {
    const int np = s.np, dpn = s.dpn;
    const int64_t n = s.n;
    // interior dofs per subdomain
    s.int_ptr.assign(np + 1, 0);
    for (int64_t v = 0; v < s.nn; ++v)
        if (!s.is_gamma[v]) s.int_ptr[s.part[v] + 1] += dpn;
    for (int i = 0; i < np; ++i) s.int_ptr[i + 1] += s.int_ptr[i];
    s.int_idx.resize(s.int_ptr[np]);
    {
        std::vector<int64_t> fill(s.int_ptr.begin(), s.int_ptr.end() - 1);
        for (int64_t v = 0; v < s.nn; ++v)
            if (!s.is_gamma[v])
                for (int k = 0; k < dpn; ++k) s.int_idx[fill[s.part[v]]++] = int32_t(v * dpn + k);
    }
    const int64_t nint = s.int_ptr[np];
    s.max_nii = 0;
    for (int i = 0; i < np; ++i) s.max_nii = std::max<int32_t>(s.max_nii, int32_t(s.int_ptr[i + 1] - s.int_ptr[i]));
    // dof -> position in its component block
    std::vector<int32_t> comp_lr(n, -1);
    for (int32_t c = 0; c < s.nc; ++c)
        for (int64_t q = s.comp_ptr[c]; q < s.comp_ptr[c + 1]; ++q)
            for (int k = 0; k < dpn; ++k)
                comp_lr[int64_t(s.comp_nodes[q]) * dpn + k] = int32_t((q - s.comp_ptr[c]) * dpn + k);
    const bool coarse = s.opt.coarse != GDSW_COARSE_NONE && s.n0 > 0;
    // adjacent coarse columns of each interior block and the couplings
    s.scol_ptr.assign(np + 1, 0);
    s.scol.clear();
    s.cpl_ptr.assign(nint + 1, 0);
    s.cpl_apos.clear(); s.cpl_phi.clear(); s.cpl_stride.clear(); s.cpl_rank.clear(); s.cpl_slot.clear();
    s.cpl_slotmap.clear();
    std::vector<int32_t> slot_of_comp(s.nc, -1);   // start of the component's slots in cpl_slotmap
    std::vector<int32_t> slot_of_col(coarse ? s.n0 : 0, -1);
    for (int i = 0; i < np; ++i) {
        std::vector<int32_t> comps;
        for (int64_t q = s.int_ptr[i]; q < s.int_ptr[i + 1]; ++q) {
            int32_t d = s.int_idx[q];
            for (int64_t p = s.rowptr[d]; p < s.rowptr[d + 1]; ++p) {
                int32_t node = s.col[p] / dpn;
                if (s.is_gamma[node] && coarse && s.comp_rank[s.comp_of_node[node]] > 0)
                    comps.push_back(s.comp_of_node[node]);
            }
        }
        std::sort(comps.begin(), comps.end());
        comps.erase(std::unique(comps.begin(), comps.end()), comps.end());
        // the coarse columns of the adjacent components, ascending, each once
        const size_t sc0 = s.scol.size();
        for (int32_t c : comps)
            for (int64_t q = s.ccol_ptr[c]; q < s.ccol_ptr[c + 1]; ++q) s.scol.push_back(s.ccol[q]);
        std::sort(s.scol.begin() + sc0, s.scol.end());
        s.scol.erase(std::unique(s.scol.begin() + sc0, s.scol.end()), s.scol.end());
        for (size_t q = sc0; q < s.scol.size(); ++q) slot_of_col[s.scol[q]] = int32_t(q - sc0);
        for (int32_t c : comps) {
            slot_of_comp[c] = int32_t(s.cpl_slotmap.size());
            for (int64_t q = s.ccol_ptr[c]; q < s.ccol_ptr[c + 1]; ++q) s.cpl_slotmap.push_back(slot_of_col[s.ccol[q]]);
        }
        for (size_t q = sc0; q < s.scol.size(); ++q) slot_of_col[s.scol[q]] = -1;
        s.scol_ptr[i + 1] = int64_t(s.scol.size());
        for (int64_t q = s.int_ptr[i]; q < s.int_ptr[i + 1]; ++q) {
            int32_t d = s.int_idx[q];
            for (int64_t p = s.rowptr[d]; p < s.rowptr[d + 1]; ++p) {
                int32_t g = s.col[p];
                int32_t node = g / dpn;
                if (!s.is_gamma[node] || !coarse) continue;
                int32_t c = s.comp_of_node[node];
                if (s.comp_rank[c] == 0) continue;
                s.cpl_apos.push_back(p);
                s.cpl_phi.push_back(s.phig_off[c] + comp_lr[g]);
                s.cpl_stride.push_back(int32_t((s.comp_ptr[c + 1] - s.comp_ptr[c]) * dpn));
                s.cpl_rank.push_back(s.comp_rank[c]);
                s.cpl_slot.push_back(slot_of_comp[c]);
            }
            s.cpl_ptr[q + 1] = int64_t(s.cpl_apos.size());
        }
        for (int32_t c : comps) slot_of_comp[c] = -1;
    }
    s.ext_off.assign(np + 1, 0);
    for (int i = 0; i < np; ++i)
        s.ext_off[i + 1] = s.ext_off[i] + (s.int_ptr[i + 1] - s.int_ptr[i]) * (s.scol_ptr[i + 1] - s.scol_ptr[i]);
    // band profiles of the interior blocks (needed only with a coarse space)
    s.ibw.assign(np, 0);
    s.iband_off.assign(np + 1, 0);
    s.ibscat_dst.clear();
    s.ibscat_src.clear();
    if (coarse) {
        std::vector<int32_t> g2l(n, -1);
        for (int i = 0; i < np; ++i) {
            const int64_t o = s.int_ptr[i], ni = s.int_ptr[i + 1] - o;
            for (int64_t l = 0; l < ni; ++l) g2l[s.int_idx[o + l]] = int32_t(l);
            int32_t b = 0;
            for (int64_t l = 0; l < ni; ++l) {
                int32_t d = s.int_idx[o + l];
                for (int64_t p = s.rowptr[d]; p < s.rowptr[d + 1]; ++p) {
                    int32_t q = g2l[s.col[p]];
                    if (q >= 0 && q < l) b = std::max<int32_t>(b, int32_t(l - q));
                }
            }
            s.ibw[i] = b;
            s.iband_off[i + 1] = s.iband_off[i] + ni * int64_t(b + 1);
            for (int64_t l = 0; l < ni; ++l) {
                int32_t d = s.int_idx[o + l];
                for (int64_t p = s.rowptr[d]; p < s.rowptr[d + 1]; ++p) {
                    int32_t q = g2l[s.col[p]];
                    if (q >= 0 && q <= l) {
                        s.ibscat_dst.push_back(s.iband_off[i] + l * int64_t(b + 1) + (q - l + b));
                        s.ibscat_src.push_back(p);
                    }
                }
            }
            for (int64_t l = 0; l < ni; ++l) g2l[s.int_idx[o + l]] = -1;
        }
    }
    s.max_ibw = 0;
    for (int i = 0; i < np; ++i) s.max_ibw = std::max(s.max_ibw, s.ibw[i]);

    // coarse blocks: interior blocks (subdomains with k_i > 0), then interface
    // component blocks
    PhiBlocks &B = s.blk;
    B = PhiBlocks();
    B.row_ptr.assign(1, 0);
    B.col_ptr.assign(1, 0);
    B.val_off.assign(1, 0);
    if (coarse) {
        for (int i = 0; i < np; ++i) {
            int64_t nr = s.int_ptr[i + 1] - s.int_ptr[i];
            int64_t k = s.scol_ptr[i + 1] - s.scol_ptr[i];
            if (nr == 0 || k == 0) continue;
            B.rows.insert(B.rows.end(), s.int_idx.begin() + s.int_ptr[i], s.int_idx.begin() + s.int_ptr[i + 1]);
            B.cols.insert(B.cols.end(), s.scol.begin() + s.scol_ptr[i], s.scol.begin() + s.scol_ptr[i + 1]);
            B.row_ptr.push_back(int64_t(B.rows.size()));
            B.col_ptr.push_back(int64_t(B.cols.size()));
            B.val_off.push_back(B.val_off.back() + nr * k);
            B.kind.push_back(0);
            B.owner.push_back(i);
        }
        for (int32_t c = 0; c < s.nc; ++c) {
            int64_t k = s.comp_rank[c];
            if (k == 0) continue;
            for (int64_t q = s.comp_ptr[c]; q < s.comp_ptr[c + 1]; ++q)
                for (int kk = 0; kk < dpn; ++kk) B.rows.push_back(int32_t(int64_t(s.comp_nodes[q]) * dpn + kk));
            for (int64_t q = s.ccol_ptr[c]; q < s.ccol_ptr[c + 1]; ++q) B.cols.push_back(s.ccol[q]);
            int64_t nr = (s.comp_ptr[c + 1] - s.comp_ptr[c]) * dpn;
            B.row_ptr.push_back(int64_t(B.rows.size()));
            B.col_ptr.push_back(int64_t(B.cols.size()));
            B.val_off.push_back(B.val_off.back() + nr * k);
            B.kind.push_back(1);
            B.owner.push_back(c);
        }
    }
    B.nb = int32_t(B.kind.size());
    // reduction lists (partials of each coarse column, ascending block order)
    const int32_t n0 = coarse ? s.n0 : 0;
    // coarse columns and A_0 blocks of every problem (problems never couple,
    // and components are ordered by their smallest node, so the columns of a
    // problem are contiguous)
    s.prob_c0.assign(s.nprob + 1, 0);
    s.cprob.assign(n0, 0);
    {
        auto prob_of_dof = [&](int64_t d) {
            return int32_t(std::upper_bound(s.prob_ptr.begin(), s.prob_ptr.end(), d) - s.prob_ptr.begin() - 1);
        };
        std::vector<int32_t> cnt(s.nprob, 0);
        for (int32_t col = 0; col < n0; ++col) {
            const int32_t c = s.col_comp[col];
            const int32_t k = prob_of_dof(int64_t(s.comp_nodes[s.comp_ptr[c]]) * dpn);
            s.cprob[col] = k;
            cnt[k] += 1;
        }
        for (int32_t c = 1; c < n0; ++c)
            if (s.cprob[c] < s.cprob[c - 1]) fail(GDSW_ERR_INTERNAL, "coarse columns of a problem not contiguous");
        for (int k = 0; k < s.nprob; ++k) s.prob_c0[k + 1] = s.prob_c0[k] + cnt[k];
        s.a0_off.assign(s.nprob + 1, 0);
        for (int k = 0; k < s.nprob; ++k) {
            const int64_t nk = s.prob_c0[k + 1] - s.prob_c0[k];
            s.a0_off[k + 1] = s.a0_off[k] + nk * nk;
        }
    }
    auto a0_index = [&](int32_t a, int32_t b) {
        const int32_t k = s.cprob[a];
        const int64_t c0 = s.prob_c0[k], nk = s.prob_c0[k + 1] - c0;
        return s.a0_off[k] + (a - c0) * nk + (b - c0);
    };
    s.red_ptr.assign(n0 + 1, 0);
    for (int64_t q = 0; q < int64_t(B.cols.size()); ++q) s.red_ptr[B.cols[q] + 1]++;
    for (int32_t c = 0; c < n0; ++c) s.red_ptr[c + 1] += s.red_ptr[c];
    s.red_idx.resize(B.cols.size());
    {
        std::vector<int64_t> fill(s.red_ptr.begin(), s.red_ptr.end() - 1);
        for (int64_t q = 0; q < int64_t(B.cols.size()); ++q) s.red_idx[fill[B.cols[q]]++] = int32_t(q);
    }
    s.dof_blk.assign(n, -1);
    s.dof_lr.assign(n, 0);
    for (int32_t g = 0; g < B.nb; ++g)
        for (int64_t q = B.row_ptr[g]; q < B.row_ptr[g + 1]; ++q) {
            s.dof_blk[B.rows[q]] = g;
            s.dof_lr[B.rows[q]] = int32_t(q - B.row_ptr[g]);
        }
    // ---- A_0 assembly lists -------------------------------------------------
    s.pair_c.clear(); s.pair_d.clear(); s.pair_off.assign(1, 0); s.pair_eptr.assign(1, 0);
    s.pair_apos.clear(); s.pair_lr_c.clear(); s.pair_lr_d.clear(); s.a0pair_tgt.clear();
    s.t1_off.assign(np + 1, 0);
    s.a0seg_tgt.clear(); s.a0seg_ptr.assign(1, 0); s.a0seg_src.clear();
    if (!coarse) return;
    // interface-interface: Phi_G^T A_GG Phi_G by component pairs
    for (int32_t c = 0; c < s.nc; ++c) {
        if (s.comp_rank[c] == 0) continue;
        std::map<int32_t, std::vector<std::array<int64_t, 3>>> by;
        for (int64_t q = s.comp_ptr[c]; q < s.comp_ptr[c + 1]; ++q)
            for (int kk = 0; kk < dpn; ++kk) {
                int64_t g = int64_t(s.comp_nodes[q]) * dpn + kk;
                for (int64_t p = s.rowptr[g]; p < s.rowptr[g + 1]; ++p) {
                    int32_t u = s.col[p];
                    int32_t node = u / dpn;
                    if (!s.is_gamma[node]) continue;
                    int32_t d = s.comp_of_node[node];
                    if (s.comp_rank[d] == 0) continue;
                    by[d].push_back({p, comp_lr[g], comp_lr[u]});
                }
            }
        for (auto &kv : by) {
            int32_t d = kv.first;
            s.pair_c.push_back(c);
            s.pair_d.push_back(d);
            for (auto &e : kv.second) {
                s.pair_apos.push_back(e[0]);
                s.pair_lr_c.push_back(int32_t(e[1]));
                s.pair_lr_d.push_back(int32_t(e[2]));
            }
            s.pair_eptr.push_back(int64_t(s.pair_apos.size()));
            int64_t rc = s.comp_rank[c], rd = s.comp_rank[d];
            s.pair_off.push_back(s.pair_off.back() + rc * rd);
            for (int64_t a = 0; a < rc; ++a)
                for (int64_t b = 0; b < rd; ++b)
                    s.a0pair_tgt.push_back(a0_index(s.ccol[s.ccol_ptr[c] + a], s.ccol[s.ccol_ptr[d] + b]));
        }
    }
    // T2 values by target, ascending pair order (one value per target unless
    // components share coarse columns)
    s.a0seg2_tgt.clear(); s.a0seg2_ptr.assign(1, 0); s.a0seg2_src.clear();
    {
        std::vector<int64_t> order(s.a0pair_tgt.size());
        std::iota(order.begin(), order.end(), int64_t(0));
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t x, int64_t y) { return s.a0pair_tgt[x] < s.a0pair_tgt[y]; });
        for (size_t q = 0; q < order.size(); ++q) {
            if (q == 0 || s.a0pair_tgt[order[q]] != s.a0pair_tgt[order[q - 1]]) {
                if (q) s.a0seg2_ptr.push_back(int64_t(q));
                s.a0seg2_tgt.push_back(s.a0pair_tgt[order[q]]);
            }
            s.a0seg2_src.push_back(order[q]);
        }
        if (!order.empty()) s.a0seg2_ptr.push_back(int64_t(order.size()));
    }
    // subdomain terms E_i^T X_i: segments by target, ascending subdomain
    for (int i = 0; i < np; ++i) {
        int64_t k = s.scol_ptr[i + 1] - s.scol_ptr[i];
        if (s.int_ptr[i + 1] == s.int_ptr[i]) k = 0;
        s.t1_off[i + 1] = s.t1_off[i] + k * k;
    }
    std::vector<std::pair<int64_t, int64_t>> contrib;   // (target, source)
    contrib.reserve(s.t1_off[np]);
    for (int i = 0; i < np; ++i) {
        int64_t k = (s.t1_off[i + 1] - s.t1_off[i]);
        if (!k) continue;
        int64_t kk = int64_t(std::llround(std::sqrt(double(k))));
        const int32_t *cols = s.scol.data() + s.scol_ptr[i];
        for (int64_t a = 0; a < kk; ++a)
            for (int64_t b = 0; b < kk; ++b)
                contrib.push_back({a0_index(cols[a], cols[b]), s.t1_off[i] + a * kk + b});
    }
    std::stable_sort(contrib.begin(), contrib.end(),
                     [](const auto &x, const auto &y) { return x.first < y.first; });
    for (size_t q = 0; q < contrib.size(); ++q) {
        if (q == 0 || contrib[q].first != contrib[q - 1].first) {
            if (q) s.a0seg_ptr.push_back(int64_t(q));
            s.a0seg_tgt.push_back(contrib[q].first);
        }
        s.a0seg_src.push_back(contrib[q].second);
    }
    if (!contrib.empty()) s.a0seg_ptr.push_back(int64_t(contrib.size()));
}

}  // namespace

gdsw_status analyze(gdsw_handle_s *h, const gdsw_csr *A, const int32_t *part, int32_t n_parts,
                    int32_t dpn, const double *Z, int32_t n_null, const gdsw_options *opt,
                    const int64_t *share_ptr, const int32_t *share_sub) {
    auto t0 = std::chrono::steady_clock::now();
    try {
        Symbolic &s = h->sym;
        validate_and_copy(s, A, part, n_parts, dpn, Z, n_null, opt);
        if (share_ptr || share_sub) {
            if (!share_ptr || !share_sub) fail(GDSW_ERR_INVALID_ARG, "sharing sets: both arrays are needed");
            if (share_ptr[0] != 0) fail(GDSW_ERR_INVALID_ARG, "sharing sets: share_ptr[0] must be 0");
            for (int64_t v = 0; v < s.nn; ++v)
                if (share_ptr[v + 1] < share_ptr[v]) fail(GDSW_ERR_INVALID_ARG, "sharing sets: share_ptr not ascending");
            s.share_ptr.assign(share_ptr, share_ptr + s.nn + 1);
            s.share_sub.assign(share_sub, share_sub + share_ptr[s.nn]);
            for (int32_t q : s.share_sub)
                if (q < 0 || q >= s.np) fail(GDSW_ERR_INVALID_ARG, "sharing sets: subdomain id out of range");
        }
        if (s.prob_ptr.empty()) {
            s.nprob = 1;
            s.prob_ptr = {0, s.n};
            s.prob_sub = {0, s.np};
        }
        s.sub_prob.assign(s.np, 0);
        for (int k = 0; k < s.nprob; ++k)
            for (int32_t i = s.prob_sub[k]; i < s.prob_sub[k + 1]; ++i) s.sub_prob[i] = k;
        build_graph(s);
        build_overlap(s);
        build_interface(s);
        build_local(s);
        s.nd_mask.assign(s.np, 0);
        if (s.opt.local == GDSW_LOCAL_EXACT && s.opt.exact_order != GDSW_ORDER_NATURAL) build_nd(s);
        build_coarse(s);
        if (s.opt.local == GDSW_LOCAL_ILU0 && s.max_ni > 65535)
            fail(GDSW_ERR_INVALID_ARG, "ILU(0) local solver supports subdomains of at most 65535 dofs");
    } catch (const Fail &f) {
        h->err = f.msg;
        return f.st;
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed in analysis";
        return GDSW_ERR_BUDGET;
    } catch (const std::runtime_error &e) {
        h->err = e.what();
        return GDSW_ERR_INTERNAL;
    }
    h->sym.t_analyze = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    h->analyzed = true;
    return GDSW_OK;
}

gdsw_status analyze_batch(gdsw_handle_s *h, int32_t count, const gdsw_csr *A, const int32_t *const *part,
                          const int32_t *n_parts, int32_t dpn, const double *const *Z, int32_t n_null,
                          const gdsw_options *opt) {
    try {
        if (count <= 0 || !A || !part || !n_parts) fail(GDSW_ERR_INVALID_ARG, "batch: bad arguments");
        if (dpn <= 0) fail(GDSW_ERR_INVALID_ARG, "batch: dpn");
        if ((Z == nullptr) != (n_null <= 0) && !(Z == nullptr && n_null <= 1))
            fail(GDSW_ERR_INVALID_ARG, "batch: null space arguments");
        // block-diagonal concatenation; subdomain ids and dofs offset per problem
        int64_t n = 0, nnz = 0, np = 0;
        for (int k = 0; k < count; ++k) {
            if (!A[k].rowptr || !A[k].col || !A[k].val || !part[k] || A[k].n <= 0 || A[k].n % dpn || n_parts[k] <= 0)
                fail(GDSW_ERR_INVALID_ARG, "batch: problem " + std::to_string(k) + " malformed");
            n += A[k].n;
            nnz += A[k].rowptr[A[k].n];
            np += n_parts[k];
        }
        if (n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 31) || np >= (int64_t(1) << 31))
            fail(GDSW_ERR_INVALID_ARG, "batch too large");
        std::vector<int64_t> rowptr(n + 1, 0);
        std::vector<int32_t> col(nnz);
        std::vector<double> val(nnz);
        std::vector<int32_t> prt(n / dpn);
        std::vector<double> Zc;
        const int nz = Z ? n_null : 1;
        if (Z) Zc.assign(size_t(n) * nz, 0.0);
        Symbolic &s = h->sym;
        s.nprob = count;
        s.prob_ptr.assign(count + 1, 0);
        s.prob_sub.assign(count + 1, 0);
        int64_t ro = 0, eo = 0;
        int32_t so = 0;
        for (int k = 0; k < count; ++k) {
            const int64_t nk = A[k].n;
            for (int64_t i = 0; i < nk; ++i) {
                for (int64_t p = A[k].rowptr[i]; p < A[k].rowptr[i + 1]; ++p) {
                    const int32_t c = A[k].col[p];
                    if (c < 0 || c >= nk) fail(GDSW_ERR_INVALID_ARG, "batch: column out of range");
                    col[eo] = int32_t(c + ro);
                    val[eo] = A[k].val[p];
                    ++eo;
                }
                rowptr[ro + i + 1] = eo;
            }
            for (int64_t v = 0; v < nk / dpn; ++v) {
                const int32_t pv = part[k][v];
                if (pv < 0 || pv >= n_parts[k]) fail(GDSW_ERR_INVALID_ARG, "batch: part out of range");
                prt[ro / dpn + v] = so + pv;
            }
            if (Z) {
                if (!Z[k]) fail(GDSW_ERR_INVALID_ARG, "batch: missing null space");
                for (int j = 0; j < nz; ++j)
                    for (int64_t i = 0; i < nk; ++i) Zc[size_t(j) * n + ro + i] = Z[k][size_t(j) * nk + i];
            }
            ro += nk;
            so += n_parts[k];
            s.prob_ptr[k + 1] = ro;
            s.prob_sub[k + 1] = so;
        }
        gdsw_csr big{n, rowptr.data(), col.data(), val.data()};
        return analyze(h, &big, prt.data(), int32_t(np), dpn, Z ? Zc.data() : nullptr, Z ? nz : 0, opt);
    } catch (const Fail &f) {
        h->err = f.msg;
        return f.st;
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed in batch analysis";
        return GDSW_ERR_BUDGET;
    }
}

}  // namespace gdsw
