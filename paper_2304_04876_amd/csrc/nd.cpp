// Nested-dissection ordering and supernodal symbolic factorization of the
// local matrices A_i, for the exact local solver (Sec. V-B, sparse direct
// factorization after a fill-reducing ordering; Sec. VI on its cost).
//
// Ordering: recursive vertex-separator bisection of the graph of A_i.  A
// part is split at one level set of a breadth-first search from a
// pseudo-peripheral row (no edge joins the rows before that level to the
// rows after it): the level with the fewest rows among those that leave
// between 35 % and 75 % of the part before them.  Parts of at most ND_LEAF
// rows are not split.  Each leaf part and each separator is a supernode;
// the new numbering lists the supernodes children first, so a separator
// follows both halves it separates.
//
// Symbolic factorization: the struct of a supernode J (the rows of L below
// its diagonal block) is the set of later rows adjacent to J in A_i joined
// with the structs of its children, restricted to rows after J; with a
// separator tree every such row lies in J's ancestors.  From it follow the
// panel layout, the row gathers of the forward solve, the rows by height in
// the tree (independent supernodes of one height are solved together), the
// left-looking update lists of the numerical factorization and the map that
// scatters A_i's lower entries into the panels.
#include <algorithm>
#include <cstdint>
#include <stdexcept>
#include <vector>

#include "gdsw_impl.hpp"

namespace gdsw {
namespace {

struct LocalGraph {
    const int64_t *ptr;   // local CSR rows (diagonal included)
    const int32_t *col;
    int n;
};

// Per-subdomain result, merged into NDSym afterwards.
struct SubND {
    std::vector<int32_t> perm;            // new -> old
    std::vector<int32_t> first, ncol, height, parent;
    std::vector<std::vector<int32_t>> st;
};

class Dissector {
  public:
    explicit Dissector(const LocalGraph &g) : g_(g), mark_(g.n, 0), lev_(g.n, -1) {}

    // Splits `nodes` (one connected part or several), appending supernodes in
    // children-first order; returns the roots of the parts' trees.
    std::vector<int> run(std::vector<int> nodes) {
        std::vector<int> roots;
        while (!nodes.empty()) {
            const int tag = ++tag_;
            for (int v : nodes) mark_[v] = tag;
            // the connected piece of nodes[0]
            std::vector<int> order;
            bfs(tag, nodes[0], order);
            std::vector<int> rest;
            if (order.size() < nodes.size())
                for (int v : nodes)
                    if (lev_[v] < 0) rest.push_back(v);
            for (int v : order) lev_[v] = -1;
            std::vector<int> piece(order.begin(), order.end());
            roots.push_back(split_connected(std::move(piece)));
            nodes.swap(rest);
        }
        return roots;
    }

    std::vector<std::vector<int32_t>> rows;   // supernode rows (old local), children first
    std::vector<int32_t> parent;

  private:
    int add(std::vector<int> r, const std::vector<int> &kids) {
        std::sort(r.begin(), r.end());
        const int id = int(rows.size());
        rows.emplace_back(r.begin(), r.end());
        parent.push_back(-1);
        for (int k : kids) parent[k] = id;
        return id;
    }

    void bfs(int tag, int start, std::vector<int> &order) {
        order.clear();
        order.push_back(start);
        lev_[start] = 0;
        for (size_t h = 0; h < order.size(); ++h) {
            const int u = order[h];
            for (int64_t e = g_.ptr[u]; e < g_.ptr[u + 1]; ++e) {
                const int v = g_.col[e];
                if (v != u && mark_[v] == tag && lev_[v] < 0) {
                    lev_[v] = lev_[u] + 1;
                    order.push_back(v);
                }
            }
        }
    }

    int degree_in(int v, int tag) const {
        int d = 0;
        for (int64_t e = g_.ptr[v]; e < g_.ptr[v + 1]; ++e) d += (g_.col[e] != v && mark_[g_.col[e]] == tag);
        return d;
    }

    // `nodes` connected; returns the root supernode of its tree
    int split_connected(std::vector<int> nodes) {
        const int n = int(nodes.size());
        if (n <= ND_LEAF) return add(std::move(nodes), {});
        const int tag = ++tag_;
        for (int v : nodes) mark_[v] = tag;
        // pseudo-peripheral row: repeated searches from a row of the last
        // level with the fewest neighbours, while the depth grows
        int start = *std::min_element(nodes.begin(), nodes.end());
        std::vector<int> order;
        int depth = -1;
        for (int it = 0; it < 6; ++it) {
            bfs(tag, start, order);
            const int d = lev_[order.back()];
            int best = order.back(), bdeg = degree_in(best, tag);
            for (int k = int(order.size()) - 1; k >= 0 && lev_[order[k]] == d; --k) {
                const int dg = degree_in(order[k], tag);
                if (dg < bdeg || (dg == bdeg && order[k] < best)) {
                    best = order[k];
                    bdeg = dg;
                }
            }
            const bool grew = d > depth;
            depth = std::max(depth, d);
            for (int v : order) lev_[v] = -1;
            if (!grew) break;
            start = best;
        }
        bfs(tag, start, order);
        const int L = lev_[order.back()];
        if (L < 2) {   // no level separates two nonempty halves
            for (int v : order) lev_[v] = -1;
            return add(std::move(nodes), {});
        }
        std::vector<int> cnt(L + 1, 0);
        for (int v : order) ++cnt[lev_[v]];
        int m = -1;
        int before = cnt[0];
        for (int l = 1; l < L; ++l) {
            const int after = n - before - cnt[l];
            if (100 * int64_t(before) >= 35 * int64_t(n) && 100 * int64_t(before + cnt[l]) <= 75 * int64_t(n) &&
                after > 0 &&
                (m < 0 || cnt[l] < cnt[m]))
                m = l;
            before += cnt[l];
        }
        if (m < 0) {   // the level holding the median row
            int c = 0;
            for (m = 0; m < L && c + cnt[m] <= n / 2; ++m) c += cnt[m];
            m = std::min(std::max(m, 1), L - 1);
        }
        std::vector<int> a, b, sep;
        for (int v : order) (lev_[v] < m ? a : lev_[v] > m ? b : sep).push_back(v);
        for (int v : order) lev_[v] = -1;
        std::vector<int> kids = run(std::move(a));
        std::vector<int> kb = run(std::move(b));
        kids.insert(kids.end(), kb.begin(), kb.end());
        return add(std::move(sep), kids);
    }

    const LocalGraph &g_;
    std::vector<int> mark_, lev_;
    int tag_ = 0;
};

void subdomain_nd(const LocalGraph &g, SubND &out) {
    Dissector d(g);
    std::vector<int> all(g.n);
    for (int v = 0; v < g.n; ++v) all[v] = v;
    d.run(std::move(all));
    const int ns = int(d.rows.size());
    // heights in the tree (the dissector lists children first), then the
    // supernodes by height, so that those of one height (independent of
    // each other) hold consecutive columns; a child still precedes its
    // parent, and any such order of the tree gives the same fill
    std::vector<int32_t> h(ns, 0);
    for (int J = 0; J < ns; ++J)
        if (d.parent[J] >= 0) h[d.parent[J]] = std::max(h[d.parent[J]], h[J] + 1);
    std::vector<int> ord(ns), at(ns);
    for (int J = 0; J < ns; ++J) ord[J] = J;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return h[a] < h[b]; });
    for (int k = 0; k < ns; ++k) at[ord[k]] = k;
    out.perm.clear();
    out.first.assign(ns, 0);
    out.ncol.assign(ns, 0);
    out.height.assign(ns, 0);
    out.parent.assign(ns, -1);
    for (int k = 0; k < ns; ++k) {
        const int J = ord[k];
        out.first[k] = int32_t(out.perm.size());
        out.ncol[k] = int32_t(d.rows[J].size());
        out.height[k] = h[J];
        out.parent[k] = d.parent[J] >= 0 ? at[d.parent[J]] : -1;
        out.perm.insert(out.perm.end(), d.rows[J].begin(), d.rows[J].end());
    }
    std::vector<int32_t> iperm(g.n);
    for (int p = 0; p < g.n; ++p) iperm[out.perm[p]] = p;
    // structs, children first
    std::vector<std::vector<int>> kids(ns);
    for (int J = 0; J < ns; ++J)
        if (out.parent[J] >= 0) kids[out.parent[J]].push_back(J);
    out.st.assign(ns, {});
    std::vector<int> seen(g.n, -1);
    for (int J = 0; J < ns; ++J) {
        const int end = out.first[J] + out.ncol[J];
        std::vector<int32_t> &S = out.st[J];
        for (int p = out.first[J]; p < end; ++p) {
            const int v = out.perm[p];
            for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
                const int q = iperm[g.col[e]];
                if (q >= end && seen[q] != J) {
                    seen[q] = J;
                    S.push_back(q);
                }
            }
        }
        for (int C : kids[J])
            for (int32_t q : out.st[C])
                if (q >= end && seen[q] != J) {
                    seen[q] = J;
                    S.push_back(q);
                }
        std::sort(S.begin(), S.end());
    }
}

}  // namespace

void build_nd(Symbolic &s) {
    const int np = s.np;
    const int64_t nloc = s.ov_ptr[np];
    std::vector<SubND> sub(np);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < np; ++i) {
        const int64_t o = s.ov_ptr[i];
        const int ni = int(s.ov_ptr[i + 1] - o);
        // local CSR of subdomain i with row pointers relative to its first entry
        std::vector<int64_t> ptr(ni + 1);
        const int64_t base = s.lrowptr[o];
        for (int l = 0; l <= ni; ++l) ptr[l] = s.lrowptr[o + l] - base;
        LocalGraph g{ptr.data(), s.lcol.data() + base, ni};
        if (ni > 0) subdomain_nd(g, sub[i]);
    }
    // Which subdomains take the supernodal factor: those whose solve fits a
    // gfx950 compute unit's 160 KiB of LDS (nd_lds_bytes with 8-byte
    // accumulators for FP64 factors, 4 otherwise; at most
    // ND_MAX_SUPERNODES supernodes and ND_MAX_TROWS rows of one height above
    // the leaves; panel values of one subdomain below 2^31) and whose
    // leaves hold at most ND_LEAF rows (a part the level search cannot split
    // stays whole), all of them (GDSW_ORDER_ND) or (GDSW_ORDER_AUTO) those
    // whose panels hold fewer values than their band (both read twice per
    // apply); the others keep the band.  The choice depends on the
    // subdomain alone, so a problem's results do not depend on what it is
    // packed with.
    const bool all_nd = s.opt.exact_order == GDSW_ORDER_ND;
    const size_t acc = s.opt.local_prec == GDSW_FP64 ? 8 : 4;
    s.nd_mask.assign(np, 0);
    for (int i = 0; i < np; ++i) {
        const int64_t ni = s.ov_ptr[i + 1] - s.ov_ptr[i];
        const SubND &u = sub[i];
        if (ni == 0 || int(u.first.size()) > ND_MAX_SUPERNODES ||
            nd_lds_bytes(int(ni), ND_MAX_TROWS, ND_MAX_SUPERNODES, acc) > size_t(160) * 1024)
            continue;
        {   // rows of one height above the leaves
            std::vector<int64_t> rows_at;
            for (size_t J = 0; J < u.first.size(); ++J) {
                if (size_t(u.height[J]) >= rows_at.size()) rows_at.resize(u.height[J] + 1, 0);
                rows_at[u.height[J]] += u.ncol[J];
            }
            bool ok = true;
            for (size_t hh = 1; hh < rows_at.size(); ++hh) ok &= rows_at[hh] <= ND_MAX_TROWS;
            if (!ok) continue;
        }
        int64_t vals = 0;
        bool small_leaves = true;
        for (size_t J = 0; J < u.first.size(); ++J) {
            vals += int64_t(u.ncol[J]) * (u.ncol[J] + int64_t(u.st[J].size()));
            if (u.height[J] == 0 && u.ncol[J] > ND_LEAF) small_leaves = false;
        }
        if (vals >= (int64_t(1) << 31) || !small_leaves) continue;
        s.nd_mask[i] = all_nd || vals < ni * int64_t(s.bw[i] + 1);
    }
    for (int i = 0; i < np; ++i)
        if (!s.nd_mask[i]) sub[i] = SubND{};
    NDSym &d = s.nd;
    d = NDSym{};
    d.perm.resize(nloc);
    d.sn_ptr.assign(np + 1, 0);
    for (int i = 0; i < np; ++i) d.sn_ptr[i + 1] = d.sn_ptr[i] + int64_t(sub[i].first.size());
    const int64_t nsn = d.sn_ptr[np];
    d.nsn = nsn;
    d.first.resize(nsn);
    d.ncol.resize(nsn);
    d.nrow.resize(nsn);
    d.height.resize(nsn);
    d.voff.assign(nsn + 1, 0);
    d.st_ptr.assign(nsn + 1, 0);
    d.row_sn.resize(nloc);
    for (int i = 0; i < np; ++i) {
        const SubND &u = sub[i];
        const int64_t o = s.ov_ptr[i];
        if (s.nd_mask[i]) std::copy(u.perm.begin(), u.perm.end(), d.perm.begin() + o);
        else
            for (int64_t p = 0; p < s.ov_ptr[i + 1] - o; ++p) d.perm[o + p] = int32_t(p);   // (band subdomain)
        for (size_t J = 0; J < u.first.size(); ++J) {
            const int64_t g = d.sn_ptr[i] + int64_t(J);
            d.first[g] = u.first[J];
            d.ncol[g] = u.ncol[J];
            d.nrow[g] = u.ncol[J] + int32_t(u.st[J].size());
            d.height[g] = u.height[J];
            d.voff[g + 1] = d.voff[g] + int64_t(d.nrow[g]) * d.ncol[g];
            d.st_ptr[g + 1] = d.st_ptr[g] + int64_t(u.st[J].size());
            d.max_ncol = std::max(d.max_ncol, u.ncol[J]);
            d.max_sn = std::max(d.max_sn, int32_t(u.first.size()));
            for (int p = u.first[J]; p < u.first[J] + u.ncol[J]; ++p) d.row_sn[o + p] = int32_t(g);
        }
    }
    d.st_row.resize(d.st_ptr[nsn]);
    for (int i = 0; i < np; ++i)
        for (size_t J = 0; J < sub[i].st.size(); ++J) {
            const int64_t g = d.sn_ptr[i] + int64_t(J);
            std::copy(sub[i].st[J].begin(), sub[i].st[J].end(), d.st_row.begin() + d.st_ptr[g]);
        }
    // position of new row r in the panel of supernode J (r in J's columns or struct)
    auto panel_row = [&](int64_t J, int32_t r) -> int64_t {
        if (r >= d.first[J] && r < d.first[J] + d.ncol[J]) return r - d.first[J];
        const int32_t *b = d.st_row.data() + d.st_ptr[J], *e = d.st_row.data() + d.st_ptr[J + 1];
        const int32_t *it = std::lower_bound(b, e, r);
        if (it == e || *it != r) return -1;
        return d.ncol[J] + int64_t(it - b);
    };
    // forward row gathers: contributor K and row position, ascending K
    d.rc_ptr.assign(nloc + 1, 0);
    for (int i = 0; i < np; ++i) {
        const int64_t o = s.ov_ptr[i];
        for (int64_t K = d.sn_ptr[i]; K < d.sn_ptr[i + 1]; ++K)
            for (int64_t t = d.st_ptr[K]; t < d.st_ptr[K + 1]; ++t) ++d.rc_ptr[o + d.st_row[t] + 1];
    }
    for (int64_t p = 0; p < nloc; ++p) d.rc_ptr[p + 1] += d.rc_ptr[p];
    d.rc_sn.resize(d.rc_ptr[nloc]);
    d.rc_pos.resize(d.rc_ptr[nloc]);
    d.rc_w.resize(d.rc_ptr[nloc]);
    d.st_sn.resize(d.st_ptr[nsn]);
    {
        std::vector<int64_t> fill(d.rc_ptr.begin(), d.rc_ptr.end() - 1);
        for (int i = 0; i < np; ++i) {
            const int64_t o = s.ov_ptr[i], sb = d.st_ptr[d.sn_ptr[i]];
            for (int64_t K = d.sn_ptr[i]; K < d.sn_ptr[i + 1]; ++K)
                for (int64_t t = d.st_ptr[K]; t < d.st_ptr[K + 1]; ++t) {
                    const int64_t q = fill[o + d.st_row[t]]++;
                    d.rc_sn[q] = int32_t(K);
                    d.rc_pos[q] = d.ncol[K] + int32_t(t - d.st_ptr[K]);
                    if (t - sb >= (int64_t(1) << 31)) throw std::runtime_error("nested dissection: struct too large");
                    d.rc_w[q] = int32_t(t - sb);
                    d.st_sn[t] = int32_t(K);
                }
        }
    }
    // rows by height
    d.lv_base.assign(np + 1, 0);
    d.lv_rows.resize(nloc);
    d.ch_base.assign(np + 1, 0);
    d.ch_row.clear();
    {
        std::vector<int32_t> lp;
        for (int i = 0; i < np; ++i) {
            const int64_t o = s.ov_ptr[i];
            if (!s.nd_mask[i]) {   // a band subdomain: no levels
                d.lv_base[i + 1] = d.lv_base[i];
                d.ch_base[i + 1] = int64_t(d.ch_row.size());
                for (int64_t p = o; p < s.ov_ptr[i + 1]; ++p) d.lv_rows[p] = int32_t(p - o);
                continue;
            }
            int H = 0;
            for (int64_t J = d.sn_ptr[i]; J < d.sn_ptr[i + 1]; ++J) H = std::max(H, d.height[J] + 1);
            std::vector<int32_t> ptr(H + 1, 0);
            for (int64_t J = d.sn_ptr[i]; J < d.sn_ptr[i + 1]; ++J) ptr[d.height[J] + 1] += d.ncol[J];
            for (int h = 0; h < H; ++h) ptr[h + 1] += ptr[h];
            std::vector<int32_t> f(ptr.begin(), ptr.end() - 1);
            for (int64_t J = d.sn_ptr[i]; J < d.sn_ptr[i + 1]; ++J)
                for (int c = 0; c < d.ncol[J]; ++c) {
                    const int32_t p = f[d.height[J]]++;
                    d.lv_rows[o + p] = d.first[J] + c;
                    // (supernodes by height: the rows of a height are consecutive)
                    if (d.lv_rows[o + p] != p) throw std::runtime_error("nested dissection: rows not ordered by height");
                }
            // per height: first struct entry of its supernodes (relative to
            // the subdomain's first) and the multiply-adds of its diagonal
            // blocks and of its struct parts (saturated; a launch heuristic)
            std::vector<int64_t> st0(H + 1, -1), dm(H + 1, 0), sm(H + 1, 0);
            const int64_t sb = d.st_ptr[d.sn_ptr[i]];
            for (int64_t J = d.sn_ptr[i]; J < d.sn_ptr[i + 1]; ++J) {
                const int hJ = d.height[J];
                if (st0[hJ] < 0) st0[hJ] = d.st_ptr[J] - sb;
                const int64_t nJ = d.ncol[J], nsJ = d.nrow[J] - nJ;
                dm[hJ] += nJ * (nJ + 1) / 2;
                sm[hJ] += nJ * nsJ;
            }
            st0[H] = d.st_ptr[d.sn_ptr[i + 1]] - sb;
            const int64_t cap = (int64_t(1) << 31) - 1;
            for (int hh = 0; hh <= H; ++hh) {
                d.lv_info.push_back(int32_t(st0[hh]));
                d.lv_info.push_back(int32_t(std::min(dm[hh], cap)));
                d.lv_info.push_back(int32_t(std::min(sm[hh], cap)));
                d.lv_info.push_back(0);
            }
            d.lv_base[i + 1] = d.lv_base[i] + H + 1;
            lp.insert(lp.end(), ptr.begin(), ptr.end());
            d.max_levels = std::max(d.max_levels, H);
            for (int hh = 1; hh < H; ++hh) d.max_t = std::max(d.max_t, ptr[hh + 1] - ptr[hh]);
            // the leaves' rows (height 0, rows 0 .. ptr[1]) in chunks of at
            // most 64 rows that split no leaf: one wavefront solves a chunk
            d.ch_row.push_back(0);
            int32_t b0 = 0, cur = 0;
            for (int64_t J = d.sn_ptr[i]; J < d.sn_ptr[i + 1] && d.height[J] == 0; ++J) {
                if (cur + d.ncol[J] - b0 > 64) {
                    d.ch_row.push_back(cur);
                    b0 = cur;
                }
                cur += d.ncol[J];
            }
            if (cur > b0) d.ch_row.push_back(cur);
            d.ch_base[i + 1] = int64_t(d.ch_row.size());
        }
        d.lv_ptr = std::move(lp);
    }
    // left-looking update lists: for each J the earlier K whose struct meets
    // J's columns (ascending K), with the panel rows of struct(K) from s0 on
    {
        std::vector<std::vector<int64_t>> ups(nsn);   // K ids per J
        for (int i = 0; i < np; ++i) {
            const int64_t o = s.ov_ptr[i];
            for (int64_t K = d.sn_ptr[i]; K < d.sn_ptr[i + 1]; ++K) {
                int64_t last = -1;
                for (int64_t t = d.st_ptr[K]; t < d.st_ptr[K + 1]; ++t) {
                    const int64_t J = d.row_sn[o + d.st_row[t]];
                    if (J != last) {
                        ups[J].push_back(K);
                        last = J;
                    }
                }
            }
        }
        d.up_ptr.assign(nsn + 1, 0);
        for (int64_t J = 0; J < nsn; ++J) d.up_ptr[J + 1] = d.up_ptr[J] + int64_t(ups[J].size());
        const int64_t nup = d.up_ptr[nsn];
        d.up_k.resize(nup);
        d.up_s0.resize(nup);
        d.up_n1.resize(nup);
        d.up_rel.resize(nup);
        int64_t nrel = 0;
        for (int64_t J = 0; J < nsn; ++J)
            for (size_t q = 0; q < ups[J].size(); ++q) {
                const int64_t K = ups[J][q], u = d.up_ptr[J] + int64_t(q);
                const int32_t *b = d.st_row.data() + d.st_ptr[K], *e = d.st_row.data() + d.st_ptr[K + 1];
                const int32_t *s0 = std::lower_bound(b, e, d.first[J]);
                const int32_t *s1 = std::lower_bound(s0, e, d.first[J] + d.ncol[J]);
                d.up_k[u] = int32_t(K);
                d.up_s0[u] = int32_t(s0 - b);
                d.up_n1[u] = int32_t(s1 - s0);
                d.up_rel[u] = nrel;
                nrel += int64_t(e - s0);
            }
        d.rel.resize(nrel);
        for (int64_t J = 0; J < nsn; ++J)
            for (int64_t u = d.up_ptr[J]; u < d.up_ptr[J + 1]; ++u) {
                const int64_t K = d.up_k[u];
                const int64_t t0 = d.st_ptr[K] + d.up_s0[u];
                for (int64_t t = t0; t < d.st_ptr[K + 1]; ++t) {
                    const int64_t pr = panel_row(J, d.st_row[t]);
                    if (pr < 0) throw std::runtime_error("nested dissection: a struct row outside the parent panel");
                    d.rel[d.up_rel[u] + (t - t0)] = int32_t(pr);
                }
            }
    }
    // assembly of the lower entries of A_i into the panels
    {
        std::vector<int64_t> cnt(np + 1, 0);
        for (int i = 0; i < np; ++i) {
            if (!s.nd_mask[i]) continue;
            const int64_t o = s.ov_ptr[i];
            const int ni = int(s.ov_ptr[i + 1] - o);
            std::vector<int32_t> iperm(ni);
            for (int p = 0; p < ni; ++p) iperm[d.perm[o + p]] = p;
            for (int l = 0; l < ni; ++l)
                for (int64_t e = s.lrowptr[o + l]; e < s.lrowptr[o + l + 1]; ++e)
                    if (iperm[l] >= iperm[s.lcol[e]]) ++cnt[i + 1];
        }
        for (int i = 0; i < np; ++i) cnt[i + 1] += cnt[i];
        d.asm_src.resize(cnt[np]);
        d.asm_dst.resize(cnt[np]);
#pragma omp parallel for schedule(dynamic)
        for (int i = 0; i < np; ++i) {
            if (!s.nd_mask[i]) continue;
            const int64_t o = s.ov_ptr[i];
            const int ni = int(s.ov_ptr[i + 1] - o);
            std::vector<int32_t> iperm(ni);
            for (int p = 0; p < ni; ++p) iperm[d.perm[o + p]] = p;
            int64_t q = cnt[i];
            for (int l = 0; l < ni; ++l)
                for (int64_t e = s.lrowptr[o + l]; e < s.lrowptr[o + l + 1]; ++e) {
                    const int32_t pr = iperm[l], pc = iperm[s.lcol[e]];
                    if (pr < pc) continue;
                    const int64_t J = d.row_sn[o + pc];
                    const int64_t pos = panel_row(J, pr);
                    d.asm_src[q] = s.lgpos[e];
                    d.asm_dst[q] = pos < 0 ? -1 : d.voff[J] + int64_t(pc - d.first[J]) * d.nrow[J] + pos;
                    ++q;
                }
        }
        for (int64_t q = 0; q < int64_t(d.asm_dst.size()); ++q)
            if (d.asm_dst[q] < 0) throw std::runtime_error("nested dissection: an entry of A_i outside the panels");
    }
    // the band keeps only the subdomains without the supernodal factor
    if (!s.band_off.empty() && s.band_off[np] > 0) {
        std::vector<int64_t> off(np + 1, 0), dst, src;
        for (int i = 0; i < np; ++i)
            off[i + 1] = off[i] + (s.nd_mask[i] ? 0 : s.band_off[i + 1] - s.band_off[i]);
        int64_t q = 0;
        for (int i = 0; i < np; ++i) {
            // this subdomain's band scatter entries: its lower entries of A_i
            const int64_t o = s.ov_ptr[i];
            int64_t cnt = 0;
            for (int64_t l = 0; l < s.ov_ptr[i + 1] - o; ++l)
                for (int64_t e = s.lrowptr[o + l]; e < s.lrowptr[o + l + 1]; ++e) cnt += s.lcol[e] <= l;
            if (!s.nd_mask[i])
                for (int64_t k = q; k < q + cnt; ++k) {
                    dst.push_back(s.bscat_dst[k] - s.band_off[i] + off[i]);
                    src.push_back(s.bscat_src[k]);
                }
            q += cnt;
        }
        s.band_off.swap(off);
        s.bscat_dst.swap(dst);
        s.bscat_src.swap(src);
    }
}

}  // namespace gdsw
