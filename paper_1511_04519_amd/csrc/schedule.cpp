// Host builders of the sweep schedules (see schedule.hpp). Plain C++: the
// library uploads what these produce, and a host check replays it.
#include "schedule.hpp"

#include <algorithm>

namespace matex {

Contrib contributions(const Symbolic& s)
{
    Contrib C;
    C.pos_base.resize(s.sn.size());
    C.cptr.push_back(0);
    std::vector<std::vector<int32_t>> contrib;
    for (size_t k = 0; k < s.sn.size(); ++k) {
        const Supernode& q = s.sn[k];
        contrib.assign(q.nr, {});
        for (int32_t cp = s.child_ptr[k]; cp < s.child_ptr[k + 1]; ++cp) {
            const Supernode& c = s.sn[s.child_idx[cp]];
            for (int32_t t = 0; t < c.nr - c.nc; ++t) contrib[s.relidx[c.u + t]].push_back(int32_t(c.u + t));
        }
        C.pos_base[k] = int32_t(C.cptr.size()) - 1;
        for (int32_t p = 0; p < q.nr; ++p) {
            C.cidx.insert(C.cidx.end(), contrib[p].begin(), contrib[p].end());
            C.cptr.push_back(int32_t(C.cidx.size()));
        }
    }
    if (C.cidx.empty()) C.cidx.push_back(0);
    return C;
}

TreeHost build_tree_host(const Symbolic& s, const Contrib& C, int32_t limit)
{
    const std::vector<int32_t>&pos_base = C.pos_base, &cptr = C.cptr, &cidx = C.cidx;
    const int L = s.n_levels;
    const int32_t nsn = int32_t(s.sn.size());
    int E = 0;
    for (; E < L && limit >= 0; ++E) {
        bool ok = true;
        for (int32_t k : s.level_sn[E]) {
            const Supernode& q = s.sn[k];
            ok = ok && q.nc <= 64 && q.nr <= TREE_MAX_NR;
            for (int32_t p = 0; p < q.nr && ok; ++p) ok = cptr[pos_base[k] + p + 1] - cptr[pos_base[k] + p] <= 2;
        }
        if (!ok) break;
    }
    if (limit > 0) E = std::min(E, int(limit));
    auto is_root = [&](int32_t k, int S) {
        const int32_t par = s.sn[k].parent;
        return s.sn[k].level < S && (par < 0 || s.sn[par].level >= S);
    };
    auto n_roots = [&](int S) {
        int64_t r = 0;
        for (int32_t k = 0; k < nsn; ++k) r += is_root(k, S) ? 1 : 0;
        return r;
    };
    // subtree of each root: its supernodes and shared LDS need
    std::vector<int32_t> stack, nodes;
    auto subtree = [&](int32_t root) {
        nodes.clear();
        stack.assign(1, root);
        while (!stack.empty()) {
            const int32_t c = stack.back();
            stack.pop_back();
            nodes.push_back(c);
            for (int32_t cp = s.child_ptr[c]; cp < s.child_ptr[c + 1]; ++cp) stack.push_back(s.child_idx[cp]);
        }
    };
    auto shared_need = [&](int32_t root) {
        subtree(root);
        int64_t d = 0;
        for (int32_t c : nodes) d += s.sn[c].nc + (c == root ? 0 : s.sn[c].nr - s.sn[c].nc);
        return d;
    };
    int S = 0;
    if (E > 0) {
        const int64_t r1 = n_roots(1);
        for (int k = 1; k <= E; ++k)
            if (r1 < TREE_MIN_BLOCKS || n_roots(k) >= TREE_MIN_BLOCKS) S = k;
        // every subtree must fit one block's shared LDS
        while (S > 0) {
            bool fits = true;
            for (int32_t k = 0; k < nsn && fits; ++k)
                if (is_root(k, S)) fits = shared_need(k) <= TREE_MAX_SHARED;
            if (fits) break;
            --S;
        }
    }
    TreeHost T;
    T.n_levels = S;
    if (S == 0) return T;
    // pack roots into blocks; LDS offsets of each block's supernodes
    std::vector<int32_t> block_of(nsn, -1), lds_u(nsn, -1), lds_x(nsn, -1);
    std::vector<std::vector<int32_t>> blocks;
    std::vector<int64_t> bshared;
    int64_t cur_nodes = 0, cur_shared = 0;
    for (int32_t lv = S - 1; lv >= 0; --lv)
        for (int32_t k : s.level_sn[lv]) {
            if (!is_root(k, S)) continue;
            const int64_t need = shared_need(k);   // fills nodes
            if (blocks.empty() || cur_nodes + int64_t(nodes.size()) > TREE_MAX_NODES ||
                cur_shared + need > TREE_MAX_SHARED) {
                blocks.emplace_back();
                bshared.push_back(0);
                cur_nodes = cur_shared = 0;
            }
            const int32_t bi = int32_t(blocks.size()) - 1;
            for (int32_t c : nodes) {
                block_of[c] = bi;
                blocks.back().push_back(c);
                lds_u[c] = c == k ? -1 : 0;   // placed below
            }
            cur_nodes += int64_t(nodes.size());
            cur_shared += need;
            bshared.back() = cur_shared;
        }
    int32_t max_nr = 64;
    for (size_t bi = 0; bi < blocks.size(); ++bi) {
        int32_t off = 0;
        for (int32_t c : blocks[bi])
            if (lds_u[c] >= 0) { lds_u[c] = off; off += s.sn[c].nr - s.sn[c].nc; }
        for (int32_t c : blocks[bi]) { lds_x[c] = off; off += s.sn[c].nc; }
        for (int32_t c : blocks[bi]) max_nr = std::max(max_nr, s.sn[c].nr);
    }
    // LDS offsets of contributions and off rows
    std::vector<int32_t> trow(s.rows.size() + 1, 0);   // one spare: clamped reads stay inside
    std::vector<int32_t> owner(s.n);
    for (int32_t k = 0; k < nsn; ++k)
        for (int32_t c = 0; c < s.sn[k].nc; ++c) owner[s.sn[k].c0 + c] = k;
    std::vector<int32_t> slot_lds(std::max<int64_t>(1, s.n_upd), -1);
    for (int32_t k = 0; k < nsn; ++k)
        if (block_of[k] >= 0 && lds_u[k] >= 0)
            for (int32_t t = 0; t < s.sn[k].nr - s.sn[k].nc; ++t) slot_lds[s.sn[k].u + t] = lds_u[k] + t;
    for (int32_t k = 0; k < nsn; ++k) {
        if (block_of[k] < 0) continue;
        const Supernode& q = s.sn[k];
        for (int32_t t = 0; t < q.nr - q.nc; ++t) {
            const int32_t r = s.rows[q.roff + t], a = owner[r];
            trow[q.roff + t] = block_of[a] == block_of[k] ? -1 - (lds_x[a] + r - s.sn[a].c0) : r;
        }
    }
    // steps: forward items are 64-row slabs, children's levels first;
    // backward items column groups with at most 16 rows per lane, root first
    std::vector<TItem> fi, bi_;
    std::vector<int32_t> fblk{0}, bblk{0};
    std::vector<TItem> lvl;
    auto flush = [&](std::vector<TItem>& out) {
        for (size_t i = 0; i < lvl.size(); i += TW)
            for (size_t w = i; w < i + TW; ++w) out.push_back(w < lvl.size() ? lvl[w] : TItem{});
        lvl.clear();
    };
    for (const auto& blk : blocks) {
        for (int32_t lv = 0; lv < S; ++lv) {
            for (int32_t c : blk) {
                const Supernode& q = s.sn[c];
                if (q.level != lv) continue;
                for (int32_t r = 0; r < q.nr; r += 64)
                    lvl.push_back({q.w, q.u, q.c0, q.nc, q.nr, r, std::min(q.nr, r + 64), pos_base[c],
                                   lds_u[c], lds_x[c]});
            }
            flush(fi);
        }
        fblk.push_back(int32_t(fi.size() / TW));
        for (int32_t lv = S - 1; lv >= 0; --lv) {
            for (int32_t c : blk) {
                const Supernode& q = s.sn[c];
                if (q.level != lv) continue;
                int32_t lpc = 1;
                while (lpc < 64 && int64_t(lpc) * 16 < q.nr) lpc *= 2;
                const int32_t cpi = 64 / lpc;
                for (int32_t c1 = 0; c1 < q.nc; c1 += cpi)
                    lvl.push_back({q.w, q.roff, q.c0, q.nc, q.nr, c1, std::min(q.nc, c1 + cpi), 0,
                                   lds_u[c], lds_x[c]});
            }
            flush(bi_);
        }
        bblk.push_back(int32_t(bi_.size() / TW));
    }
    // per forward item and lane: the LDS slots adding into its btilde column
    // and its panel row
    auto desc = [&](const TItem& t, int32_t p) {
        int32_t d = 0, sh = 0;
        if (p >= t.nr) return 0;
        const int64_t base = t.pos + p;
        for (int32_t j = cptr[base]; j < cptr[base + 1]; ++j, sh += 16) d |= (slot_lds[cidx[j]] + 1) << sh;
        return d;
    };
    std::vector<I2> fd(fi.size() * 64, I2{0, 0});
    for (size_t i = 0; i < fi.size(); ++i) {
        const TItem& t = fi[i];
        if (t.nr == 0) continue;
        for (int32_t lane = 0; lane < 64; ++lane) {
            const int32_t row = t.first + lane;
            fd[i * 64 + lane] = I2{lane < t.nc ? desc(t, lane) : 0,
                                   row >= t.nc && row < t.last ? desc(t, row) : 0};
        }
    }
    int64_t shared = 0, steps = 0;
    for (int64_t v : bshared) shared = std::max(shared, v);
    for (size_t b = 0; b + 1 < fblk.size(); ++b)
        steps = std::max<int64_t>(steps, std::max(fblk[b + 1] - fblk[b], bblk[b + 1] - bblk[b]));
    T.fdesc = std::move(fd);
    T.fitems = std::move(fi);
    T.bitems = std::move(bi_);
    T.fblk = std::move(fblk);
    T.bblk = std::move(bblk);
    T.trow = std::move(trow);
    T.shared = std::move(bshared);
    T.n_blocks = int32_t(blocks.size());
    T.ws = (max_nr + 15) / 16 * 16;
    T.item_doubles = int32_t(steps * TW * int64_t(sizeof(TItem)) / 8);
    T.lds_doubles = int32_t(T.item_doubles + TW * T.ws + shared);
    return T;
}

}  // namespace matex
