// C-ABI entry points, device factor handle, segment planner and the
// transient driver of the R-MATEX library (see include/matex.h).
//
// Everything numeric after the one-time factorisation runs in the HIP kernels
// of kernels.hip, in the nested-dissection ordering (vectors are permuted
// once on the way in and out). The host only plans steps (transition spots,
// output times, shift choice) and reads back the few integers that decide
// control flow (converged or not, Krylov dimension).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <map>
#include <unordered_map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/matex.h"
#include "batched.hpp"
#include "factor.hpp"
#include "kernels.hpp"
#include "schedule.hpp"

using namespace matex;

namespace {

thread_local std::string g_err;

matex_status fail(matex_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

struct HipError {
    hipError_t e;
    const char* what;
};

#define HIPCHK(expr)                                                      \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) throw HipError{e_, #expr};                  \
    } while (0)

struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    explicit DevMem(size_t b) : bytes(b) {
        if (b) HIPCHK(hipMalloc(&p, b));
    }
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    DevMem(DevMem&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevMem& operator=(DevMem&& o) noexcept {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        return *this;
    }
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

template <class T>
DevMem upload(const std::vector<T>& v)
{
    DevMem m(sizeof(T) * v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(m.p, v.data(), m.bytes, hipMemcpyHostToDevice));
    return m;
}

struct PinnedMem {
    void* p = nullptr;
    explicit PinnedMem(size_t b) { HIPCHK(hipHostMalloc(&p, b, hipHostMallocDefault)); }
    ~PinnedMem() {
        if (p) (void)hipHostFree(p);
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Pinned staging slots for host-to-device copies on one stream: a slot is
// reused only after the copy that last read it has completed (its event),
// so filling the next one never drains the stream.
struct StageRing {
    static constexpr int SLOTS = 4;
    std::unique_ptr<PinnedMem> mem;
    size_t slot_bytes = 0;
    hipEvent_t ev[SLOTS] = {};
    bool used[SLOTS] = {};
    int next = 0;
    explicit StageRing(size_t bytes) : slot_bytes(bytes) {
        mem.reset(new PinnedMem(SLOTS * slot_bytes));
        for (auto& e : ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    StageRing(const StageRing&) = delete;
    StageRing& operator=(const StageRing&) = delete;
    ~StageRing() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    // Copies `bytes` from host src to device dst on st through a free slot.
    void copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
        if (bytes > slot_bytes) {
            HIPCHK(hipStreamSynchronize(st));
            slot_bytes = bytes * 2;
            mem.reset(new PinnedMem(SLOTS * slot_bytes));
            for (bool& u : used) u = false;
        }
        const int s = next;
        next = (next + 1) % SLOTS;
        if (used[s]) HIPCHK(hipEventSynchronize(ev[s]));
        char* slot = mem->as<char>() + size_t(s) * slot_bytes;
        std::memcpy(slot, src, bytes);
        HIPCHK(hipMemcpyAsync(dst, slot, bytes, hipMemcpyHostToDevice, st));
        HIPCHK(hipEventRecord(ev[s], st));
        used[s] = true;
    }
};

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Names of the arrays (count, device pointer) holding a NaN or an infinite
// value; empty when all are finite. Synchronises st.
std::string nonfinite_arrays(const std::vector<std::tuple<const char*, int64_t, const double*>>& arrs,
                             hipStream_t st)
{
    DevMem flags(sizeof(int32_t) * std::max<size_t>(1, arrs.size()));
    HIPCHK(hipMemsetAsync(flags.p, 0, flags.bytes, st));
    for (size_t k = 0; k < arrs.size(); ++k)
        if (std::get<2>(arrs[k])) launch_flag_nonfinite(std::get<1>(arrs[k]), std::get<2>(arrs[k]), flags.as<int32_t>() + k, st);
    std::vector<int32_t> h(arrs.size(), 0);
    if (!h.empty()) HIPCHK(hipMemcpyAsync(h.data(), flags.p, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::string bad;
    for (size_t k = 0; k < arrs.size(); ++k)
        if (h[k]) bad += std::string(bad.empty() ? "" : ", ") + std::get<0>(arrs[k]);
    return bad;
}

}  // namespace

struct matex_factor_s {
    Symbolic sym;
    double gamma = 0.0;
    std::vector<double> gammas;       // shift ladder
    double vdd = 1.0;
    std::vector<double> c_host;       // node capacitances, natural order
    int device = 0;
    // device structure
    DevMem d_c0, d_nc, d_nr, d_roff, d_w, d_u, d_rows, d_child_ptr, d_child_idx, d_relidx;
    DevMem d_perm, d_iperm, d_cperm;
    DevMem d_grp, d_gci, d_gv;        // G in the permuted order (CSR), for the adjoint
    std::vector<DevMem> d_W;          // [n_shifts] M factors, then G
    DevMem d_fdesc, d_gsrc;
    DevMem d_fwd_tasks, d_bwd_tasks, d_tree_f, d_tree_b, d_tree_fblk, d_tree_bblk, d_tree_fdesc,
        d_tree_trow;
    std::vector<LevelTasks> fwd, bwd;   // levels tree.n_levels .. n_levels - 1
    TreeTasks tree{};
    // batched (multi-subtask) sweeps
    DevMem d_b_pos, d_b_cptr, d_b_cidx, d_b_ft, d_b_fr, d_b_bt, d_b_br, d_b_wave;
    BatchAssembly bas{};
    std::vector<BatchLevel> blevels;               // the schedule in use, per level
    struct BatchCand {
        BatchLevel lv;
        std::string name;
    };
    std::vector<std::vector<BatchCand>> bcand;     // candidates per level
    std::vector<std::pair<int, int>> bchoice;      // forward, backward candidate kept
    int64_t b_slots = 0;   // partial-result slots one batched sweep needs
    DevSym dsym{};
    matex_factor_info info{};
    int64_t held_bytes() const {
        int64_t b = 0;
        for (const DevMem* m : {&d_c0, &d_nc, &d_nr, &d_roff, &d_w, &d_u, &d_rows, &d_child_ptr, &d_child_idx,
                                &d_relidx, &d_perm, &d_iperm, &d_cperm, &d_grp, &d_gci, &d_gv, &d_fwd_tasks, &d_bwd_tasks, &d_fdesc, &d_gsrc, &d_tree_f, &d_tree_b,
                                &d_tree_fblk, &d_tree_bblk, &d_tree_fdesc, &d_tree_trow, &d_b_pos,
                                &d_b_cptr, &d_b_cidx, &d_b_ft, &d_b_fr, &d_b_bt, &d_b_br, &d_b_wave})
            b += int64_t(m->bytes);
        for (const DevMem& m : d_W) b += int64_t(m.bytes);
        return b;
    }
};

// gamma of factor index k as the check kernels take it: gamma_k for a shift
// of the ladder, 0 for G (the inverted space of Sec. 3.3.1, X1 = G).
inline double shift_gamma(const matex_factor_s& F, int k)
{
    return k < int(F.gammas.size()) ? F.gammas[k] : 0.0;
}

namespace {

// Blocks the device holds at once at 256 threads each (256 compute units x 8).
constexpr int64_t RESIDENT_BLOCKS = 2048;

// Uploads the subtree schedule of the bottom levels (schedule.cpp).
void build_tree(matex_factor_s& F, const Contrib& C, int32_t limit)
{
    TreeHost h = build_tree_host(F.sym, C, limit);
    F.tree = TreeTasks{};
    F.tree.n_levels = h.n_levels;
    if (h.n_levels == 0) return;
    static_assert(sizeof(I2) == sizeof(int2), "I2 is read as int2");
    F.d_tree_fdesc = upload(h.fdesc);
    F.d_tree_f = upload(h.fitems);
    F.d_tree_b = upload(h.bitems);
    F.d_tree_fblk = upload(h.fblk);
    F.d_tree_bblk = upload(h.bblk);
    F.d_tree_trow = upload(h.trow);
    TreeTasks& T = F.tree;
    T.fitems = F.d_tree_f.as<TItem>();
    T.bitems = F.d_tree_b.as<TItem>();
    T.fblk = F.d_tree_fblk.as<int32_t>();
    T.bblk = F.d_tree_bblk.as<int32_t>();
    T.fdesc = F.d_tree_fdesc.as<int2>();
    T.trow = F.d_tree_trow.as<int32_t>();
    T.n_blocks = h.n_blocks;
    T.ws = h.ws;
    T.item_doubles = h.item_doubles;
    T.lds_doubles = h.lds_doubles;
}

void build_tasks(matex_factor_s& F, int32_t subtree_limit)
{
    const Symbolic& s = F.sym;
    const int L = s.n_levels;
    // every panel position's contributing child update slots, in child order
    // (the inverse of relidx), shared by the one-vector and batched sweeps
    const Contrib C = contributions(s);
    const std::vector<int32_t>&pos_base = C.pos_base, &cptr = C.cptr, &cidx = C.cidx;
    F.d_b_pos = upload(pos_base); F.d_b_cptr = upload(cptr); F.d_b_cidx = upload(cidx);
    F.bas = BatchAssembly{F.d_b_pos.as<int32_t>(), F.d_b_cptr.as<int32_t>(), F.d_b_cidx.as<int32_t>()};
    build_tree(F, C, subtree_limit);
    const int32_t S = F.tree.n_levels;
    // levels above: the forward sweep takes 16 panel rows per block, 64 when
    // that many blocks would not all be resident at once, 4 on levels with
    // few such blocks; the backward sweep one wavefront per column, 16 lanes
    // per column when four-column blocks would not all be resident.
    std::vector<PTask> ft, bt;
    std::vector<int64_t> fo(L + 1, 0), bo(L + 1, 0);
    std::vector<int32_t> fkind(L), bkind(L), flds(L, 1), blds(L, 1);
    auto ceil_div = [](int64_t a, int64_t b) { return (a + b - 1) / b; };
    for (int lv = S; lv < L; ++lv) {
        int32_t mx_nr = 0, mx_nc = 0;
        int64_t r16 = 0, c4 = 0;
        for (int32_t k : s.level_sn[lv]) {
            const Supernode& q = s.sn[k];
            mx_nr = std::max(mx_nr, q.nr);
            mx_nc = std::max(mx_nc, q.nc);
            r16 += ceil_div(q.nr, 16);
            c4 += ceil_div(q.nc, 4);
        }
        fkind[lv] = r16 > RESIDENT_BLOCKS ? 64 : (r16 < 128 ? 4 : 16);
        bkind[lv] = c4 > RESIDENT_BLOCKS ? 16 : 64;
        flds[lv] = std::max(1, mx_nc);
        blds[lv] = std::max(1, mx_nr);
        const int32_t cols_per = 256 / bkind[lv];
        for (int32_t k : s.level_sn[lv]) {
            const Supernode& q = s.sn[k];
            for (int32_t r = 0; r < q.nr; r += fkind[lv])
                ft.push_back({q.w, q.u, q.c0, q.nc, q.nr, r, pos_base[k], 0});
            for (int32_t c = 0; c < q.nc; c += cols_per)
                bt.push_back({q.w, q.roff, q.c0, q.nc, q.nr, c, 0, 0});
        }
        fo[lv + 1] = int64_t(ft.size());
        bo[lv + 1] = int64_t(bt.size());
    }
    for (int lv = 0; lv < S; ++lv) fo[lv + 1] = bo[lv + 1] = 0;
    F.d_fwd_tasks = upload(ft.empty() ? std::vector<PTask>(1, PTask{}) : ft);
    F.d_bwd_tasks = upload(bt.empty() ? std::vector<PTask>(1, PTask{}) : bt);
    // block-indexed tables: forward contributor slots (levels whose panel
    // positions have at most two contributors), backward sources of g
    std::vector<int2> fdesc;
    std::vector<int32_t> gsrc;
    std::vector<int64_t> fdo(L, -1), gso(L, 0);
    std::vector<int32_t> fslot(L, 0), gslot(L, 0);
    for (int lv = S; lv < L; ++lv) {
        bool two = true;
        for (int32_t k : s.level_sn[lv])
            for (int32_t p = 0; p < s.sn[k].nr && two; ++p)
                two = cptr[pos_base[k] + p + 1] - cptr[pos_base[k] + p] <= 2;
        if (two) {
            const int32_t nc_max = flds[lv], sl = nc_max + fkind[lv];
            fslot[lv] = sl;
            fdo[lv] = int64_t(fdesc.size());
            auto entry = [&](const PTask& t, int32_t p) {
                int2 d = make_int2(-1, -1);
                if (p < 0 || p >= t.nr) return d;
                const int32_t j0 = cptr[t.pos + p], j1 = cptr[t.pos + p + 1];
                if (j1 > j0) d.x = cidx[j0];
                if (j1 > j0 + 1) d.y = cidx[j0 + 1];
                return d;
            };
            for (int64_t i = fo[lv]; i < fo[lv + 1]; ++i) {
                const PTask& t = ft[i];
                for (int32_t k = 0; k < nc_max; ++k) fdesc.push_back(k < t.nc ? entry(t, k) : make_int2(-1, -1));
                for (int32_t r = 0; r < fkind[lv]; ++r) {
                    const int32_t row = t.first + r;
                    fdesc.push_back(row >= t.nc ? entry(t, row) : make_int2(-1, -1));
                }
            }
        }
        int32_t sl = 0;
        for (int64_t i = bo[lv]; i < bo[lv + 1]; ++i) sl = std::max(sl, bt[i].nr - bt[i].first);
        gslot[lv] = sl;
        gso[lv] = int64_t(gsrc.size());
        for (int64_t i = bo[lv]; i < bo[lv + 1]; ++i) {
            const PTask& t = bt[i];
            for (int32_t q = 0; q < sl; ++q) {
                const int32_t k = t.first + q;
                int32_t v = INT32_MIN;
                if (k < t.nc) v = -1 - (t.c0 + k);
                else if (k < t.nr) v = s.rows[t.aux + k - t.nc];
                gsrc.push_back(v);
            }
        }
    }
    F.d_fdesc = upload(fdesc.empty() ? std::vector<int2>(1, make_int2(-1, -1)) : fdesc);
    F.d_gsrc = upload(gsrc.empty() ? std::vector<int32_t>(1, INT32_MIN) : gsrc);
    for (int lv = S; lv < L; ++lv) {
        LevelTasks f{F.d_fwd_tasks.as<PTask>() + fo[lv], int32_t(fo[lv + 1] - fo[lv]), flds[lv], fkind[lv],
                     fslot[lv], fdo[lv] >= 0 ? F.d_fdesc.as<int2>() + fdo[lv] : nullptr, nullptr};
        LevelTasks b{F.d_bwd_tasks.as<PTask>() + bo[lv], int32_t(bo[lv + 1] - bo[lv]), blds[lv], bkind[lv],
                     gslot[lv], nullptr, F.d_gsrc.as<int32_t>() + gso[lv]};
        F.fwd.push_back(f);
        F.bwd.push_back(b);
    }
    // batched sweeps: per level, candidate schedules of the 64-right-hand-side
    // pair, picked by tune_batched: forward blocks of 64 panel rows and
    // backward blocks of 64 panel columns, each split into tasks of at most
    // `chunk` panel columns / rows whose partial results are summed (chunk
    // 64, 128 or 256), and on levels of narrow supernodes one wavefront per
    // supernode
    {
        std::vector<BTask> ft, bt;
        std::vector<BRed> fr, br;
        std::vector<int32_t> wv;
        struct Off { int64_t f, fr, b, br; };
        std::vector<std::vector<Off>> off(L);
        std::vector<int64_t> wo(L, -1);
        for (int lv = 0; lv < L; ++lv) {
            for (int32_t chunk : BATCH_CHUNKS) {
                Off o{int64_t(ft.size()), int64_t(fr.size()), int64_t(bt.size()), int64_t(br.size())};
                int32_t fslots = 0, bslots = 0;
                for (int32_t k : s.level_sn[lv]) {
                    const Supernode& q = s.sn[k];
                    for (int32_t r0 = 0; r0 < q.nr; r0 += BR) {
                        const int32_t K = std::min(q.nc, r0 + BR);
                        const int32_t nch = (K + chunk - 1) / chunk;
                        if (nch == 1) {
                            ft.push_back({k, r0, 0, K, -1});
                        } else {
                            fr.push_back({k, r0, fslots, nch});
                            for (int32_t c = 0; c < nch; ++c)
                                ft.push_back({k, r0, c * chunk, std::min(K, (c + 1) * chunk), fslots++});
                        }
                    }
                    for (int32_t c0 = 0; c0 < q.nc; c0 += BR) {
                        const int32_t nch = (q.nr - c0 + chunk - 1) / chunk;
                        if (nch == 1) {
                            bt.push_back({k, c0, c0, q.nr, -1});
                        } else {
                            br.push_back({k, c0, bslots, nch});
                            for (int32_t c = 0; c < nch; ++c)
                                bt.push_back({k, c0, c0 + c * chunk, std::min(q.nr, c0 + (c + 1) * chunk),
                                              bslots++});
                        }
                    }
                }
                F.b_slots = std::max<int64_t>(F.b_slots, std::max(fslots, bslots));
                off[lv].push_back(o);
            }
            off[lv].push_back({int64_t(ft.size()), int64_t(fr.size()), int64_t(bt.size()), int64_t(br.size())});
            bool narrow = true;
            for (int32_t k : s.level_sn[lv]) narrow = narrow && s.sn[k].nc <= WAVE_MAX_NC;
            if (narrow && !s.level_sn[lv].empty()) {
                wo[lv] = int64_t(wv.size());
                wv.insert(wv.end(), s.level_sn[lv].begin(), s.level_sn[lv].end());
            }
        }
        if (fr.empty()) fr.push_back({0, 0, 0, 0});
        if (br.empty()) br.push_back({0, 0, 0, 0});
        if (wv.empty()) wv.push_back(0);
        F.d_b_ft = upload(ft); F.d_b_fr = upload(fr); F.d_b_bt = upload(bt); F.d_b_br = upload(br);
        F.d_b_wave = upload(wv);
        F.bcand.assign(L, {});
        for (int lv = 0; lv < L; ++lv) {
            for (size_t v = 0; v + 1 < off[lv].size(); ++v) {
                const Off& o = off[lv][v];
                const Off& e = off[lv][v + 1];
                BatchLevel b;
                b.fwd = F.d_b_ft.as<BTask>() + o.f;
                b.n_fwd = int32_t(e.f - o.f);
                b.fred = F.d_b_fr.as<BRed>() + o.fr;
                b.n_fred = int32_t(e.fr - o.fr);
                b.bwd = F.d_b_bt.as<BTask>() + o.b;
                b.n_bwd = int32_t(e.b - o.b);
                b.bred = F.d_b_br.as<BRed>() + o.br;
                b.n_bred = int32_t(e.br - o.br);
                F.bcand[lv].push_back({b, "split" + std::to_string(BATCH_CHUNKS[v])});
            }
            if (wo[lv] >= 0) {
                BatchLevel b = F.bcand[lv].back().lv;
                b.fwave = b.bwave = F.d_b_wave.as<int32_t>() + wo[lv];
                b.n_fwave = b.n_bwave = int32_t(s.level_sn[lv].size());
                for (int32_t k : s.level_sn[lv]) b.wave_nc = std::max(b.wave_nc, s.sn[k].nc);
                F.bcand[lv].push_back({b, "wave"});
            }
            // until tuned: the largest chunk (the candidate of fewest tasks)
            F.blevels.push_back(F.bcand[lv][BATCH_CHUNKS.size() - 1].lv);
            F.bchoice.push_back({int(BATCH_CHUNKS.size()) - 1, int(BATCH_CHUNKS.size()) - 1});
        }
    }
}

// The autotuner of the 64-right-hand-side pair: for every level, each
// candidate schedule's forward and backward launches are timed on the
// factor of C + gamma_0 G (HIP events on `st`, the best of a few repeats,
// after one untimed launch), and the fastest forward and the fastest
// backward are kept. The choice depends on the structure and the device
// only; values do not change the timing (zero right-hand sides).
void keep_batched_choice(matex_factor_s& F, int lv, int bf, int bb)
{
    const auto& cand = F.bcand[size_t(lv)];
    BatchLevel m = cand[size_t(bf)].lv;
    const BatchLevel& mb = cand[size_t(bb)].lv;
    m.bwd = mb.bwd; m.n_bwd = mb.n_bwd; m.bred = mb.bred; m.n_bred = mb.n_bred;
    m.bwave = mb.bwave; m.n_bwave = mb.n_bwave;
    m.fwave = cand[size_t(bf)].lv.fwave;
    m.n_fwave = cand[size_t(bf)].lv.n_fwave;
    m.wave_nc = std::max(cand[size_t(bf)].lv.wave_nc, mb.wave_nc);
    F.blevels[size_t(lv)] = m;
    F.bchoice[size_t(lv)] = {bf, bb};
}

// The tuner's cache (file named by MATEX_TUNE_CACHE; none when unset): one
// line per factor structure, "key L f_0 b_0 ... f_{L-1} b_{L-1}", the key
// made of the sizes that fix the candidates (nodes, supernodes, levels,
// stored panel entries, structural nonzeros, update rows) and the candidate
// counts per level. A factor of a structure found there takes the recorded
// choices instead of timing them, so that every process that shares the
// file runs the same schedule.
std::string tune_key(const matex_factor_s& F)
{
    std::string k = std::to_string(F.sym.n) + ":" + std::to_string(F.sym.sn.size()) + ":" +
                    std::to_string(F.sym.n_levels) + ":" + std::to_string(F.sym.n_w) + ":" +
                    std::to_string(F.sym.nnz_exact) + ":" + std::to_string(F.sym.n_upd) + ":";
    for (const auto& c : F.bcand) k += std::to_string(c.size());
    return k;
}

bool load_tuned(matex_factor_s& F)
{
    const char* path = std::getenv("MATEX_TUNE_CACHE");
    if (!path || !path[0]) return false;
    std::FILE* fp = std::fopen(path, "r");
    if (!fp) return false;
    const std::string key = tune_key(F);
    const int L = F.sym.n_levels;
    bool found = false;
    char buf[8192];
    while (!found && std::fgets(buf, sizeof buf, fp)) {
        std::string line(buf);
        if (line.compare(0, key.size() + 1, key + " ") != 0) continue;
        std::vector<int> v;
        const char* q = buf + key.size() + 1;
        char* end = nullptr;
        for (long x = std::strtol(q, &end, 10); end != q; x = std::strtol(q, &end, 10)) {
            v.push_back(int(x));
            q = end;
        }
        if (int(v.size()) != 1 + 2 * L || v[0] != L) continue;
        bool ok = true;
        for (int lv = 0; lv < L && ok; ++lv) {
            const int nc = int(F.bcand[size_t(lv)].size());
            ok = v[1 + 2 * lv] >= 0 && v[1 + 2 * lv] < nc && v[2 + 2 * lv] >= 0 && v[2 + 2 * lv] < nc;
        }
        if (!ok) continue;
        for (int lv = 0; lv < L; ++lv) keep_batched_choice(F, lv, v[1 + 2 * lv], v[2 + 2 * lv]);
        found = true;
    }
    std::fclose(fp);
    return found;
}

void store_tuned(const matex_factor_s& F)
{
    const char* path = std::getenv("MATEX_TUNE_CACHE");
    if (!path || !path[0]) return;
    std::FILE* fp = std::fopen(path, "a");
    if (!fp) return;
    std::fprintf(fp, "%s %d", tune_key(F).c_str(), F.sym.n_levels);
    for (const auto& c : F.bchoice) std::fprintf(fp, " %d %d", c.first, c.second);
    std::fprintf(fp, "\n");
    std::fclose(fp);
}

void tune_batched(matex_factor_s& F, hipStream_t st)
{
    if (load_tuned(F)) {
        F.info.seconds_tune = 0.0;
        return;
    }
    const int L = F.sym.n_levels;
    const int R = RMAX;
    const int64_t n = F.sym.n;
    const double t0 = now_s();
    DevMem B(sizeof(double) * size_t(n) * R), Y(sizeof(double) * size_t(n) * R), X(sizeof(double) * size_t(n) * R),
        U(sizeof(double) * std::max<int64_t>(1, F.sym.n_upd) * R),
        P(sizeof(double) * std::max<int64_t>(1, F.b_slots) * PSLOT);
    for (DevMem* m : {&B, &Y, &X, &U}) HIPCHK(hipMemsetAsync(m->p, 0, m->bytes, st));
    const double* W = F.d_W[0].as<double>();
    const double* sc = F.d_cperm.as<double>();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    constexpr int REPS = 3;
    auto time_it = [&](auto&& launch) {
        launch();
        float best = 1e30f;
        for (int r = 0; r < REPS; ++r) {
            HIPCHK(hipEventRecord(e0, st));
            launch();
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return best;
    };
    for (int lv = 0; lv < L; ++lv) {
        const auto& cand = F.bcand[lv];
        int bf = 0, bb = 0;
        float tf = 1e30f, tb = 1e30f;
        for (size_t c = 0; c < cand.size(); ++c) {
            const BatchLevel& b = cand[c].lv;
            const float f = time_it([&]() {
                launch_b_forward(F.dsym, F.bas, b, R, W, B.as<double>(), sc, Y.as<double>(), U.as<double>(),
                                 P.as<double>(), st);
            });
            const float g = time_it([&]() {
                launch_b_backward(F.dsym, b, R, W, Y.as<double>(), X.as<double>(), P.as<double>(), st);
            });
            if (f < tf) { tf = f; bf = int(c); }
            if (g < tb) { tb = g; bb = int(c); }
        }
        keep_batched_choice(F, lv, bf, bb);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipStreamSynchronize(st));
    F.info.seconds_tune = now_s() - t0;
    store_tuned(F);
}

// One line per level: the supernodes' widths and the schedules kept.
std::string describe_batched(const matex_factor_s& F)
{
    std::string out;
    for (int lv = 0; lv < F.sym.n_levels; ++lv) {
        int mx = 0;
        for (int32_t k : F.sym.level_sn[size_t(lv)]) mx = std::max(mx, F.sym.sn[size_t(k)].nc);
        const auto& c = F.bcand[size_t(lv)];
        out += "level " + std::to_string(lv) + ": " + std::to_string(F.sym.level_sn[size_t(lv)].size()) +
               " supernodes (nc <= " + std::to_string(mx) + "), forward " +
               c[size_t(F.bchoice[size_t(lv)].first)].name + ", backward " +
               c[size_t(F.bchoice[size_t(lv)].second)].name + "\n";
    }
    return out;
}

// x = A_which^-1 (scale .* b), all in the permuted ordering. tmp: [n], upd: [n_upd].
void dev_solve(const matex_factor_s& F, int which, const double* b, const double* scale,
               double* x, double* tmp, double* upd, const int32_t* done, hipStream_t st)
{
    const double* W = F.d_W[which].as<double>();
    launch_forward_tree(F.tree, W, b, scale, tmp, upd, done, st);
    for (const LevelTasks& lv : F.fwd)
        launch_forward(lv, F.bas.cptr, F.bas.cidx, W, b, scale, tmp, upd, done, st);
    const int32_t* rows = F.d_rows.as<int32_t>();
    for (auto it = F.bwd.rbegin(); it != F.bwd.rend(); ++it)
        launch_backward(*it, rows, W, tmp, x, done, st);
    launch_backward_tree(F.tree, W, tmp, x, done, st);
}

// Multi-subtask pair: x = A_which^-1 (scale .* B) for R row-interleaved
// right-hand sides (n x R). T, yf: n x R scratch; U: n_upd x R scratch.
// P: F.b_slots * PSLOT doubles of partial results.
void dev_solve_batched(const matex_factor_s& F, int which, int R, const double* B,
                       const double* scale, double* x, double* yf, double* U, double* P,
                       hipStream_t st)
{
    const double* W = F.d_W[which].as<double>();
    const int L = F.sym.n_levels;
    for (int lv = 0; lv < L; ++lv) launch_b_forward(F.dsym, F.bas, F.blevels[lv], R, W, B, scale, yf, U, P, st);
    for (int lv = L - 1; lv >= 0; --lv) launch_b_backward(F.dsym, F.blevels[lv], R, W, yf, x, P, st);
}

// Scratch of one batched pair.
struct BatchScratch {
    DevMem yf, U, P;
    BatchScratch(const matex_factor_s& F, int R) {
        const size_t nr = sizeof(double) * size_t(F.sym.n) * R;
        yf = DevMem(nr);
        U = DevMem(sizeof(double) * std::max<int64_t>(1, F.sym.n_upd) * R);
        P = DevMem(sizeof(double) * std::max<int64_t>(1, F.b_slots) * PSLOT);
    }
};

void dev_solve_batched(const matex_factor_s& F, int which, int R, const double* B,
                       const double* scale, double* x, const BatchScratch& sc, hipStream_t st)
{
    dev_solve_batched(F, which, R, B, scale, x, sc.yf.as<double>(), sc.U.as<double>(), sc.P.as<double>(), st);
}

// Scratch of one Krylov process.
struct Work {
    int64_t n = 0;
    DevMem V, w, tmp, upd, partial, ks, u, est, taus, sel;
    int64_t max_checks = 0;
    // checks run on their own stream beside the next iteration; a check waits
    // for its iteration's ticket (the number gs_finish publishes), not for a
    // cross-stream event: such an event wait slowed every iteration of the
    // main stream by about 20 us on MI355X
    hipStream_t cs = nullptr;
    int32_t ticket = 0;                // number of the last iteration launched
    // iteration graphs (MATEX_GRAPHS=1), keyed by shift and iteration
    bool use_graphs = false;
    hipStream_t gs = nullptr;          // capture stream
    std::map<int, hipGraphExec_t> graphs;
    Work(const Work&) = delete;
    Work& operator=(const Work&) = delete;
    ~Work() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        if (gs) (void)hipStreamDestroy(gs);
        if (cs) (void)hipStreamDestroy(cs);
    }
    Work(const matex_factor_s& F, int64_t max_chk) {
        HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        n = F.sym.n;
        V = DevMem(sizeof(double) * n * (MAXM + 1));
        w = DevMem(sizeof(double) * n);
        tmp = DevMem(sizeof(double) * n);
        upd = DevMem(sizeof(double) * std::max<int64_t>(1, F.sym.n_upd));
        partial = DevMem(sizeof(double) * 2 * RED_BLOCKS * (MAXM + 2));
        ks = DevMem(sizeof(KState));
        HIPCHK(hipMemset(ks.p, 0, sizeof(KState)));
        max_checks = std::max<int64_t>(1, max_chk);
        u = DevMem(sizeof(double) * max_checks * MAXM);
        est = DevMem(sizeof(double) * max_checks);
        taus = DevMem(sizeof(double) * max_checks);
        sel = DevMem(sizeof(int32_t) * 2);
        const char* ge = std::getenv("MATEX_GRAPHS");
        use_graphs = ge && ge[0] == '1';
    }
    KState* kst() const { return ks.as<KState>(); }
    const int32_t* done() const { return &ks.as<KState>()->done; }
};

struct KsHost {
    int32_t done, converged, m, breakdown, counter, mdec, ticket, wait_err;   // KState's leading fields
    double beta, est;
};
static_assert(offsetof(KsHost, wait_err) == offsetof(KState, wait_err) &&
              offsetof(KsHost, beta) == offsetof(KState, beta) &&
              offsetof(KsHost, est) == offsetof(KState, est), "KsHost mirrors KState's head");

// A check waits at most this long (100 MHz device clock ticks, 20 s) for its
// iteration; far beyond any one iteration, so reaching it means a fault.
constexpr int64_t TICKET_WAIT_MAX = int64_t(2000000000);

KsHost read_state(const Work& wk, KsHost* pinned, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(pinned, wk.ks.p, sizeof(KsHost), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return *pinned;
}

double read_est(const Work& wk, double* pinned, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(pinned, &wk.kst()->est, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return *pinned;
}

// One Krylov iteration j (0-based): w = M^-1 C v_j, two Gram-Schmidt passes,
// v_{j+1} and column j of Ht.
void iteration_launches(const matex_factor_s& F, int shift, Work& wk, int j, hipStream_t st)
{
    const int64_t n = wk.n;
    double* V = wk.V.as<double>();
    dev_solve(F, shift, V + int64_t(j) * n, F.d_cperm.as<double>(), wk.w.as<double>(),
              wk.tmp.as<double>(), wk.upd.as<double>(), wk.done(), st);
    launch_gs_dots(n, V, n, j + 1, wk.w.as<double>(), wk.partial.as<double>(), wk.kst(), wk.done(), st);
    launch_gs_update(n, V, n, j + 1, wk.w.as<double>(), wk.partial.as<double>(), wk.kst(), wk.done(), st);
    launch_gs_finish(n, V, n, j + 1, wk.w.as<double>(), wk.partial.as<double>(), wk.kst(), wk.done(), st);
}

// With graphs on (MATEX_GRAPHS=1 when the work is made), the launches of
// iteration j with shift k are captured once on the work's capture stream
// (kernels only: no copy or fill) and replayed on st as one graph; every
// argument is fixed for the work's lifetime (the ticket is counted on the
// device).

void krylov_iteration(const matex_factor_s& F, int shift, Work& wk, int j, hipStream_t st)
{
    ++wk.ticket;
    if (!wk.use_graphs) {
        iteration_launches(F, shift, wk, j, st);
        return;
    }
    const int key = shift * (MAXM + 1) + j;
    auto it = wk.graphs.find(key);
    if (it == wk.graphs.end()) {
        if (!wk.gs) HIPCHK(hipStreamCreateWithFlags(&wk.gs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(wk.gs, hipStreamCaptureModeThreadLocal));
        iteration_launches(F, shift, wk, j, wk.gs);
        HIPCHK(hipStreamEndCapture(wk.gs, &g));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        it = wk.graphs.emplace(key, ex).first;
    }
    HIPCHK(hipGraphLaunch(it->second, st));
}

// Host-side timing of the iteration loop (diagnostics, MATEX_HOST_TIMES=1):
// seconds spent enqueuing iterations and waiting for check results.
// With stamps on, the device clock is also written at each iteration's
// start (tag 0), a basis's set-up (tag 1) and its reconstruction's end (tag 2).
struct HostTimes {
    double enqueue_s = 0.0, wait_s = 0.0;
    int64_t iterations = 0, waits = 0;
    int64_t* d_stamps = nullptr;
    int64_t cap = 0;
    std::vector<int8_t> tags;
    void stamp(int tag, hipStream_t st) {
        if (!d_stamps || int64_t(tags.size()) >= cap) return;
        launch_stamp(d_stamps, int64_t(tags.size()), st);
        tags.push_back(int8_t(tag));
    }
};
thread_local HostTimes g_host_times;

// Runs Alg. 1 from the (already normalised) V_0 until a check stops it.
// The estimate of dimension j + 1 runs on the work's check stream while
// the main stream already computes iteration j + 1: the decision lands a
// check later on the host, the next iteration never waits for it, and an
// iteration computed past the decision is discarded (the dimension is set
// back to the decided one). An iteration goes ahead unless the decay of the
// last estimates predicts that the pending check stops: the next estimate
// is taken as the last one times the mean ratio per dimension over the last
// two (at most 1), and a prediction below PRED_KAPPA * tol holds the
// iteration back until the check has landed. A wrong hold costs one check's
// latency, a wrong go-ahead one discarded iteration. With more than two check offsets the
// iterations test only the first and the last; once those pass, one
// evaluation of every offset confirms the decision, and if it fails the
// process continues with every offset tested. This stops at the same
// dimension as testing every offset each time: a failing subset implies a
// failing full set, and the evaluation leaves every offset's vector of the
// current dimension for the next iteration's difference term. Returns the
// final host view of the state (m the decided dimension).
constexpr double PRED_KAPPA = 1.5;

KsHost run_arnoldi(const matex_factor_s& F, int shift, Work& wk, int n_tau, double tol, int m_max,
                   KsHost* pinned, hipStream_t st, int* n_launched = nullptr,
                   std::vector<double>* ests = nullptr)
{
    int launched = 0;
    bool full = n_tau <= 2;
    if (!full) launch_set_ends(wk.sel.as<int32_t>(), n_tau - 1, st);
    // a zero start vector has the state done already: the first check then
    // returns at once and its read shows it
    KsHost h{};
    const double gamma = shift_gamma(F, shift);
    auto launch_iter = [&](int i) {
        const double t0 = now_s();
        g_host_times.stamp(0, st);
        krylov_iteration(F, shift, wk, i, st);
        launched++;
        g_host_times.enqueue_s += now_s() - t0;
        g_host_times.iterations++;
    };
    auto launch_check = [&](int i) {   // dimension i + 1, after iteration i (the last launched)
        launch_wait_ticket(wk.kst(), wk.ticket, TICKET_WAIT_MAX, wk.cs);
        launch_checks(wk.kst(), gamma, wk.taus.as<double>(), full ? nullptr : wk.sel.as<int32_t>(),
                      full ? n_tau : 2, tol, wk.u.as<double>(), wk.est.as<double>(), m_max, 1, i + 1, wk.cs);
        HIPCHK(hipMemcpyAsync(pinned, wk.ks.p, sizeof(KsHost), hipMemcpyDeviceToHost, wk.cs));
    };
    int j = 0;   // next iteration
    double e[3] = {0.0, 0.0, 0.0};   // the last estimates, newest first
    int n_e = 0;
    auto predicts_stop = [&]() {
        if (n_e < 2 || !(e[0] > 0.0) || !(e[1] > 0.0)) return false;
        const double r = n_e >= 3 && e[2] > 0.0 ? std::sqrt(e[0] / e[2]) : e[0] / e[1];
        return e[0] * std::min(r, 1.0) < PRED_KAPPA * tol;
    };
    while (true) {
        if (h.done || j >= m_max) break;
        launch_iter(j);
        launch_check(j);
        ++j;
        int mdec = 0;
        while (true) {
            // iteration j goes ahead of the decision on dimension j unless
            // that decision is predicted to stop
            const bool ahead = j < m_max && !predicts_stop();
            if (ahead) launch_iter(j);
            const double t0 = now_s();
            HIPCHK(hipStreamSynchronize(wk.cs));
            g_host_times.wait_s += now_s() - t0;
            g_host_times.waits++;
            h = *pinned;
            if (h.wait_err) throw HipError{hipErrorLaunchTimeOut, "a check timed out waiting for its iteration"};
            if (ests) ests->push_back(h.est);
            e[2] = e[1];
            e[1] = e[0];
            e[0] = h.est;
            n_e++;
            if (h.done || j >= m_max) { mdec = h.mdec; break; }
            if (!ahead) launch_iter(j);
            launch_check(j);
            ++j;
        }
        // the check stream is idle: the host has seen its last copy land
        launch_set_m(wk.kst(), mdec, st);
        h.m = mdec;
        if (full || !h.converged || mdec == 0) break;
        launch_checks(wk.kst(), gamma, wk.taus.as<double>(), nullptr, n_tau, tol, wk.u.as<double>(),
                      wk.est.as<double>(), m_max, 0, -1, st);
        h = read_state(wk, pinned, st);
        if (h.converged) break;
        full = true;
        if (h.m >= m_max) break;
        launch_resume(wk.kst(), st);
        h.done = 0;
        j = mdec;   // the iteration launched past the decision may have been cut short
    }
    if (n_launched) *n_launched = launched;
    return h;
}

// Algorithmic bytes of one substitution pair on nrhs right-hand sides: every
// nonzero of L read once per sweep (8 B; the exact structural count, not the
// stored panel entries with their explicit zeros) and, per right-hand side,
// each sweep's right-hand side and result (4 x 8 B per row). The panel
// format's own overheads (explicit zeros, update slots, indices) are not
// algorithmic.
int64_t solve_pair_bytes(const Symbolic& s, int nrhs)
{
    return 2 * 8 * s.nnz_exact + int64_t(nrhs) * 4 * 8 * s.n;
}

}  // namespace

// ------------------------------------------------ allocation-free solves

// Scratch of matex_solve_noalloc: a file-scope device array, one per GPU the
// library runs on, held until the process ends. Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address): each device's address comes from hipGetSymbolAddress, taken
// once per device with that device current, and is used instead.
constexpr int64_t NOALLOC_DOUBLES = int64_t(8) << 20;   // 64 MiB
static __device__ __align__(256) double g_noalloc_scratch[NOALLOC_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[MAX_DEVICES] = {};

// The scratch's address on the current device (nullptr and the error text
// set when HIP cannot resolve it).
double* noalloc_scratch(int dev)
{
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_noalloc_scratch));
        if (e != hipSuccess || !ptr) {
            g_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_noalloc_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_noalloc_ptr[dev];
}

}  // namespace

// --------------------------------------------------------------------- ABI

extern "C" {

const char* matex_version(void) { return "matex-mi355x 0.2 (gfx950, fp64)"; }

matex_status matex_sync(void* stream)
{
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(MATEX_E_HIP, std::string("matex_sync: ") + hipGetErrorString(e));
    return MATEX_OK;
}

size_t matex_last_error(char* buf, size_t len)
{
    if (!buf || len == 0) return g_err.size();
    size_t k = std::min(len - 1, g_err.size());
    std::memcpy(buf, g_err.data(), k);
    buf[k] = 0;
    return g_err.size();
}

matex_status matex_factor(const matex_netlist* nl, double gamma, const matex_factor_opts* opts,
                          void* stream, matex_factor_t* out)
{
    (void)stream;
    if (!nl || !out) return fail(MATEX_E_INVALID, "null argument");
    *out = nullptr;
    const int64_t n = nl->n;
    if (n <= 0 || n > INT32_MAX - 1) return fail(MATEX_E_INVALID, "n out of range");
    if (!(gamma > 0.0)) return fail(MATEX_E_INVALID, "gamma must be > 0");
    if (nl->n_branch < 0 || nl->n_pad < 0) return fail(MATEX_E_INVALID, "negative count");
    if ((nl->n_branch && (!nl->br_a || !nl->br_b || !nl->br_g)) || !nl->c_node ||
        (nl->n_pad && (!nl->pad_node || !nl->pad_g)))
        return fail(MATEX_E_INVALID, "null array");
    for (int64_t k = 0; k < nl->n_branch; ++k) {
        if (nl->br_a[k] < 0 || nl->br_a[k] >= n || nl->br_b[k] < 0 || nl->br_b[k] >= n ||
            nl->br_a[k] == nl->br_b[k])
            return fail(MATEX_E_INVALID, "branch " + std::to_string(k) + " has a bad node id");
        if (!(nl->br_g[k] > 0.0)) return fail(MATEX_E_INVALID, "branch conductance must be > 0");
    }
    for (int64_t i = 0; i < n; ++i)
        if (!(nl->c_node[i] > 0.0)) return fail(MATEX_E_INVALID, "capacitance must be > 0");
    for (int32_t k = 0; k < nl->n_pad; ++k) {
        if (nl->pad_node[k] < 0 || nl->pad_node[k] >= n) return fail(MATEX_E_INVALID, "pad node id");
        if (!(nl->pad_g[k] > 0.0)) return fail(MATEX_E_INVALID, "pad conductance must be > 0");
    }
    int n_shifts = (opts && opts->n_shifts > 0) ? opts->n_shifts : 6;
    int leaf = (opts && opts->leaf_max > 0) ? opts->leaf_max : 16;
    const int32_t subtree = opts ? opts->subtree_levels : 0;
    const int32_t bsched = opts ? opts->batched_schedule : 0;
    if (bsched < 0 || bsched > 2) return fail(MATEX_E_INVALID, "batched_schedule must be 0, 1 or 2");
    if (n_shifts > 12) return fail(MATEX_E_INVALID, "n_shifts must be <= 12");
    try {
        auto F = std::make_unique<matex_factor_s>();
        HIPCHK(hipGetDevice(&F->device));
        F->gamma = gamma;
        F->vdd = nl->vdd;
        for (int k = 0; k < n_shifts; ++k) F->gammas.push_back(gamma * std::pow(10.0, -k));
        double t0 = now_s();
        Csr G = assemble_g(n, nl->n_branch, nl->br_a, nl->br_b, nl->br_g, nl->n_pad,
                           nl->pad_node, nl->pad_g);
        F->sym = analyse(G, nl->coord, leaf);
        const Symbolic& s = F->sym;
        if (int64_t(s.max_nr) * 8 > 60 * 1024)
            return fail(MATEX_E_UNSUPPORTED, "a supernode has more rows than the sweep kernels stage in LDS");
        double t1 = now_s();
        // numeric: all shifts and G in parallel host threads
        std::vector<std::vector<double>> Wh(n_shifts + 1);
        std::vector<int64_t> bad(n_shifts + 1, 0);
        std::vector<double> zero(n, 0.0);
        std::vector<std::thread> th;
        for (int k = 0; k <= n_shifts; ++k) {
            th.emplace_back([&, k]() {
                if (k < n_shifts) bad[k] = factor_panels(s, G, F->gammas[k], nl->c_node, Wh[k], 1);
                else bad[k] = factor_panels(s, G, 1.0, zero.data(), Wh[k], 1);
            });
        }
        for (auto& t : th) t.join();
        for (int k = 0; k <= n_shifts; ++k)
            if (bad[k])
                return fail(MATEX_E_NOT_SPD, std::string(k < n_shifts ? "C + gamma G" : "G") +
                                                 " is not positive definite (pivot at column " +
                                                 std::to_string(bad[k] - 1) + ")");
        double t2 = now_s();
        // upload
        std::vector<int32_t> c0, nc, nr;
        std::vector<int64_t> roff, w, u;
        for (auto& q : s.sn) {
            c0.push_back(q.c0); nc.push_back(q.nc); nr.push_back(q.nr);
            roff.push_back(q.roff); w.push_back(q.w); u.push_back(q.u);
        }
        F->d_c0 = upload(c0); F->d_nc = upload(nc); F->d_nr = upload(nr);
        F->d_roff = upload(roff); F->d_w = upload(w); F->d_u = upload(u);
        F->d_rows = upload(s.rows.empty() ? std::vector<int32_t>{0} : s.rows);
        F->d_child_ptr = upload(s.child_ptr);
        F->d_child_idx = upload(s.child_idx.empty() ? std::vector<int32_t>{0} : s.child_idx);
        F->d_relidx = upload(s.relidx.empty() ? std::vector<int32_t>{0} : s.relidx);
        F->d_perm = upload(s.perm);
        F->d_iperm = upload(s.iperm);
        std::vector<double> cperm(n);
        for (int64_t k = 0; k < n; ++k) cperm[k] = nl->c_node[s.perm[k]];
        F->d_cperm = upload(cperm);
        F->c_host.assign(nl->c_node, nl->c_node + n);
        {
            // G with rows and columns in the factor's order
            std::vector<int32_t> rp(n + 1, 0), ci;
            std::vector<double> gv;
            ci.reserve(G.ci.size());
            gv.reserve(G.v.size());
            for (int64_t r = 0; r < n; ++r) {
                const int32_t o = s.perm[r];
                for (int64_t q = G.rp[o]; q < G.rp[o + 1]; ++q) {
                    ci.push_back(s.iperm[G.ci[q]]);
                    gv.push_back(G.v[q]);
                }
                rp[r + 1] = int32_t(ci.size());
            }
            F->d_grp = upload(rp);
            F->d_gci = upload(ci);
            F->d_gv = upload(gv);
        }
        for (int k = 0; k <= n_shifts; ++k) {
            F->d_W.push_back(upload(Wh[k]));
            std::vector<double>().swap(Wh[k]);
        }
        F->dsym = DevSym{n, F->d_c0.as<int32_t>(), F->d_nc.as<int32_t>(), F->d_nr.as<int32_t>(),
                         F->d_roff.as<int64_t>(), F->d_w.as<int64_t>(), F->d_u.as<int64_t>(),
                         F->d_rows.as<int32_t>(), F->d_child_ptr.as<int32_t>(),
                         F->d_child_idx.as<int32_t>(), F->d_relidx.as<int32_t>()};
        build_tasks(*F, subtree);
        if (bsched == 0) tune_batched(*F, static_cast<hipStream_t>(stream));
        if (bsched == 2)
            for (int lv = 0; lv < F->sym.n_levels; ++lv) {
                const int c = int(F->bcand[size_t(lv)].size()) - 1;
                const int k = F->bcand[size_t(lv)][size_t(c)].name == "wave" ? c : 0;
                F->blevels[size_t(lv)] = F->bcand[size_t(lv)][size_t(k)].lv;
                F->bchoice[size_t(lv)] = {k, k};
            }
        matex_factor_info& I = F->info;
        I.n = n;
        I.nnz_l = s.nnz_l;
        I.panel_doubles = s.n_w;
        I.n_supernodes = int32_t(s.sn.size());
        I.n_levels = s.n_levels;
        I.n_shifts = n_shifts;
        I.max_nr = s.max_nr;
        I.gamma = gamma;
        I.seconds_analyse = t1 - t0;
        I.seconds_numeric = t2 - t1;
        I.device_bytes = F->held_bytes();
        I.subtree_levels = F->tree.n_levels;
        I.subtree_blocks = F->tree.n_blocks;
        I.nnz_l_exact = s.nnz_exact;
        I.n_upd = s.n_upd;
        *out = F.release();
        return MATEX_OK;
    } catch (const HipError& e) {
        return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc&) {
        return fail(MATEX_E_OOM, "host allocation failed");
    }
}

matex_status matex_factor_free(matex_factor_t f)
{
    delete f;
    return MATEX_OK;
}

size_t matex_factor_describe(matex_factor_t f, char* buf, size_t len)
{
    if (!f) return 0;
    const std::string d = describe_batched(*f);
    if (buf && len) {
        const size_t k = std::min(len - 1, d.size());
        std::memcpy(buf, d.data(), k);
        buf[k] = 0;
    }
    return d.size();
}

matex_status matex_factor_get_info(matex_factor_t f, matex_factor_info* info)
{
    if (!f || !info) return fail(MATEX_E_INVALID, "null argument");
    *info = f->info;
    return MATEX_OK;
}

matex_status matex_solve_noalloc(matex_factor_t f, int32_t which, const double* d_b, const double* d_scale,
                                 double* d_x, void* stream)
{
    if (!f || !d_b || !d_x) return fail(MATEX_E_INVALID, "bad argument");
    const int n_shifts = int(f->gammas.size());
    if (which < -1 || which >= n_shifts) return fail(MATEX_E_INVALID, "factor index out of range");
    if (d_b == d_x) return fail(MATEX_E_INVALID, "d_b and d_x may not alias");
    const int64_t n = f->sym.n, n_upd = std::max<int64_t>(1, f->sym.n_upd);
    // b, x (also the scale until the backward sweep), the forward result and
    // the update slots
    const int64_t need = 3 * n + n_upd;
    if (need > NOALLOC_DOUBLES)
        return fail(MATEX_E_INVALID, "matex_solve_noalloc: the factor needs " + std::to_string(need) +
                                         " doubles of scratch (3 n + update slots), more than its " +
                                         std::to_string(NOALLOC_DOUBLES) + " (64 MiB)");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return fail(MATEX_E_HIP, "matex_solve_noalloc: no usable current device");
    double* sp = noalloc_scratch(dev);
    if (!sp) return MATEX_E_HIP;
    const int idx = which < 0 ? n_shifts : which;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* bp = sp;
    double* xp = sp + n;
    double* tmp = sp + 2 * n;
    double* upd = sp + 3 * n;
    const int32_t* perm = f->d_perm.as<int32_t>();
    try {
        launch_gather_perm(n, perm, d_b, bp, n, n, 1, st);
        const double* scale_p = nullptr;
        if (d_scale) {
            // the scale is read by the forward sweep only; the backward sweep
            // then writes x over it
            launch_gather_perm(n, perm, d_scale, xp, n, n, 1, st);
            scale_p = xp;
        }
        dev_solve(*f, idx, bp, scale_p, xp, tmp, upd, nullptr, st);
        launch_scatter_perm(n, perm, xp, d_x, n, n, 1, st);
        HIPCHK(hipGetLastError());
        return MATEX_OK;
    } catch (const HipError& e) {
        return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
}

matex_status matex_solve(matex_factor_t f, int32_t which, int32_t nrhs, const double* d_b,
                         const double* d_scale, double* d_x, void* stream)
{
    if (!f || !d_b || !d_x || nrhs < 0) return fail(MATEX_E_INVALID, "bad argument");
    const int n_shifts = int(f->gammas.size());
    if (which < -1 || which >= n_shifts) return fail(MATEX_E_INVALID, "factor index out of range");
    if (d_b == d_x) return fail(MATEX_E_INVALID, "d_b and d_x may not alias");
    const int idx = which < 0 ? n_shifts : which;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = f->sym.n;
    try {
        DevMem bp(sizeof(double) * n), xp(sizeof(double) * n), tmp(sizeof(double) * n),
            upd(sizeof(double) * std::max<int64_t>(1, f->sym.n_upd)), sc;
        const double* scale_p = nullptr;
        if (d_scale) {
            sc = DevMem(sizeof(double) * n);
            launch_gather_perm(n, f->d_perm.as<int32_t>(), d_scale, sc.as<double>(), n, n, 1, st);
            scale_p = sc.as<double>();
        }
        if (nrhs > 1) {
            // multi-right-hand-side sweeps, RMAX columns at a time
            const int Rm = std::min<int>(RMAX, nrhs);
            const size_t nr = sizeof(double) * size_t(n) * Rm;
            DevMem Bi(nr), Xi(nr);
            BatchScratch bs(*f, Rm);
            for (int r0 = 0; r0 < nrhs; r0 += RMAX) {
                const int R = std::min<int>(RMAX, nrhs - r0);
                launch_b_interleave(n, R, f->d_perm.as<int32_t>(), d_b + int64_t(r0) * n, Bi.as<double>(), st);
                dev_solve_batched(*f, idx, R, Bi.as<double>(), scale_p, Xi.as<double>(), bs, st);
                launch_b_deinterleave(n, R, f->d_perm.as<int32_t>(), Xi.as<double>(), d_x + int64_t(r0) * n,
                                      st);
            }
            HIPCHK(hipStreamSynchronize(st));
            return MATEX_OK;
        }
        for (int r = 0; r < nrhs; ++r) {
            launch_gather_perm(n, f->d_perm.as<int32_t>(), d_b + int64_t(r) * n, bp.as<double>(), n,
                               n, 1, st);
            dev_solve(*f, idx, bp.as<double>(), scale_p, xp.as<double>(), tmp.as<double>(),
                      upd.as<double>(), nullptr, st);
            launch_scatter_perm(n, f->d_perm.as<int32_t>(), xp.as<double>(), d_x + int64_t(r) * n,
                                n, n, 1, st);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        return MATEX_OK;
    } catch (const HipError& e) {
        return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
}

matex_status matex_time_solves(matex_factor_t f, int32_t which, int32_t nrhs, int32_t reps,
                               double* seconds, double* bytes, void* stream)
{
    if (!f || !seconds || !bytes || reps <= 0) return fail(MATEX_E_INVALID, "bad argument");
    if (nrhs < 1 || nrhs > RMAX) return fail(MATEX_E_INVALID, "nrhs must be in 1..64");
    const int n_shifts = int(f->gammas.size());
    if (which < -1 || which >= n_shifts) return fail(MATEX_E_INVALID, "factor index out of range");
    const int idx = which < 0 ? n_shifts : which;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = f->sym.n;
    if (nrhs > 1) {
        try {
            const size_t nr = sizeof(double) * size_t(n) * nrhs;
            DevMem b(nr), x(nr);
            BatchScratch bs(*f, nrhs);
            HIPCHK(hipMemsetAsync(b.p, 0, b.bytes, st));
            const double* sc = idx < n_shifts ? f->d_cperm.as<double>() : nullptr;
            auto pair = [&]() { dev_solve_batched(*f, idx, nrhs, b.as<double>(), sc, x.as<double>(), bs, st); };
            pair();   // warm
            hipEvent_t e0, e1;
            HIPCHK(hipEventCreate(&e0));
            HIPCHK(hipEventCreate(&e1));
            HIPCHK(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) pair();
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            *seconds = 1e-3 * double(ms) / reps;
            *bytes = double(solve_pair_bytes(f->sym, nrhs));
            return MATEX_OK;
        } catch (const HipError& e) {
            return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
        }
    }
    try {
        DevMem b(sizeof(double) * n), x(sizeof(double) * n), tmp(sizeof(double) * n),
            upd(sizeof(double) * std::max<int64_t>(1, f->sym.n_upd));
        HIPCHK(hipMemsetAsync(b.p, 0, b.bytes, st));
        const double* sc = idx < n_shifts ? f->d_cperm.as<double>() : nullptr;
        dev_solve(*f, idx, b.as<double>(), sc, x.as<double>(), tmp.as<double>(), upd.as<double>(),
                  nullptr, st);   // warm
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r)
            dev_solve(*f, idx, b.as<double>(), sc, x.as<double>(), tmp.as<double>(), upd.as<double>(),
                      nullptr, st);
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipStreamSynchronize(st));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *seconds = 1e-3 * double(ms) / reps;
        *bytes = double(solve_pair_bytes(f->sym, 1));
        return MATEX_OK;
    } catch (const HipError& e) {
        return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
}

matex_status matex_krylov_step(matex_factor_t f, int32_t shift, int32_t nrhs, const double* d_v,
                               int32_t n_tau, const double* tau, int32_t m_max, double tol,
                               double* d_out, int32_t* m_used, double* est, void* stream)
{
    if (!f || !d_v || !d_out || !tau || nrhs < 0 || n_tau <= 0)
        return fail(MATEX_E_INVALID, "bad argument");
    if (shift < -1 || shift >= int(f->gammas.size())) return fail(MATEX_E_INVALID, "shift out of range");
    if (shift < 0) shift = int(f->gammas.size());   // the inverted space, X1 = G
    if (m_max < 1 || m_max > MAXM) return fail(MATEX_E_INVALID, "m_max must be in 1..32");
    if (!(tol >= 0.0)) return fail(MATEX_E_INVALID, "tol must be >= 0");
    for (int k = 0; k < n_tau; ++k)
        if (!(tau[k] > 0.0)) return fail(MATEX_E_INVALID, "tau must be > 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = f->sym.n;
    bool all_conv = true;
    try {
        Work wk(*f, n_tau);
        PinnedMem pin(256);
        DevMem zero(sizeof(double) * n), acc(sizeof(double) * n);
        HIPCHK(hipMemsetAsync(zero.p, 0, zero.bytes, st));
        HIPCHK(hipMemcpyAsync(wk.taus.p, tau, sizeof(double) * n_tau, hipMemcpyHostToDevice, st));
        double* V = wk.V.as<double>();
        for (int r = 0; r < nrhs; ++r) {
            // V_0 = P v_r / ||v_r|| (setup with y0 = z2 = 0)
            launch_gather_perm(n, f->d_perm.as<int32_t>(), d_v + int64_t(r) * n, acc.as<double>(),
                               n, n, 1, st);
            launch_setup_v(n, acc.as<double>(), zero.as<double>(), zero.as<double>(), V,
                           wk.partial.as<double>(), wk.kst(), st);
            launch_normalize_v(n, V, wk.partial.as<double>(), wk.kst(), st);
            KsHost h = run_arnoldi(*f, shift, wk, n_tau, tol, m_max, pin.as<KsHost>(), st);
            if (!h.converged) all_conv = false;
            if (m_used) m_used[r] = h.m;
            if (est) est[r] = read_est(wk, pin.as<double>() + 8, st);
            for (int k = 0; k < n_tau; ++k) {
                // out = beta V u(tau_k), reconstructed with y0 = z1 = z2 = 0
                launch_recon_full(n, 0.0, wk.u.as<double>() + int64_t(k) * MAXM, wk.kst(), V, n,
                                  acc.as<double>(), zero.as<double>(), zero.as<double>(),
                                  zero.as<double>(), st);
                launch_scatter_perm(n, f->d_perm.as<int32_t>(), acc.as<double>(),
                                    d_out + n * (r + int64_t(nrhs) * k), n, n, 1, st);
            }
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    } catch (const HipError& e) {
        return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    if (!all_conv) return fail(MATEX_E_NOCONV, "estimate >= tol at m_max");
    return MATEX_OK;
}

}  // extern "C"

// ------------------------------------------------------------ transient

namespace {

constexpr double FS = 1e-15;

struct Segment {
    // planner output for one transition spot: slope changes at that time
    int64_t t;
    std::vector<int32_t> node;   // permuted rows
    std::vector<double> dslope;  // A/s
};

// Transition spots of one subtask and the slope changes of its sources at
// each (Sec. 2.2: the input is linear between spots; Sec. 3.1: LTS).
std::vector<Segment> plan_spots(const matex_problem* p, const std::vector<int32_t>& srcs,
                                const std::vector<int32_t>& iperm)
{
    std::map<int64_t, std::map<int32_t, double>> ev;
    ev[0];
    ev[p->t_end];
    for (int32_t k : srcs) {
        const int64_t d = p->delay[k], r = p->rise[k], w = p->width[k], f = p->fall[k];
        const double a = p->amp[k];
        const int32_t row = iperm[p->node[k]];
        const int64_t t[4] = {d, d + r, d + r + w, d + r + w + f};
        const double ds[4] = {a / (double(r) * FS), -a / (double(r) * FS), -a / (double(f) * FS),
                              a / (double(f) * FS)};
        for (int q = 0; q < 4; ++q)
            if (t[q] >= 0 && t[q] < p->t_end) ev[t[q]][row] += ds[q];
    }
    std::vector<Segment> out;
    for (auto& kv : ev) {
        Segment s;
        s.t = kv.first;
        for (auto& e : kv.second) {
            s.node.push_back(e.first);
            s.dslope.push_back(e.second);
        }
        out.push_back(std::move(s));
    }
    return out;
}

// Check offsets of a step from t_a towards the next spot t_next: the output
// times in (t_a, t_next] and the spot itself (Alg. 2 reuses one basis for
// every snapshot before the next spot). *snap0: index of the first output
// after t_a.
std::vector<int64_t> step_offsets(const std::vector<int64_t>& tout, int64_t t_a, int64_t t_next,
                                  int32_t* snap0)
{
    auto lo = std::upper_bound(tout.begin(), tout.end(), t_a);
    auto hi = std::upper_bound(tout.begin(), tout.end(), t_next);
    std::vector<int64_t> offs;
    for (auto it = lo; it != hi; ++it) offs.push_back(*it - t_a);
    if (offs.empty() || offs.back() != t_next - t_a) offs.push_back(t_next - t_a);
    *snap0 = int32_t(lo - tout.begin());
    return offs;
}

// Shift ladder: the largest gamma_k with tau_1 >= ratio * gamma_k, else the
// smallest shift.
int ladder_shift(const std::vector<double>& gammas, int64_t off0, double ratio)
{
    for (size_t k = 0; k < gammas.size(); ++k)
        if (double(off0) * FS >= ratio * gammas[k]) return int(k);
    return int(gammas.size()) - 1;
}

// Below the top shift a step ends at its last check offset <= 10 gamma_k.
void ladder_cut(std::vector<int64_t>& offs, const std::vector<double>& gammas, int k)
{
    if (k == 0) return;
    const double lim = 10.0 * gammas[k];
    size_t cnt = 0;
    while (cnt < offs.size() && double(offs[cnt]) * FS <= lim) cnt++;
    offs.resize(std::max<size_t>(1, cnt));
}

// Offsets of a halved step: those below hstep, then hstep.
std::vector<int64_t> halved_offsets(const std::vector<int64_t>& offs, int64_t hstep)
{
    std::vector<int64_t> o2;
    for (int64_t v : offs)
        if (v < hstep) o2.push_back(v);
    o2.push_back(hstep);
    return o2;
}

struct NoConv {
    std::string msg;
};

// ------------------------------------------------- batched subtasks

// Host staging of one device table: consecutive typed arrays packed into a
// pinned buffer and uploaded with one copy; the device copy has the same
// layout.
struct Packer {
    char* h;
    char* d;
    size_t size, off = 0;
    Packer(const PinnedMem& hm, const DevMem& dm, size_t sz)
        : h(hm.as<char>()), d(static_cast<char*>(dm.p)), size(sz) {}
    template <class T> T* take(size_t count, T** dev) {
        off = (off + 15) & ~size_t(15);
        if (off + sizeof(T) * count > size) throw HipError{hipErrorInvalidValue, "staging table overflow"};
        T* hp = reinterpret_cast<T*>(h + off);
        *dev = reinterpret_cast<T*>(d + off);
        off += sizeof(T) * count;
        return hp;
    }
    void upload(hipStream_t st) {
        if (off) HIPCHK(hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, st));
    }
};

// Per-subtask planner state.
struct BCol {
    std::vector<Segment> spots;
    size_t k_spot = 0;
    int64_t t_a = 0;
    std::vector<int64_t> offs, cand;
    int32_t snap0 = 0;
    int ksh = 0;
    int64_t hstep = 0;
};

// Buffers of one batch of up to RMAX subtasks; n x R arrays row-interleaved.
struct BatchWork {
    int64_t n;
    int Rmax, cap;
    DevMem V, w, partial, ks, y, y0, z1, z2, s, u, est, Yout, probe_perm;
    BatchScratch sc;
    size_t tab_bytes, ev_bytes;
    PinnedMem h_pre, h_post, h_ks;
    DevMem d_pre, d_post;
    std::unique_ptr<PinnedMem> h_ev;
    DevMem d_ev;
    static size_t table_bytes(int R, int cap) {
        const size_t e = size_t(R) * cap;
        return e * (2 * sizeof(double) + 3 * sizeof(int32_t)) + size_t(R) * 8 * sizeof(double) + 16 * 16;
    }
    BatchWork(const matex_factor_s& F, int Rmax_, int cap_, int64_t n_po)
        : n(F.sym.n), Rmax(Rmax_), cap(cap_), sc(F, Rmax_), tab_bytes(table_bytes(Rmax_, cap_)),
          ev_bytes(1 << 16), h_pre(tab_bytes), h_post(tab_bytes), h_ks(sizeof(KState) * RMAX)
    {
        const size_t nr = sizeof(double) * size_t(n) * Rmax;
        V = DevMem(nr * (MAXM + 1));
        HIPCHK(hipMemset(V.p, 0, V.bytes));
        w = DevMem(nr);
        partial = DevMem(sizeof(double) * size_t(B_RED_BLOCKS) * Rmax * (MAXM + 2));
        ks = DevMem(sizeof(KState) * Rmax);
        HIPCHK(hipMemset(ks.p, 0, ks.bytes));
        y = DevMem(nr); y0 = DevMem(nr); z1 = DevMem(nr); z2 = DevMem(nr); s = DevMem(nr);
        u = DevMem(sizeof(double) * size_t(Rmax) * cap * MAXM);
        est = DevMem(sizeof(double) * size_t(Rmax) * cap);
        Yout = DevMem(sizeof(double) * std::max<int64_t>(1, n_po) * Rmax);
        d_pre = DevMem(tab_bytes);
        d_post = DevMem(tab_bytes);
        h_ev.reset(new PinnedMem(ev_bytes));
        d_ev = DevMem(ev_bytes);
    }
    double* Vd() const { return V.as<double>(); }
    KState* kst() const { return ks.as<KState>(); }
};

std::vector<KsHost> read_states(const BatchWork& bw, int R, hipStream_t st)
{
    KsHost* h = bw.h_ks.as<KsHost>();
    HIPCHK(hipMemcpy2DAsync(h, sizeof(KsHost), bw.ks.p, sizeof(KState), sizeof(KsHost), R,
                            hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return std::vector<KsHost>(h, h + R);
}

// Checks table of the columns in cols_in: every offset off_of(r) is
// uploaded; the checked ones are all of them when all_of(r), else the first
// and the last. `extra` is packed after the table (ext = its device copy).
struct CheckTab {
    double* taus = nullptr;
    int32_t *off = nullptr, *active = nullptr, *col = nullptr, *idx = nullptr, *coff = nullptr,
            *ccnt = nullptr, *ext = nullptr;
    int n_chk = 0;
};

template <class OffsOf, class AllOf>
CheckTab build_checks(BatchWork& bw, int R, const std::vector<int>& cols_in, OffsOf off_of, AllOf all_of,
                      const std::vector<int32_t>& extra, hipStream_t st)
{
    size_t tot = 0, nsel = 0;
    for (int r : cols_in) {
        const size_t c = off_of(r).size();
        tot += c;
        nsel += (all_of(r) || c <= 2) ? c : 2;
    }
    Packer pk(bw.h_pre, bw.d_pre, bw.tab_bytes);
    CheckTab t;
    double* ht = pk.take<double>(std::max<size_t>(1, tot), &t.taus);
    int32_t* hoff = pk.take<int32_t>(R, &t.off);
    int32_t* hact = pk.take<int32_t>(R, &t.active);
    int32_t* hcoff = pk.take<int32_t>(R, &t.coff);
    int32_t* hccnt = pk.take<int32_t>(R, &t.ccnt);
    int32_t* hcol = pk.take<int32_t>(std::max<size_t>(1, nsel), &t.col);
    int32_t* hidx = pk.take<int32_t>(std::max<size_t>(1, nsel), &t.idx);
    int32_t* hext = pk.take<int32_t>(std::max<size_t>(1, extra.size()), &t.ext);
    std::fill(hoff, hoff + R, 0);
    std::fill(hact, hact + R, 0);
    std::fill(hcoff, hcoff + R, 0);
    std::fill(hccnt, hccnt + R, 0);
    std::copy(extra.begin(), extra.end(), hext);
    size_t q = 0, e = 0;
    for (int r : cols_in) {
        const std::vector<int64_t>& of = off_of(r);
        const int32_t c = int32_t(of.size());
        hoff[r] = int32_t(q);
        hact[r] = 1;
        for (int32_t k = 0; k < c; ++k) ht[q + k] = double(of[k]) * FS;
        q += c;
        hcoff[r] = int32_t(e);
        if (all_of(r) || c <= 2) {
            for (int32_t k = 0; k < c; ++k, ++e) { hcol[e] = r; hidx[e] = k; }
        } else {
            hcol[e] = r; hidx[e] = 0; ++e;
            hcol[e] = r; hidx[e] = c - 1; ++e;
        }
        hccnt[r] = int32_t(e) - hcoff[r];
    }
    t.n_chk = int(e);
    pk.upload(st);
    return t;
}

void launch_tab_checks(const matex_factor_s& F, BatchWork& bw, const CheckTab& t, int k, double tol, int m_max,
                       int update, hipStream_t st)
{
    launch_b_checks(bw.kst(), shift_gamma(F, k), t.taus, t.off, bw.cap, t.col, t.idx, t.coff, t.ccnt, t.n_chk, tol,
                    bw.u.as<double>(), bw.est.as<double>(), m_max, update, st);
}

// One lockstep pass of Alg. 1 with shift k for the subtasks in grp (the
// others inactive): one multi-right-hand-side substitution pair per Krylov
// iteration for the whole batch, then per-subtask Gram-Schmidt and checks.
// Check offsets as in the one-subtask path: the first and the last while
// iterating, every offset to confirm, every offset from then on for a
// subtask whose confirmation failed.
std::vector<KsHost> run_pass(const matex_factor_s& F, BatchWork& bw, int R, int k,
                             const std::vector<int>& grp, std::vector<BCol>& cols, double tol,
                             int m_max, int& m_guess, matex_stats& S, hipStream_t st)
{
    const int64_t n = bw.n;
    std::vector<char> full(R, 0);
    auto offs_of = [&](int r) -> const std::vector<int64_t>& { return cols[r].offs; };
    auto mode_of = [&](int r) { return full[r] != 0; };
    CheckTab t = build_checks(bw, R, grp, offs_of, mode_of, {}, st);
    double* V = bw.Vd();
    launch_b_setup(n, R, bw.y.as<double>(), bw.y0.as<double>(), bw.z2.as<double>(), V,
                   bw.partial.as<double>(), bw.kst(), t.active, st);
    std::vector<KsHost> hs = read_states(bw, R, st);
    auto all_done = [&]() {
        for (int r : grp)
            if (!hs[r].done) return false;
        return true;
    };
    int j = 0, chunk = std::max(1, std::min(m_guess, m_max));
    while (true) {
        while (!all_done() && j < m_max) {
            const int stop = std::min(m_max, j + chunk);
            for (; j < stop; ++j) {
                dev_solve_batched(F, k, R, V + int64_t(j) * n * R, F.d_cperm.as<double>(), bw.w.as<double>(),
                                  bw.sc, st);
                launch_b_gs(n, R, V, j + 1, bw.w.as<double>(), bw.partial.as<double>(), bw.kst(), st);
                launch_tab_checks(F, bw, t, k, tol, m_max, 1, st);
                S.solve_pairs_m++;
            }
            hs = read_states(bw, R, st);
            chunk = 1;
        }
        std::vector<int> ver;
        for (int r : grp)
            if (!full[r] && hs[r].converged && hs[r].m > 0 && cols[r].offs.size() > 2) ver.push_back(r);
        if (ver.empty()) break;
        CheckTab tv = build_checks(bw, R, ver, offs_of, [](int) { return true; }, {}, st);
        launch_tab_checks(F, bw, tv, k, tol, m_max, 0, st);
        hs = read_states(bw, R, st);
        std::vector<int32_t> res;
        for (int r : ver) {
            full[r] = 1;
            if (!hs[r].converged && hs[r].m < m_max) res.push_back(r);
        }
        if (res.empty()) break;
        t = build_checks(bw, R, grp, offs_of, mode_of, res, st);
        launch_b_resume(bw.kst(), t.ext, int(res.size()), st);
        for (int r : res) hs[r].done = 0;
    }
    int mx = 0;
    for (int r : grp) {
        S.bases++;
        S.krylov_dims += hs[r].m;
        S.m_peak = std::max(S.m_peak, hs[r].m);
        mx = std::max(mx, hs[r].m);
    }
    if (mx > 0) m_guess = mx;
    return hs;
}

// Snapshots at the probes and the step-end state of the subtasks in fin.
void reconstruct(BatchWork& bw, int R, const std::vector<int>& fin, std::vector<BCol>& cols,
                 const std::vector<int64_t>& tout, int n_probe, int n_out, matex_stats& S,
                 hipStream_t st)
{
    size_t n_ent = 0;
    for (int r : fin) {
        const BCol& c = cols[r];
        const int64_t t_b = c.t_a + c.offs.back();
        for (int32_t q = c.snap0; q < int32_t(tout.size()) && tout[q] <= t_b; ++q) n_ent++;
    }
    Packer pk(bw.h_post, bw.d_post, bw.tab_bytes);
    double *d_tau, *d_ctau;
    int32_t *d_col, *d_t, *d_u, *d_cu, *d_fin;
    double* h_tau = pk.take<double>(std::max<size_t>(1, n_ent), &d_tau);
    double* h_ctau = pk.take<double>(R, &d_ctau);
    int32_t* h_col = pk.take<int32_t>(std::max<size_t>(1, n_ent), &d_col);
    int32_t* h_t = pk.take<int32_t>(std::max<size_t>(1, n_ent), &d_t);
    int32_t* h_u = pk.take<int32_t>(std::max<size_t>(1, n_ent), &d_u);
    int32_t* h_cu = pk.take<int32_t>(R, &d_cu);
    int32_t* h_fin = pk.take<int32_t>(R, &d_fin);
    std::fill(h_ctau, h_ctau + R, 0.0);
    std::fill(h_cu, h_cu + R, 0);
    std::fill(h_fin, h_fin + R, 0);
    size_t e = 0;
    for (int r : fin) {
        const BCol& c = cols[r];
        const int64_t t_b = c.t_a + c.offs.back();
        for (int32_t q = c.snap0; q < int32_t(tout.size()) && tout[q] <= t_b; ++q, ++e) {
            h_col[e] = r;
            h_t[e] = q;
            h_tau[e] = double(c.offs[q - c.snap0]) * FS;
            h_u[e] = r * bw.cap + (q - c.snap0);
        }
        h_ctau[r] = double(c.offs.back()) * FS;
        h_cu[r] = r * bw.cap + int32_t(c.offs.size()) - 1;
        h_fin[r] = 1;
    }
    pk.upload(st);
    launch_b_recon_probes(bw.n, R, n_probe, bw.probe_perm.as<int32_t>(), int(n_ent), d_col, d_t, d_tau, d_u,
                          bw.u.as<double>(), bw.kst(), bw.Vd(), bw.y0.as<double>(), bw.z1.as<double>(),
                          bw.z2.as<double>(), bw.Yout.as<double>(), n_out, st);
    launch_b_recon_full(bw.n, R, d_ctau, d_cu, bw.u.as<double>(), bw.kst(), d_fin, bw.Vd(),
                        bw.y.as<double>(), bw.y0.as<double>(), bw.z1.as<double>(), bw.z2.as<double>(), st);
    for (int r : fin) {
        cols[r].t_a += cols[r].offs.back();
        S.segments++;
    }
}

// One multi-right-hand-side pair on the batch's basis with ragged inputs
// (right-hand side r is block ks[r].m of V): w = (C + gamma_k G)^-1 C v.
void dev_solve_batched_ragged(const matex_factor_s& F, int which, int R, BatchWork& bw, hipStream_t st)
{
    const double* W = F.d_W[size_t(which)].as<double>();
    const int L = F.sym.n_levels;
    double* yf = bw.sc.yf.as<double>();
    double* U = bw.sc.U.as<double>();
    double* P = bw.sc.P.as<double>();
    for (int lv = 0; lv < L; ++lv)
        launch_b_forward(F.dsym, F.bas, F.blevels[size_t(lv)], R, W, bw.Vd(), F.d_cperm.as<double>(), yf, U, P, st,
                         bw.kst());
    for (int lv = L - 1; lv >= 0; --lv) launch_b_backward(F.dsym, F.blevels[size_t(lv)], R, W, yf, bw.w.as<double>(), P, st);
}

// Solved columns of the pulse timings (subtasks that advance independently):
// within each subtask of a batch, the sources of one timing (delay, rise,
// width, fall) form one column q with weight vector b_q (their amplitudes at
// their rows), and Z1[:, q] = G^-1 b_q, Z2[:, q] = G^-1 C Z1[:, q]. The
// subtask's slope vector is sum_q sigma_q(t) b_q with sigma_q the unit
// pulse's slope, so at a transition spot its z1 and z2 (Eq. 6) change by the
// change of sigma_q times these columns: no solve with G during the run.
struct TimingCols {
    struct Col {
        int32_t sub;                 // subtask (column of the batch)
        int64_t d, r, w, f;          // pulse timing (fs)
    };
    std::vector<Col> col;
    DevMem Z;                        // Z1 then Z2, n x columns each
    int64_t n = 0;
    const double* Z1() const { return Z.as<double>(); }
    const double* Z2() const { return Z.as<double>() + n * int64_t(col.size()); }
};

// The timing columns of subtasks b0 .. b0 + R - 1 and their solves (64 at a
// time with the G factor). Returns false, with nothing allocated, when they
// would take more than half the free device memory.
bool timing_cols(const matex_factor_s& F, const matex_problem* p,
                 const std::vector<std::vector<int32_t>>& subtasks, int b0, int R, BatchWork& bw,
                 TimingCols& tc, matex_stats& S, hipStream_t st)
{
    const int64_t n = F.sym.n;
    tc = TimingCols{};
    tc.n = n;
    std::vector<std::map<int32_t, double>> rows;   // per column: row -> weight
    for (int r = 0; r < R; ++r) {
        std::map<std::array<int64_t, 4>, int32_t> idx;
        for (int32_t k : subtasks[size_t(b0 + r)]) {
            const std::array<int64_t, 4> key = {p->delay[k], p->rise[k], p->width[k], p->fall[k]};
            auto it = idx.find(key);
            if (it == idx.end()) {
                it = idx.emplace(key, int32_t(tc.col.size())).first;
                tc.col.push_back({r, key[0], key[1], key[2], key[3]});
                rows.emplace_back();
            }
            rows[size_t(it->second)][F.sym.iperm[p->node[k]]] += p->amp[k];
        }
    }
    const int64_t nq = int64_t(tc.col.size());
    if (nq == 0) return true;
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    if (sizeof(double) * size_t(n) * size_t(2 * nq) > fr / 2) return false;
    tc.Z = DevMem(sizeof(double) * size_t(n) * size_t(2 * nq));
    std::vector<int32_t> id(n);
    for (int64_t i = 0; i < n; ++i) id[size_t(i)] = int32_t(i);
    DevMem ident = upload(id);
    double* Z1 = tc.Z.as<double>();
    double* Z2 = Z1 + n * nq;
    double* E = bw.s.as<double>();
    double* X1 = bw.w.as<double>();
    double* X2 = bw.y.as<double>();
    for (int64_t q0 = 0; q0 < nq; q0 += bw.Rmax) {
        const int Rc = int(std::min<int64_t>(bw.Rmax, nq - q0));
        size_t cnt = 0;
        for (int c = 0; c < Rc; ++c) cnt += rows[size_t(q0 + c)].size();
        std::vector<int32_t> hr, hc;
        std::vector<double> hd;
        for (int c = 0; c < Rc; ++c)
            for (auto& e : rows[size_t(q0 + c)]) { hr.push_back(e.first); hc.push_back(c); hd.push_back(e.second); }
        DevMem dr = upload(hr), dc = upload(hc), dd = upload(hd);
        launch_b_fill(n * Rc, 0.0, E, st);
        launch_b_events(int(cnt), Rc, dr.as<int32_t>(), dc.as<int32_t>(), dd.as<double>(), E, st);
        dev_solve_batched(F, int(F.gammas.size()), Rc, E, nullptr, X1, bw.sc, st);
        launch_b_deinterleave(n, Rc, ident.as<int32_t>(), X1, Z1 + q0 * n, st);
        dev_solve_batched(F, int(F.gammas.size()), Rc, X1, F.d_cperm.as<double>(), X2, bw.sc, st);
        launch_b_deinterleave(n, Rc, ident.as<int32_t>(), X2, Z2 + q0 * n, st);
        HIPCHK(hipStreamSynchronize(st));   // the small uploads are released here
        S.solve_pairs_g += 2;
    }
    return true;
}

// Alg. 2 for up to RMAX subtasks at a time, each advancing on its own: a
// subtask whose basis has converged is reconstructed and starts its next
// step at once, while the others go on iterating. Every Krylov iteration
// advances the largest group of running subtasks that use the same shift
// (one factor per substitution pair), each at its own dimension; a subtask's
// decisions (offsets, shift, step-down, halving) are those of the plain mode,
// so both take the same steps. Slope changes come from the timing columns.
// The shift of consecutive iterations stays the same while any subtask runs
// with it, so the pair's columns fill up as they would in one lockstep pass,
// and subtasks that finish and start their next step with that shift are
// taken at once instead of idling to the end of the pass.
void transient_batched_async(const matex_factor_s& F, const matex_problem* p, const matex_run_opts* o,
                             const std::vector<std::vector<int32_t>>& subtasks, int64_t h_min, double ratio,
                             bool trace, double* d_probe_out, double* d_final, matex_stats& S, hipStream_t st,
                             bool* fell_back)
{
    const int64_t n = F.sym.n;
    const int n_shifts = int(F.gammas.size());
    const int32_t n_out = p->n_out, n_probe = p->n_probe;
    const int64_t npo = int64_t(n_probe) * n_out;
    const std::vector<int64_t> tout(p->t_out, p->t_out + n_out);
    const int G = int(subtasks.size());
    BatchWork bw(F, std::min(RMAX, G), n_out + 1, npo);
    {
        std::vector<int32_t> pp(std::max(1, n_probe));
        for (int32_t k = 0; k < n_probe; ++k) pp[k] = F.sym.iperm[p->probe[k]];
        bw.probe_perm = upload(pp);
    }
    const double base = o->output_droop ? 0.0 : F.vdd, sgn = o->output_droop ? 1.0 : -1.0;
    launch_b_fill(npo, base, d_probe_out, st);
    if (d_final) launch_b_fill(n, base, d_final, st);
    enum Phase { SETUP, RESTART, RUN, FIN, DONE };
    for (int b0 = 0; b0 < G; b0 += RMAX) {
        const int R = std::min(RMAX, G - b0);
        TimingCols tc;
        if (!timing_cols(F, p, subtasks, b0, R, bw, tc, S, st)) {
            *fell_back = true;
            return;
        }
        std::vector<std::vector<int32_t>> my_cols(R);
        for (size_t q = 0; q < tc.col.size(); ++q) my_cols[size_t(tc.col[q].sub)].push_back(int32_t(q));
        std::vector<BCol> cols(R);
        std::vector<int> ph(R, SETUP);
        std::vector<char> full(R, 0);
        for (int r = 0; r < R; ++r) {
            cols[r].spots = plan_spots(p, subtasks[size_t(b0 + r)], F.sym.iperm);
            S.subtasks++;
        }
        const size_t nr = sizeof(double) * size_t(n) * R;
        for (DevMem* b : {&bw.y, &bw.y0, &bw.z1, &bw.z2, &bw.s, &bw.w}) HIPCHK(hipMemsetAsync(b->p, 0, nr, st));
        if (npo) HIPCHK(hipMemsetAsync(bw.Yout.p, 0, sizeof(double) * npo * R, st));
        std::vector<KsHost> hs(R, KsHost{});
        auto offs_of = [&](int r) -> const std::vector<int64_t>& { return cols[r].offs; };
        auto full_of = [&](int r) { return full[r] != 0; };
        int cur_shift = -1;
        while (true) {
            // (1) subtasks starting a step: spot events, step plan, start vector
            std::vector<int> su;
            for (int r = 0; r < R; ++r)
                if (ph[r] == SETUP || ph[r] == RESTART) su.push_back(r);
            if (!su.empty()) {
                std::vector<int32_t> eptr(R + 1, 0), eq;
                std::vector<double> ecoef;
                for (int r = 0; r < R; ++r) {
                    if (ph[r] == SETUP) {
                        BCol& c = cols[r];
                        if (c.k_spot < c.spots.size() && c.spots[c.k_spot].t == c.t_a) {
                            for (int32_t q : my_cols[r]) {
                                const TimingCols::Col& tq = tc.col[size_t(q)];
                                const int64_t te[4] = {tq.d, tq.d + tq.r, tq.d + tq.r + tq.w, tq.d + tq.r + tq.w + tq.f};
                                const double ds[4] = {1.0 / (double(tq.r) * FS), -1.0 / (double(tq.r) * FS),
                                                      -1.0 / (double(tq.f) * FS), 1.0 / (double(tq.f) * FS)};
                                double coef = 0.0;
                                bool any = false;
                                for (int e = 0; e < 4; ++e)
                                    if (te[e] == c.t_a && te[e] >= 0 && te[e] < p->t_end) { coef += ds[e]; any = true; }
                                if (any) { eq.push_back(q); ecoef.push_back(coef); }
                            }
                            c.k_spot++;
                        }
                        c.offs = step_offsets(tout, c.t_a, c.spots[c.k_spot].t, &c.snap0);
                        c.ksh = ladder_shift(F.gammas, c.offs[0], ratio);
                        ladder_cut(c.offs, F.gammas, c.ksh);
                    }
                    eptr[r + 1] = int32_t(eq.size());
                }
                Packer pk(*bw.h_ev, bw.d_ev, bw.ev_bytes);
                int32_t *d_ptr, *d_q, *d_act;
                double* d_coef;
                int32_t* h_ptr = pk.take<int32_t>(R + 1, &d_ptr);
                int32_t* h_q = pk.take<int32_t>(std::max<size_t>(1, eq.size()), &d_q);
                double* h_coef = pk.take<double>(std::max<size_t>(1, ecoef.size()), &d_coef);
                int32_t* h_act = pk.take<int32_t>(R, &d_act);
                std::copy(eptr.begin(), eptr.end(), h_ptr);
                std::copy(eq.begin(), eq.end(), h_q);
                std::copy(ecoef.begin(), ecoef.end(), h_coef);
                std::fill(h_act, h_act + R, 0);
                for (int r : su) { h_act[r] = 1; full[r] = 0; ph[r] = RUN; }
                pk.upload(st);
                if (!eq.empty())
                    launch_b_spot_cols(n, R, d_ptr, d_q, d_coef, tc.Z1(), tc.Z2(), bw.z1.as<double>(),
                                       bw.z2.as<double>(), st);
                launch_b_setup(n, R, bw.y.as<double>(), bw.y0.as<double>(), bw.z2.as<double>(), bw.Vd(),
                               bw.partial.as<double>(), bw.kst(), d_act, st, true);
                hs = read_states(bw, R, st);   // the staging table is free again
            }
            // (2) one iteration of the running subtasks of one shift: the
            // shift of the previous iteration while any subtask still runs
            // with it (subtasks that start a step with that shift join at
            // once), else the shift that most running subtasks use
            std::vector<int> cnt_k(n_shifts, 0);
            bool any_run = false;
            for (int r = 0; r < R; ++r)
                if (ph[r] == RUN && !hs[r].done) { cnt_k[cols[r].ksh]++; any_run = true; }
            std::vector<int> grp;
            if (any_run) {
                if (cur_shift < 0 || cnt_k[cur_shift] == 0)
                    cur_shift = int(std::max_element(cnt_k.begin(), cnt_k.end()) - cnt_k.begin());
                const int k = cur_shift;
                int nv = 1;
                for (int r = 0; r < R; ++r)
                    if (ph[r] == RUN && !hs[r].done && cols[r].ksh == k) { grp.push_back(r); nv = std::max(nv, hs[r].m + 1); }
                CheckTab t = build_checks(bw, R, grp, offs_of, full_of, {}, st);
                dev_solve_batched_ragged(F, k, R, bw, st);
                launch_b_gs(n, R, bw.Vd(), nv, bw.w.as<double>(), bw.partial.as<double>(), bw.kst(), st, t.active, 1);
                launch_tab_checks(F, bw, t, k, o->tol, o->m_max, 1, st);
                S.solve_pairs_m++;
                hs = read_states(bw, R, st);
            }
            // (3) decisions of the finished subtasks (the group's, and those
            // whose start vector was zero)
            std::vector<int> ver, fin, halve;
            for (int r = 0; r < R; ++r) {
                if (ph[r] != RUN || !hs[r].done) continue;
                if (hs[r].converged) {
                    if (!full[r] && hs[r].m > 0 && cols[r].offs.size() > 2) ver.push_back(r);
                    else fin.push_back(r);
                } else if (cols[r].ksh + 1 < n_shifts) {
                    cols[r].ksh++;
                    ladder_cut(cols[r].offs, F.gammas, cols[r].ksh);
                    S.shift_downs++;
                    S.bases++;
                    S.krylov_dims += hs[r].m;
                    ph[r] = RESTART;
                } else {
                    cols[r].hstep = cols[r].offs.back();
                    halve.push_back(r);
                }
            }
            if (!ver.empty()) {
                // every offset evaluated once at the decided dimension (one
                // table per shift)
                std::vector<int> res;
                std::vector<int> shifts;
                for (int r : ver) shifts.push_back(cols[r].ksh);
                std::sort(shifts.begin(), shifts.end());
                shifts.erase(std::unique(shifts.begin(), shifts.end()), shifts.end());
                for (int k : shifts) {
                    std::vector<int> vk;
                    for (int r : ver)
                        if (cols[r].ksh == k) vk.push_back(r);
                    CheckTab tv = build_checks(bw, R, vk, offs_of, [](int) { return true; }, {}, st);
                    launch_tab_checks(F, bw, tv, k, o->tol, o->m_max, 0, st);
                    std::vector<KsHost> hv = read_states(bw, R, st);
                    for (int r : vk) {
                        full[r] = 1;
                        if (hv[r].converged) fin.push_back(r);
                        else if (hv[r].m < o->m_max) res.push_back(r);
                        else if (cols[r].ksh + 1 < n_shifts) {
                            cols[r].ksh++;
                            ladder_cut(cols[r].offs, F.gammas, cols[r].ksh);
                            S.shift_downs++;
                            S.bases++;
                            S.krylov_dims += hv[r].m;
                            ph[r] = RESTART;
                        } else {
                            cols[r].hstep = cols[r].offs.back();
                            halve.push_back(r);
                        }
                        hs[r] = hv[r];
                    }
                }
                if (!res.empty()) {
                    std::vector<int32_t> ext(res.begin(), res.end());
                    CheckTab tr = build_checks(bw, R, res, offs_of, full_of, ext, st);
                    launch_b_resume(bw.kst(), tr.ext, int(res.size()), st);
                    hs = read_states(bw, R, st);
                }
            }
            // halve the step with the same basis until the checks pass
            while (!halve.empty()) {
                for (int r : halve) {
                    BCol& c = cols[r];
                    c.hstep /= 2;
                    S.halvings++;
                    if (c.hstep < h_min)
                        throw NoConv{"no convergence at t = " + std::to_string(c.t_a) + " fs (subtask " +
                                     std::to_string(b0 + r) + ")"};
                    c.cand = halved_offsets(c.offs, c.hstep);
                }
                const int k = n_shifts - 1;
                CheckTab t = build_checks(
                    bw, R, halve, [&](int r) -> const std::vector<int64_t>& { return cols[r].cand; },
                    [](int) { return true; }, {}, st);
                launch_tab_checks(F, bw, t, k, o->tol, o->m_max, 0, st);
                std::vector<KsHost> hh = read_states(bw, R, st);
                std::vector<int> still;
                for (int r : halve) {
                    if (hh[r].converged) {
                        cols[r].offs = cols[r].cand;
                        fin.push_back(r);
                    } else {
                        still.push_back(r);
                    }
                }
                halve.swap(still);
            }
            // (4) reconstruction of the finished steps; their next step starts
            if (!fin.empty()) {
                for (int r : fin) {
                    S.bases++;
                    S.krylov_dims += hs[r].m;
                    S.m_peak = std::max(S.m_peak, hs[r].m);
                }
                reconstruct(bw, R, fin, cols, tout, n_probe, n_out, S, st);
                for (int r : fin) ph[r] = cols[r].t_a < p->t_end ? SETUP : DONE;
                HIPCHK(hipStreamSynchronize(st));   // the staging table of the reconstruction is free again
            }
            if (trace)
                fprintf(stderr, "[matex] async batch %d: group %zu, verified %zu, finished %zu\n", b0 / RMAX,
                        grp.size(), ver.size(), fin.size());
            bool all_done = true;
            for (int r = 0; r < R; ++r) all_done = all_done && ph[r] == DONE;
            if (all_done) break;
        }
        launch_b_sum_out(npo, R, bw.Yout.as<double>(), sgn, d_probe_out, st);
        if (d_final) launch_b_sum_final(n, R, F.d_perm.as<int32_t>(), bw.y.as<double>(), sgn, d_final, st);
    }
    HIPCHK(hipStreamSynchronize(st));
}

// Alg. 2 for all subtasks, up to RMAX at a time in lockstep generations: in
// each generation every unfinished subtask takes one step. Subtasks that
// ask for different shifts of the ladder run in separate passes (the
// substitution pair of a pass uses one factor); a subtask's decisions
// (offsets, shift, step-down, halving) are those of the one-subtask path.
void transient_batched(const matex_factor_s& F, const matex_problem* p, const matex_run_opts* o,
                       const std::vector<std::vector<int32_t>>& subtasks, int64_t h_min, double ratio,
                       bool trace, double* d_probe_out, double* d_final, matex_stats& S, hipStream_t st)
{
    const int64_t n = F.sym.n;
    const int n_shifts = int(F.gammas.size());
    const int32_t n_out = p->n_out, n_probe = p->n_probe;
    const int64_t npo = int64_t(n_probe) * n_out;
    const std::vector<int64_t> tout(p->t_out, p->t_out + n_out);
    const int G = int(subtasks.size());
    BatchWork bw(F, std::min(RMAX, G), n_out + 1, npo);
    {
        std::vector<int32_t> pp(std::max(1, n_probe));
        for (int32_t k = 0; k < n_probe; ++k) pp[k] = F.sym.iperm[p->probe[k]];
        bw.probe_perm = upload(pp);
    }
    // outputs start at Vdd and each batch subtracts its droops (x), or start
    // at 0 and add them (droop)
    const double base = o->output_droop ? 0.0 : F.vdd, sgn = o->output_droop ? 1.0 : -1.0;
    launch_b_fill(npo, base, d_probe_out, st);
    if (d_final) launch_b_fill(n, base, d_final, st);
    const bool inverted = o->krylov == MATEX_INVERTED;
    int m_guess = 6;
    for (int b0 = 0; b0 < G; b0 += RMAX) {
        const int R = std::min(RMAX, G - b0);
        std::vector<BCol> cols(R);
        for (int r = 0; r < R; ++r) {
            cols[r].spots = plan_spots(p, subtasks[b0 + r], F.sym.iperm);
            S.subtasks++;
        }
        const size_t nr = sizeof(double) * size_t(n) * R;
        for (DevMem* b : {&bw.y, &bw.y0, &bw.z1, &bw.z2, &bw.s}) HIPCHK(hipMemsetAsync(b->p, 0, nr, st));
        if (npo) HIPCHK(hipMemsetAsync(bw.Yout.p, 0, sizeof(double) * npo * R, st));
        while (true) {
            std::vector<int> act;
            for (int r = 0; r < R; ++r)
                if (cols[r].t_a < p->t_end) act.push_back(r);
            if (act.empty()) break;
            // new input slopes at transition spots: s += ds, then z1 = G^-1 s
            // and z2 = G^-1 C z1 for the whole batch (unchanged columns
            // reproduce their values)
            size_t cnt = 0;
            for (int r : act) {
                const BCol& c = cols[r];
                if (c.k_spot < c.spots.size() && c.spots[c.k_spot].t == c.t_a) cnt += c.spots[c.k_spot].node.size();
            }
            if (cnt > 0) {
                const size_t need = cnt * (sizeof(double) + 2 * sizeof(int32_t)) + 64;
                if (need > bw.ev_bytes) {
                    HIPCHK(hipStreamSynchronize(st));
                    bw.ev_bytes = need * 2;
                    bw.h_ev.reset(new PinnedMem(bw.ev_bytes));
                    bw.d_ev = DevMem(bw.ev_bytes);
                }
            }
            Packer pk(*bw.h_ev, bw.d_ev, bw.ev_bytes);
            double* d_d;
            int32_t *d_row, *d_col;
            double* h_d = pk.take<double>(std::max<size_t>(1, cnt), &d_d);
            int32_t* h_row = pk.take<int32_t>(std::max<size_t>(1, cnt), &d_row);
            int32_t* h_col = pk.take<int32_t>(std::max<size_t>(1, cnt), &d_col);
            size_t e = 0;
            for (int r : act) {
                BCol& c = cols[r];
                if (c.k_spot < c.spots.size() && c.spots[c.k_spot].t == c.t_a) {
                    const Segment& sg = c.spots[c.k_spot];
                    for (size_t q = 0; q < sg.node.size(); ++q, ++e) {
                        h_d[e] = sg.dslope[q];
                        h_row[e] = sg.node[q];
                        h_col[e] = r;
                    }
                    c.k_spot++;
                }
            }
            if (cnt > 0) {
                pk.upload(st);
                launch_b_events(int(cnt), R, d_row, d_col, d_d, bw.s.as<double>(), st);
                dev_solve_batched(F, n_shifts, R, bw.s.as<double>(), nullptr, bw.z1.as<double>(), bw.sc, st);
                dev_solve_batched(F, n_shifts, R, bw.z1.as<double>(), F.d_cperm.as<double>(),
                                  bw.z2.as<double>(), bw.sc, st);
                S.solve_pairs_g += 2;
            }
            // step plans
            for (int r : act) {
                BCol& c = cols[r];
                c.offs = step_offsets(tout, c.t_a, c.spots[c.k_spot].t, &c.snap0);
                if (inverted) {
                    c.ksh = n_shifts;   // G: no ladder
                } else {
                    c.ksh = ladder_shift(F.gammas, c.offs[0], ratio);
                    ladder_cut(c.offs, F.gammas, c.ksh);
                }
            }
            std::vector<int> pending = act;
            while (!pending.empty()) {
                int k = n_shifts;
                for (int r : pending) k = std::min(k, cols[r].ksh);
                std::vector<int> grp, rest;
                for (int r : pending) (cols[r].ksh == k ? grp : rest).push_back(r);
                std::vector<KsHost> hs = run_pass(F, bw, R, k, grp, cols, o->tol, o->m_max, m_guess, S, st);
                std::vector<int> fin, halve;
                for (int r : grp) {
                    if (hs[r].converged) {
                        fin.push_back(r);
                    } else if (k + 1 < n_shifts) {
                        cols[r].ksh = k + 1;
                        ladder_cut(cols[r].offs, F.gammas, k + 1);
                        S.shift_downs++;
                        rest.push_back(r);
                    } else {
                        cols[r].hstep = cols[r].offs.back();
                        halve.push_back(r);
                    }
                }
                // halve the step with the same basis until the checks pass
                while (!halve.empty()) {
                    for (int r : halve) {
                        BCol& c = cols[r];
                        c.hstep /= 2;
                        S.halvings++;
                        if (c.hstep < h_min)
                            throw NoConv{"no convergence at t = " + std::to_string(c.t_a) + " fs (subtask " +
                                         std::to_string(b0 + r) + ")"};
                        c.cand = halved_offsets(c.offs, c.hstep);
                    }
                    CheckTab t = build_checks(
                        bw, R, halve, [&](int r) -> const std::vector<int64_t>& { return cols[r].cand; },
                        [](int) { return true; }, {}, st);
                    launch_tab_checks(F, bw, t, k, o->tol, o->m_max, 0, st);
                    std::vector<KsHost> hh = read_states(bw, R, st);
                    std::vector<int> still;
                    for (int r : halve) {
                        if (hh[r].converged) {
                            cols[r].offs = cols[r].cand;
                            fin.push_back(r);
                        } else {
                            still.push_back(r);
                        }
                    }
                    halve.swap(still);
                }
                if (trace)
                    fprintf(stderr, "[matex] batch %d pass shift=%d cols=%zu fin=%zu\n", b0 / RMAX, k, grp.size(),
                            fin.size());
                reconstruct(bw, R, fin, cols, tout, n_probe, n_out, S, st);
                pending.swap(rest);
            }
        }
        launch_b_sum_out(npo, R, bw.Yout.as<double>(), sgn, d_probe_out, st);
        if (d_final) launch_b_sum_final(n, R, F.d_perm.as<int32_t>(), bw.y.as<double>(), sgn, d_final, st);
    }
    HIPCHK(hipStreamSynchronize(st));
}

}  // namespace

// Recorder of a plain run's segments for the adjoint: per segment its
// start and end, shift and dimension, and (device checkpoint) the basis's
// normalised start vector followed by its norm, so that the basis can be
// rebuilt exactly as the run built it.
struct FwdRecord {
    int64_t n = 0;
    std::vector<int64_t> ta, tb;
    std::vector<int> ksh, m;
    std::vector<DevMem> blocks;     // checkpoints, CK_BLOCK of n + 1 doubles each
    static constexpr int CK_BLOCK = 256;
    int64_t max_bytes = 0;
    void add(int64_t a, int64_t b, int k, int mm, const double* v0, const double* beta, hipStream_t st) {
        const size_t i = ta.size();
        if (i % CK_BLOCK == 0) {
            if (int64_t(blocks.size() + 1) * CK_BLOCK * (n + 1) * 8 > max_bytes)
                throw std::bad_alloc();
            blocks.emplace_back(sizeof(double) * size_t(n + 1) * CK_BLOCK);
        }
        HIPCHK(hipMemcpyAsync(state(i), v0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(state(i) + n, beta, sizeof(double), hipMemcpyDeviceToDevice, st));
        ta.push_back(a); tb.push_back(b); ksh.push_back(k); m.push_back(mm);
    }
    double* state(size_t i) const {
        return blocks[i / CK_BLOCK].as<double>() + int64_t(i % CK_BLOCK) * (n + 1);
    }
};

// The plain mode (Alg. 2 per subtask, one after another). Throws HipError
// and NoConv; rec (optional) records every segment.
static void transient_plain(matex_factor_s* f, const matex_problem* p, const matex_run_opts* o,
                            const std::map<int32_t, std::vector<int32_t>>& groups, int64_t h_min,
                            double shift_ratio, bool trace, double* d_probe_out, double* d_final,
                            matex_stats& S, hipStream_t st, FwdRecord* rec)
{
    const int64_t n = f->sym.n;
    const int n_shifts = int(f->gammas.size());
    const bool inverted = o->krylov == MATEX_INVERTED;
    const int32_t n_out = p->n_out, n_probe = p->n_probe;
    // largest check set: outputs inside one spot interval + 1
    Work wk(*f, int64_t(n_out) + 1);
    PinnedMem pin(4096);
    KsHost* hks = pin.as<KsHost>();
    double* hest = pin.as<double>() + 16;
    StageRing ring(size_t(1) << 16);
    int64_t ev_cap = 1 << 16;
    DevMem d_ev(ev_cap);
    DevMem y(sizeof(double) * n), y0(sizeof(double) * n), z1(sizeof(double) * n),
        z2(sizeof(double) * n), sl(sizeof(double) * n), ysum(sizeof(double) * n);
    DevMem probe_perm(sizeof(int32_t) * std::max(1, n_probe));
    {
        std::vector<int32_t> pp(n_probe);
        for (int32_t k = 0; k < n_probe; ++k) pp[k] = f->sym.iperm[p->probe[k]];
        if (n_probe)
            HIPCHK(hipMemcpy(probe_perm.p, pp.data(), sizeof(int32_t) * n_probe, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemsetAsync(d_probe_out, 0, sizeof(double) * int64_t(n_probe) * n_out, st));
    HIPCHK(hipMemsetAsync(ysum.p, 0, ysum.bytes, st));
    const std::vector<int64_t> tout(p->t_out, p->t_out + n_out);
    const double* cperm = f->d_cperm.as<double>();
    double* V = wk.V.as<double>();
    const char* ht_env = std::getenv("MATEX_HOST_TIMES");
    const bool host_times = ht_env && ht_env[0] == '1';
    if (host_times) {
        g_host_times = HostTimes{};
        g_host_times.cap = int64_t(1) << 20;
        HIPCHK(hipMalloc(&g_host_times.d_stamps, sizeof(int64_t) * g_host_times.cap));
    }

    for (auto& grp : groups) {
        S.subtasks++;
        std::vector<Segment> spots = plan_spots(p, grp.second, f->sym.iperm);
        for (DevMem* b : {&y, &y0, &z1, &z2, &sl}) HIPCHK(hipMemsetAsync(b->p, 0, b->bytes, st));
        // z1 = G^-1 s and z2 = G^-1 C z1 are linear in the slopes s, which
        // change only at the subtask's source rows: G^-1 e_k and
        // G^-1 C G^-1 e_k for every source row k come from the
        // 64-right-hand-side sweeps once, and a spot then adds its changed
        // slopes' columns instead of solving twice. Done when the columns
        // fit half the free device memory and the spots outnumber eight
        // per 64 columns (a 64-column pair costs about six one-vector ones).
        std::vector<int32_t> srows;
        for (const Segment& sg : spots) srows.insert(srows.end(), sg.node.begin(), sg.node.end());
        std::sort(srows.begin(), srows.end());
        srows.erase(std::unique(srows.begin(), srows.end()), srows.end());
        const int64_t nq = int64_t(srows.size());
        DevMem Zc;
        std::unordered_map<int32_t, int32_t> qof;
        {
            size_t fr = 0, tot = 0;
            HIPCHK(hipMemGetInfo(&fr, &tot));
            const size_t need = sizeof(double) * size_t(n) * size_t(2 * nq + 3 * RMAX);
            int64_t n_chg = 0;
            for (const Segment& sg : spots) n_chg += sg.node.empty() ? 0 : 1;
            if (nq > 0 && need <= fr / 2 && n_chg > 8 * ((nq + RMAX - 1) / RMAX)) {
                Zc = DevMem(sizeof(double) * size_t(n) * size_t(2 * nq));
                const int Rm = int(std::min<int64_t>(RMAX, nq));
                BatchScratch bsc(*f, Rm);
                DevMem E(sizeof(double) * size_t(n) * Rm), X1(sizeof(double) * size_t(n) * Rm),
                    X2(sizeof(double) * size_t(n) * Rm), ident(sizeof(int32_t) * size_t(n)),
                    ones(sizeof(int32_t) * RMAX + sizeof(double) * RMAX);
                {
                    std::vector<int32_t> id(n);
                    for (int64_t i = 0; i < n; ++i) id[i] = int32_t(i);
                    HIPCHK(hipMemcpyAsync(ident.p, id.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
                    HIPCHK(hipStreamSynchronize(st));
                }
                double* Z1 = Zc.as<double>();
                double* Z2 = Z1 + n * nq;
                for (int64_t q0 = 0; q0 < nq; q0 += RMAX) {
                    const int R = int(std::min<int64_t>(RMAX, nq - q0));
                    std::vector<char> hb(sizeof(double) * RMAX + sizeof(int32_t) * RMAX);
                    double* hv = reinterpret_cast<double*>(hb.data());
                    int32_t* hi = reinterpret_cast<int32_t*>(hv + RMAX);
                    for (int r = 0; r < R; ++r) {
                        hv[r] = 1.0;
                        hi[r] = int32_t(int64_t(srows[q0 + r]) * R + r);
                    }
                    ring.copy(ones.p, hb.data(), hb.size(), st);
                    launch_b_fill(n * R, 0.0, E.as<double>(), st);
                    launch_scatter_add(R, reinterpret_cast<int32_t*>(ones.as<double>() + RMAX), ones.as<double>(),
                                       E.as<double>(), st);
                    dev_solve_batched(*f, n_shifts, R, E.as<double>(), nullptr, X1.as<double>(), bsc, st);
                    launch_b_deinterleave(n, R, ident.as<int32_t>(), X1.as<double>(), Z1 + q0 * n, st);
                    dev_solve_batched(*f, n_shifts, R, X1.as<double>(), cperm, X2.as<double>(), bsc, st);
                    launch_b_deinterleave(n, R, ident.as<int32_t>(), X2.as<double>(), Z2 + q0 * n, st);
                }
                HIPCHK(hipStreamSynchronize(st));   // the scratch is released below
                for (int64_t q = 0; q < nq; ++q) qof[srows[q]] = int32_t(q);
                S.solve_pairs_g += 2 * nq;
            }
        }
        int64_t t_a = 0;
        size_t k_spot = 0;
        SpotArgs pend{};   // a spot update applied by the next basis's start
        while (t_a < p->t_end) {
            // new input slope at a transition spot: z1 = G^-1 s, z2 = G^-1 C z1
            if (k_spot < spots.size() && spots[k_spot].t == t_a) {
                const Segment& sg = spots[k_spot];
                const int32_t cnt = int32_t(sg.node.size());
                if (cnt > 0 && Zc.p && cnt <= SPOT_ARGS) {
                    pend.cnt = cnt;
                    for (int32_t c = 0; c < cnt; ++c) {
                        pend.q[c] = qof.at(sg.node[c]);
                        pend.coef[c] = sg.dslope[c];
                    }
                } else if (cnt > 0) {
                    const size_t need = cnt * (sizeof(int32_t) + sizeof(double)) + 16;
                    if (int64_t(need) > ev_cap) {
                        HIPCHK(hipStreamSynchronize(st));
                        ev_cap = int64_t(need) * 2;
                        d_ev = DevMem(ev_cap);
                    }
                    std::vector<char> buf(need);
                    std::memcpy(buf.data(), sg.dslope.data(), sizeof(double) * cnt);
                    int32_t* bi = reinterpret_cast<int32_t*>(buf.data() + sizeof(double) * cnt);
                    for (int32_t c = 0; c < cnt; ++c) bi[c] = Zc.p ? qof.at(sg.node[c]) : sg.node[c];
                    ring.copy(d_ev.p, buf.data(), need, st);
                    double* dv = d_ev.as<double>();
                    const int32_t* di = reinterpret_cast<int32_t*>(dv + cnt);
                    if (Zc.p) {
                        launch_spot_update(n, cnt, di, dv, Zc.as<double>(), Zc.as<double>() + n * nq,
                                           z1.as<double>(), z2.as<double>(), st);
                    } else {
                        launch_scatter_add(cnt, di, dv, sl.as<double>(), st);
                        dev_solve(*f, n_shifts, sl.as<double>(), nullptr, z1.as<double>(),
                                  wk.tmp.as<double>(), wk.upd.as<double>(), nullptr, st);
                        dev_solve(*f, n_shifts, z1.as<double>(), cperm, z2.as<double>(),
                                  wk.tmp.as<double>(), wk.upd.as<double>(), nullptr, st);
                        S.solve_pairs_g += 2;
                    }
                }
                k_spot++;
            }
            int32_t snap0 = 0;
            std::vector<int64_t> offs = step_offsets(tout, t_a, spots[k_spot].t, &snap0);
            int ksh = n_shifts;   // the inverted space: G, no ladder
            if (!inverted) {
                ksh = ladder_shift(f->gammas, offs[0], shift_ratio);
                ladder_cut(offs, f->gammas, ksh);
            }
            KsHost h{};
            int launched = 0;
            std::vector<double> ests;
            while (true) {
                std::vector<double> taus(offs.size());
                for (size_t q = 0; q < offs.size(); ++q) taus[q] = double(offs[q]) * FS;
                // the spot update, the start vector and few offsets in one
                // launch, by value; more offsets through the staging ring
                TauArgs ta{};
                if (taus.size() <= size_t(TAU_ARGS)) {
                    ta.n = int32_t(taus.size());
                    for (size_t q = 0; q < taus.size(); ++q) ta.t[q] = taus[q];
                } else {
                    ring.copy(wk.taus.p, taus.data(), sizeof(double) * taus.size(), st);
                }
                g_host_times.stamp(1, st);
                launch_spot_setup(n, pend, Zc.p ? Zc.as<double>() : nullptr,
                                  Zc.p ? Zc.as<double>() + n * nq : nullptr, z1.as<double>(), z2.as<double>(),
                                  y.as<double>(), y0.as<double>(), V, wk.partial.as<double>(),
                                  wk.taus.as<double>(), ta, st);
                pend.cnt = 0;   // a retry at a lower shift only sets up again
                launch_normalize_v(n, V, wk.partial.as<double>(), wk.kst(), st);
                ests.clear();
                h = run_arnoldi(*f, ksh, wk, int(taus.size()), o->tol, o->m_max, hks, st, &launched,
                                trace ? &ests : nullptr);
                S.bases++;
                S.solve_pairs_m += launched;
                S.krylov_dims += h.m;
                S.m_peak = std::max(S.m_peak, h.m);
                if (trace && !h.converged)
                    fprintf(stderr, "[matex] not converged t_a=%lld shift=%d m=%d est=%.3e checks=%zu first=%lld last=%lld\n",
                            (long long)t_a, ksh, h.m, read_est(wk, hest, st), offs.size(),
                            (long long)offs[0], (long long)offs.back());
                if (h.converged || ksh + 1 >= n_shifts) break;
                ksh++;
                S.shift_downs++;
                ladder_cut(offs, f->gammas, ksh);
            }
            if (!h.converged) {
                // halve the step with the same basis until the checks pass
                int64_t hstep = offs.back();
                while (true) {
                    hstep /= 2;
                    S.halvings++;
                    if (hstep < h_min)
                        throw NoConv{"no convergence at t = " + std::to_string(t_a) + " fs"};
                    std::vector<int64_t> o2 = halved_offsets(offs, hstep);
                    std::vector<double> taus(o2.size());
                    for (size_t q = 0; q < o2.size(); ++q) taus[q] = double(o2[q]) * FS;
                    ring.copy(wk.taus.p, taus.data(), sizeof(double) * taus.size(), st);
                    launch_checks(wk.kst(), shift_gamma(*f, ksh), wk.taus.as<double>(), nullptr, int(taus.size()),
                                  o->tol, wk.u.as<double>(), wk.est.as<double>(), o->m_max, 0, -1, st);
                    KsHost hh = read_state(wk, hks, st);
                    if (trace)
                        fprintf(stderr, "[matex] halving t_a=%lld step=%lld est=%.3e\n", (long long)t_a,
                                (long long)hstep, read_est(wk, hest, st));
                    if (hh.converged) { offs = o2; break; }
                }
            }
            const int64_t t_b = t_a + offs.back();
            if (trace) {
                const double e = read_est(wk, hest, st);
                fprintf(stderr, "[matex] seg t_a=%lld t_b=%lld shift=%d m=%d conv=%d est=%.3e checks=%zu launched=%d ests",
                        (long long)t_a, (long long)t_b, ksh, h.m, h.converged, e, offs.size(), launched);
                for (double v : ests) fprintf(stderr, " %.3e", v);
                fprintf(stderr, "\n");
            }
            if (rec) rec->add(t_a, t_b, ksh, h.m, V, &wk.kst()->beta, st);
            // snapshots (Alg. 2 reuse) at the probes, then the full state at t_b
            int n_snap = 0;
            while (snap0 + n_snap < n_out && tout[snap0 + n_snap] <= t_b) n_snap++;
            launch_recon_probes(n_probe, probe_perm.as<int32_t>(), n_snap, snap0, wk.taus.as<double>(),
                                wk.u.as<double>(), wk.kst(), V, n, y0.as<double>(), z1.as<double>(),
                                z2.as<double>(), d_probe_out, n_out, st);
            launch_recon_full(n, double(offs.back()) * FS,
                              wk.u.as<double>() + int64_t(offs.size() - 1) * MAXM, wk.kst(), V, n,
                              y.as<double>(), y0.as<double>(), z1.as<double>(), z2.as<double>(), st);
            g_host_times.stamp(2, st);
            S.segments++;
            t_a = t_b;
        }
        launch_axpy_scaled(n, 1.0, y.as<double>(), ysum.as<double>(), st);
    }
    if (host_times) {
        HostTimes& t = g_host_times;
        fprintf(stderr, "[matex] host: %lld iterations enqueued in %.3f s (%.1f us each), %lld check waits %.3f s (%.1f us each)\n",
                (long long)t.iterations, t.enqueue_s, 1e6 * t.enqueue_s / std::max<int64_t>(1, t.iterations),
                (long long)t.waits, t.wait_s, 1e6 * t.wait_s / std::max<int64_t>(1, t.waits));
        HIPCHK(hipStreamSynchronize(st));
        std::vector<int64_t> ts(t.tags.size());
        if (!ts.empty())
            HIPCHK(hipMemcpy(ts.data(), t.d_stamps, sizeof(int64_t) * ts.size(), hipMemcpyDeviceToHost));
        // intervals (10 ns ticks) by the tags that open and close them
        double sum[3][3] = {}, cnt[3][3] = {};
        for (size_t i = 1; i < ts.size(); ++i) {
            sum[t.tags[i - 1]][t.tags[i]] += double(ts[i] - ts[i - 1]) * 1e-2;
            cnt[t.tags[i - 1]][t.tags[i]] += 1;
        }
        const char* nm[3] = {"iter", "setup", "recon_end"};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (cnt[a][b] > 0)
                    fprintf(stderr, "[matex] stamps %s -> %s: %.0f intervals, %.3f s, %.1f us each\n", nm[a], nm[b],
                            cnt[a][b], 1e-6 * sum[a][b], sum[a][b] / cnt[a][b]);
        HIPCHK(hipFree(t.d_stamps));
        g_host_times = HostTimes{};
    }
    if (!o->output_droop) launch_vdd_minus(int64_t(n_probe) * n_out, f->vdd, d_probe_out, st);
    if (d_final) {
        launch_scatter_perm(n, f->d_perm.as<int32_t>(), ysum.as<double>(), d_final, n, n, 1, st);
        if (!o->output_droop) launch_vdd_minus(n, f->vdd, d_final, st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
}

// Argument checks shared by matex_transient and matex_adjoint.
static matex_status check_problem(matex_factor_t f, const matex_problem* p, const matex_run_opts* o)
{
    if (!f || !p || !o) return fail(MATEX_E_INVALID, "null argument");
    const int64_t n = f->sym.n;
    if (p->n_src < 0 || p->n_out <= 0 || p->n_probe < 0 || p->t_end <= 0)
        return fail(MATEX_E_INVALID, "bad sizes");
    if (p->n_src > 0 && (!p->node || !p->amp || !p->delay || !p->rise || !p->width || !p->fall))
        return fail(MATEX_E_INVALID, "null source array");
    if (!p->t_out || (p->n_probe > 0 && !p->probe)) return fail(MATEX_E_INVALID, "null array");
    if (o->mode != MATEX_PLAIN && o->mode != MATEX_BATCHED) return fail(MATEX_E_INVALID, "unknown mode");
    if (o->krylov != MATEX_RATIONAL && o->krylov != MATEX_INVERTED)
        return fail(MATEX_E_INVALID, "unknown Krylov subspace");
    if (o->m_max < 1 || o->m_max > MAXM) return fail(MATEX_E_INVALID, "m_max must be in 1..32");
    if (!(o->tol > 0.0)) return fail(MATEX_E_INVALID, "tol must be > 0");
    for (int32_t k = 0; k < p->n_src; ++k) {
        if (p->node[k] < 0 || p->node[k] >= n) return fail(MATEX_E_INVALID, "source node out of range");
        if (p->delay[k] < 0 || p->rise[k] <= 0 || p->fall[k] <= 0 || p->width[k] < 0)
            return fail(MATEX_E_INVALID, "pulse timing out of range");
        if (p->group && p->group[k] < 0) return fail(MATEX_E_INVALID, "negative group");
    }
    for (int32_t k = 0; k < p->n_out; ++k) {
        if (p->t_out[k] < 0 || p->t_out[k] > p->t_end) return fail(MATEX_E_INVALID, "t_out outside [0, t_end]");
        if (k && p->t_out[k] <= p->t_out[k - 1]) return fail(MATEX_E_INVALID, "t_out not increasing");
    }
    for (int32_t k = 0; k < p->n_probe; ++k)
        if (p->probe[k] < 0 || p->probe[k] >= n) return fail(MATEX_E_INVALID, "probe out of range");
    return MATEX_OK;
}

// MATEX_E_NONFINITE if a probe output or the final state is NaN or infinite.
static matex_status check_outputs(const matex_problem* p, int64_t n, const double* d_probe_out,
                                  const double* d_final, hipStream_t st)
{
    try {
        const std::string bad = nonfinite_arrays(
            {{"probe outputs", int64_t(p->n_probe) * p->n_out, d_probe_out}, {"final state", n, d_final}}, st);
        if (!bad.empty()) return fail(MATEX_E_NONFINITE, "non-finite values in the " + bad);
    } catch (const HipError& e) {
        return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    return MATEX_OK;
}

extern "C" matex_status matex_transient(matex_factor_t f, const matex_problem* p,
                                        const matex_run_opts* o, double* d_probe_out,
                                        double* d_final, matex_stats* stats, void* stream)
{
    const double t_start = now_s();
    if (!d_probe_out) return fail(MATEX_E_INVALID, "null argument");
    if (matex_status cs = check_problem(f, p, o)) return cs;
    const int64_t n = f->sym.n;
    const int64_t h_min = std::max<int64_t>(1, o->h_min);
    const double shift_ratio = o->shift_ratio > 0.0 ? o->shift_ratio : 1.0;

    // subtasks (Sec. 3.1)
    std::map<int32_t, std::vector<int32_t>> groups;
    for (int32_t k = 0; k < p->n_src; ++k) groups[p->group ? p->group[k] : 0].push_back(k);
    if (groups.empty()) groups[0];

    matex_stats S{};
    const char* trace_env = std::getenv("MATEX_TRACE");
    const bool trace = trace_env && trace_env[0] == '1';
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n_shifts = int(f->gammas.size());
    const int32_t n_out = p->n_out, n_probe = p->n_probe;
    if (o->mode == MATEX_BATCHED) {
        std::vector<std::vector<int32_t>> subs;
        for (auto& g : groups) subs.push_back(g.second);
        try {
            bool fell_back = o->batched_independent == 0 || o->krylov == MATEX_INVERTED;
            if (!fell_back)
                transient_batched_async(*f, p, o, subs, h_min, shift_ratio, trace, d_probe_out, d_final, S, st,
                                        &fell_back);
            if (fell_back) {
                S = matex_stats{};
                transient_batched(*f, p, o, subs, h_min, shift_ratio, trace, d_probe_out, d_final, S, st);
            }
        } catch (const NoConv& e) {
            return fail(MATEX_E_NOCONV, e.msg);
        } catch (const HipError& e) {
            return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
        } catch (const std::bad_alloc&) {
            return fail(MATEX_E_OOM, "host allocation failed");
        }
        S.seconds = now_s() - t_start;
        if (stats) *stats = S;
        return check_outputs(p, n, d_probe_out, d_final, st);
    }
    try {
        transient_plain(f, p, o, groups, h_min, shift_ratio, trace, d_probe_out, d_final, S, st, nullptr);
    } catch (const NoConv& e) {
        return fail(MATEX_E_NOCONV, e.msg);
    } catch (const HipError& e) {
        return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc&) {
        return fail(MATEX_E_OOM, "host allocation failed");
    }
    S.seconds = now_s() - t_start;
    if (stats) *stats = S;
    return check_outputs(p, n, d_probe_out, d_final, st);
}

// The trapezoidal rule at a fixed step (Eq. 2), the paper's comparator: every
// step forms its right-hand side on the device (one fused kernel), then one
// substitution pair with the factor of C + (h/2) G, then gathers the probes
// when the step ends at an output time.
extern "C" matex_status matex_trapezoidal(matex_factor_t f, const matex_problem* p, int64_t h_fs,
                                          const matex_run_opts* o, double* d_probe_out, double* d_final,
                                          matex_stats* stats, void* stream)
{
    const double t_start = now_s();
    if (!d_probe_out || !o) return fail(MATEX_E_INVALID, "null argument");
    matex_run_opts oo = *o;
    oo.mode = MATEX_PLAIN;
    oo.krylov = MATEX_RATIONAL;
    if (!(oo.tol > 0.0)) oo.tol = 1.0;
    if (oo.m_max < 1) oo.m_max = 1;
    if (matex_status cs = check_problem(f, p, &oo)) return cs;
    if (h_fs <= 0 || p->t_end % h_fs != 0) return fail(MATEX_E_INVALID, "h must be > 0 and divide t_end");
    for (int32_t k = 0; k < p->n_out; ++k)
        if (p->t_out[k] % h_fs != 0) return fail(MATEX_E_INVALID, "every output time must be a multiple of h");
    const double hs = double(h_fs) * FS;
    if (!(std::fabs(f->gammas[0] - 0.5 * hs) <= 1e-12 * hs))
        return fail(MATEX_E_INVALID, "the factor's first shift must be h / 2 (factor C + (h/2) G)");
    const int64_t n = f->sym.n;
    const int32_t n_out = p->n_out, n_probe = p->n_probe, n_src = p->n_src;
    hipStream_t st = static_cast<hipStream_t>(stream);
    matex_stats S{};
    try {
        // sources grouped by row (factor order), each row's in source order
        std::vector<int32_t> order(n_src);
        for (int32_t k = 0; k < n_src; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return f->sym.iperm[p->node[a]] < f->sym.iperm[p->node[b]];
        });
        std::vector<int32_t> sptr(n + 1, 0);
        std::vector<double> amp;
        std::vector<int64_t> sd, sr, sw, sf;
        for (int32_t q : order) {
            sptr[f->sym.iperm[p->node[q]] + 1]++;
            amp.push_back(p->amp[q]);
            sd.push_back(p->delay[q]); sr.push_back(p->rise[q]); sw.push_back(p->width[q]); sf.push_back(p->fall[q]);
        }
        for (int64_t i = 0; i < n; ++i) sptr[i + 1] += sptr[i];
        if (amp.empty()) { amp.push_back(0.0); sd.push_back(0); sr.push_back(1); sw.push_back(0); sf.push_back(1); }
        DevMem d_sptr = upload(sptr), d_amp = upload(amp), d_sd = upload(sd), d_sr = upload(sr), d_sw = upload(sw),
               d_sf = upload(sf);
        std::vector<int32_t> pp(std::max(1, n_probe), 0);
        for (int32_t k = 0; k < n_probe; ++k) pp[k] = f->sym.iperm[p->probe[k]];
        DevMem d_pp = upload(pp);
        DevMem y(sizeof(double) * n), rhs(sizeof(double) * n), tmp(sizeof(double) * n),
            upd(sizeof(double) * std::max<int64_t>(1, f->sym.n_upd));
        HIPCHK(hipMemsetAsync(d_probe_out, 0, sizeof(double) * int64_t(n_probe) * n_out, st));
        // initial state: y(0) = G^-1 i(0) (0 when no pulse is on at t = 0)
        {
            std::vector<double> i0(n, 0.0);
            bool any = false;
            for (int32_t k = 0; k < n_src; ++k) {
                const int64_t d = p->delay[k], r = p->rise[k], w = p->width[k], fl = p->fall[k];
                double u = 0.0;
                if (0 > d && 0 <= d + r) u = double(0 - d) / double(r);
                else if (0 > d + r && 0 <= d + r + w) u = 1.0;
                else if (0 > d + r + w && 0 < d + r + w + fl) u = 1.0 - double(0 - d - r - w) / double(fl);
                if (u != 0.0) { i0[f->sym.iperm[p->node[k]]] += p->amp[k] * u; any = true; }
            }
            if (any) {
                DevMem d_i0 = upload(i0);
                dev_solve(*f, int(f->gammas.size()), d_i0.as<double>(), nullptr, y.as<double>(), tmp.as<double>(),
                          upd.as<double>(), nullptr, st);
                S.solve_pairs_g++;
                HIPCHK(hipStreamSynchronize(st));
            } else {
                HIPCHK(hipMemsetAsync(y.p, 0, y.bytes, st));
            }
        }
        int32_t k_out = 0;
        while (k_out < n_out && p->t_out[k_out] == 0)
            launch_gather_probes(n_probe, d_pp.as<int32_t>(), y.as<double>(), d_probe_out, n_out, k_out++, st);
        const int64_t steps = p->t_end / h_fs;
        for (int64_t k = 1; k <= steps; ++k) {
            const int64_t t0 = (k - 1) * h_fs, t1 = k * h_fs;
            launch_tr_rhs(n, f->d_grp.as<int32_t>(), f->d_gci.as<int32_t>(), f->d_gv.as<double>(),
                          f->d_cperm.as<double>(), y.as<double>(), 0.5 * hs, t0, t1, d_sptr.as<int32_t>(),
                          d_amp.as<double>(), d_sd.as<int64_t>(), d_sr.as<int64_t>(), d_sw.as<int64_t>(),
                          d_sf.as<int64_t>(), rhs.as<double>(), st);
            dev_solve(*f, 0, rhs.as<double>(), nullptr, y.as<double>(), tmp.as<double>(), upd.as<double>(), nullptr,
                      st);
            while (k_out < n_out && p->t_out[k_out] == t1)
                launch_gather_probes(n_probe, d_pp.as<int32_t>(), y.as<double>(), d_probe_out, n_out, k_out++, st);
            S.solve_pairs_m++;
            S.segments++;
        }
        if (!o->output_droop) launch_vdd_minus(int64_t(n_probe) * n_out, f->vdd, d_probe_out, st);
        if (d_final) {
            launch_scatter_perm(n, f->d_perm.as<int32_t>(), y.as<double>(), d_final, n, n, 1, st);
            if (!o->output_droop) launch_vdd_minus(n, f->vdd, d_final, st);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    } catch (const HipError& e) {
        return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc&) {
        return fail(MATEX_E_OOM, "host allocation failed");
    }
    S.subtasks = 1;
    S.seconds = now_s() - t_start;
    if (stats) *stats = S;
    return check_outputs(p, n, d_probe_out, d_final, st);
}

extern "C" matex_status matex_transient_many(int32_t n_inst, const matex_factor_t* f,
                                             const matex_problem* p, const matex_run_opts* o,
                                             double* const* d_probe_out, double* const* d_final,
                                             matex_stats* stats, int32_t n_streams, void* stream)
{
    if (n_inst < 0 || (n_inst > 0 && (!f || !p || !o || !d_probe_out)))
        return fail(MATEX_E_INVALID, "null argument");
    if (n_streams < 0 || n_streams > 16) return fail(MATEX_E_INVALID, "n_streams must be in 0..16");
    if (n_inst == 0) return MATEX_OK;
    const int workers = std::min<int>(n_inst, n_streams > 0 ? n_streams : 4);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MATEX_E_HIP, "hipGetDevice failed");
    // the caller's stream may hold work that produced the inputs
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(MATEX_E_HIP, "stream synchronisation failed");
    // largest work first: nodes times transition spots
    std::vector<int32_t> order(n_inst);
    std::vector<double> work(n_inst);
    for (int32_t k = 0; k < n_inst; ++k) {
        order[k] = k;
        work[k] = f[k] ? double(f[k]->sym.n) * (4.0 * std::max(1, p[k].n_src) + 2.0) : 0.0;
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
    std::atomic<int32_t> next{0};
    std::mutex mu;
    matex_status first = MATEX_OK;
    std::string first_msg;
    auto run = [&]() {
        if (hipSetDevice(dev) != hipSuccess) return;
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            std::lock_guard<std::mutex> g(mu);
            if (first == MATEX_OK) { first = MATEX_E_HIP; first_msg = "stream creation failed"; }
            return;
        }
        while (true) {
            const int32_t q = next.fetch_add(1);
            if (q >= n_inst) break;
            const int32_t k = order[q];
            matex_stats sk{};
            const matex_status r = matex_transient(f[k], &p[k], &o[k], d_probe_out[k],
                                                   d_final ? d_final[k] : nullptr, &sk, st);
            if (stats) stats[k] = sk;
            if (r != MATEX_OK) {
                std::lock_guard<std::mutex> g(mu);
                if (first == MATEX_OK) {
                    first = r;
                    first_msg = "instance " + std::to_string(k) + ": " + g_err;
                }
                next.store(n_inst);
            }
        }
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    };
    std::vector<std::thread> th;
    for (int w = 0; w < workers; ++w) th.emplace_back(run);
    for (auto& t : th) t.join();
    if (first != MATEX_OK) return fail(first, first_msg);
    return MATEX_OK;
}

// Adjoint sweep (continuous adjoint of C y' = -G y + i(t)): lambda is zero
// after the last sample time, jumps by C^-1 g_s at every sample time t_s
// (g_s = dJ/dy(t_s) = -dJ/dx(t_s) at the probes) and between them satisfies
// C lambda' = G lambda, i.e. lambda(t_hi - sigma) = e^{sigma A} lambda(t_hi)
// with the forward operator A = -C^-1 G: the same rational Krylov steps as
// the forward run, backwards in time, with no input terms. Steps break at
// the sample times and at every source's transition spots, so each pulse
// is linear on a step and its amplitude gradient
// dJ/da_k = int u_k(t) lambda_{n_k}(t) dt accumulates step by step from the
// step's exact integrals of e^{sigma H} e1 and sigma e^{sigma H} e1.
extern "C" matex_status matex_adjoint(matex_factor_t f, const matex_problem* p, const matex_run_opts* o,
                                      const double* d_dJdx, double* d_grad_amp, double* d_grad_c,
                                      void* stream)
{
    if (!d_dJdx) return fail(MATEX_E_INVALID, "null argument");
    if (matex_status cs = check_problem(f, p, o)) return cs;
    if (o->m_max > MAXM - 2) return fail(MATEX_E_INVALID, "m_max must be <= 30 for the adjoint");
    if (o->krylov != MATEX_RATIONAL) return fail(MATEX_E_INVALID, "the adjoint runs the rational space only");
    const int64_t n = f->sym.n;
    const int n_shifts = int(f->gammas.size());
    const int32_t n_out = p->n_out, n_probe = p->n_probe, n_src = p->n_src;
    const int64_t h_min = std::max<int64_t>(1, o->h_min);
    const double ratio = o->shift_ratio > 0.0 ? o->shift_ratio : 1.0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    try {
        // sample times: output times > 0 whose column of dJ/dx is not zero
        std::vector<double> g(size_t(n_probe) * n_out);
        if (!g.empty())
            HIPCHK(hipMemcpyAsync(g.data(), d_dJdx, sizeof(double) * g.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::map<int64_t, int32_t> sample;   // time -> output column
        for (int32_t c = 0; c < n_out; ++c) {
            if (p->t_out[c] <= 0) continue;
            bool nz = false;
            for (int32_t q = 0; q < n_probe && !nz; ++q) nz = g[size_t(q) * n_out + c] != 0.0;
            if (nz) sample[p->t_out[c]] = c;
        }
        if (d_grad_amp && n_src > 0) HIPCHK(hipMemsetAsync(d_grad_amp, 0, sizeof(double) * n_src, st));
        if (d_grad_c) HIPCHK(hipMemsetAsync(d_grad_c, 0, sizeof(double) * n, st));
        if (sample.empty() || (n_src == 0 && !d_grad_c)) {
            HIPCHK(hipStreamSynchronize(st));
            return MATEX_OK;
        }
        const int64_t t_last = sample.rbegin()->first;
        // lambda is carried divided by the largest jump norm max_s ||C^-1 g_s||,
        // so the tolerance is relative to the strongest sensitivity
        double lscale = 0.0;
        for (auto& kv : sample) {
            std::map<int32_t, double> jv;
            for (int32_t q = 0; q < n_probe; ++q) jv[p->probe[q]] -= g[size_t(q) * n_out + kv.second];
            double s2 = 0.0;
            for (auto& e : jv) s2 += (e.second / f->c_host[e.first]) * (e.second / f->c_host[e.first]);
            lscale = std::max(lscale, std::sqrt(s2));
        }
        // step boundaries below t_last: sample times and transition spots
        std::vector<int64_t> bnd{0};
        for (auto& kv : sample) bnd.push_back(kv.first);
        for (int32_t k = 0; k < n_src; ++k) {
            const int64_t d = p->delay[k], r = p->rise[k], w = p->width[k], fl = p->fall[k];
            for (int64_t t : {d, d + r, d + r + w, d + r + w + fl})
                if (t > 0 && t < t_last) bnd.push_back(t);
        }
        std::sort(bnd.begin(), bnd.end());
        bnd.erase(std::unique(bnd.begin(), bnd.end()), bnd.end());
        // probes grouped by permuted row (fixed summation order for repeats)
        std::map<int32_t, std::vector<int32_t>> by_row;
        for (int32_t q = 0; q < n_probe; ++q) by_row[f->sym.iperm[p->probe[q]]].push_back(q);
        std::vector<int32_t> rows, ptr{0}, pidx;
        for (auto& kv : by_row) {
            rows.push_back(kv.first);
            pidx.insert(pidx.end(), kv.second.begin(), kv.second.end());
            ptr.push_back(int32_t(pidx.size()));
        }
        DevMem d_rows = upload(rows), d_ptr = upload(ptr), d_pidx = upload(pidx);
        std::vector<int32_t> srow(n_src);
        for (int32_t k = 0; k < n_src; ++k) srow[k] = f->sym.iperm[p->node[k]];
        DevMem d_srow = upload(srow);
        DevMem d_del = upload(std::vector<int64_t>(p->delay, p->delay + n_src));
        DevMem d_ris = upload(std::vector<int64_t>(p->rise, p->rise + n_src));
        DevMem d_wid = upload(std::vector<int64_t>(p->width, p->width + n_src));
        DevMem d_fal = upload(std::vector<int64_t>(p->fall, p->fall + n_src));
        Work wk(*f, 2);
        PinnedMem pin(4096);
        KsHost* hks = pin.as<KsHost>();
        DevMem lam(sizeof(double) * n), zero(sizeof(double) * n), I(sizeof(double) * 2 * MAXM);
        HIPCHK(hipMemsetAsync(lam.p, 0, lam.bytes, st));
        HIPCHK(hipMemsetAsync(zero.p, 0, zero.bytes, st));
        double* V = wk.V.as<double>();
        const double* cperm = f->d_cperm.as<double>();
        auto jump = [&](int64_t t) {
            auto it = sample.find(t);
            if (it != sample.end())
                launch_adj_jump(int(rows.size()), d_rows.as<int32_t>(), d_ptr.as<int32_t>(), d_pidx.as<int32_t>(),
                                d_dJdx, n_out, it->second, cperm, 1.0 / lscale, lam.as<double>(), st);
        };
        auto set_tau = [&](int64_t dt) {
            HIPCHK(hipStreamSynchronize(st));
            double* h = pin.as<double>() + 64;
            *h = double(dt) * FS;
            HIPCHK(hipMemcpyAsync(wk.taus.p, h, sizeof(double), hipMemcpyHostToDevice, st));
        };
        const char* trace_env = std::getenv("MATEX_TRACE");
        const bool trace = trace_env && trace_env[0] == '1';
        int64_t t_hi = t_last;
        jump(t_hi);
        // a jump puts weight on modes much faster than the steps; the step
        // integrals need them resolved, so after a jump the steps grow
        // geometrically from 1 fs (a step never exceeds the time since the
        // jump), each with the shift of the ladder that fits it
        int64_t since = 0;
        size_t b = bnd.size() - 1;   // bnd[b] == t_last

        // capacitance gradients: dJ/dc_i = -int lambda_i y_i' dt, integrated by
        // parts. A forward run over [0, t_last] (all sources as one subtask:
        // the sum of the subtasks' droops) records every segment with its
        // basis's start vector; the sweep rebuilds each forward basis exactly
        // (recorded shift and dimension) and integrates every overlap of an
        // adjoint step with a forward segment exactly (Van Loan).
        std::unique_ptr<FwdRecord> rec;
        std::unique_ptr<Work> wf;
        DevMem gcp, Wq, fy0, fz1, fz2, fi, fsl, fev, GV;
        std::unique_ptr<PinnedMem> fstage, dbg;
        size_t fev_cap = 0;
        int64_t fseg = 0;
        auto unit_val = [&](int32_t k, int64_t t) -> double {
            const int64_t d = p->delay[k], r = p->rise[k], w = p->width[k], fl = p->fall[k];
            if (t <= d) return 0.0;
            if (t < d + r) return double(t - d) / double(r);
            if (t <= d + r + w) return 1.0;
            if (t < d + r + w + fl) return 1.0 - double(t - d - r - w) / double(fl);
            return 0.0;
        };
        auto unit_slope = [&](int32_t k, double tm) -> double {   // per second
            const double d = double(p->delay[k]), r = double(p->rise[k]), w = double(p->width[k]),
                         fl = double(p->fall[k]);
            if (tm > d && tm < d + r) return 1.0 / (r * FS);
            if (tm > d + r + w && tm < d + r + w + fl) return -1.0 / (fl * FS);
            return 0.0;
        };
        auto build_fwd = [&](int64_t i) {
            const int64_t ta = rec->ta[size_t(i)], tb = rec->tb[size_t(i)];
            if (trace)
                fprintf(stderr, "[matex-adj] %.4f s rebuild forward segment %lld [%lld, %lld] shift=%d m=%d\n",
                        now_s(), (long long)i, (long long)ta, (long long)tb, rec->ksh[size_t(i)], rec->m[size_t(i)]);
            const double tm = 0.5 * (double(ta) + double(tb));
            std::vector<int32_t> rr;
            std::vector<double> iv, sv;
            for (int32_t k = 0; k < n_src; ++k) {
                const double a = p->amp[k] * unit_val(k, ta), sl = p->amp[k] * unit_slope(k, tm);
                if (a != 0.0 || sl != 0.0) {
                    rr.push_back(int32_t(f->sym.iperm[p->node[k]]));
                    iv.push_back(a);
                    sv.push_back(sl);
                }
            }
            const size_t cnt = rr.size();
            const size_t need = cnt * (2 * sizeof(double) + sizeof(int32_t)) + 64;
            HIPCHK(hipStreamSynchronize(st));
            if (need > fev_cap) {
                fev_cap = need * 2;
                fstage.reset(new PinnedMem(fev_cap));
                fev = DevMem(fev_cap);
            }
            double* hv = fstage->as<double>();
            std::memcpy(hv, iv.data(), sizeof(double) * cnt);
            std::memcpy(hv + cnt, sv.data(), sizeof(double) * cnt);
            std::memcpy(reinterpret_cast<int32_t*>(hv + 2 * cnt), rr.data(), sizeof(int32_t) * cnt);
            HIPCHK(hipMemsetAsync(fi.p, 0, fi.bytes, st));
            HIPCHK(hipMemsetAsync(fsl.p, 0, fsl.bytes, st));
            if (cnt) {
                HIPCHK(hipMemcpyAsync(fev.p, fstage->p, need, hipMemcpyHostToDevice, st));
                double* dv = fev.as<double>();
                const int32_t* drow = reinterpret_cast<const int32_t*>(dv + 2 * cnt);
                launch_scatter_add(int32_t(cnt), drow, dv, fi.as<double>(), st);
                launch_scatter_add(int32_t(cnt), drow, dv + cnt, fsl.as<double>(), st);
            }
            // y0 = G^-1 i(t_a), z1 = G^-1 s, z2 = G^-1 C z1 (Eq. 6)
            dev_solve(*f, n_shifts, fi.as<double>(), nullptr, fy0.as<double>(), wf->tmp.as<double>(),
                      wf->upd.as<double>(), nullptr, st);
            dev_solve(*f, n_shifts, fsl.as<double>(), nullptr, fz1.as<double>(), wf->tmp.as<double>(),
                      wf->upd.as<double>(), nullptr, st);
            dev_solve(*f, n_shifts, fz1.as<double>(), cperm, fz2.as<double>(), wf->tmp.as<double>(),
                      wf->upd.as<double>(), nullptr, st);
            // the run's own start vector and norm: the same basis, bit for bit
            double* Vf = wf->V.as<double>();
            HIPCHK(hipMemcpyAsync(Vf, rec->state(size_t(i)), sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            launch_restore_start(wf->kst(), rec->state(size_t(i)) + n, st);
            const int sh = rec->ksh[size_t(i)];
            for (int j = 0; j < rec->m[size_t(i)]; ++j) {
                dev_solve(*f, sh, Vf + int64_t(j) * n, cperm, wf->w.as<double>(), wf->tmp.as<double>(),
                          wf->upd.as<double>(), wf->done(), st);
                launch_gs_dots(n, Vf, n, j + 1, wf->w.as<double>(), wf->partial.as<double>(), wf->kst(),
                               wf->done(), st);
                launch_gs_update(n, Vf, n, j + 1, wf->w.as<double>(), wf->partial.as<double>(), wf->kst(),
                                 wf->done(), st);
                launch_gs_finish(n, Vf, n, j + 1, wf->w.as<double>(), wf->partial.as<double>(), wf->kst(),
                                 wf->done(), st);
                ++wf->ticket;
            }
        };
        if (d_grad_c) {
            rec.reset(new FwdRecord());
            rec->n = n;
            size_t fr = 0, tot = 0;
            HIPCHK(hipMemGetInfo(&fr, &tot));
            rec->max_bytes = int64_t(0.8 * double(fr));
            matex_problem q = *p;
            q.t_end = t_last;
            q.n_out = 0;
            while (q.n_out < n_out && p->t_out[q.n_out] <= t_last) q.n_out++;
            std::map<int32_t, std::vector<int32_t>> one;
            for (int32_t k = 0; k < n_src; ++k) one[0].push_back(k);
            if (one.empty()) one[0];
            DevMem xo(sizeof(double) * std::max<int64_t>(1, int64_t(n_probe) * q.n_out));
            matex_stats S2{};
            // the gradient's sample and integral terms partly cancel, so the
            // recorded droop is taken two digits tighter than the adjoint
            matex_run_opts ro = *o;
            ro.output_droop = 1;
            ro.tol = o->tol * 1e-2;
            transient_plain(f, &q, &ro, one, h_min, ratio, false, xo.as<double>(), nullptr, S2, st, rec.get());
            wf.reset(new Work(*f, 2));
            gcp = DevMem(sizeof(double) * n);
            HIPCHK(hipMemsetAsync(gcp.p, 0, gcp.bytes, st));
            Wq = DevMem(sizeof(double) * (MAXM * MAXM + 2 * MAXM));
            HIPCHK(hipMemsetAsync(Wq.p, 0, Wq.bytes, st));
            GV = DevMem(sizeof(double) * n * (MAXM + 1));
            // sample term: -(1/c_i) sum_s g_{s,i} y_i(t_s) = (1/c_i) sum dJ/dx * y at
            // the probes (g = -dJ/dx), with the droop of the recorded run
            std::vector<double> yp(size_t(n_probe) * q.n_out);
            if (!yp.empty())
                HIPCHK(hipMemcpyAsync(yp.data(), xo.p, sizeof(double) * yp.size(), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            std::map<int32_t, double> term;
            for (auto& kv : sample)
                for (int32_t qq = 0; qq < n_probe; ++qq)
                    term[f->sym.iperm[p->probe[qq]]] += g[size_t(qq) * n_out + kv.second] *
                                                         yp[size_t(qq) * q.n_out + kv.second] /
                                                         f->c_host[p->probe[qq]];
            std::vector<int32_t> trow;
            std::vector<double> tval;
            for (auto& e : term) { trow.push_back(e.first); tval.push_back(e.second); }
            if (!trow.empty()) {
                DevMem dr = upload(trow), dv = upload(tval);
                launch_scatter_add(int32_t(trow.size()), dr.as<int32_t>(), dv.as<double>(), gcp.as<double>(), st);
                HIPCHK(hipStreamSynchronize(st));
            }
            for (DevMem* v : {&fy0, &fz1, &fz2, &fi, &fsl}) *v = DevMem(sizeof(double) * n);
            fseg = int64_t(rec->ta.size()) - 1;
            build_fwd(fseg);
        }
        while (t_hi > 0) {
            while (bnd[b] >= t_hi) --b;
            int64_t dt = std::min(t_hi - bnd[b], std::max<int64_t>(1, since));
            int ksh = ladder_shift(f->gammas, dt, ratio);
            set_tau(dt);
            KsHost h{};
            while (true) {
                launch_setup_v(n, lam.as<double>(), zero.as<double>(), zero.as<double>(), V,
                               wk.partial.as<double>(), wk.kst(), st);
                launch_normalize_v(n, V, wk.partial.as<double>(), wk.kst(), st);
                h = run_arnoldi(*f, ksh, wk, 1, o->tol, o->m_max, hks, st);
                if (h.converged || ksh + 1 >= n_shifts) break;
                ksh++;
            }
            if (trace)
                fprintf(stderr, "[matex-adj] %.4f s t_hi=%lld dt=%lld shift=%d m=%d conv=%d est=%.3e\n", now_s(),
                        (long long)t_hi, (long long)dt, ksh, h.m, h.converged,
                        read_est(wk, pin.as<double>() + 128, st));
            while (!h.converged) {
                dt /= 2;
                if (dt < h_min)
                    return fail(MATEX_E_NOCONV, "adjoint: no convergence at t = " + std::to_string(t_hi) + " fs");
                set_tau(dt);
                launch_checks(wk.kst(), f->gammas[ksh], wk.taus.as<double>(), nullptr, 1, o->tol,
                              wk.u.as<double>(), wk.est.as<double>(), o->m_max, 0, -1, st);
                h = read_state(wk, hks, st);
            }
            if (d_grad_amp) {
                launch_adj_integrals(wk.kst(), f->gammas[ksh], double(dt) * FS, I.as<double>(), st);
                launch_adj_amp(n_src, d_srow.as<int32_t>(), d_del.as<int64_t>(), d_ris.as<int64_t>(),
                               d_wid.as<int64_t>(), d_fal.as<int64_t>(), t_hi, dt, V, n, wk.kst(),
                               I.as<double>(), lscale, d_grad_amp, st);
            }
            if (d_grad_c) {
                const int64_t t_lo = t_hi - dt;
                launch_spmv_cols(n, f->d_grp.as<int32_t>(), f->d_gci.as<int32_t>(), f->d_gv.as<double>(), V, n,
                                 wk.kst(), GV.as<double>(), st);
                while (fseg > 0 && rec->ta[size_t(fseg)] >= t_hi) build_fwd(--fseg);
                while (true) {
                    const int64_t ta = rec->ta[size_t(fseg)], tb = rec->tb[size_t(fseg)];
                    const int64_t t1 = std::max(t_lo, ta), t2 = std::min(t_hi, tb);
                    if (t2 > t1) {
                        const double gl = f->gammas[ksh], gf = f->gammas[rec->ksh[size_t(fseg)]];
                        const double sb = double(t_hi - t2) * FS, ta_s = double(t1 - ta) * FS,
                                     hh = double(t2 - t1) * FS;
                        launch_cg_block(wk.kst(), gl, wf->kst(), gf, sb, ta_s, hh, Wq.as<double>(), st);
                        if (trace) {
                            if (!dbg) dbg.reset(new PinnedMem(sizeof(double) * (MAXM * MAXM + 2 * MAXM)));
                            double* hw = dbg->as<double>();
                            HIPCHK(hipMemcpyAsync(hw, Wq.p, sizeof(double) * (MAXM * MAXM + 2 * MAXM),
                                                  hipMemcpyDeviceToHost, st));
                            HIPCHK(hipStreamSynchronize(st));
                            bool bad = false;
                            for (int q = 0; q < MAXM * MAXM + 2 * MAXM; ++q) bad |= !std::isfinite(hw[q]);
                            if (bad)
                                fprintf(stderr, "[matex-adj] non-finite overlap: adjoint [%lld, %lld] shift %d m %d, "
                                        "forward %lld [%lld, %lld] shift %d m %d, t1 %lld t2 %lld\n",
                                        (long long)t_lo, (long long)t_hi, ksh, h.m, (long long)fseg, (long long)ta,
                                        (long long)tb, rec->ksh[size_t(fseg)], rec->m[size_t(fseg)],
                                        (long long)t1, (long long)t2);
                        }
                        launch_cg_nodes(n, GV.as<double>(), wf->V.as<double>(), n, wk.kst(), wf->kst(),
                                        fy0.as<double>(), fz1.as<double>(), fz2.as<double>(), cperm,
                                        Wq.as<double>(), lscale, gcp.as<double>(), st);
                    }
                    if (ta > t_lo && fseg > 0) {
                        build_fwd(--fseg);
                        continue;
                    }
                    break;
                }
            }
            // lambda at the step's lower end
            launch_recon_full(n, double(dt) * FS, wk.u.as<double>(), wk.kst(), V, n, lam.as<double>(),
                              zero.as<double>(), zero.as<double>(), zero.as<double>(), st);
            t_hi -= dt;
            since += dt;
            if (sample.count(t_hi)) since = 0;
            jump(t_hi);
        }
        if (d_grad_c) launch_scatter_perm(n, f->d_perm.as<int32_t>(), gcp.as<double>(), d_grad_c, n, n, 1, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        const std::string bad = nonfinite_arrays(
            {{"amplitude gradients", n_src, d_grad_amp}, {"capacitance gradients", n, d_grad_c}}, st);
        if (!bad.empty()) return fail(MATEX_E_NONFINITE, "non-finite values in the " + bad);
    } catch (const NoConv& e) {
        return fail(MATEX_E_NOCONV, "forward run for the capacitance gradients: " + e.msg);
    } catch (const HipError& e) {
        return fail(MATEX_E_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc&) {
        return fail(MATEX_E_OOM, "host or device allocation failed (forward checkpoints need segments x n x 8 bytes)");
    }
    return MATEX_OK;
}
