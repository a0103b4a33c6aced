// Host controller and C ABI of libbfs (see include/bfs.h).
//
// The level loop is driven from the host: after every level it copies three
// device counters (next-frontier size, its edge count, entries examined) into
// pinned host memory, and applies the direction rule of Section 4.4 before
// launching the next level: top-down while the frontier's edges m_f stay at
// or below the unexplored edges m_u divided by alpha, bottom-up until the
// frontier shrinks below n / beta.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bfs.h"
#include "bfs_internal.h"

using namespace bfsk;

namespace {

thread_local std::string g_err;

bfs_status fail(bfs_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail(BFS_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

enum GraphKind { KIND_CSR = 1, KIND_DCSC = 2 };

}  // namespace

struct bfs_graph {
    int kind = 0;
    int device = 0;
    uint32_t flags = 0;
    // CSR
    int64_t n = 0, nnz = 0;
    int off_bytes = 8;
    const void* off = nullptr;
    const int32_t* cols = nullptr;
    // DCSC block
    int64_t nrows = 0, ncols = 0, row_base = 0, col_base = 0, nzc = 0, nzr = 0;
    const int32_t *jc = nullptr, *ir = nullptr, *jr = nullptr, *ic = nullptr;
    const int64_t *cp = nullptr, *rp = nullptr;
    int block_union = 0;   // bfs_block_set_union
    // derived metadata (device, library-owned, symmetric graphs only): bitmap
    // of vertices without entries, ids >= n in the last word set; their count
    uint64_t* d_iso = nullptr;
    int64_t isolated = 0;
    // row heads for the bottom-up step: {degree, first three entries} per
    // vertex, and for any-parent searches {degree, three highest-degree neighbours}
    int4* d_head = nullptr;
    int4* d_hub = nullptr;
    // hubs (the < HUB_BITS vertices of highest degree, by a degree threshold),
    // in id order, and the hub heads with the ranks of their two hubs
    int32_t* d_hubid = nullptr;
    int4* d_hubr = nullptr;
    int nhub = 0;
    int64_t max_degree = -1;   // longest row (symmetric graphs; -1 when not computed)
    bool hub_auto = false;   // frontier bitmap larger than the L2: ranked probes by default
    uint32_t* d_nbase = nullptr;   // per word: vertices with edges before it (head record index base)
    // workgroups of the persistent top-down engines that fit on the device
    int persist_groups_max = 1;
    int ms_groups_max = 1;
    int fused_groups_max = 1;
    // host metadata
    uint64_t* h_buf = nullptr;              // pinned: create-time readback only
};

namespace {

// Per-thread host state of a running search: a pinned buffer for counter
// readback and a pool of timing events.  Keeping it per thread (not per graph)
// lets several threads search the same graph at once on their own streams.
struct HostCtx {
    uint64_t* pinned = nullptr;
    // mailbox: coherent pinned memory that kernels write directly; word 0
    // carries the sequence number of the last completed readback
    uint64_t* mbox = nullptr;
    uint64_t* mbox_dev = nullptr;
    uint64_t seq = 0;
    std::vector<hipEvent_t> events;
    ~HostCtx() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        if (pinned) (void)hipHostFree(pinned);
        if (mbox) (void)hipHostFree(mbox);
    }
};
thread_local HostCtx tl_ctx;
constexpr int MBOX_WORDS = 511;   // data words of the 4 KiB mailbox

hipError_t host_ctx(HostCtx** out) {
    if (!tl_ctx.pinned) {
        hipError_t e = hipHostMalloc((void**)&tl_ctx.pinned, 4096, hipHostMallocDefault);
        if (e != hipSuccess) { tl_ctx.pinned = nullptr; return e; }
    }
    if (!tl_ctx.mbox) {
        hipError_t e = hipHostMalloc((void**)&tl_ctx.mbox, 4096, hipHostMallocCoherent | hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&tl_ctx.mbox_dev, tl_ctx.mbox, 0);
        if (e != hipSuccess) {
            if (tl_ctx.mbox) (void)hipHostFree(tl_ctx.mbox);
            tl_ctx.mbox = nullptr;
            return e;
        }
        std::memset(tl_ctx.mbox, 0, 4096);
    }
    *out = &tl_ctx;
    return hipSuccess;
}

// Wait until the mailbox shows sequence `seq`: spin (no sleep, so no wake-up
// latency), and after 2 s ask the stream, which reports a failed launch; a
// stream that completed without publishing is an error too.
bfs_status mbox_wait(HostCtx* c, hipStream_t s, uint64_t seq) {
    const auto t0 = std::chrono::steady_clock::now();
    int polls = 0;
    while (__atomic_load_n(&c->mbox[0], __ATOMIC_ACQUIRE) != seq) {
        __builtin_ia32_pause();
        if (++polls == 4096) {
            polls = 0;
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
                HIP_TRY(hipStreamSynchronize(s));
                if (__atomic_load_n(&c->mbox[0], __ATOMIC_ACQUIRE) != seq)
                    return fail(BFS_E_HIP, "readback did not arrive");
            }
        }
    }
    return BFS_OK;
}

// nw (<= MBOX_WORDS) words of device memory, read after all earlier work on s
bfs_status readback(HostCtx* c, hipStream_t s, const void* src, int nw, const uint64_t** out) {
    if (nw < 0 || nw > MBOX_WORDS) return fail(BFS_E_INVALID_ARG, "readback of %d words", nw);
    const uint64_t seq = ++c->seq;
    launch_post(s, (const uint64_t*)src, nw, c->mbox_dev, seq);
    HIP_TRY(hipGetLastError());
    bfs_status st = mbox_wait(c, s, seq);
    *out = c->mbox + 1;
    return st;
}

// -------------------------------------------------------------- workspace layout
struct SingleLayout {
    size_t counters, pctl, pctr, small, ctl_end, rec, visited, vprev, fbits, nbits, claim, q0, q1, scan, tiles, partial,
        hb, pcsum, segpos, segtot, total;
};

SingleLayout single_layout(const bfs_graph* g) {
    SingleLayout L{};
    const int64_t n = g->n;
    const int64_t W = (n + 63) / 64;
    const int64_t ntiles = (g->nnz + TD_TILE - 1) / TD_TILE;
    size_t o = 0;
    // control block, cleared as one range: level counters, engine barrier
    // words and counters, engine state; the engine's level records follow
    // the state so one copy brings both back
    L.counters = o; o = align_up(o + sizeof(uint64_t) * SLOTS * SLOT_WORDS);
    L.pctl = o; o = align_up(o + sizeof(PersistCtl));
    L.pctr = o; o = align_up(o + sizeof(uint64_t) * SLOTS * SLOT_WORDS);
    L.small = o; o = align_up(o + sizeof(SmallState));
    L.ctl_end = o;
    L.rec = o; o = align_up(o + sizeof(int64_t) * 6 * BFS_STATS_MAX_LEVELS);   // 4 per level (top-down engine), 6 (fused)
    L.visited = o; o = align_up(o + sizeof(uint64_t) * (size_t)W);
    L.vprev = o; o = align_up(o + sizeof(uint64_t) * (size_t)W);
    L.fbits = o; o = align_up(o + sizeof(uint64_t) * (size_t)W);
    L.nbits = o; o = align_up(o + sizeof(uint64_t) * (size_t)W);
    L.claim = o; o = align_up(o + sizeof(uint64_t) * (size_t)W);
    L.q0 = o; o = align_up(o + sizeof(int32_t) * (size_t)(n + 1));
    L.q1 = o; o = align_up(o + sizeof(int32_t) * (size_t)(n + 1));
    L.scan = o; o = align_up(o + sizeof(int64_t) * (size_t)(n + 2));
    L.tiles = o; o = align_up(o + sizeof(int32_t) * (size_t)(ntiles + 2));
    L.partial = o; o = align_up(o + sizeof(int64_t) * (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 2));
    L.hb = o; o = align_up(o + sizeof(uint64_t) * (HUB_BITS / 64));
    // per-workgroup edge totals of the engine's edge-balanced levels
    L.pcsum = o; o = align_up(o + sizeof(int64_t) * (size_t)(g->persist_groups_max > 0 ? g->persist_groups_max : 1));
    // top-down column segments: each queue entry's first entry in the
    // segment, and the segment's edge total
    L.segpos = o; o = align_up(o + sizeof(int32_t) * (size_t)(n + 1));
    L.segtot = o; o = align_up(o + sizeof(int64_t));
    L.total = o;
    return L;
}

struct BlockLayout {
    size_t header, q, scan, tiles, partial, spa, occ, fmark, bpar, bmask, total;
};

BlockLayout block_layout(const bfs_graph* g) {
    BlockLayout L{};
    const int64_t qmax = g->ncols < g->nzc ? g->ncols : g->nzc;
    const int64_t wr = (g->nrows + 63) / 64;
    const int64_t chunks = (g->nzr + 63) / 64;
    int64_t scan_len = g->ncols;
    if (wr > scan_len) scan_len = wr;
    if (chunks > scan_len) scan_len = chunks;
    size_t o = 0;
    L.header = o; o = align_up(o + sizeof(uint64_t) * 8);
    L.q = o; o = align_up(o + sizeof(int32_t) * (size_t)(qmax + 1));
    L.scan = o; o = align_up(o + sizeof(int64_t) * (size_t)(qmax + 2));
    L.tiles = o; o = align_up(o + sizeof(int32_t) * (size_t)((g->nnz + TD_TILE - 1) / TD_TILE + 2));
    L.partial = o; o = align_up(o + sizeof(int64_t) * (size_t)((scan_len + SCAN_TILE - 1) / SCAN_TILE + 2));
    L.spa = o; o = align_up(o + sizeof(uint32_t) * (size_t)g->nrows);
    L.occ = o; o = align_up(o + sizeof(uint64_t) * (size_t)wr);
    L.fmark = o; o = align_up(o + sizeof(uint64_t) * (size_t)((g->ncols + 63) / 64 + 1));
    L.bpar = o; o = align_up(o + sizeof(int32_t) * (size_t)(chunks * 64 + 1));
    L.bmask = o; o = align_up(o + sizeof(uint64_t) * (size_t)(chunks + 1));
    L.total = o;
    return L;
}

BlockWs block_ws(const bfs_graph* g, char* ws) {
    const BlockLayout Lo = block_layout(g);
    BlockWs W{};
    W.header = (uint64_t*)(ws + Lo.header);
    W.qlen = W.header;
    W.total = (int64_t*)(W.header + 1);
    W.range = W.header + 2;
    W.skip = W.header + 5;
    W.q = (int32_t*)(ws + Lo.q);
    W.scan = (int64_t*)(ws + Lo.scan);
    W.tiles = (int32_t*)(ws + Lo.tiles);
    W.partial = (int64_t*)(ws + Lo.partial);
    W.spa = (uint32_t*)(ws + Lo.spa);
    W.occ = (uint64_t*)(ws + Lo.occ);
    W.fmark = (uint64_t*)(ws + Lo.fmark);
    W.bpar = (int32_t*)(ws + Lo.bpar);
    W.bmask = (uint64_t*)(ws + Lo.bmask);
    return W;
}

BlockArgs block_args(const bfs_graph* g) {
    BlockArgs B{};
    B.nrows = g->nrows; B.ncols = g->ncols; B.col_base = g->col_base;
    B.nzc = g->nzc; B.nzr = g->nzr; B.nnz = g->nnz;
    B.jc = g->jc; B.ir = g->ir; B.jr = g->jr; B.ic = g->ic; B.cp = g->cp; B.rp = g->rp;
    B.sorted = (g->flags & BFS_GRAPH_SORTED) != 0;
    B.sort_union = g->block_union;
    return B;
}

struct MultiLayout {
    size_t counters, pctl, pctr, mstate, ctl_end, mrec, src, visited, F, N, hubmark, qa, qb, scan, tiles, partial,
        par, lvl, total;
};

MultiLayout multi_layout(const bfs_graph* g) {
    MultiLayout L{};
    const int64_t n = g->n;
    size_t o = 0;
    L.counters = o; o = align_up(o + sizeof(uint64_t) * SLOTS * SLOT_WORDS);
    // the persistent engine's control block (cleared before each launch) and level records
    L.pctl = o; o = align_up(o + sizeof(PersistCtl));
    L.pctr = o; o = align_up(o + sizeof(uint64_t) * SLOTS * SLOT_WORDS);
    L.mstate = o; o = align_up(o + sizeof(MsState));
    L.ctl_end = o;
    L.mrec = o; o = align_up(o + sizeof(int64_t) * 5 * BFS_STATS_MAX_LEVELS);
    L.src = o; o = align_up(o + sizeof(int64_t) * 64);
    L.visited = o; o = align_up(o + sizeof(uint64_t) * (size_t)n);
    L.F = o; o = align_up(o + sizeof(uint64_t) * (size_t)n);
    L.N = o; o = align_up(o + sizeof(uint64_t) * (size_t)n);
    L.hubmark = o; o = align_up(o + sizeof(uint64_t) * (size_t)((n + 63) / 64 + 1));
    L.qa = o; o = align_up(o + sizeof(int32_t) * (size_t)(n + 1));
    L.qb = o; o = align_up(o + sizeof(int32_t) * (size_t)(n + 1));
    L.scan = o; o = align_up(o + sizeof(int64_t) * (size_t)(n + 2));
    L.tiles = o; o = align_up(o + sizeof(int32_t) * (size_t)((g->nnz + TD_TILE - 1) / TD_TILE + 2));
    L.partial = o; o = align_up(o + sizeof(int64_t) * (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 2));
    L.par = o; o = align_up(o + sizeof(int32_t) * 64 * (size_t)n);
    L.lvl = o; o = align_up(o + sizeof(uint16_t) * 64 * (size_t)n);
    L.total = o;
    return L;
}

size_t multi_bytes(const bfs_graph* g, int) { return multi_layout(g).total; }

// -------------------------------------------------------------- timing
struct Timer {
    HostCtx* g;
    hipStream_t s;
    int mode;   // bfs_opts.timing: 0 off, 1 every kernel, 2 the bottom-up sweep only
    struct Rec { int kind; int level; size_t ev; };
    std::vector<Rec> recs;
    size_t used = 0;

    hipError_t ensure(size_t k) {
        while (g->events.size() < k) {
            // timing only (read after a stream synchronisation): no system-scope
            // fence, whose cache writeback and invalidation would slow the
            // kernel that follows the event
            hipEvent_t e;
            hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
            if (r != hipSuccess) return r;
            g->events.push_back(e);
        }
        return hipSuccess;
    }
    bool on = false;   // the bracket being recorded
    bool wants(int kind) const { return mode == 1 || (mode == 2 && kind == BFS_K_BU_SWEEP); }
    // brackets one launch (or a few launches of one kind)
    hipError_t begin(int kind) {
        on = wants(kind);
        if (!on) return hipSuccess;
        hipError_t r = ensure(used + 2);
        if (r != hipSuccess) return r;
        return hipEventRecord(g->events[used], s);
    }
    hipError_t end(int kind, int level) {
        if (!on) return hipSuccess;
        on = false;
        hipError_t r = hipEventRecord(g->events[used + 1], s);
        recs.push_back({kind, level, used});
        used += 2;
        return r;
    }
    void collect(bfs_stats* st) {
        for (auto& r : recs) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, g->events[r.ev], g->events[r.ev + 1]) != hipSuccess) ms = 0.f;
            st->kernel_ms[r.kind] += ms;
            if (r.level >= 0 && r.level < BFS_STATS_MAX_LEVELS &&
                (r.kind == BFS_K_TD_EXPAND || r.kind == BFS_K_BU_SWEEP || r.kind == BFS_K_MS_LEVEL))
                st->level_ms[r.level] += ms;
        }
    }
};

bfs_status check_csr_graph(const bfs_graph* g) {
    if (!g || g->kind != KIND_CSR) return fail(BFS_E_INVALID_ARG, "graph handle is not a CSR graph");
    return BFS_OK;
}

template <typename OffT>
bfs_status run_single(bfs_graph* g, int64_t src, const bfs_opts& o, int32_t* parent, int32_t* depth, char* ws,
                      hipStream_t stream, bfs_stats* st) {
    const auto t_start = std::chrono::steady_clock::now();
    const OffT* off = (const OffT*)g->off;
    const int64_t n = g->n, W = (n + 63) / 64;
    const SingleLayout Lo = single_layout(g);
    uint64_t* counters = (uint64_t*)(ws + Lo.counters);
    uint64_t* visited = (uint64_t*)(ws + Lo.visited);
    uint64_t* vprev = (uint64_t*)(ws + Lo.vprev);
    uint64_t* fbits = (uint64_t*)(ws + Lo.fbits);
    uint64_t* nbits = (uint64_t*)(ws + Lo.nbits);
    uint64_t* claim = (uint64_t*)(ws + Lo.claim);
    int32_t* qcur = (int32_t*)(ws + Lo.q0);
    int32_t* qnext = (int32_t*)(ws + Lo.q1);
    int64_t* scan = (int64_t*)(ws + Lo.scan);
    int32_t* tiles = (int32_t*)(ws + Lo.tiles);
    int64_t* partial = (int64_t*)(ws + Lo.partial);
    const int claim_mode = o.parent_mode == BFS_PARENT_MIN ? CLAIM_MIN
                           : o.td_claim == 1             ? CLAIM_CAS
                           : o.td_claim == 2             ? CLAIM_BENIGN
                                                         : CLAIM_BITMAP;
    const bool any_bitmap = claim_mode == CLAIM_BITMAP || claim_mode == CLAIM_BENIGN;
    const int serial = o.bu_serial > 0 ? o.bu_serial : 16;
    Launch L{stream, o.grid_blocks > 0 ? o.grid_blocks : 2048};
    HostCtx* ctx = nullptr;
    HIP_TRY(host_ctx(&ctx));
    Timer T{ctx, stream, o.timing, {}, 0};

    // a small graph: the whole search in one persistent launch
    const int64_t fused_max = o.fused_max_n > 0                            ? o.fused_max_n
                              : o.fused_max_n == 0 && o.dir != BFS_DIR_TD ? FUSED_MAX_N
                                                                          : -1;
    if (n <= fused_max && (g->flags & BFS_GRAPH_SYMMETRIC) && g->d_iso &&
        (claim_mode == CLAIM_BITMAP || claim_mode == CLAIM_MIN) && o.bu_head == 0 && o.td_prepass <= 0 &&
        o.bu_segments == 0 && o.td_segments == 0) {
        int64_t groups = o.persist_groups > 0 ? o.persist_groups : FUSED_GROUPS;
        groups = std::min<int64_t>(groups, g->fused_groups_max);
        groups = std::min<int64_t>(groups, (W + 3) / 4);   // at least one word per wave
        if (groups < 1) groups = 1;
        const int rec_cap = st ? BFS_STATS_MAX_LEVELS : 0;
        FusedState* d_fs = (FusedState*)(ws + Lo.small);
        int64_t* d_rec = (int64_t*)(ws + Lo.rec);
        HIP_TRY(T.begin(BFS_K_FUSED));
        launch_clear_words(L, counters, (int64_t)((Lo.ctl_end - Lo.counters) / sizeof(uint64_t)));
        launch_search_fused<OffT>(L, claim_mode == CLAIM_MIN, (int)groups, off, g->cols, g->d_iso, n, g->nnz, src, parent,
                                  depth, visited, fbits, nbits, vprev, o.dir, o.alpha, o.beta, serial, d_fs, counters,
                                  (PersistCtl*)(ws + Lo.pctl), d_rec, rec_cap);
        HIP_TRY(hipGetLastError());
        HIP_TRY(T.end(BFS_K_FUSED, -1));
        const uint64_t* hb = nullptr;
        {
            const int nw = (int)(((Lo.rec - Lo.small) + sizeof(int64_t) * 6 * (size_t)rec_cap) / sizeof(uint64_t));
            bfs_status rs = readback(ctx, stream, d_fs, nw, &hb);
            if (rs != BFS_OK) return rs;
        }
        FusedState fs;
        std::memcpy(&fs, hb, sizeof(fs));
        if (fs.reason == ENG_TIMEOUT) return fail(BFS_E_HIP, "fused search: grid barrier timed out");
        if (fs.reason != ENG_NOT_RUN) {
            if (st) {
                const int64_t* r = (const int64_t*)((const char*)hb + (Lo.rec - Lo.small));
                for (int64_t d = 0; d < fs.levels_done && d < rec_cap; ++d, r += 6) {
                    st->level_dir[d] = (int8_t)r[0];
                    st->level_nf[d] = r[1];
                    st->level_mf[d] = r[2];
                    st->level_mu[d] = r[3];
                    st->level_unvisited[d] = r[4];
                    st->level_examined[d] = r[5];
                    if (r[0]) st->bu_levels++; else st->td_levels++;
                }
                st->launches[BFS_K_FUSED] += 1;
                st->levels = (int32_t)fs.levels_done;
                st->fill_level = -1;
                st->reached = fs.reached;
                st->isolated = g->isolated;
                st->edges_examined = fs.examined;
                if (T.mode) {
                    if (!T.recs.empty()) HIP_TRY(hipEventSynchronize(ctx->events[T.recs.back().ev + 1]));
                    T.collect(st);
                }
                st->total_ms =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
            }
            return BFS_OK;
        }
        // the workgroups could not all be resident: level by level instead
    }

    // degree of the source: the first frontier's edge count.  The
    // initialisation does not need it and is queued behind the request, so
    // it runs while the host waits for the answer.
    const uint64_t* h = nullptr;   // the last level's counters, in the mailbox
    const uint64_t row_seq = ++ctx->seq;
    launch_post_row<OffT>(stream, off, src, ctx->mbox_dev, row_seq);
    HIP_TRY(hipGetLastError());

    // ANY parents with fetch-or claims never read parent/depth, so their -1
    // fill moves into the first bottom-up sweep (whole lines, once), or to a
    // fill pass at the end when no bottom-up level runs; the other claim
    // modes compare against -1 and need it before the first top-down level
    const bool lazy_out = any_bitmap && o.dir != BFS_DIR_TD && g->d_iso != nullptr;
    bool out_filled = !lazy_out;
    // Before the outputs are filled, a top-down level's winners (the next
    // frontier) may leave their depth unwritten: the next level writes it,
    // with whole lines when it is the sweep that fills the outputs (or the
    // hub pre-pass that fills them), else from the frontier queue.  Only
    // fetch-or claims on symmetric graphs, where every winner has an edge and
    // so enters the queue.
    const bool defer_depth = lazy_out && claim_mode == CLAIM_BITMAP && (g->flags & BFS_GRAPH_SYMMETRIC);
    bool depth_pending = false;
    int32_t fill_level = -1;   // reported in stats: who wrote the -1 of the vertices not reached
    HIP_TRY(T.begin(BFS_K_INIT));
    launch_init(L, parent, depth, n, visited, vprev, fbits, claim, g->d_iso, W, qcur, src, counters,
                (int64_t)((Lo.ctl_end - Lo.counters) / sizeof(uint64_t)), !lazy_out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(T.end(BFS_K_INIT, -1));
    if (st) st->launches[BFS_K_INIT] += 1;
    {
        bfs_status ws_ = mbox_wait(ctx, stream, row_seq);
        if (ws_ != BFS_OK) return ws_;
    }
    const int64_t deg_s = (int64_t)ctx->mbox[2] - (int64_t)ctx->mbox[1];

    int64_t n_f = 1, m_f = deg_s, m_u = g->nnz - deg_s;
    int64_t qlen = deg_s > 0 ? 1 : 0;     // exact queue length when qlen_dev is NULL
    const uint64_t* qlen_dev = nullptr;   // set when the queue came from a bitmap conversion
    int64_t unvisited = n - 1;
    int cur_dir = (o.dir == BFS_DIR_BU) ? 1 : 0;
    bool fmt_queue = true;   // frontier as queue (true) or only as bitmap (false)
    bool fbits_stale = false;   // after the small-frontier engine fbits lags the queue
    // persistent engine: one workgroup up to cap_one frontier edges, pgroups
    // workgroups up to cap_multi (no engine when small_edges < 0)
    bool engine_on = o.small_edges >= 0;
    const int64_t cap_one = o.small_edges > 0 ? o.small_edges : 1024;
    const int64_t cap_multi = o.persist_edges > 0 ? std::max<int64_t>(o.persist_edges, cap_one) : 65536;
    const int64_t prepass_edges = o.td_prepass > 0 ? o.td_prepass : o.td_prepass == 0 ? ((int64_t)1 << 24) : -1;
    int pgroups = o.persist_groups > 0 ? o.persist_groups : 64;
    pgroups = std::min(pgroups, g->persist_groups_max);
    if (pgroups < 1) pgroups = 1;
    SmallState* d_small = (SmallState*)(ws + Lo.small);
    int64_t* d_rec = (int64_t*)(ws + Lo.rec);
    int level = 0;
    int64_t reached = 1, examined = 0;
    bool prev_bu = false;      // the previous level ran bottom-up
    bool same_level = false;   // retrying this level: its direction is already chosen
    bool skip_engine = false;  // ... and it goes through the per-level kernels
    for (;;) {
        // ---- direction for this level (Section 4.4)
        if (same_level) same_level = false;
        else if (o.dir == BFS_DIR_TD) cur_dir = 0;
        else if (o.dir == BFS_DIR_BU) cur_dir = 1;
        else if (cur_dir == 0) { if ((double)m_f * o.alpha > (double)m_u) cur_dir = 1; }
        else { if ((double)n_f * o.beta < (double)n) cur_dir = 0; }

        if (cur_dir == 0 && !fmt_queue) {
            uint64_t* cslot = counters + (size_t)(level % SLOTS) * SLOT_WORDS;
            // bottom-up -> top-down: the frontier bitmap becomes a queue in
            // vertex order.  Its length is n_f exactly (the sweep counted one
            // per bit it set), so the host knows it and the persistent engine
            // may take the following small levels; the device copy goes to
            // slot word 4.
            HIP_TRY(T.begin(BFS_K_CONVERT));
            const int nl = launch_bitmap_to_queue(L, fbits, W, qcur, cslot + 4, partial);
            HIP_TRY(hipGetLastError());
            HIP_TRY(T.end(BFS_K_CONVERT, level));
            if (st) st->launches[BFS_K_CONVERT] += nl;
            qlen_dev = nullptr;
            qlen = n_f;
            fmt_queue = true;
        }

        const bool engine_ok = engine_on && !skip_engine;
        skip_engine = false;
        // ---- small top-down levels: run them back to back on the device
        if (cur_dir == 0 && fmt_queue && !qlen_dev && m_f > 0 && engine_ok && m_f <= cap_multi) {
            // one workgroup while the frontier is tiny, many once it grows
            const bool multi = m_f > cap_one;
            const int groups = multi ? pgroups : 1;
            SmallIn in{qlen, n_f, m_f, m_u, level};
            const int rec_cap = (st && level < BFS_STATS_MAX_LEVELS) ? BFS_STATS_MAX_LEVELS - level : 0;
            // forced top-down never switches: with alpha = 0 the rule m_f * alpha > m_u cannot fire
            const double eng_alpha = o.dir == BFS_DIR_TD ? 0.0 : o.alpha;
            if (depth_pending) {
                HIP_TRY(T.begin(BFS_K_CONVERT));
                launch_queue_depth(L, qcur, nullptr, qlen, depth, level);
                HIP_TRY(hipGetLastError());
                HIP_TRY(T.end(BFS_K_CONVERT, level));
                if (st) st->launches[BFS_K_CONVERT] += 1;
                depth_pending = false;
            }
            HIP_TRY(T.begin(BFS_K_TD_EXPAND));
            // the engine's small levels keep exact claims in the benign mode
            launch_td_persist<OffT>(L, claim_mode == CLAIM_BENIGN ? CLAIM_BITMAP : claim_mode, groups, off, g->cols, parent, depth, visited, vprev, claim, qcur,
                                    qnext, n, in, d_small, (uint64_t*)(ws + Lo.pctr), (PersistCtl*)(ws + Lo.pctl),
                                    d_rec, rec_cap, eng_alpha, multi ? cap_multi : cap_one, multi ? cap_one / 2 : 0,
                                    (int64_t)1 << 40, scan, tiles, (int64_t*)(ws + Lo.pcsum));
            HIP_TRY(hipGetLastError());
            HIP_TRY(T.end(BFS_K_TD_EXPAND, -1));
            // state and level records in one copy, then the whole control
            // block is cleared: the level counters (the level index moved on),
            // the engine's barrier words and its state (reason 0 = not run)
            const uint64_t* hb = nullptr;
            {
                const int nw = (int)(((Lo.rec - Lo.small) + sizeof(int64_t) * 4 * (size_t)rec_cap) / sizeof(uint64_t));
                bfs_status rs = readback(ctx, stream, d_small, nw, &hb);
                if (rs != BFS_OK) return rs;
            }
            SmallState hs;
            std::memcpy(&hs, hb, sizeof(hs));
            // a search that goes on needs the control block cleared (level
            // counters: the level index moved on; barrier words; state)
            if (hs.reason != ENG_EMPTY) {
                launch_clear_words(L, counters, (int64_t)((Lo.ctl_end - Lo.counters) / sizeof(uint64_t)));
                HIP_TRY(hipGetLastError());
            }
            const int64_t* recs = (const int64_t*)((const char*)hb + (Lo.rec - Lo.small));
            if (st) st->launches[BFS_K_TD_EXPAND] += 1;
            if (hs.reason == ENG_NOT_RUN) {
                // the workgroups could not all be resident at once (a busy
                // device): nothing was touched, continue level by level
                engine_on = false;
                same_level = true;
                continue;
            }
            if (hs.reason == ENG_TIMEOUT) return fail(BFS_E_HIP, "top-down engine: grid barrier timed out");
            if (st) {
                st->td_levels += (int32_t)hs.levels_done;
                int64_t unv = unvisited;
                const int64_t* r = recs;
                for (int64_t i = 0; i < hs.levels_done && i < rec_cap; ++i, r += 4) {
                    const int lv = level + (int)i;
                    st->level_dir[lv] = 0;
                    st->level_nf[lv] = r[0];
                    st->level_mf[lv] = r[1];
                    st->level_mu[lv] = r[2];
                    st->level_unvisited[lv] = unv;
                    st->level_examined[lv] = r[1];
                    unv -= r[3];
                }
            }
            examined += hs.examined;
            reached += hs.found;
            unvisited -= hs.found;
            level += (int)hs.levels_done;
            if (hs.cur_is_b) { int32_t* t = qcur; qcur = qnext; qnext = t; }
            if (hs.levels_done > 0) {
                fbits_stale = true;
                prev_bu = false;
            }
            if (hs.reason == ENG_EMPTY) break;   // the next frontier is empty
            qlen = hs.qlen;
            n_f = hs.n_f;
            m_f = hs.m_f;
            m_u = hs.m_u;
            if (level > n + 1) return fail(BFS_E_HIP, "level loop did not terminate");
            if (hs.levels_done == 0) {
                // nothing ran (a cap hit at entry): this level, in the
                // direction already chosen, goes through the per-level kernels
                same_level = true;
                skip_engine = true;
            }
            continue;   // the host decides the next level
        }

        uint64_t* slot = counters + (size_t)(level % SLOTS) * SLOT_WORDS;
        uint64_t* zslot = counters + (size_t)((level + 1) % SLOTS) * SLOT_WORDS;

        const int32_t next_depth = level + 1;
        bool prepass = false;
        bool skipped_depth = false;   // this level's winners left their depth to the next level
        if (cur_dir == 0) {
            if (m_f > 0) {
                // a heavy top-down level of an any-parent search first lets
                // every unvisited vertex check its two hub neighbours in the
                // on-chip copy of the hubs' frontier bits; those it finds are
                // visited before the edge pass, whose probes then skip them,
                // which saves most of its claim atomics
                prepass = any_bitmap && o.dir == BFS_DIR_DO && g->nhub > 0 && prepass_edges >= 0 &&
                          m_f >= prepass_edges;
                if (prepass) {
                    HIP_TRY(T.begin(BFS_K_CONVERT));
                    if (fbits_stale) {
                        launch_clear_words(L, fbits, W);
                        launch_queue_to_bitmap(L, qcur, qlen, fbits);
                        fbits_stale = false;
                    }
                    uint64_t* hb = (uint64_t*)(ws + Lo.hb);
                    launch_hub_gather(L, fbits, g->d_hubid, g->nhub, hb);
                    HIP_TRY(hipGetLastError());
                    HIP_TRY(T.end(BFS_K_CONVERT, level));
                    HIP_TRY(T.begin(BFS_K_TD_EXPAND));
                    launch_bu_sweep<OffT>(L, g->d_hubr, 3, g->d_iso, g->d_nbase, off, g->cols, fbits, hb, nbits,
                                          visited, vprev, parent, depth, W, next_depth, serial, slot, zslot,
                                          !out_filled, n, src, nullptr, 0, 0, depth_pending);
                    depth_pending = false;
                    if (!out_filled) fill_level = level;
                    out_filled = true;
                    HIP_TRY(hipGetLastError());
                    HIP_TRY(T.end(BFS_K_TD_EXPAND, level));
                    if (st) { st->launches[BFS_K_CONVERT] += 1; st->launches[BFS_K_TD_EXPAND] += 1; }
                }
                int nl = 0;
                const int64_t seg_min = o.td_seg_edges > 0 ? o.td_seg_edges : TD_SEG_MIN_EDGES;
                const int tds = m_f >= seg_min ? o.td_segments : 0;
                if (depth_pending) {
                    // the frontier's depths, left by the level before
                    HIP_TRY(T.begin(BFS_K_CONVERT));
                    launch_queue_depth(L, qcur, nullptr, qlen, depth, level);
                    HIP_TRY(hipGetLastError());
                    HIP_TRY(T.end(BFS_K_CONVERT, level));
                    if (st) st->launches[BFS_K_CONVERT] += 1;
                    depth_pending = false;
                }
                skipped_depth = defer_depth && !out_filled && tds == 0;
                if (tds > 0) {
                    // column segments in ascending order: each pass expands
                    // only the frontier's entries inside its id range, so
                    // its probes and claims touch only that slice of the
                    // visited bitmap; the claims are exact in every mode,
                    // so the order does not change the result
                    int32_t* segpos = (int32_t*)(ws + Lo.segpos);
                    int64_t* segtot = (int64_t*)(ws + Lo.segtot);
                    const int64_t segw = (W + tds - 1) / tds;
                    HIP_TRY(T.begin(BFS_K_TD_EXPAND));
                    for (int sg = 0; sg < tds; ++sg) {
                        const int64_t lo = std::min<int64_t>(n, sg * segw * 64);
                        const int64_t hi = sg == tds - 1 ? n : std::min<int64_t>(n, (sg + 1) * segw * 64);
                        nl += launch_td_scan_seg<OffT>(L, off, g->cols, qcur, qlen_dev, qlen, lo, hi, scan, tiles,
                                                       partial, segpos, segtot);
                        launch_td_expand<OffT>(L, claim_mode, off, g->cols, g->nnz, qcur, qlen_dev, qlen, scan, tiles,
                                               m_f, parent, depth, visited, claim, qnext, slot, zslot, next_depth,
                                               segtot, segpos, o.td_block);
                    }
                    HIP_TRY(hipGetLastError());
                    HIP_TRY(T.end(BFS_K_TD_EXPAND, level));
                } else {
                    HIP_TRY(T.begin(BFS_K_TD_SCAN));
                    nl = launch_td_scan<OffT>(L, off, qcur, qlen_dev, qlen, scan, tiles, partial, nullptr);
                    HIP_TRY(hipGetLastError());
                    HIP_TRY(T.end(BFS_K_TD_SCAN, level));
                    HIP_TRY(T.begin(BFS_K_TD_EXPAND));
                    launch_td_expand<OffT>(L, claim_mode, off, g->cols, g->nnz, qcur, qlen_dev, qlen, scan, tiles,
                                           m_f, parent, skipped_depth ? nullptr : depth, visited, claim, qnext, slot,
                                           zslot, next_depth, nullptr, nullptr, o.td_block);
                    HIP_TRY(hipGetLastError());
                    HIP_TRY(T.end(BFS_K_TD_EXPAND, level));
                }
                HIP_TRY(T.begin(BFS_K_CONVERT));
                fbits_stale = false;
                if (claim_mode == CLAIM_BENIGN) launch_merge_exact<OffT>(L, off, visited, vprev, fbits, W, slot);
                else launch_merge(L, claim_mode == CLAIM_MIN, visited, vprev, claim, fbits, W);
                HIP_TRY(hipGetLastError());
                HIP_TRY(T.end(BFS_K_CONVERT, level));
                if (st) {
                    st->launches[BFS_K_TD_SCAN] += nl;
                    st->launches[BFS_K_TD_EXPAND] += tds > 0 ? tds : 1;
                    st->launches[BFS_K_CONVERT] += 1;
                }
            }
            // with m_f == 0 nothing is launched: the slot was cleared by the
            // previous level (or by init) and reads as an empty next frontier
        } else {
            if (fbits_stale) {
                HIP_TRY(T.begin(BFS_K_CONVERT));
                launch_clear_words(L, fbits, W);
                launch_queue_to_bitmap(L, qcur, qlen, fbits);
                HIP_TRY(hipGetLastError());
                HIP_TRY(T.end(BFS_K_CONVERT, level));
                if (st) st->launches[BFS_K_CONVERT] += 2;
                fbits_stale = false;
            }
            const bool from_td = !prev_bu;   // the previous level ran top-down
            fmt_queue = false;
            // any-parent searches probe the highest-degree neighbours first.
            // On a bottom-up level entered from top-down (small frontier, many
            // misses) of a graph whose frontier bitmap exceeds the L2, the two
            // hub neighbours are probed in an LDS copy of the hubs' frontier
            // bits; later levels (large frontiers, nearly all hits on the first
            // hub) keep three hubs and skip the per-level gather.
            const bool ranked = g->nhub > 0 && (o.bu_head == 3 || (o.bu_head == 0 && from_td && g->hub_auto));
            const int hk = claim_mode == CLAIM_MIN || o.bu_head == 1 ? 0 : ranked ? 2 : 1;
            uint64_t* hb = (uint64_t*)(ws + Lo.hb);
            if (hk == 2) {
                HIP_TRY(T.begin(BFS_K_CONVERT));
                launch_hub_gather(L, fbits, g->d_hubid, g->nhub, hb);
                HIP_TRY(hipGetLastError());
                HIP_TRY(T.end(BFS_K_CONVERT, level));
                if (st) st->launches[BFS_K_CONVERT] += 1;
            }
            // column-blocked level: the sweep leaves the row scans to one
            // sub-step per column segment, in ascending order; the pending
            // lists live in the queue and scan areas, unused by a
            // bottom-up level
            const int segs = o.bu_segments;
            uint64_t* pend_a = segs ? (uint64_t*)(ws + Lo.q0) : nullptr;
            uint64_t* pend_b = (uint64_t*)(ws + Lo.scan);
            HIP_TRY(T.begin(BFS_K_BU_SWEEP));
            launch_bu_sweep<OffT>(L, hk == 2 ? g->d_hubr : hk == 1 ? g->d_hub : g->d_head, hk, g->d_iso, g->d_nbase,
                                  off, g->cols, fbits, hb, nbits, visited, vprev, parent, depth, W, next_depth, serial,
                                  slot, zslot, !out_filled, n, src, pend_a, o.bu_block, o.bu_group, depth_pending);
            depth_pending = false;
            if (!out_filled) fill_level = level;
            out_filled = true;
            const int64_t segw = segs ? (W + segs - 1) / segs : 0;
            for (int sg = 0; sg < segs; ++sg) {
                const int64_t seg_end = sg == segs - 1 ? n : std::min<int64_t>(n, (sg + 1) * segw * 64);
                launch_bu_segment<OffT>(L, off, g->cols, fbits, sg % 2 ? pend_b : pend_a, slot + S_PEND0 + sg,
                                        sg % 2 ? pend_a : pend_b, slot + S_PEND0 + sg + 1, seg_end, parent, depth,
                                        nbits, visited, vprev, next_depth, serial, slot);
            }
            HIP_TRY(hipGetLastError());
            HIP_TRY(T.end(BFS_K_BU_SWEEP, level));
            if (st) st->launches[BFS_K_BU_SWEEP] += 1 + segs;
        }
        {
            bfs_status rs = readback(ctx, stream, slot, SLOT_WORDS, &h);
            if (rs != BFS_OK) return rs;
        }
        int64_t n_next = (int64_t)slot_sum(h, S_NNEXT);
        int64_t m_next = (int64_t)slot_sum(h, S_MNEXT);
        const bool benign_td = claim_mode == CLAIM_BENIGN && cur_dir == 0 && m_f > 0;
        if (benign_td) {
            // the expansion counted every copy a thread took; the merge
            // counted the new vertices and their edges once
            const int64_t distinct = (int64_t)slot_sum(h, S_DISTINCT);
            if (st) {
                st->td_claims += n_next;
                st->td_duplicates += n_next - distinct;
            }
            n_next = distinct;
            m_next = (int64_t)slot_sum(h, S_MDISTINCT);
        }
        const int64_t lvl_examined = cur_dir == 0 ? m_f : (int64_t)slot_sum(h, S_EXAMINED);
        examined += lvl_examined;
        if (st && level < BFS_STATS_MAX_LEVELS) {
            st->level_dir[level] = (int8_t)cur_dir;
            st->level_nf[level] = n_f;
            st->level_mf[level] = m_f;
            st->level_mu[level] = m_u;
            st->level_unvisited[level] = unvisited;
            st->level_examined[level] = lvl_examined;
        }
        if (st) {
            if (cur_dir == 0) st->td_levels++; else st->bu_levels++;
        }
        ++level;
        if (n_next == 0) break;
        depth_pending = skipped_depth;
        reached += n_next;
        unvisited -= n_next;
        m_u -= m_next;
        n_f = n_next;
        m_f = m_next;
        prev_bu = cur_dir == 1;
        if (prepass || benign_td) {
            // the next frontier is the merge's bitmap (the queue holds only
            // the edge pass's winners, or nothing after a benign-race level)
            fmt_queue = false;
            qlen_dev = nullptr;
        } else if (cur_dir == 0) {
            qlen = (int64_t)h[S_QLEN];
            qlen_dev = nullptr;
            int32_t* t = qcur; qcur = qnext; qnext = t;
        } else {
            uint64_t* t = fbits; fbits = nbits; nbits = t;
        }
        if (level > n + 1) return fail(BFS_E_HIP, "level loop did not terminate");
    }
    if (depth_pending) {
        // not reached: a level with no winners ends the search, and the
        // winners of the level before had their depth written at its start
        return fail(BFS_E_HIP, "internal: a frontier's depths were left unwritten");
    }
    if (!out_filled) {
        fill_level = -2;
        HIP_TRY(T.begin(BFS_K_INIT));
        launch_fill_unreached(L, parent, depth, n, visited, g->d_iso, src);
        HIP_TRY(hipGetLastError());
        HIP_TRY(T.end(BFS_K_INIT, -1));
        if (st) st->launches[BFS_K_INIT] += 1;
    }
    if (st) {
        st->levels = level;
        st->fill_level = fill_level;
        st->reached = reached;
        st->isolated = g->isolated;
        st->edges_examined = examined;
        if (T.mode) {
            // the last timed kernel's end event is enough: the events are
            // read, nothing else on the stream is waited for
            if (!T.recs.empty()) HIP_TRY(hipEventSynchronize(ctx->events[T.recs.back().ev + 1]));
            T.collect(st);
        }
        st->total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return BFS_OK;
}

template <typename OffT>
bfs_status run_multi(bfs_graph* g, const int64_t* h_src, int k, const bfs_opts& o, int32_t* parent, int32_t* depth,
                     char* ws, hipStream_t stream, bfs_stats* st) {
    const auto t_start = std::chrono::steady_clock::now();
    const OffT* off = (const OffT*)g->off;
    const int64_t n = g->n;
    const MultiLayout Lo = multi_layout(g);
    uint64_t* counters = (uint64_t*)(ws + Lo.counters);
    int64_t* d_src = (int64_t*)(ws + Lo.src);
    uint64_t* visited = (uint64_t*)(ws + Lo.visited);
    uint64_t* F = (uint64_t*)(ws + Lo.F);
    uint64_t* N = (uint64_t*)(ws + Lo.N);
    uint64_t* hubmark = (uint64_t*)(ws + Lo.hubmark);
    int32_t* qa = (int32_t*)(ws + Lo.qa);
    int32_t* qb = (int32_t*)(ws + Lo.qb);
    int64_t* scan = (int64_t*)(ws + Lo.scan);
    int32_t* tiles = (int32_t*)(ws + Lo.tiles);
    int64_t* partial = (int64_t*)(ws + Lo.partial);
    int32_t* par_vm = (int32_t*)(ws + Lo.par);
    uint16_t* lvl_vm = (uint16_t*)(ws + Lo.lvl);
    const uint64_t full = k == 64 ? ~0ull : ((1ull << k) - 1);
    const int serial = o.bu_serial > 0 ? o.bu_serial : 16;
    Launch L{stream, o.grid_blocks > 0 ? o.grid_blocks : 2048};
    HostCtx* ctx = nullptr;
    HIP_TRY(host_ctx(&ctx));
    Timer T{ctx, stream, o.timing, {}, 0};
    uint64_t* hp = ctx->pinned;
    const uint64_t* h = nullptr;   // counters of the last readback, in the mailbox

    // sources travel through the pinned buffer (k <= 64 ids)
    std::memcpy(hp, h_src, sizeof(int64_t) * (size_t)k);
    HIP_TRY(hipMemcpyAsync(d_src, hp, sizeof(int64_t) * (size_t)k, hipMemcpyHostToDevice, stream));
    uint64_t* slot_init = counters + (size_t)(SLOTS - 1) * SLOT_WORDS;   // "level -1"
    HIP_TRY(T.begin(BFS_K_INIT));
    launch_ms_init<OffT>(L, off, n, k, d_src, g->d_iso, visited, F, N, par_vm, lvl_vm, qa, counters, slot_init);
    launch_clear_words(L, hubmark, (n + 63) / 64 + 1);
    HIP_TRY(hipGetLastError());
    HIP_TRY(T.end(BFS_K_INIT, -1));
    {
        bfs_status rs = readback(ctx, stream, slot_init, SLOT_WORDS, &h);
        if (rs != BFS_OK) return rs;
    }
    if (st) st->launches[BFS_K_INIT] += 2;

    int64_t n_f = (int64_t)slot_sum(h, M_SLOT_NNEXT), m_f = (int64_t)slot_sum(h, M_SLOT_MNEXT);
    int64_t qlen = (int64_t)h[M_SLOT_QLEN];   // frontier vertices with edges (all of them after level 0)
    int64_t m_u = g->nnz - (k == 1 ? m_f : 0);
    int cur_dir = (o.dir == BFS_DIR_BU) ? 1 : 0;
    bool fq_valid = true;          // qa lists the vertices with F != 0 (n_f of them)
    int n_dirty = 0;               // N: 0 clean, 1 dirty at the qb list (nd_len), 2 dirty anywhere
    int64_t nd_len = 0;
    int level = 0;
    int64_t examined = 0, reached_pairs = 0;
    // persistent engine for runs of small top-down levels (the same knobs as
    // the single-source engine: small_edges < 0 switches it off)
    // on graphs whose rows are all short the level kernels take one frontier
    // vertex per thread, and the engine is off unless asked for
    const bool short_rows = g->max_degree >= 0 && g->max_degree <= MS_ROWS_MAX_DEG;
    bool engine_on = o.small_edges > 0 || (o.small_edges == 0 && !short_rows);
    // edge cap of an engine level: the first level of a run is also held to
    // 2^16 edges and the later ones to rows of at most 4096 entries
    const int64_t eng_cap = o.persist_edges > 0 ? o.persist_edges : ((int64_t)1 << 18);
    int eng_groups = o.persist_groups > 0 ? o.persist_groups : 64;
    eng_groups = std::max(1, std::min(eng_groups, g->ms_groups_max));
    bool skip_engine = false;
    int64_t fmaxdeg = -1;   // longest row of the current frontier, -1 when not known
    for (;;) {
        if (level >= 65535) return fail(BFS_E_UNSUPPORTED, "more than 65535 levels");
        if (o.dir == BFS_DIR_TD) cur_dir = 0;
        else if (o.dir == BFS_DIR_BU) cur_dir = 1;
        else if (cur_dir == 0) { if ((double)m_f * o.alpha > (double)m_u) cur_dir = 1; }
        else { if ((double)n_f * o.beta < (double)n) cur_dir = 0; }
        uint64_t* slot = counters + (size_t)(level % SLOTS) * SLOT_WORDS;
        uint64_t* zslot = counters + (size_t)((level + 1) % SLOTS) * SLOT_WORDS;
        uint64_t* pslot = counters + (size_t)((level + SLOTS - 1) % SLOTS) * SLOT_WORDS;
        const uint16_t next_level = (uint16_t)(level + 1);
        // the engine's own entry test: rows known to be short, or few edges
        const bool eng_fits = fmaxdeg < 0 ? m_f <= std::min(eng_cap, MS_ENGINE_FIRST_CAP)
                                          : m_f <= eng_cap && fmaxdeg <= MS_ENGINE_MAX_DEG;
        if (cur_dir == 0 && engine_on && !skip_engine && m_f > 0 && eng_fits) {
            // the engine needs the frontier as a queue and N clean
            HIP_TRY(T.begin(BFS_K_CONVERT));
            if (!fq_valid) {
                launch_ms_mask_to_queue(L, F, n, qa, slot + M_SLOT_CONV);
                fq_valid = true;
                qlen = n_f;
            }
            if (n_dirty == 2) launch_clear_words(L, N, n);
            else if (n_dirty == 1 && nd_len > 0) launch_ms_clear_queue(L, qb, nullptr, nd_len, N);
            n_dirty = 0;
            launch_clear_words(L, (uint64_t*)(ws + Lo.pctl), (int64_t)((Lo.ctl_end - Lo.pctl) / sizeof(uint64_t)));
            HIP_TRY(hipGetLastError());
            HIP_TRY(T.end(BFS_K_CONVERT, level));
            const int rec_cap = (st && level < BFS_STATS_MAX_LEVELS) ? BFS_STATS_MAX_LEVELS - level : 0;
            const double eng_alpha = o.dir == BFS_DIR_TD ? 0.0 : o.alpha;
            HIP_TRY(T.begin(BFS_K_MS_LEVEL));
            launch_ms_persist<OffT>(L, eng_groups, off, g->cols, n, full, F, N, visited, qa, qb, par_vm, lvl_vm,
                                    hubmark, serial, MsIn{qlen, n_f, m_f, m_u, level, fmaxdeg},
                                    (MsState*)(ws + Lo.mstate),
                                    (uint64_t*)(ws + Lo.pctr), (PersistCtl*)(ws + Lo.pctl), (int64_t*)(ws + Lo.mrec),
                                    rec_cap, eng_alpha, eng_cap, 65535 - level, counters);
            HIP_TRY(hipGetLastError());
            HIP_TRY(T.end(BFS_K_MS_LEVEL, -1));
            const uint64_t* hb = nullptr;
            {
                // the state, then (after its alignment) the level records, in one copy
                const int nw = (int)((Lo.mrec - Lo.mstate) / sizeof(uint64_t)) + 5 * rec_cap;
                bfs_status rs = readback(ctx, stream, ws + Lo.mstate, nw, &hb);
                if (rs != BFS_OK) return rs;
            }
            MsState es;
            std::memcpy(&es, hb, sizeof(es));
            const int64_t* recs = (const int64_t*)((const char*)hb + (Lo.mrec - Lo.mstate));
            if (st) st->launches[BFS_K_MS_LEVEL] += 1;
            if (es.reason == ENG_NOT_RUN) {
                // the workgroups could not all be resident at once: nothing
                // was touched, this level goes through the per-level kernels
                engine_on = false;
                continue;
            }
            if (es.reason == ENG_TIMEOUT) return fail(BFS_E_HIP, "multi-source engine: grid barrier timed out");
            if (st) {
                for (int64_t i = 0; i < es.levels_done && i < rec_cap; ++i) {
                    const int lv = level + (int)i;
                    const int64_t* r = recs + i * 5;
                    st->level_dir[lv] = 0;
                    st->level_nf[lv] = r[0];
                    st->level_mf[lv] = r[1];
                    st->level_mu[lv] = r[2];
                    st->level_unvisited[lv] = -1;
                    st->level_examined[lv] = r[4];
                }
                st->td_levels += (int32_t)es.levels_done;
            }
            if (es.swapped) {
                uint64_t* t = F; F = N; N = t;
                int32_t* tq = qa; qa = qb; qb = tq;
            }
            level += (int)es.levels_done;
            examined += es.examined;
            reached_pairs += es.reached;
            qlen = es.qlen;
            n_f = es.n_f;
            m_f = es.m_f;
            m_u = es.m_u;
            fmaxdeg = es.maxdeg;
            fq_valid = true;
            if (es.reason == ENG_EMPTY) break;
            // a cap hit at entry: this level through the per-level kernels
            skip_engine = es.levels_done == 0;
            continue;
        }
        skip_engine = false;
        if (cur_dir == 0) {
            HIP_TRY(T.begin(BFS_K_CONVERT));
            int conv = 0;
            if (!fq_valid) {
                launch_ms_mask_to_queue(L, F, n, qa, slot + M_SLOT_CONV);
                fq_valid = true;
                qlen = n_f;
                ++conv;
            }
            if (n_dirty == 2) { launch_clear_words(L, N, n); ++conv; }
            else if (n_dirty == 1 && nd_len > 0) { launch_ms_clear_queue(L, qb, nullptr, nd_len, N); ++conv; }
            HIP_TRY(hipGetLastError());
            HIP_TRY(T.end(BFS_K_CONVERT, level));
            HIP_TRY(T.begin(BFS_K_MS_LEVEL));
            if (m_f > 0)
                launch_ms_td<OffT>(L, off, g->cols, g->nnz, qa, qlen, m_f, scan, tiles, partial, F, N, visited, full,
                                   qb, par_vm, lvl_vm, next_level, serial, hubmark, slot, zslot, g->max_degree);
            HIP_TRY(hipGetLastError());
            HIP_TRY(T.end(BFS_K_MS_LEVEL, level));
            if (st) { st->launches[BFS_K_CONVERT] += conv; st->launches[BFS_K_MS_LEVEL] += m_f > 0 ? 3 : 0; }
        } else {
            HIP_TRY(T.begin(BFS_K_MS_LEVEL));
            launch_ms_bu<OffT>(L, off, g->cols, n, F, N, visited, full, pslot + M_SLOT_OR, par_vm, lvl_vm,
                               next_level, serial, slot, zslot);
            HIP_TRY(hipGetLastError());
            HIP_TRY(T.end(BFS_K_MS_LEVEL, level));
            if (st) st->launches[BFS_K_MS_LEVEL] += 1;
        }
        {
            bfs_status rs = readback(ctx, stream, slot, SLOT_WORDS, &h);
            if (rs != BFS_OK) return rs;
        }
        const int64_t n_next = (int64_t)slot_sum(h, M_SLOT_NNEXT), m_next = (int64_t)slot_sum(h, M_SLOT_MNEXT);
        const int64_t lvl_exam = cur_dir == 0 ? m_f + (int64_t)slot_sum(h, M_SLOT_EXAM) : (int64_t)slot_sum(h, M_SLOT_EXAM);
        examined += lvl_exam;
        if (st && level < BFS_STATS_MAX_LEVELS) {
            st->level_dir[level] = (int8_t)cur_dir;
            st->level_nf[level] = n_f;
            st->level_mf[level] = m_f;
            st->level_mu[level] = m_u;
            st->level_unvisited[level] = -1;
            st->level_examined[level] = lvl_exam;
        }
        if (st) { if (cur_dir == 0) st->td_levels++; else st->bu_levels++; }
        // the longest row of the next frontier: recorded by a top-down
        // level's resolve pass, not known after a bottom-up level
        fmaxdeg = cur_dir == 0 ? (int64_t)slot_max(h, M_SLOT_MAXDEG) : -1;
        // frontier <- next; the old frontier array becomes the next buffer
        uint64_t* t = F; F = N; N = t;
        if (cur_dir == 0) {
            int32_t* tq = qa; qa = qb; qb = tq;   // qa: new frontier list, qb: dirty list of N
            n_dirty = 1;
            nd_len = qlen;
            qlen = n_next;
            fq_valid = true;
        } else {
            if (fq_valid) {
                int32_t* tq = qa; qa = qb; qb = tq;
                n_dirty = 1;
                nd_len = qlen;
            } else {
                n_dirty = 2;
            }
            fq_valid = false;
        }
        ++level;
        if (n_next == 0) break;
        reached_pairs += n_next;
        m_u -= (int64_t)slot_sum(h, M_SLOT_MFULL);
        n_f = n_next;
        m_f = m_next;
    }
    HIP_TRY(T.begin(BFS_K_MS_OUTPUT));
    launch_ms_output(L, n, k, d_src, visited, g->d_iso, par_vm, lvl_vm, parent, depth);
    HIP_TRY(hipGetLastError());
    HIP_TRY(T.end(BFS_K_MS_OUTPUT, -1));
    HIP_TRY(hipStreamSynchronize(stream));
    if (st) {
        st->launches[BFS_K_MS_OUTPUT] += 1;
        st->levels = level;
        st->fill_level = -1;
        st->reached = reached_pairs;
        st->isolated = g->isolated;
        st->edges_examined = examined;
        if (T.mode) T.collect(st);
        st->total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return BFS_OK;
}

template <typename OffT>
bfs_status build_derived(bfs_graph* g, hipStream_t s) {
    const int64_t W = (g->n + 63) / 64;
    HIP_TRY(hipMalloc((void**)&g->d_iso, sizeof(uint64_t) * (size_t)(W + 1)));
    uint64_t* d_count = g->d_iso + W;
    HIP_TRY(hipMemsetAsync(d_count, 0, sizeof(uint64_t), s));
    Launch L{s, 4096};
    launch_isolated_mask<OffT>(L, (const OffT*)g->off, g->n, W, g->d_iso, d_count);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(g->h_buf, d_count, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    g->isolated = (int64_t)g->h_buf[0];
    const int64_t nrec = g->n - g->isolated;
    HIP_TRY(hipMalloc((void**)&g->d_nbase, sizeof(uint32_t) * (size_t)W));
    struct Scratch {   // scan partials, released on every return
        int64_t* p = nullptr;
        ~Scratch() { if (p) (void)hipFree(p); }
    } partial;
    HIP_TRY(hipMalloc((void**)&partial.p, sizeof(int64_t) * (size_t)((W + SCAN_TILE - 1) / SCAN_TILE + 2)));
    launch_head_index(L, g->d_iso, W, g->d_nbase, partial.p);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMalloc((void**)&g->d_head, sizeof(int4) * (size_t)(nrec > 0 ? nrec : 1)));
    launch_row_heads<OffT>(L, (const OffT*)g->off, g->cols, g->n, g->d_iso, g->d_nbase, g->d_head);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMalloc((void**)&g->d_hub, sizeof(int4) * (size_t)(nrec > 0 ? nrec : 1)));
    launch_hub_heads<OffT>(L, (const OffT*)g->off, g->cols, g->n, g->d_iso, g->d_nbase, g->d_hub);
    HIP_TRY(hipGetLastError());
    // hubs: the smallest degree threshold that leaves fewer than HUB_BITS
    // vertices at or above it (none when even the top histogram bin is larger)
    struct Tmp {
        void* p = nullptr;
        ~Tmp() { if (p) (void)hipFree(p); }
    } hist, mask, hbase;
    HIP_TRY(hipMalloc(&hist.p, sizeof(uint32_t) * HUB_HIST_BINS));
    HIP_TRY(hipMemsetAsync(hist.p, 0, sizeof(uint32_t) * HUB_HIST_BINS, s));
    launch_deg_hist<OffT>(L, (const OffT*)g->off, g->n, (uint32_t*)hist.p, HUB_HIST_BINS);
    HIP_TRY(hipGetLastError());
    std::vector<uint32_t> hh(HUB_HIST_BINS);
    HIP_TRY(hipMemcpyAsync(hh.data(), hist.p, sizeof(uint32_t) * HUB_HIST_BINS, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int64_t nhub = 0, thr = 0;
    g->max_degree = 0;
    for (int64_t d = HUB_HIST_BINS - 1; d >= 1; --d)
        if (hh[d]) { g->max_degree = d; break; }   // the last bin holds every longer row too
    for (int64_t d = HUB_HIST_BINS - 1; d >= 1; --d) {
        if (nhub + hh[d] > HUB_BITS - 1) break;
        nhub += hh[d];
        thr = d;
    }
    if (nhub > 0) {
        HIP_TRY(hipMalloc(&mask.p, sizeof(uint64_t) * (size_t)W));
        HIP_TRY(hipMalloc(&hbase.p, sizeof(uint32_t) * (size_t)W));
        HIP_TRY(hipMalloc((void**)&g->d_hubid, sizeof(int32_t) * (size_t)nhub));
        HIP_TRY(hipMalloc((void**)&g->d_hubr, sizeof(int4) * (size_t)(nrec > 0 ? nrec : 1)));
        launch_hub_ranks<OffT>(L, (const OffT*)g->off, g->n, thr, g->d_hub, nrec, (uint64_t*)mask.p,
                               (uint32_t*)hbase.p, partial.p, g->d_hubid, g->d_hubr);
        HIP_TRY(hipGetLastError());
        g->nhub = (int)nhub;
    }
    HIP_TRY(hipStreamSynchronize(s));
    return BFS_OK;
}

}  // namespace

namespace bfsk {
int64_t graph_vertices(const bfs_graph* g) { return (g && g->kind == KIND_CSR) ? g->n : 0; }
void set_last_error(const char* msg) { g_err = msg ? msg : ""; }
}  // namespace bfsk

// ---------------------------------------------------------- allocation-free block top-down
// bfs_block_td_noalloc works in this file-scope device array instead of a
// caller workspace.  Host code never passes `scratch` itself to a kernel (its
// host-side name is not a device address): the device address is looked up
// once per device with hipGetSymbolAddress and kept in g_na[device].ptr.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
struct NoAllocDevice {
    bool ready = false;       // ptr looked up
    void* ptr = nullptr;      // device address of `scratch` on this device
    bool zeroed = false;      // the accumulator regions of `last` hold zeros
    BlockLayout last{};       // layout of the previous call on this device
};
std::mutex g_na_mu;
NoAllocDevice g_na[NOALLOC_MAX_DEVICES];

bool same_layout(const BlockLayout& a, const BlockLayout& b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }
}  // namespace

// ================================================================== C ABI
extern "C" {

void bfs_opts_default(bfs_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->dir = BFS_DIR_DO;
    o->parent_mode = BFS_PARENT_ANY;
    o->alpha = 15.0;
    o->beta = 18.0;
}

const char* bfs_last_error(void) { return g_err.c_str(); }

const char* bfs_status_string(bfs_status s) {
    switch (s) {
        case BFS_OK: return "ok";
        case BFS_E_INVALID_ARG: return "invalid argument";
        case BFS_E_OUT_OF_RANGE: return "id out of range";
        case BFS_E_UNSORTED: return "rows not sorted";
        case BFS_E_NOT_SYMMETRIC: return "graph not symmetric";
        case BFS_E_NO_MEMORY: return "out of host memory";
        case BFS_E_HIP: return "HIP runtime error";
        case BFS_E_BUDGET: return "workspace too small";
        case BFS_E_UNSUPPORTED: return "unsupported for this graph or mode";
    }
    return "unknown status";
}

bfs_status bfs_create_graph_csr(int64_t n, const void* d_offsets, int offset_bytes, const int32_t* d_cols,
                                int64_t nnz, uint32_t flags, void* hip_stream, bfs_graph** out) {
    if (!out) return fail(BFS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 0 || n > 2147483647LL) return fail(BFS_E_INVALID_ARG, "n=%lld outside [0, 2^31-1]", (long long)n);
    if (nnz < 0) return fail(BFS_E_INVALID_ARG, "nnz < 0");
    if (offset_bytes != 4 && offset_bytes != 8) return fail(BFS_E_INVALID_ARG, "offset_bytes must be 4 or 8");
    if (offset_bytes == 4 && nnz > 2147483647LL) return fail(BFS_E_INVALID_ARG, "nnz needs int64 offsets");
    if (!d_offsets) return fail(BFS_E_INVALID_ARG, "offsets is NULL");
    if (nnz > 0 && !d_cols) return fail(BFS_E_INVALID_ARG, "cols is NULL");
    if (flags & ~(BFS_GRAPH_SYMMETRIC | BFS_GRAPH_SORTED | BFS_GRAPH_VALIDATE))
        return fail(BFS_E_INVALID_ARG, "unknown flag bits 0x%x", flags);
    bfs_graph* g = new (std::nothrow) bfs_graph();
    if (!g) return fail(BFS_E_NO_MEMORY, "graph handle");
    g->kind = KIND_CSR;
    g->n = n;
    g->nnz = nnz;
    g->off_bytes = offset_bytes;
    g->off = d_offsets;
    g->cols = d_cols;
    g->flags = flags & (BFS_GRAPH_SYMMETRIC | BFS_GRAPH_SORTED);
    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess) e = hipHostMalloc((void**)&g->h_buf, 4096, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete g;
        return fail(BFS_E_HIP, "create: %s", hipGetErrorString(e));
    }
    if ((flags & BFS_GRAPH_VALIDATE) && n > 0) {
        hipStream_t s = (hipStream_t)hip_stream;
        uint32_t* d_err = nullptr;
        e = hipMalloc((void**)&d_err, sizeof(uint32_t));
        if (e == hipSuccess) e = hipMemsetAsync(d_err, 0, sizeof(uint32_t), s);
        if (e == hipSuccess) {
            Launch L{s, 4096};
            if (offset_bytes == 4)
                launch_validate_csr<int32_t>(L, (const int32_t*)d_offsets, d_cols, n, nnz, g->flags, d_err);
            else
                launch_validate_csr<int64_t>(L, (const int64_t*)d_offsets, d_cols, n, nnz, g->flags, d_err);
            e = hipGetLastError();
        }
        uint32_t herr = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&herr, d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipStreamSynchronize(s);
        if (d_err) (void)hipFree(d_err);
        if (e != hipSuccess) {
            bfs_destroy_graph(g);
            return fail(BFS_E_HIP, "validation: %s", hipGetErrorString(e));
        }
        bfs_status bad = BFS_OK;
        if (herr & VE_OFFSETS) bad = fail(BFS_E_INVALID_ARG, "offsets not monotone or not ending at nnz");
        else if (herr & VE_RANGE) bad = fail(BFS_E_OUT_OF_RANGE, "column id outside [0, n)");
        else if (herr & VE_UNSORTED) bad = fail(BFS_E_UNSORTED, "a row is not ascending");
        else if (herr & VE_ASYM) bad = fail(BFS_E_NOT_SYMMETRIC, "an entry (u,v) has no (v,u)");
        if (bad != BFS_OK) {
            bfs_destroy_graph(g);
            return bad;
        }
    }
    g->persist_groups_max = g->off_bytes == 4 ? persist_max_groups<int32_t>() : persist_max_groups<int64_t>();
    g->ms_groups_max = g->off_bytes == 4 ? ms_persist_max_groups<int32_t>() : ms_persist_max_groups<int64_t>();
    g->fused_groups_max = g->off_bytes == 4 ? fused_max_groups<int32_t>() : fused_max_groups<int64_t>();
    {
        // hub-ranked probes pay off only when the frontier bitmap does not fit in L2
        int l2 = 0;
        if (hipDeviceGetAttribute(&l2, hipDeviceAttributeL2CacheSize, g->device) != hipSuccess) l2 = 0;
        g->hub_auto = l2 > 0 && (n + 7) / 8 > (int64_t)l2;
    }
    // only in a symmetric graph is a vertex without row entries unreachable
    if (n > 0 && (g->flags & BFS_GRAPH_SYMMETRIC)) {
        bfs_status bs = g->off_bytes == 4 ? build_derived<int32_t>(g, (hipStream_t)hip_stream)
                                          : build_derived<int64_t>(g, (hipStream_t)hip_stream);
        if (bs != BFS_OK) {
            bfs_destroy_graph(g);
            return bs;
        }
    }
    *out = g;
    return BFS_OK;
}

bfs_status bfs_create_graph_dcsc(int64_t nrows, int64_t ncols, int64_t row_base, int64_t col_base, int64_t nzc,
                                 const int32_t* d_jc, const int64_t* d_cp, const int32_t* d_ir, int64_t nzr,
                                 const int32_t* d_jr, const int64_t* d_rp, const int32_t* d_ic, int64_t nnz,
                                 uint32_t flags, void* hip_stream, bfs_graph** out) {
    (void)hip_stream;
    if (!out) return fail(BFS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nrows < 1 || ncols < 1 || nrows > 2147483647LL || ncols > 2147483647LL)
        return fail(BFS_E_INVALID_ARG, "block shape %lld x %lld", (long long)nrows, (long long)ncols);
    if (row_base < 0 || col_base < 0 || col_base + ncols > 2147483648LL)
        return fail(BFS_E_INVALID_ARG, "block base out of range");
    if (nzc < 0 || nzc > ncols || nnz < 0 || (nnz > 0 && (!d_jc || !d_cp || !d_ir)) || !d_cp)
        return fail(BFS_E_INVALID_ARG, "bad DCSC arrays");
    if (d_jr && (nzr < 0 || nzr > nrows || !d_rp || (nnz > 0 && !d_ic)))
        return fail(BFS_E_INVALID_ARG, "bad row-major arrays");
    bfs_graph* g = new (std::nothrow) bfs_graph();
    if (!g) return fail(BFS_E_NO_MEMORY, "graph handle");
    g->kind = KIND_DCSC;
    g->nrows = nrows; g->ncols = ncols; g->row_base = row_base; g->col_base = col_base;
    g->nzc = nzc; g->jc = d_jc; g->cp = d_cp; g->ir = d_ir;
    g->nzr = d_jr ? nzr : 0; g->jr = d_jr; g->rp = d_rp; g->ic = d_ic;
    g->nnz = nnz;
    g->flags = flags & (BFS_GRAPH_SYMMETRIC | BFS_GRAPH_SORTED);
    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess) e = hipHostMalloc((void**)&g->h_buf, 4096, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete g;
        return fail(BFS_E_HIP, "create: %s", hipGetErrorString(e));
    }
    if (flags & BFS_GRAPH_VALIDATE) {
        hipStream_t s = (hipStream_t)hip_stream;
        uint32_t* d_err = nullptr;
        e = hipMalloc((void**)&d_err, sizeof(uint32_t));
        if (e == hipSuccess) e = hipMemsetAsync(d_err, 0, sizeof(uint32_t), s);
        if (e == hipSuccess) {
            Launch L{s, 4096};
            const bool sorted = (g->flags & BFS_GRAPH_SORTED) != 0;
            launch_validate_dcs(L, d_jc, d_cp, d_ir, nzc, ncols, nrows, nnz, sorted, d_err);
            if (d_jr) launch_validate_dcs(L, d_jr, d_rp, d_ic, nzr, nrows, ncols, nnz, sorted, d_err);
            e = hipGetLastError();
        }
        uint32_t herr = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&herr, d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipStreamSynchronize(s);
        if (d_err) (void)hipFree(d_err);
        if (e != hipSuccess) {
            bfs_destroy_graph(g);
            return fail(BFS_E_HIP, "validation: %s", hipGetErrorString(e));
        }
        bfs_status bad = BFS_OK;
        if (herr & VE_OFFSETS) bad = fail(BFS_E_INVALID_ARG, "pointers not monotone or not ending at nnz");
        else if (herr & VE_RANGE) bad = fail(BFS_E_OUT_OF_RANGE, "an id is out of range or the ids are not ascending");
        else if (herr & VE_UNSORTED) bad = fail(BFS_E_UNSORTED, "a column (row) is not ascending");
        if (bad != BFS_OK) {
            bfs_destroy_graph(g);
            return bad;
        }
    }
    *out = g;
    return BFS_OK;
}

void bfs_destroy_graph(bfs_graph* g) {
    if (!g) return;
    if (g->d_iso) (void)hipFree(g->d_iso);
    if (g->d_head) (void)hipFree(g->d_head);
    if (g->d_hub) (void)hipFree(g->d_hub);
    if (g->d_hubid) (void)hipFree(g->d_hubid);
    if (g->d_hubr) (void)hipFree(g->d_hubr);
    if (g->d_nbase) (void)hipFree(g->d_nbase);
    if (g->h_buf) (void)hipHostFree(g->h_buf);
    delete g;
}

size_t bfs_workspace_bytes(const bfs_graph* g, int k) {
    if (!g) return 0;
    if (g->kind == KIND_CSR) {
        if (k < 1 || k > 64) return 0;
        if (k == 1) return single_layout(g).total;
        return multi_bytes(g, k);
    }
    if (g->kind == KIND_DCSC) return block_layout(g).total;
    return 0;
}

bfs_status bfs_run(bfs_graph* g, int64_t source, const bfs_opts* opts, int32_t* d_parent, int32_t* d_depth,
                   void* d_workspace, size_t workspace_bytes, void* hip_stream, bfs_stats* stats) {
    bfs_status s = check_csr_graph(g);
    if (s != BFS_OK) return s;
    bfs_opts o;
    bfs_opts_default(&o);
    if (opts) o = *opts;
    if (o.dir < BFS_DIR_DO || o.dir > BFS_DIR_BU) return fail(BFS_E_INVALID_ARG, "bad dir %d", o.dir);
    if (o.parent_mode != BFS_PARENT_ANY && o.parent_mode != BFS_PARENT_MIN)
        return fail(BFS_E_INVALID_ARG, "bad parent_mode %d", o.parent_mode);
    if (o.td_claim < 0 || o.td_claim > 2) return fail(BFS_E_INVALID_ARG, "bad td_claim %d", o.td_claim);
    if (o.bu_segments < 0 || o.bu_segments > BU_MAX_SEGMENTS)
        return fail(BFS_E_INVALID_ARG, "bu_segments %d outside [0, %d]", o.bu_segments, BU_MAX_SEGMENTS);
    if (o.td_seg_edges < 0) return fail(BFS_E_INVALID_ARG, "td_seg_edges %d < 0", o.td_seg_edges);
    if (o.td_segments < 0 || o.td_segments > TD_MAX_SEGMENTS)
        return fail(BFS_E_INVALID_ARG, "td_segments %d outside [0, %d]", o.td_segments, TD_MAX_SEGMENTS);
    if (o.td_block != 0 && o.td_block != 128 && o.td_block != 256 && o.td_block != 512)
        return fail(BFS_E_INVALID_ARG, "td_block %d not 0, 128, 256 or 512", o.td_block);
    if (o.bu_block != 0 && o.bu_block != 128 && o.bu_block != 256 && o.bu_block != 512)
        return fail(BFS_E_INVALID_ARG, "bu_block %d not 0, 128, 256 or 512", o.bu_block);
    if (o.bu_group < 0 || o.bu_group > WAVE || (o.bu_group & (o.bu_group - 1)))
        return fail(BFS_E_INVALID_ARG, "bu_group %d not 0 or a power of two up to 64", o.bu_group);
    if (!(o.alpha > 0) || !(o.beta > 0)) return fail(BFS_E_INVALID_ARG, "alpha and beta must be > 0");
    if (source < 0 || source >= g->n)
        return fail(BFS_E_OUT_OF_RANGE, "source %lld outside [0, %lld)", (long long)source, (long long)g->n);
    if (!d_parent || !d_depth || !d_workspace) return fail(BFS_E_INVALID_ARG, "NULL output or workspace");
    if ((uintptr_t)d_workspace % ALIGN) return fail(BFS_E_INVALID_ARG, "workspace not 256-byte aligned");
    if (workspace_bytes < single_layout(g).total)
        return fail(BFS_E_BUDGET, "workspace %zu < %zu bytes", workspace_bytes, single_layout(g).total);
    if (o.dir != BFS_DIR_TD && !(g->flags & BFS_GRAPH_SYMMETRIC))
        return fail(BFS_E_UNSUPPORTED, "bottom-up levels need a graph created with BFS_GRAPH_SYMMETRIC");
    if (o.dir != BFS_DIR_TD && o.parent_mode == BFS_PARENT_MIN && !(g->flags & BFS_GRAPH_SORTED))
        return fail(BFS_E_UNSUPPORTED, "minimum parents with bottom-up levels need BFS_GRAPH_SORTED");
    if ((o.bu_segments > 0 || o.td_segments > 0) && !(g->flags & BFS_GRAPH_SORTED))
        return fail(BFS_E_UNSUPPORTED, "column segments need BFS_GRAPH_SORTED (a segment is a sub-range of a row)");
    if (stats) std::memset(stats, 0, sizeof(*stats));
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev != g->device) {
        if (hipSetDevice(g->device) != hipSuccess) return fail(BFS_E_HIP, "hipSetDevice(%d) failed", g->device);
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if (g->off_bytes == 4)
        s = run_single<int32_t>(g, source, o, d_parent, d_depth, (char*)d_workspace, st, stats);
    else
        s = run_single<int64_t>(g, source, o, d_parent, d_depth, (char*)d_workspace, st, stats);
    if (dev != g->device) (void)hipSetDevice(dev);
    return s;
}

bfs_status bfs_run_multi(bfs_graph* g, const int64_t* h_sources, int k, const bfs_opts* opts, int32_t* d_parent,
                         int32_t* d_depth, void* d_workspace, size_t workspace_bytes, void* hip_stream,
                         bfs_stats* stats) {
    bfs_status s = check_csr_graph(g);
    if (s != BFS_OK) return s;
    bfs_opts o;
    bfs_opts_default(&o);
    if (opts) o = *opts;
    if (k < 1 || k > 64) return fail(BFS_E_INVALID_ARG, "k=%d outside [1, 64]", k);
    if (!h_sources) return fail(BFS_E_INVALID_ARG, "sources is NULL");
    for (int j = 0; j < k; ++j)
        if (h_sources[j] < 0 || h_sources[j] >= g->n)
            return fail(BFS_E_OUT_OF_RANGE, "source %d = %lld outside [0, %lld)", j, (long long)h_sources[j],
                        (long long)g->n);
    if (o.dir < BFS_DIR_DO || o.dir > BFS_DIR_BU) return fail(BFS_E_INVALID_ARG, "bad dir %d", o.dir);
    if (!(o.alpha > 0) || !(o.beta > 0)) return fail(BFS_E_INVALID_ARG, "alpha and beta must be > 0");
    if (!d_depth || !d_workspace) return fail(BFS_E_INVALID_ARG, "NULL depth output or workspace");
    if ((uintptr_t)d_workspace % ALIGN) return fail(BFS_E_INVALID_ARG, "workspace not 256-byte aligned");
    if (!(g->flags & BFS_GRAPH_SYMMETRIC) || !(g->flags & BFS_GRAPH_SORTED))
        return fail(BFS_E_UNSUPPORTED, "multi-source search needs a SYMMETRIC and SORTED graph");
    const size_t need = multi_layout(g).total;
    if (workspace_bytes < need) return fail(BFS_E_BUDGET, "workspace %zu < %zu bytes", workspace_bytes, need);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev != g->device) {
        if (hipSetDevice(g->device) != hipSuccess) return fail(BFS_E_HIP, "hipSetDevice(%d) failed", g->device);
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if (g->off_bytes == 4)
        s = run_multi<int32_t>(g, h_sources, k, o, d_parent, d_depth, (char*)d_workspace, st, stats);
    else
        s = run_multi<int64_t>(g, h_sources, k, o, d_parent, d_depth, (char*)d_workspace, st, stats);
    if (dev != g->device) (void)hipSetDevice(dev);
    return s;
}

bfs_status bfs_block_td(bfs_graph* g, const int32_t* d_frontier, int64_t nf, int32_t* d_out_rows,
                        int32_t* d_out_parents, int64_t* d_nout, void* d_workspace, size_t workspace_bytes,
                        void* hip_stream) {
    if (!g || g->kind != KIND_DCSC) return fail(BFS_E_INVALID_ARG, "graph handle is not a DCSC block");
    if (nf < 0 || nf > g->ncols) return fail(BFS_E_INVALID_ARG, "nf=%lld outside [0, ncols]", (long long)nf);
    if ((nf > 0 && !d_frontier) || !d_out_rows || !d_out_parents || !d_nout || !d_workspace)
        return fail(BFS_E_INVALID_ARG, "NULL frontier, output or workspace");
    if ((uintptr_t)d_workspace % ALIGN) return fail(BFS_E_INVALID_ARG, "workspace not 256-byte aligned");
    const BlockLayout Lo = block_layout(g);
    if (workspace_bytes < Lo.total)
        return fail(BFS_E_BUDGET, "workspace %zu < %zu bytes", workspace_bytes, Lo.total);
    hipStream_t st = (hipStream_t)hip_stream;
    Launch L{st, 2048};
    const BlockWs W = block_ws(g, (char*)d_workspace);
    launch_clear_words(L, W.header, 8);
    launch_block_td(L, block_args(g), d_frontier, nf, d_out_rows, d_out_parents, d_nout, W);
    HIP_TRY(hipGetLastError());
    return BFS_OK;
}

bfs_status bfs_block_td_noalloc(bfs_graph* g, const int32_t* d_frontier, int64_t nf, int32_t* d_out_rows,
                                int32_t* d_out_parents, int64_t* d_nout, void* hip_stream) {
    if (!g || g->kind != KIND_DCSC) return fail(BFS_E_INVALID_ARG, "graph handle is not a DCSC block");
    if (nf < 0 || nf > g->ncols) return fail(BFS_E_INVALID_ARG, "nf=%lld outside [0, ncols]", (long long)nf);
    if ((nf > 0 && !d_frontier) || !d_out_rows || !d_out_parents || !d_nout)
        return fail(BFS_E_INVALID_ARG, "NULL frontier or output");
    const BlockLayout Lo = block_layout(g);
    if (Lo.total > NOALLOC_SCRATCH_BYTES)
        return fail(BFS_E_BUDGET, "block needs %zu bytes of scratch, the static array holds %zu", Lo.total,
                    NOALLOC_SCRATCH_BYTES);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != g->device) return fail(BFS_E_INVALID_ARG, "the block lives on device %d, device %d is current",
                                      g->device, dev);
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(BFS_E_UNSUPPORTED, "device %d: too many devices", dev);
    std::lock_guard<std::mutex> lock(g_na_mu);
    NoAllocDevice& D = g_na[dev];
    if (!D.ready) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (uintptr_t)p % ALIGN) return fail(BFS_E_HIP, "scratch array has no usable device address");
        D.ptr = p;
        D.ready = true;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    Launch L{st, 2048};
    // the accumulator, occupied and frontier-mark regions must hold zeros;
    // a call leaves them zeroed at its own layout's offsets, so a different
    // layout (another block shape), the first call, or a failed call clears
    // the whole range this layout uses, with a kernel
    const bool need_clear = !D.zeroed || !same_layout(D.last, Lo);
    D.zeroed = false;   // until this call has been issued completely
    if (need_clear) {
        launch_clear_words(L, (uint64_t*)D.ptr, (int64_t)(Lo.total / sizeof(uint64_t)));
        HIP_TRY(hipGetLastError());
    }
    const BlockWs W = block_ws(g, (char*)D.ptr);
    launch_clear_words(L, W.header, 8);
    launch_block_td(L, block_args(g), d_frontier, nf, d_out_rows, d_out_parents, d_nout, W);
    HIP_TRY(hipGetLastError());
    D.last = Lo;
    D.zeroed = true;
    return BFS_OK;
}

bfs_status bfs_block_set_union(bfs_graph* g, int mode) {
    if (!g || g->kind != KIND_DCSC) return fail(BFS_E_INVALID_ARG, "graph handle is not a DCSC block");
    if (mode < -1 || mode > 1) return fail(BFS_E_INVALID_ARG, "union mode %d outside [-1, 1]", mode);
    g->block_union = mode;
    return BFS_OK;
}

bfs_status bfs_block_bu(bfs_graph* g, const uint64_t* d_fbits, uint64_t* d_completed, int64_t row_lo,
                        int64_t row_hi, int32_t* d_out_rows, int32_t* d_out_parents, int64_t* d_nout,
                        void* d_workspace, size_t workspace_bytes, void* hip_stream) {
    if (!g || g->kind != KIND_DCSC) return fail(BFS_E_INVALID_ARG, "graph handle is not a DCSC block");
    if (!g->jr) return fail(BFS_E_UNSUPPORTED, "the block was created without its row-major copy");
    if (!(g->flags & BFS_GRAPH_SORTED))
        return fail(BFS_E_UNSUPPORTED, "a first-hit row scan needs ascending rows: create with BFS_GRAPH_SORTED");
    if (row_lo < 0 || row_hi > g->nrows || row_lo > row_hi)
        return fail(BFS_E_INVALID_ARG, "row range [%lld, %lld) outside [0, %lld]", (long long)row_lo,
                    (long long)row_hi, (long long)g->nrows);
    if (!d_fbits || !d_completed || !d_out_rows || !d_out_parents || !d_nout || !d_workspace)
        return fail(BFS_E_INVALID_ARG, "NULL bitmap, output or workspace");
    if ((uintptr_t)d_workspace % ALIGN) return fail(BFS_E_INVALID_ARG, "workspace not 256-byte aligned");
    const BlockLayout Lo = block_layout(g);
    if (workspace_bytes < Lo.total)
        return fail(BFS_E_BUDGET, "workspace %zu < %zu bytes", workspace_bytes, Lo.total);
    hipStream_t st = (hipStream_t)hip_stream;
    Launch L{st, 2048};
    const BlockWs W = block_ws(g, (char*)d_workspace);
    launch_clear_words(L, W.header, 8);
    launch_block_bu(L, block_args(g), d_fbits, d_completed, row_lo, row_hi, 16, d_out_rows, d_out_parents,
                    d_nout, W);
    HIP_TRY(hipGetLastError());
    return BFS_OK;
}

}  // extern "C"
