// Internal interface between the host controller (bfs_api.hip) and the
// gfx950 kernels (bfs_kernels.hip, bfs_multi.hip, bfs_block.hip).  Not part
// of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct bfs_graph;

namespace bfsk {

// number of vertices of a CSR graph handle (0 for other handles)
int64_t graph_vertices(const bfs_graph* g);
// sets the calling thread's bfs_last_error() message
void set_last_error(const char* msg);

constexpr int WAVE = 64;
constexpr int TD_BLOCK = 256;                 // threads per top-down expand workgroup
constexpr int TD_EPT = 4;                     // edges per thread per tile
constexpr int TD_TILE = TD_BLOCK * TD_EPT;    // edges per tile
constexpr int HUB_BITS = 65536;               // hub ranks 0..HUB_BITS-2; HUB_BITS-1 marks "not a hub"
constexpr int HUB_HIST_BINS = 1 << 20;        // degree histogram for the hub threshold
constexpr int SCAN_BLOCK = 1024;              // threads per scan workgroup
constexpr int SCAN_IPT = 4;                   // items per scan thread
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_IPT;
constexpr int BU_BLOCK = 256;                 // 4 waves, one 64-vertex word per wave

// Per-level counter slot (uint64 words).  A ring of SLOTS slots lets level
// d write slot d % SLOTS while any kernel of level d clears slot (d+1) % SLOTS.
// A slot is SLOT_SPREAD lines of SLOT_LINE words.  Sums that every workgroup
// adds to (S_NNEXT, S_MNEXT, S_EXAMINED) go to line blockIdx % SLOT_SPREAD of
// their word, and the host adds the lines up: one address taking an atomic
// from each of thousands of workgroups serialises them.  Counters whose
// running value matters on the device (the queue append position S_QLEN,
// word 4 = queue length of a conversion) live in line 0 only.
// S_PEND0 + s (line 0) = length of the pending list of a column-blocked
// bottom-up level's sub-step s (at most BU_MAX_SEGMENTS sub-steps).
enum { S_QLEN = 0, S_NNEXT = 1, S_MNEXT = 2, S_EXAMINED = 3, S_DISTINCT = 5, S_PEND0 = 6, S_MDISTINCT = 15,
       SLOT_LINE = 16, SLOT_SPREAD = 16, SLOT_WORDS = SLOT_LINE * SLOT_SPREAD, SLOTS = 3 };
constexpr int BU_MAX_SEGMENTS = 8;
// top-down column segments: at most this many, by default on levels of at
// least this many frontier edges
constexpr int TD_MAX_SEGMENTS = 8;
constexpr int64_t TD_SEG_MIN_EDGES = (int64_t)1 << 20;
static_assert(S_PEND0 + BU_MAX_SEGMENTS < S_MDISTINCT, "pending counts must fit line 0 of a slot");

// sum of word `w` over the lines of a slot copied to the host
inline uint64_t slot_sum(const uint64_t* h, int w) {
    uint64_t s = 0;
    for (int j = 0; j < SLOT_SPREAD; ++j) s += h[j * SLOT_LINE + w];
    return s;
}

// maximum of word `w` over the lines of a slot copied to the host
inline uint64_t slot_max(const uint64_t* h, int w) {
    uint64_t s = 0;
    for (int j = 0; j < SLOT_SPREAD; ++j) s = h[j * SLOT_LINE + w] > s ? h[j * SLOT_LINE + w] : s;
    return s;
}

// Validation error bits.
enum { VE_OFFSETS = 1, VE_RANGE = 2, VE_UNSORTED = 4, VE_ASYM = 8 };

struct Launch {
    hipStream_t stream;
    int grid_cap;   // workgroup cap for grid-stride kernels
};

// Top-down claim modes.  BENIGN takes a child with no atomic test: every
// thread that saw it unvisited writes its parent (several may, any of them is
// valid) and sets its visited bit with an atomic whose result is unused; the
// level queues nothing, its next frontier is the merge's exact bitmap.
enum { CLAIM_BITMAP = 0, CLAIM_CAS = 1, CLAIM_MIN = 2, CLAIM_BENIGN = 3 };

// ---- single source -------------------------------------------------------
template <typename OffT>
void launch_isolated_mask(const Launch& L, const OffT* off, int64_t n, int64_t W, uint64_t* iso, uint64_t* count);

void launch_init(const Launch& L, int32_t* parent, int32_t* depth, int64_t n, uint64_t* visited, uint64_t* vprev,
                 uint64_t* fbits, uint64_t* claim, const uint64_t* iso, int64_t W, int32_t* queue, int64_t src,
                 uint64_t* counters, int64_t counter_words, bool write_out);
// parent = depth = -1 for every vertex not reached (the source excepted)
void launch_fill_unreached(const Launch& L, int32_t* parent, int32_t* depth, int64_t n, const uint64_t* visited,
                           const uint64_t* iso, int64_t src);
// depth[q[i]] = d for every entry of a queue (qlen_dev, if given, holds its length)
void launch_queue_depth(const Launch& L, const int32_t* q, const uint64_t* qlen_dev, int64_t qlen_host,
                        int32_t* depth, int32_t d);

// degree prefix sum of the frontier queue + tile partition for the expand
// (scan[i] = sum of degrees of q[0..i), tile_start[t] = queue index owning
// edge t*TD_TILE, tile_start[ntiles] = qlen-1).  The queue length is read
// from qlen_dev when it is not NULL (qlen_host is then an upper bound).
// partial needs ceil(qlen_host/SCAN_TILE)+2 int64; total_out (device, may be
// NULL) receives the edge total.
template <typename OffT>
int launch_td_scan(const Launch& L, const OffT* off, const int32_t* q, const uint64_t* qlen_dev, int64_t qlen_host,
                   int64_t* scan, int32_t* tile_start, int64_t* partial, int64_t* total_out);

// total_dev (may be NULL): the edge count on the device (total then bounds
// the grid); segpos (may be NULL): per queue entry, the row position where
// its edges start (a column segment's first entry); block: threads per
// workgroup (128, 512; anything else = TD_BLOCK), the tile stays TD_TILE edges.
// depth may be NULL: the winners' depths are then not written (see the caller)
template <typename OffT>
void launch_td_expand(const Launch& L, int mode, const OffT* off, const int32_t* cols, int64_t nnz,
                      const int32_t* q, const uint64_t* qlen_dev, int64_t qlen_host, const int64_t* scan,
                      const int32_t* tile_start, int64_t total, int32_t* parent, int32_t* depth,
                      uint64_t* visited, uint64_t* claim, int32_t* qnext, uint64_t* slot, uint64_t* zslot,
                      int32_t next_depth, const int64_t* total_dev = nullptr, const int32_t* segpos = nullptr,
                      int block = 0);
// the degree scan of one column segment: each queue entry's entries with ids
// in [lo, hi) (its sorted row's sub-range, found by binary search); their
// start positions go to segpos, the segment's edge total to *total_out
template <typename OffT>
int launch_td_scan_seg(const Launch& L, const OffT* off, const int32_t* cols, const int32_t* q,
                       const uint64_t* qlen_dev, int64_t qlen_host, int64_t lo, int64_t hi, int64_t* scan,
                       int32_t* tile_start, int64_t* partial, int32_t* segpos, int64_t* total_out);

// head kinds (hub): 0 row heads, 1 hub heads, 2 hub heads with hub ranks
// (then hb holds the hubs' frontier bits, HUB_BITS bits), 3 the same probes
// only, as a pre-pass of a top-down level (visited updated, nbits/vprev not).  fill: the outputs
// were not initialised; the sweep also writes -1 to every entry of the
// unreached and isolated vertices (the source, of id src, excepted)
// pend (may be NULL): column-blocked level; rows that need scanning past
// their head are appended to pend (count in slot[S_PEND0]) for the sub-steps.
// block: threads per workgroup (128, 512; anything else = BU_BLOCK);
// group_cap > 0 caps the 64-vertex words per wave's work unit.
// frontier_depth (with fill): the frontier's vertices were reached by a
// top-down level that left their depth unwritten; the sweep writes it
// (next_depth - 1) with the fill
template <typename OffT>
void launch_bu_sweep(const Launch& L, const int4* head, int hub, const uint64_t* iso, const uint32_t* nbase,
                     const OffT* off, const int32_t* cols, const uint64_t* fbits, const uint64_t* hb, uint64_t* nbits,
                     uint64_t* visited, uint64_t* vprev, int32_t* parent, int32_t* depth, int64_t W,
                     int32_t next_depth, int serial_len, uint64_t* slot, uint64_t* zslot, bool fill, int64_t n,
                     int64_t src, uint64_t* pend = nullptr, int block = 0, int group_cap = 0,
                     bool frontier_depth = false);
// one column-segment sub-step: pending rows (count *cin) scanned over their
// entries < seg_end; rows that reach a later segment go to pout (count *cout)
template <typename OffT>
void launch_bu_segment(const Launch& L, const OffT* off, const int32_t* cols, const uint64_t* fbits,
                       const uint64_t* pin, const uint64_t* cin, uint64_t* pout, uint64_t* cout, int64_t seg_end,
                       int32_t* parent, int32_t* depth, uint64_t* nbits, uint64_t* visited, uint64_t* vprev,
                       int32_t next_depth, int serial_len, uint64_t* slot);
// Hub ranks: hist[min(deg, nbins-1)] counts the vertices with edges; the hubs
// are the vertices of degree >= thr (fewer than HUB_BITS); mask (W words),
// hbase (W) and partial (scan scratch) are temporaries; hubid receives the
// hubs in id order and out the rank heads {deg, c0, c1, rank(c0) | rank(c1) << 16}.
template <typename OffT>
void launch_deg_hist(const Launch& L, const OffT* off, int64_t n, uint32_t* hist, int nbins);
template <typename OffT>
void launch_hub_ranks(const Launch& L, const OffT* off, int64_t n, int64_t thr, const int4* hub, int64_t nrec,
                      uint64_t* mask, uint32_t* hbase, int64_t* partial, int32_t* hubid, int4* out);
// hb[r / 64] bit r%64 = frontier bit of hub r (all HUB_BITS bits written)
void launch_hub_gather(const Launch& L, const uint64_t* fbits, const int32_t* hubid, int nhub, uint64_t* hb);
// Head records exist for the vertices with edges only, stored by rank among
// them: record of v = nbase[v/64] + (vertices with edges before v in its word).
// nbase (W entries) from the isolated-vertex bitmap; partial: scan scratch
void launch_head_index(const Launch& L, const uint64_t* iso, int64_t W, uint32_t* nbase, int64_t* partial);
// row heads {degree, first three entries (-1 when absent)}
template <typename OffT>
void launch_row_heads(const Launch& L, const OffT* off, const int32_t* cols, int64_t n, const uint64_t* iso,
                      const uint32_t* nbase, int4* head);
// hub heads {degree, three highest-degree neighbours (-1 when absent)}
template <typename OffT>
void launch_hub_heads(const Launch& L, const OffT* off, const int32_t* cols, int64_t n, const uint64_t* iso,
                      const uint32_t* nbase, int4* hub);

void launch_clear_words(const Launch& L, uint64_t* w, int64_t nw);
// host mailbox: dst[1..nw] = src[0..nw), then dst[0] = seq (dst: coherent pinned host memory)
void launch_post(hipStream_t s, const uint64_t* src, int nw, uint64_t* dst, uint64_t seq);
// host mailbox: dst[1] = off[v], dst[2] = off[v+1], then dst[0] = seq
template <typename OffT>
void launch_post_row(hipStream_t s, const OffT* off, int64_t v, uint64_t* dst, uint64_t seq);
void launch_queue_to_bitmap(const Launch& L, const int32_t* q, int64_t qlen, uint64_t* bits);

// persistent top-down engine state (device memory, read and written by the engine)
struct SmallIn {
    int64_t qlen, n_f, m_f, m_u, level;
};
// why the engine stopped; ENG_NOT_RUN (0, a cleared state) when it could not assemble
enum { ENG_NOT_RUN = 0, ENG_EMPTY = 1, ENG_TO_BU = 2, ENG_EDGE_CAP = 3, ENG_LEVEL_CAP = 4, ENG_TIMEOUT = 5,
       ENG_SHRINK = 6 };
struct SmallState {                                 // written by the engine
    int64_t qlen, n_f, m_f, m_u, level, cur_is_b;   // where the search stands
    int64_t levels_done, reason;
    int64_t found, examined;                        // vertices discovered, entries expanded
};
// grid-barrier control words, cleared before every launch
struct PersistCtl {
    uint32_t roll, bar, err, pad;
};
// the fused whole-search engine's result (in the engine state area)
struct FusedState {
    int64_t levels_done, reason, reached, examined, level;
};
// graphs of at most this many vertices run the fused search by default
constexpr int64_t FUSED_MAX_N = (int64_t)1 << 18;
constexpr int FUSED_GROUPS = 128;   // default workgroups of the fused search
// most workgroups of the fused search that fit on the device at once
template <typename OffT>
int fused_max_groups();
// One whole search (every level, both directions) in one launch.  ctr and
// ctl zero at launch; st reads ENG_NOT_RUN until the engine writes it (then
// levels_done, reason, reached, examined as a FusedState); rec: 6 int64 per
// level (direction, n_f, m_f, m_u, unvisited, entries examined); b0..b2:
// three n/64-word frontier bitmaps.  dir: 0 the Section 4.4 rule, 1
// top-down only, 2 bottom-up only.
template <typename OffT>
void launch_search_fused(const Launch& L, bool min_parent, int groups, const OffT* off, const int32_t* cols,
                         const uint64_t* iso, int64_t n, int64_t nnz, int64_t src, int32_t* parent, int32_t* depth,
                         uint64_t* visited, uint64_t* b0, uint64_t* b1, uint64_t* b2, int dir, double alpha,
                         double beta, int serial, FusedState* st, uint64_t* ctr, PersistCtl* ctl, int64_t* rec,
                         int rec_cap);
// most workgroups of the engine that fit on the device at once
template <typename OffT>
int persist_max_groups();
// ctr: SLOTS * SLOT_WORDS counter words and ctl: barrier words, both zero at
// launch (the engine leaves them dirty); st reads ENG_NOT_RUN until the
// engine writes it; rec: 4 int64 per level (n_f, m_f, m_u, n_next)
template <typename OffT>
void launch_td_persist(const Launch& L, int mode, int groups, const OffT* off, const int32_t* cols, int32_t* parent,
                       int32_t* depth, uint64_t* visited, uint64_t* vprev, uint64_t* claim, int32_t* qa, int32_t* qb,
                       int64_t n, SmallIn in, SmallState* st, uint64_t* ctr, PersistCtl* ctl, int64_t* rec,
                       int rec_cap, double alpha, int64_t edge_cap, int64_t shrink_below, int64_t max_levels,
                       int64_t* gscan, int32_t* gtiles, int64_t* csum);
// queue = set bits of `bits` in ascending order, *qlen_ctr = their count;
// partial: scan scratch of ceil(W / SCAN_TILE) + 2 int64.  Returns launches.
int launch_bitmap_to_queue(const Launch& L, const uint64_t* bits, int64_t W, int32_t* q, uint64_t* qlen_ctr,
                           int64_t* partial);
void launch_merge(const Launch& L, bool min_mode, uint64_t* visited, uint64_t* vprev, uint64_t* claim,
                  uint64_t* fnext, int64_t W);
// the merge of a benign-race top-down level: also the exact next-frontier
// size (slot S_DISTINCT) and edge count (S_MDISTINCT)
template <typename OffT>
void launch_merge_exact(const Launch& L, const OffT* off, const uint64_t* visited, uint64_t* vprev, uint64_t* fnext,
                        int64_t W, uint64_t* slot);

// ---- multi-source --------------------------------------------------------
// NNEXT, MNEXT, MFULL and EXAM are spread over the slot's lines; QLEN, OR and
// CONV live in line 0.
enum { M_SLOT_QLEN = 0, M_SLOT_NNEXT = 1, M_SLOT_MNEXT = 2, M_SLOT_OR = 3, M_SLOT_MFULL = 4, M_SLOT_EXAM = 5,
       M_SLOT_CONV = 6, M_SLOT_MAXDEG = 8 };

template <typename OffT>
void launch_ms_init(const Launch& L, const OffT* off, int64_t n, int k, const int64_t* src, const uint64_t* iso,
                    uint64_t* visited, uint64_t* F, uint64_t* N, int32_t* par_vm, uint16_t* lvl_vm, int32_t* q,
                    uint64_t* counters, uint64_t* slot0);
// max_degree: the graph's longest row (-1 unknown).  Rows of at most
// MS_ROWS_MAX_DEG entries everywhere: the expand takes one frontier vertex
// per thread (no degree scan); no row longer than the hub limit: the hub
// passes are not launched.
template <typename OffT>
void launch_ms_td(const Launch& L, const OffT* off, const int32_t* cols, int64_t nnz, const int32_t* q, int64_t qlen,
                  int64_t total, int64_t* scan, int32_t* tiles, int64_t* partial, const uint64_t* F, uint64_t* N,
                  uint64_t* visited, uint64_t full, int32_t* qnext, int32_t* par_vm, uint16_t* lvl_vm,
                  uint16_t level, int serial, uint64_t* hubmark, uint64_t* slot, uint64_t* zslot,
                  int64_t max_degree);
template <typename OffT>
void launch_ms_bu(const Launch& L, const OffT* off, const int32_t* cols, int64_t n, const uint64_t* F, uint64_t* N,
                  uint64_t* visited, uint64_t full, const uint64_t* active_dev, int32_t* par_vm, uint16_t* lvl_vm,
                  uint16_t level, int serial, uint64_t* slot, uint64_t* zslot);
void launch_ms_mask_to_queue(const Launch& L, const uint64_t* N, int64_t n, int32_t* q, uint64_t* qlen);
// The persistent multi-source engine takes a level only while no frontier
// row is longer than MS_ENGINE_MAX_DEG (a workgroup expands whole rows of its
// queue chunk), and while the rows' lengths are not known only up to
// MS_ENGINE_FIRST_CAP frontier edges.
constexpr int64_t MS_ENGINE_MAX_DEG = 4096;
constexpr int MS_ROWS_MAX_DEG = 32;
constexpr int64_t MS_ENGINE_FIRST_CAP = 65536;
// persistent multi-source top-down engine: inputs, and the state it leaves
struct MsIn {
    int64_t qlen, n_f, m_f, m_u, level;
    int64_t maxdeg;    // longest row in the frontier, -1 when not known
};
struct MsState {
    int64_t qlen, n_f, m_f, m_u, level;
    int64_t levels_done, reason, reached, examined;
    int64_t swapped;   // 1: the frontier masks are now in the array passed as N (and F is clear)
    int64_t maxdeg;    // longest row in the frontier it leaves (-1 when not known)
};
template <typename OffT>
int ms_persist_max_groups();
// F holds the frontier masks (non-zero exactly for qa's qlen entries), N is
// zero.  ctr (SLOTS * SLOT_WORDS words) and ctl zero at launch; rec: 5 int64
// per level (n_f, m_f, m_u, n_next, entries examined); hring: the host's
// counter ring, left cleared except the last level's source bits (M_OR)
template <typename OffT>
void launch_ms_persist(const Launch& L, int groups, const OffT* off, const int32_t* cols, int64_t n, uint64_t full,
                       uint64_t* F, uint64_t* N, uint64_t* visited, int32_t* qa, int32_t* qb, int32_t* par_vm,
                       uint16_t* lvl_vm, uint64_t* hubmark, int serial, MsIn in, MsState* st, uint64_t* ctr,
                       PersistCtl* ctl, int64_t* rec, int rec_cap, double alpha, int64_t edge_cap,
                       int64_t max_levels, uint64_t* hring);
void launch_ms_clear_queue(const Launch& L, const int32_t* q, const uint64_t* qlen_dev, int64_t qlen_host,
                           uint64_t* M);
void launch_ms_output(const Launch& L, int64_t n, int k, const int64_t* src, const uint64_t* visited,
                      const uint64_t* iso, const int32_t* par_vm, const uint16_t* lvl_vm, int32_t* parent,
                      int32_t* depth);

// ---- DCSC block ----------------------------------------------------------
struct BlockArgs {
    int64_t nrows, ncols, col_base, nzc, nzr, nnz;
    bool sorted;   // entries ascending inside every column and row
    // top-down union of the frontier columns: -1 accumulator only, 0 chosen
    // by the expected entry count, 1 sorted union whenever it fits
    int sort_union;
    const int32_t *jc, *ir, *jr, *ic;
    const int64_t *cp, *rp;
};
struct BlockWs {
    uint64_t* header;   // 8 words cleared per call: [0] qlen, [1] total, [2..4] range, [5] skip
    uint64_t* skip;     // set by the sorted union when it wrote the output
    uint64_t* qlen;
    int64_t* total;
    uint64_t* range;
    int32_t* q;
    int64_t* scan;
    int32_t* tiles;
    int64_t* partial;
    uint32_t* spa;      // nrows complemented minimum parents, 0 = empty (kept zero between calls)
    uint64_t* occ;      // occupied rows (kept zero between calls)
    uint64_t* fmark;    // frontier columns of a dense frontier (kept zero between calls)
    int32_t* bpar;
    uint64_t* bmask;
};
void launch_block_td(const Launch& L, const BlockArgs& B, const int32_t* F, int64_t nf, int32_t* out_rows,
                     int32_t* out_parents, int64_t* nout, const BlockWs& W);
void launch_block_bu(const Launch& L, const BlockArgs& B, const uint64_t* fbits, uint64_t* completed,
                     int64_t row_lo, int64_t row_hi, int serial_len, int32_t* out_rows, int32_t* out_parents,
                     int64_t* nout, const BlockWs& W);
void launch_validate_dcs(const Launch& L, const int32_t* j, const int64_t* p, const int32_t* minor, int64_t nz,
                         int64_t nmajor, int64_t nminor, int64_t nnz, bool sorted, uint32_t* err);

template <typename OffT>
void launch_validate_csr(const Launch& L, const OffT* off, const int32_t* cols, int64_t n, int64_t nnz,
                         uint32_t flags, uint32_t* err);

}  // namespace bfsk
