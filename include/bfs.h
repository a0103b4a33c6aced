/*
 * bfs.h -- C ABI of libbfs, a direction-optimizing breadth-first search for
 * one AMD Instinct MI355X (gfx950).
 *
 * The method is the level-synchronous search of Buluc, Beamer, Madduri,
 * Asanovic and Patterson, "Distributed-Memory Breadth-First Search on
 * Massive Graphs": top-down expansion of a frontier queue (Alg. 1; the local
 * discovery and update of Alg. 3), bottom-up search in which each unvisited
 * vertex probes a frontier bitmap and stops at its first hit (Alg. 2; the
 * local discovery of Alg. 4), and the per-level choice between the two from
 * the frontier's edge count (while top-down) and its size (while bottom-up)
 * (Section 4.4).  The graph is one whole CSR graph (Section 5.1) or one
 * hypersparse DCSC block A_ij of a p_r x p_c decomposition (Eq. 1,
 * Section 5.1).
 *
 * Conventions shared by every call:
 *   - Ownership: every device buffer (graph arrays, outputs, workspace) is
 *     allocated and freed by the caller.  A graph handle borrows the graph
 *     arrays until bfs_destroy_graph; the library never frees caller
 *     memory.  The library allocates only metadata at create time: a
 *     pinned host counter buffer, HIP events, and for symmetric CSR
 *     graphs one n/8-byte device bitmap of the vertices without entries
 *     (freed by bfs_destroy_graph).
 *   - Asynchrony: kernels run on the HIP stream passed in (NULL = the null
 *     stream).  bfs_run / bfs_run_multi drive the level loop from the host
 *     and synchronise that stream once per level to read three counters, so
 *     they return with the results complete.  The block calls
 *     (bfs_block_td, bfs_block_bu) are fully asynchronous.
 *   - Errors: every call returns a bfs_status; argument errors are detected
 *     on the host before any launch.  bfs_last_error() returns a
 *     thread-local message for the last failure.  No exception crosses the
 *     ABI.  A call that fails leaves caller buffers in an unspecified state.
 *   - Vertex ids and outputs: int32.  parent[s] = s, depth[s] = 0; vertices
 *     not reached have parent = depth = -1.  Graphs may hold up to 2^31-1
 *     vertices; CSR offsets are int32 (nnz < 2^31) or int64.
 *   - Bitmaps: arrays of uint64 words; bit i of word w stands for id 64*w+i.
 */
#ifndef BFS_MI355X_H
#define BFS_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BFS_OK = 0,
    BFS_E_INVALID_ARG = 1,    /* null pointer, bad size, bad enum value      */
    BFS_E_OUT_OF_RANGE = 2,   /* source or column id outside [0, n)          */
    BFS_E_UNSORTED = 3,       /* SORTED claimed, a row is not ascending      */
    BFS_E_NOT_SYMMETRIC = 4,  /* SYMMETRIC claimed (or needed) and false     */
    BFS_E_NO_MEMORY = 5,      /* host-side metadata allocation failed        */
    BFS_E_HIP = 6,            /* a HIP runtime call or launch failed         */
    BFS_E_BUDGET = 7,         /* workspace smaller than bfs_*_workspace_bytes */
    BFS_E_UNSUPPORTED = 8     /* e.g. bottom-up on a graph not marked symmetric */
} bfs_status;

/* Direction policy (Section 4.4).  DO picks per level; TD and BU force one. */
typedef enum { BFS_DIR_DO = 0, BFS_DIR_TD = 1, BFS_DIR_BU = 2 } bfs_dir;

/* Which parent is reported.  Section 2: any vertex one level closer to the
 * source with an edge to v is a valid parent.  ANY: in top-down levels the
 * first thread to claim v wins -- an atomic fetch-or on v's bit of a claim
 * bitmap (default) or a compare-and-swap on parent[v] (bfs_opts.td_claim);
 * in bottom-up levels v takes the first frontier entry of its row.  MIN
 * reports the smallest such id:
 * the (select2nd, min) semiring of Section 4.2 in top-down levels and the
 * first hit over a sorted row in bottom-up levels.  MIN needs sorted rows
 * when a bottom-up level can run.                                          */
typedef enum { BFS_PARENT_ANY = 0, BFS_PARENT_MIN = 1 } bfs_parent_mode;

/* bfs_create_graph_* flags: what the caller claims about the graph. */
#define BFS_GRAPH_SYMMETRIC 0x1u  /* every (u,v) entry has a (v,u) entry        */
#define BFS_GRAPH_SORTED 0x2u     /* every row (column) is ascending            */
#define BFS_GRAPH_VALIDATE 0x4u   /* check structure and the claims on device   */

/* Kernel kinds reported in bfs_stats (timing mode). */
enum {
    BFS_K_INIT = 0,        /* output and bitmap initialisation                */
    BFS_K_TD_SCAN = 1,     /* frontier degree prefix sum (top-down)           */
    BFS_K_TD_EXPAND = 2,   /* top-down edge expansion and claims              */
    BFS_K_BU_SWEEP = 3,    /* bottom-up step (first-hit sweep of a level)     */
    BFS_K_CONVERT = 4,     /* queue <-> bitmap frontier conversions, merges   */
    BFS_K_MS_LEVEL = 5,    /* multi-source level kernel                       */
    BFS_K_MS_OUTPUT = 6,   /* multi-source output kernels                     */
    BFS_K_BLOCK = 7,       /* DCSC block kernels                              */
    BFS_K_FUSED = 8,       /* whole search in one persistent launch           */
    BFS_KERNEL_KINDS = 9
};

#define BFS_STATS_MAX_LEVELS 64

typedef struct {
    int32_t dir;           /* bfs_dir, default BFS_DIR_DO                         */
    int32_t parent_mode;   /* bfs_parent_mode, default BFS_PARENT_ANY             */
    double alpha;          /* top-down -> bottom-up when m_f * alpha > m_u (15)    */
    double beta;           /* bottom-up -> top-down when n_f * beta < n (18)       */
    int32_t timing;        /* HIP events -> stats: 0 none, 1 around every kernel,
                              2 around the bottom-up sweeps only               */
    int32_t bu_serial;     /* entries a lane scans alone before its wave helps
                              (0 = default 16)                                   */
    int32_t grid_blocks;   /* cap on workgroups of grid-stride kernels
                              (0 = default 2048)                                 */
    int32_t td_claim;      /* ANY parents, top-down claim: 0 = atomic fetch-or on
                              the visited bitmap, 1 = compare-and-swap on
                              parent[], 2 = benign race (Section 5.2): no
                              atomic test, every thread that saw the child
                              unvisited writes its parent (several may; the
                              repeats are counted in bfs_stats.td_duplicates)
                              and sets its visited bit with an atomic whose
                              result it does not wait for.  Such a level
                              queues nothing: its next frontier is the exact
                              bitmap of new vertices, so depths, frontier
                              sizes and edge counts stay exact and parents
                              valid.  Small levels run by the persistent
                              engine keep exact claims                          */
    int32_t small_edges;   /* top-down levels with at most this many frontier
                              edges run back to back inside one persistent
                              workgroup with no host round trip (0 = default
                              1024, negative = no persistent engine at all).
                              bfs_run_multi: > 0 engine on, negative off, 0 on
                              unless every row of the graph has at most 32
                              entries (there the level kernels take one
                              frontier vertex per thread and were measured
                              faster)                                           */
    int32_t persist_edges; /* ... and up to this many inside persist_groups
                              workgroups separated by grid barriers (0 = default
                              65536; bfs_run_multi: 2^18)                        */
    int32_t persist_groups;/* workgroups of that engine and of the fused search
                              (0 = default 64, fused search 128; capped by what
                              fits on the device at once)                        */
    int32_t bu_head;       /* bottom-up, ANY parents, what each vertex probes
                              before scanning its row: 2 = its three
                              highest-degree neighbours; 3 = its two
                              highest-degree neighbours, those among the graph's
                              hubs (fewer than 65536 vertices of highest degree)
                              in an on-chip copy of the hubs' frontier bits;
                              0 (default) = 3 on a level entered from top-down
                              when the frontier bitmap (n/8 bytes) is larger
                              than the device's L2 cache, else 2; 1 = its first
                              three row entries (MIN always uses these).  3
                              falls back to 2 on a graph without hubs (no
                              degree threshold leaves fewer than 65536)        */
    int32_t td_prepass;    /* ANY parents (fetch-or claims), direction-optimizing:
                              a top-down level with at least this many frontier
                              edges first lets every unvisited vertex probe its
                              two hub neighbours (as bu_head 3) and takes the
                              hits; the edge pass then finds them visited.
                              Needs hub ranks.  0 = default (2^24), negative =
                              never                                            */
    int32_t bu_segments;   /* bottom-up levels in column blocks (Alg. 4's
                              sub-steps, Fig. 1, inside one device): 0 (default)
                              = one sweep that scans every row to its first
                              frontier entry; S = 1..8 = the sweep probes only
                              the row heads, then S sub-steps, one per column
                              segment of about n/S ids in ascending order, scan
                              the remaining rows over that segment's entries,
                              so each sub-step probes only its slice (n/(8S)
                              bytes) of the frontier bitmap.  Rows are sorted,
                              so the first hit is the same and minimum parents
                              stay exact.  Needs BFS_GRAPH_SORTED               */
    int32_t td_segments;   /* top-down levels in column blocks: 0 (default) = one
                              edge-tiled pass over the frontier's rows; S = 1..8
                              = on levels of at least td_seg_edges frontier
                              edges, S passes, one per column segment of about
                              n/S ids,
                              each over the frontier's entries inside its
                              segment (found by binary search in the sorted
                              rows), so each pass probes and claims only its
                              slice of the visited bitmap.  Needs sorted rows
                              for the segment bounds; results do not change    */
    int32_t td_seg_edges;  /* ... on levels of at least this many frontier edges
                              (0 = default 2^20)                                */
    /* workgroup and tile shapes (tuning only; results do not change) */
    int32_t td_block;      /* threads per top-down expand workgroup: 128, 256
                              or 512 (0 = default 256).  A tile stays 1024
                              frontier edges, so a thread takes 8, 4 or 2     */
    int32_t bu_block;      /* threads per bottom-up sweep workgroup: 128, 256
                              or 512 (0 = default 256), one wave per work
                              unit; column-blocked levels keep 256             */
    int32_t bu_group;      /* bottom-up work unit: at most this many 64-vertex
                              words per wave, a power of two 1..64 (0 = default:
                              64, halved while the grid would get fewer than
                              two units per wave; the first sweep of a search
                              caps it at 8)                                    */
    int32_t fused_max_n;   /* bfs_run on a graph with at most this many vertices
                              runs the whole search, every level in both
                              directions with the Section 4.4 rule on the
                              device, in one persistent launch of
                              persist_groups workgroups (0 = default: graphs
                              up to 2^18 vertices, not with dir top-down only,
                              whose heavy levels the level kernels balance
                              better; positive = up to that many vertices in
                              every direction; negative = never).  Used on BFS_GRAPH_SYMMETRIC
                              graphs with fetch-or or minimum claims, bu_head
                              0, td_prepass <= 0 and no column segments; the
                              bottom-up scans follow row order.  When the
                              device cannot hold the workgroups at once the
                              search runs level by level instead              */
} bfs_opts;

typedef struct {
    int32_t levels;                 /* levels expanded (last one finds nothing)     */
    int32_t td_levels, bu_levels;
    int32_t fill_level;             /* bfs_run: where the -1 of the vertices not
                                       reached was written: -1 by the
                                       initialisation before level 0, d >= 0
                                       by the expansion of level d (its
                                       bottom-up sweep, or the hub pre-pass of a
                                       top-down level), -2 by a pass after the
                                       last level; -1 for bfs_run_multi       */
    int64_t reached;                /* vertices with depth >= 0                      */
    int64_t isolated;               /* symmetric graphs: vertices without entries
                                       (never scanned: they start out visited);
                                       0 for graphs not marked SYMMETRIC           */
    int64_t edges_examined;         /* adjacency entries examined (top-down: all
                                       entries of the frontier; bottom-up: entries
                                       up to and including the first hit).  Not
                                       the algorithmic byte count: any-parent
                                       bottom-up levels probe hub neighbours
                                       before the row, so this differs from the
                                       row-order scan of Alg. 2 that the byte
                                       model uses; the benchmark takes that scan
                                       from the oracle's work table instead     */
    double total_ms;                /* host wall time of the call                    */
    int64_t launches[BFS_KERNEL_KINDS];
    double kernel_ms[BFS_KERNEL_KINDS]; /* summed HIP-event time (timing mode only)  */
    /* per level d < BFS_STATS_MAX_LEVELS: direction used (0 TD, 1 BU), frontier
     * size n_f, frontier edges m_f, unexplored edges m_u when it was expanded,
     * vertices still unvisited, entries examined, and the time of the level's
     * expansion kernel (timing mode).                                          */
    int8_t level_dir[BFS_STATS_MAX_LEVELS];
    int64_t level_nf[BFS_STATS_MAX_LEVELS];
    int64_t level_mf[BFS_STATS_MAX_LEVELS];
    int64_t level_mu[BFS_STATS_MAX_LEVELS];
    int64_t level_unvisited[BFS_STATS_MAX_LEVELS];
    int64_t level_examined[BFS_STATS_MAX_LEVELS];
    float level_ms[BFS_STATS_MAX_LEVELS];
    /* td_claim = 2: children taken by per-level top-down expansions (every
     * take, with the hub pre-pass's), and how many of them repeat a child
     * already taken at the same level                                       */
    int64_t td_claims;
    int64_t td_duplicates;
} bfs_stats;

typedef struct bfs_graph bfs_graph;

/* Fill *o with defaults: DO, ANY, alpha 15, beta 18, no timing. */
void bfs_opts_default(bfs_opts* o);

/* Thread-local message describing the last failure of this thread. */
const char* bfs_last_error(void);
const char* bfs_status_string(bfs_status s);

/* Wrap a device CSR graph (Section 5.1: sorted adjacencies stored
 * contiguously, an n+1 offsets array; an undirected edge stored twice).
 *   n            vertices, 0 <= n <= 2^31-1
 *   d_offsets    device, n+1 entries of offset_bytes (4 or 8) each,
 *                offsets[0] = 0, non-decreasing, offsets[n] = nnz
 *   d_cols       device, nnz int32 column ids in [0, n)
 *   flags        BFS_GRAPH_* claims; VALIDATE checks structure and the
 *                claims with device kernels (symmetry is checked only
 *                together with SORTED, by binary search) and synchronises
 *   hip_stream   stream for validation kernels
 * Bottom-up and direction-optimizing searches need SYMMETRIC.  The arrays
 * are borrowed, not copied.                                                */
bfs_status bfs_create_graph_csr(int64_t n, const void* d_offsets, int offset_bytes, const int32_t* d_cols,
                                int64_t nnz, uint32_t flags, void* hip_stream, bfs_graph** out);

/* Wrap one device DCSC block A_ij (Section 5.1): nrows x ncols with
 * block-local ids; the block's rows are children and its columns candidate
 * parents, global parent id = col_base + local column (row_base is kept
 * for the caller's bookkeeping).
 *   d_jc[nzc]      int32 ascending ids of the non-empty columns
 *   d_cp[nzc+1]    int64 pointers into d_ir, d_cp[0] = 0, d_cp[nzc] = nnz
 *   d_ir[nnz]      int32 row ids, ascending inside each column if SORTED
 * The row-major copy (the same block compressed by rows; the paper leaves
 * open how a block is scanned by rows for Alg. 4) is optional and needed
 * only by bfs_block_bu:
 *   d_jr[nzr]      int32 ascending ids of the non-empty rows (may be NULL)
 *   d_rp[nzr+1]    int64 pointers into d_ic
 *   d_ic[nnz]      int32 column ids, ascending inside each row
 * All arrays are borrowed.                                                 */
bfs_status bfs_create_graph_dcsc(int64_t nrows, int64_t ncols, int64_t row_base, int64_t col_base,
                                 int64_t nzc, const int32_t* d_jc, const int64_t* d_cp, const int32_t* d_ir,
                                 int64_t nzr, const int32_t* d_jr, const int64_t* d_rp, const int32_t* d_ic,
                                 int64_t nnz, uint32_t flags, void* hip_stream, bfs_graph** out);

void bfs_destroy_graph(bfs_graph* g);

/* Bytes of device workspace on this graph: k = 1 gives what bfs_run needs;
 * k = 2..64 what bfs_run_multi needs for any batch size (its layout does not
 * depend on k, so a one-source bfs_run_multi also uses the k = 2 size); for
 * a DCSC graph, the bytes bfs_block_td and bfs_block_bu need (k ignored).
 * Returns 0 for a bad handle or k.                                         */
size_t bfs_workspace_bytes(const bfs_graph* g, int k);

/* Single-source search from `source` on a CSR graph (Alg. 1/2/3/4 local
 * steps, Section 4.4 switching).
 *   d_parent, d_depth   device int32[n] outputs
 *   d_workspace         device, >= bfs_workspace_bytes(g, 1) bytes, 256-B
 *                       aligned; its contents need no initialisation
 *   workspace_bytes     its size (checked)
 *   opts                NULL = defaults
 *   stats               NULL or filled on return                          */
bfs_status bfs_run(bfs_graph* g, int64_t source, const bfs_opts* opts, int32_t* d_parent, int32_t* d_depth,
                   void* d_workspace, size_t workspace_bytes, void* hip_stream, bfs_stats* stats);

/* k (1..64) searches at once on a CSR graph, one bit per source in a
 * per-vertex uint64 visited / frontier / next mask.
 *   h_sources      host int64[k] source ids (duplicates allowed)
 *   d_parent       device int32[k*n] or NULL; row j (n entries) is source
 *                  j's parent array, identical to bfs_run with MIN parents
 *   d_depth        device int32[k*n]; row j is source j's depth array
 * Parents are always the minimum-id parents (BFS_PARENT_MIN); the graph
 * must be SYMMETRIC and SORTED.  Levels are kept in 16 bits: a batch whose
 * search needs more than 65535 levels (some source has a vertex more than
 * 65534 hops away, e.g. on a path of more than 65535 vertices) fails with
 * BFS_E_UNSUPPORTED once it reaches that level; bfs_run has no such limit. */
bfs_status bfs_run_multi(bfs_graph* g, const int64_t* h_sources, int k, const bfs_opts* opts, int32_t* d_parent,
                         int32_t* d_depth, void* d_workspace, size_t workspace_bytes, void* hip_stream,
                         bfs_stats* stats);

/* Block workspace: bfs_workspace_bytes(g, 1) bytes, 256-B aligned, shared by
 * bfs_block_td and bfs_block_bu.  It must be zero-filled before its first
 * use; every successful call leaves its accumulator zeroed again (a failed
 * or interrupted call requires zero-filling it anew).  Calls that share one
 * workspace must be ordered (same stream).                                  */

/* Top-down local discovery on a DCSC block (Alg. 3, the SpMSV on the
 * (select2nd, min) semiring of Section 4.2): for every block row r with an
 * entry in a frontier column, parent(r) = min(col_base + k) over frontier
 * columns k with an entry (r, k).
 *   d_frontier     device int32[nf] distinct block-local column ids, ascending
 *   d_out_rows     device int32[nrows] capacity; rows with a candidate, ascending
 *   d_out_parents  device int32[nrows] capacity; their global parent ids
 *   d_nout         device int64[1]: number of output pairs
 * Asynchronous on hip_stream.                                              */
bfs_status bfs_block_td(bfs_graph* g, const int32_t* d_frontier, int64_t nf, int32_t* d_out_rows,
                        int32_t* d_out_parents, int64_t* d_nout, void* d_workspace, size_t workspace_bytes,
                        void* hip_stream);

/* How bfs_block_td (and bfs_block_td_noalloc) unite the frontier's columns
 * (Section 5.2 weighs a sparse accumulator against a heap-based merge):
 *   0  (default) or -1: the sparse accumulator (an atomic minimum per row,
 *      then an ordered pass over the nrows/64 occupied-bit words)
 *   1  the sorted union: one workgroup gathers the frontier columns'
 *      (row, parent) pairs into LDS, sorts them and keeps each row's
 *      smallest parent, when they are at most 8192; otherwise the
 *      accumulator runs
 * The output is the same in every mode.  The accumulator is the default
 * because it was faster at every density measured on one 2^27 x 2^27 block
 * of a scale-30 graph (0.042 vs 0.078 ms at |F| = 1342).  Returns
 * BFS_E_INVALID_ARG for a handle that is not a DCSC block or a mode outside
 * [-1, 1].                                                                 */
bfs_status bfs_block_set_union(bfs_graph* g, int mode);

/* Bottom-up local discovery on a DCSC block, one sub-step (Alg. 4): every
 * row r in [row_lo, row_hi) whose completed bit is 0 scans its columns in
 * ascending order and stops at the first column c whose frontier bit is
 * set; it emits (r, col_base + c) and sets its completed bit.
 *   d_fbits        device uint64[ceil(ncols/64)] frontier over columns
 *   d_completed    device uint64[ceil(nrows/64)] in/out
 *   outputs        as bfs_block_td, ascending rows
 * Needs the row-major copy.  Asynchronous on hip_stream.                   */
bfs_status bfs_block_bu(bfs_graph* g, const uint64_t* d_fbits, uint64_t* d_completed, int64_t row_lo,
                        int64_t row_hi, int32_t* d_out_rows, int32_t* d_out_parents, int64_t* d_nout,
                        void* d_workspace, size_t workspace_bytes, void* hip_stream);

/* Allocation-free variant of bfs_block_td, for callers that cannot
 * allocate device memory: code being captured into a HIP graph, tight
 * serving loops, harnesses that forbid hipMalloc.  The operation, the
 * arguments it shares with bfs_block_td and the outputs are the same; the
 * workspace is a file-scope device array of the library (64 MiB on every
 * device the library runs on, held until the process ends) instead of a
 * caller buffer, and the call allocates nothing.
 *   - A block whose workspace (bfs_workspace_bytes) exceeds 64 MiB is
 *     rejected with BFS_E_BUDGET before any launch.
 *   - The block's device must be the current device (BFS_E_INVALID_ARG).
 *   - Every call on one device shares that device's array and leaves its
 *     contents to the next call.  Calls that overlap on one device (on
 *     streams not ordered with each other, or from several threads at once)
 *     race and give wrong results: order them, e.g. on one stream.
 *   - The first call on a device, the call after a failed one and a call on
 *     a block whose workspace layout differs from the previous call's clear
 *     the part of the array they use with a kernel before the search.
 * Asynchronous on hip_stream.                                              */
bfs_status bfs_block_td_noalloc(bfs_graph* g, const int32_t* d_frontier, int64_t nf, int32_t* d_out_rows,
                                int32_t* d_out_parents, int64_t* d_nout, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* BFS_MI355X_H */
