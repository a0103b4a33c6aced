// Single-source direction-optimizing BFS kernels for gfx950 (wave64).
//
// Top-down level (Alg. 1; the local discovery + local update of Alg. 3):
//   a degree prefix sum over the frontier queue assigns every adjacency entry
//   of the frontier a global index; fixed tiles of TD_TILE entries are then
//   expanded by workgroups, each tile's frontier vertices staged in LDS, so a
//   hub's row is spread over many workgroups.  Each edge probes the visited
//   bitmap once.  A child v is claimed by the one thread whose atomic
//   fetch-or sets v's visited bit (CLAIM_BITMAP; the bitmap is n/8 bytes and
//   lives in L2 / Infinity Cache) or whose compare-and-swap on parent[v]
//   succeeds (CLAIM_CAS).  In MIN mode the visited bitmap stays frozen for
//   the level, every frontier neighbour applies atomicMin to parent[v] (the
//   (select2nd, min) semiring of Section 4.2) and a fetch-or on a separate
//   claim bitmap picks the one thread that records depth and enqueues v.
//   Winners are compacted in LDS (wave ballot + mbcnt, one LDS atomic per
//   wave) and appended to the next queue with one global atomicAdd per tile.
//   After the level one pass extracts the newly set bits as the next
//   frontier bitmap.
// Bottom-up level (Alg. 2; the local discovery of Alg. 4):
//   one wave owns 64 consecutive vertices = one word of the visited bitmap.
//   Vertices without edges are marked visited at initialisation, so words
//   holding only visited or isolated vertices are skipped.  Each unvisited
//   lane scans its sorted row for up to `serial_len` entries probing the
//   frontier bitmap; rows still
//   unresolved are then scanned by the whole wave 64 entries at a time,
//   keeping the first hit in row order (the minimum-id parent).  The wave's
//   ballot of found lanes is the next-frontier word and updates the visited
//   word, so the sweep needs no atomics except three counters per workgroup.
#include "bfs_device.h"

namespace bfsk {

// ------------------------------------------------------------------ init
// isolated mask: bit set for vertices without entries and for ids >= n in
// the last word; `count` receives the number of vertices without entries.
template <typename OffT>
__global__ __launch_bounds__(256) void k_isolated_mask(const OffT* __restrict__ off, int64_t n, int64_t W,
                                                       uint64_t* __restrict__ iso, uint64_t* __restrict__ count) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (256 / WAVE);
    uint64_t c = 0;
    for (int64_t w = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE; w < W; w += nwaves) {
        const int64_t v = w * WAVE + lane;
        bool empty = true;
        if (v < n) empty = off[v + 1] == off[v];
        const uint64_t m = __ballot(empty);
        if (lane == 0) iso[w] = m;
        if (v < n && empty) c += 1;
    }
    c = wave_sum(c);
    if (lane == 0 && c) atomicAdd((unsigned long long*)count, (unsigned long long)c);
}

template <typename OffT>
void launch_isolated_mask(const Launch& L, const OffT* off, int64_t n, int64_t W, uint64_t* iso, uint64_t* count) {
    hipLaunchKernelGGL(k_isolated_mask<OffT>, dim3(grid_for(W, 256 / WAVE, L.grid_cap)), dim3(256), 0, L.stream,
                       off, n, W, iso, count);
}

__global__ void k_init(int32_t* __restrict__ parent, int32_t* __restrict__ depth, int64_t n,
                       uint64_t* __restrict__ visited, uint64_t* __restrict__ vprev, uint64_t* __restrict__ fbits,
                       uint64_t* __restrict__ claim, const uint64_t* __restrict__ iso, int64_t W,
                       int32_t* __restrict__ queue, int64_t src, uint64_t* __restrict__ counters,
                       int64_t counter_words, int write_out) {
    // with write_out every output entry is written here, whole lines at a
    // time, and the search overwrites the reached ones; otherwise only the
    // source's entries are, and the first bottom-up level (or the final fill)
    // writes the rest
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (write_out) {
        for (int64_t v = tid; v < n; v += stride) {
            bool s = v == src;
            parent[v] = s ? (int32_t)src : -1;
            depth[v] = s ? 0 : -1;
        }
    } else if (tid == 0) {
        parent[src] = (int32_t)src;
        depth[src] = 0;
    }
    for (int64_t w = tid; w < W; w += stride) {
        // vertices without edges can never be reached: they start visited, and
        // ids >= n in the last word count as visited so its wave can finish
        uint64_t pad = (w == W - 1 && (n & 63)) ? (~0ull << (n & 63)) : 0ull;
        uint64_t sb = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
        const uint64_t vis = (iso ? iso[w] : pad) | sb;
        visited[w] = vis;
        vprev[w] = vis;
        fbits[w] = sb;
        claim[w] = 0;
    }
    if (tid == 0) queue[0] = (int32_t)src;
    for (int64_t i = tid; i < counter_words; i += stride) counters[i] = 0;
}

void launch_init(const Launch& L, int32_t* parent, int32_t* depth, int64_t n, uint64_t* visited, uint64_t* vprev,
                 uint64_t* fbits, uint64_t* claim, const uint64_t* iso, int64_t W, int32_t* queue, int64_t src,
                 uint64_t* counters, int64_t counter_words, bool write_out) {
    int g = grid_for(write_out && n > W ? n : W, 256, L.grid_cap * 4);
    hipLaunchKernelGGL(k_init, dim3(g), dim3(256), 0, L.stream, parent, depth, n, visited, vprev, fbits, claim, iso,
                       W, queue, src, counters, counter_words, write_out ? 1 : 0);
}

// -1 for every vertex the search did not reach (unvisited, or without edges),
// the source excepted: the end of a search whose outputs were not initialised
// and that ran no bottom-up level
__global__ void k_fill_unreached(int32_t* __restrict__ parent, int32_t* __restrict__ depth, int64_t n,
                                 const uint64_t* __restrict__ visited, const uint64_t* __restrict__ iso, int64_t src) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint64_t bit = 1ull << (v & 63);
        const bool reached = (visited[v >> 6] & bit) && !(iso && (iso[v >> 6] & bit));
        if (!reached && v != src) {
            parent[v] = -1;
            depth[v] = -1;
        }
    }
}

void launch_fill_unreached(const Launch& L, int32_t* parent, int32_t* depth, int64_t n, const uint64_t* visited,
                           const uint64_t* iso, int64_t src) {
    hipLaunchKernelGGL(k_fill_unreached, dim3(grid_for(n, 256, L.grid_cap * 4)), dim3(256), 0, L.stream, parent, depth,
                       n, visited, iso, src);
}

// depth[q[i]] = d for the qlen entries of a queue (length on the device when
// qlen_dev is given)
__global__ void k_queue_depth(const int32_t* __restrict__ q, const uint64_t* __restrict__ qlen_dev, int64_t qlen_host,
                              int32_t* __restrict__ depth, int32_t d) {
    const int64_t qlen = len_of(qlen_dev, qlen_host);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < qlen; i += stride)
        __builtin_nontemporal_store(d, &depth[q[i]]);
}

void launch_queue_depth(const Launch& L, const int32_t* q, const uint64_t* qlen_dev, int64_t qlen_host,
                        int32_t* depth, int32_t d) {
    hipLaunchKernelGGL(k_queue_depth, dim3(grid_for(qlen_host > 0 ? qlen_host : 1, 256, L.grid_cap)), dim3(256), 0,
                       L.stream, q, qlen_dev, qlen_host, depth, d);
}

// ------------------------------------------------------------------ host mailbox
// Copies nw words to a coherent pinned host buffer and then publishes `seq`
// in its word 0 (system-scope release after a system-scope fence), so the
// host can spin on word 0 instead of sleeping in a stream synchronisation.
__global__ void k_post(const uint64_t* __restrict__ src, int nw, uint64_t* dst, uint64_t seq) {
    for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[1 + i] = src[i];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&dst[0], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename OffT>
__global__ void k_post_row(const OffT* __restrict__ off, int64_t v, uint64_t* dst, uint64_t seq) {
    dst[1] = (uint64_t)(int64_t)off[v];
    dst[2] = (uint64_t)(int64_t)off[v + 1];
    __threadfence_system();
    __hip_atomic_store(&dst[0], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_post(hipStream_t s, const uint64_t* src, int nw, uint64_t* dst, uint64_t seq) {
    hipLaunchKernelGGL(k_post, dim3(1), dim3(256), 0, s, src, nw, dst, seq);
}

template <typename OffT>
void launch_post_row(hipStream_t s, const OffT* off, int64_t v, uint64_t* dst, uint64_t seq) {
    hipLaunchKernelGGL(k_post_row<OffT>, dim3(1), dim3(1), 0, s, off, v, dst, seq);
}
template void launch_post_row<int32_t>(hipStream_t, const int32_t*, int64_t, uint64_t*, uint64_t);
template void launch_post_row<int64_t>(hipStream_t, const int64_t*, int64_t, uint64_t*, uint64_t);

// ------------------------------------------------------------------ frontier degree scan
// the first pass of a multi-block scan keeps the gathered degrees in `scan`,
// so the second pass reads them in order instead of gathering the offsets
// again (each item is read and then overwritten by the same thread)
template <typename OffT>
struct QueueDegreeKeep {
    const OffT* off;
    const int32_t* q;
    int64_t* keep;
    __device__ int64_t operator()(int64_t i) const {
        const int32_t u = q[i];
        const int64_t d = (int64_t)off[u + 1] - (int64_t)off[u];
        keep[i] = d;
        return d;
    }
};
struct KeptValue {
    const int64_t* keep;
    __device__ int64_t operator()(int64_t i) const { return keep[i]; }
};

template <typename OffT>
int launch_td_scan(const Launch& L, const OffT* off, const int32_t* q, const uint64_t* qlen_dev, int64_t qlen_host,
                   int64_t* scan, int32_t* tile_start, int64_t* partial, int64_t* total_out) {
    const int64_t nb = (qlen_host + SCAN_TILE - 1) / SCAN_TILE;
    if (nb <= 1)
        return launch_scan(L.stream, QueueDegree<OffT>{off, q}, qlen_dev, qlen_host, partial,
                           TileSink{scan, tile_start, total_out});
    hipLaunchKernelGGL((k_scan_partials_g<QueueDegreeKeep<OffT>>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, L.stream,
                       QueueDegreeKeep<OffT>{off, q, scan}, qlen_dev, qlen_host, partial);
    hipLaunchKernelGGL(k_scan_top_g<0>, dim3(1), dim3(SCAN_BLOCK), 0, L.stream, partial, nb);
    hipLaunchKernelGGL((k_scan_apply_g<KeptValue, TileSink>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, L.stream,
                       KeptValue{scan}, qlen_dev, qlen_host, partial, nb, TileSink{scan, tile_start, total_out});
    return 3;
}

// ------------------------------------------------------------------ column segments
// first position p in the sorted row cols[b, e) with cols[p] >= x (e when none)
__device__ __forceinline__ int64_t row_lower_bound(const int32_t* __restrict__ cols, int64_t b, int64_t e, int64_t x) {
    while (b < e) {
        const int64_t mid = (b + e) >> 1;
        if ((int64_t)cols[mid] < x) b = mid + 1; else e = mid;
    }
    return b;
}

// queue entry i's entries with ids in [lo, hi): their count, kept in `keep`,
// and the position of the first of them in the row, in `segpos`
template <typename OffT>
struct QueueSegDegree {
    const OffT* off;
    const int32_t* cols;
    const int32_t* q;
    int64_t lo, hi;
    int64_t* keep;
    int32_t* segpos;
    __device__ int64_t operator()(int64_t i) const {
        const int32_t u = q[i];
        const int64_t b = (int64_t)off[u], e = (int64_t)off[u + 1];
        const int64_t p0 = lo > 0 ? row_lower_bound(cols, b, e, lo) : b;
        const int64_t p1 = row_lower_bound(cols, p0, e, hi);
        segpos[i] = (int32_t)(p0 - b);
        keep[i] = p1 - p0;
        return p1 - p0;
    }
};

template <typename OffT>
int launch_td_scan_seg(const Launch& L, const OffT* off, const int32_t* cols, const int32_t* q,
                       const uint64_t* qlen_dev, int64_t qlen_host, int64_t lo, int64_t hi, int64_t* scan,
                       int32_t* tile_start, int64_t* partial, int32_t* segpos, int64_t* total_out) {
    const QueueSegDegree<OffT> val{off, cols, q, lo, hi, scan, segpos};
    const int64_t nb = (qlen_host + SCAN_TILE - 1) / SCAN_TILE;
    if (nb <= 1)
        return launch_scan(L.stream, val, qlen_dev, qlen_host, partial, TileSink{scan, tile_start, total_out});
    hipLaunchKernelGGL((k_scan_partials_g<QueueSegDegree<OffT>>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, L.stream,
                       val, qlen_dev, qlen_host, partial);
    hipLaunchKernelGGL(k_scan_top_g<0>, dim3(1), dim3(SCAN_BLOCK), 0, L.stream, partial, nb);
    hipLaunchKernelGGL((k_scan_apply_g<KeptValue, TileSink>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, L.stream,
                       KeptValue{scan}, qlen_dev, qlen_host, partial, nb, TileSink{scan, tile_start, total_out});
    return 3;
}

// ------------------------------------------------------------------ top-down expand
// BLK threads per workgroup; a tile keeps TD_TILE edges, TD_TILE / BLK per thread
template <typename OffT, int MODE, int BLK>
__global__ __launch_bounds__(BLK) void k_td_expand(
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, const int32_t* __restrict__ q,
    const uint64_t* __restrict__ qlen_dev, int64_t qlen_host, const int64_t* __restrict__ scan,
    const int32_t* __restrict__ tile_start, const int64_t* __restrict__ total_dev, int64_t total_host, int64_t nnz,
    int32_t* __restrict__ parent, int32_t* __restrict__ depth, uint64_t* __restrict__ visited,
    uint64_t* __restrict__ claim, int32_t* __restrict__ qnext, uint64_t* __restrict__ slot,
    uint64_t* __restrict__ zslot, int32_t next_depth, const int32_t* __restrict__ segpos) {
    constexpr int EPT = TD_TILE / BLK;
    __shared__ int32_t s_start[TD_TILE + 1];   // first edge of staged vertex j, relative to the tile
    __shared__ int64_t s_base[TD_TILE + 1];    // off[u_j] - scan[j]: cols index = s_base[j] + edge index
    __shared__ int32_t s_u[TD_TILE + 1];
    // winners of several tiles collect here; the buffer is flushed to the next
    // queue with one global atomic whenever less than a tile's worth is free
    __shared__ int32_t s_out[2 * TD_TILE];
    __shared__ int s_cnt;
    __shared__ uint64_t s_qbase;

    zero_slot(zslot);
    const int64_t qlen = len_of(qlen_dev, qlen_host);
    const int64_t total = total_dev ? *total_dev : total_host;
    const int64_t ntiles = (total + TD_TILE - 1) / TD_TILE;
    uint64_t my_n = 0, my_m = 0;
    const int lane = lane_id();
    if (threadIdx.x == 0) s_cnt = 0;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t e0 = t * TD_TILE;
        const int64_t e1 = (e0 + TD_TILE < total) ? e0 + TD_TILE : total;
        const int i0 = tile_start[t];
        int nv = tile_start[t + 1] - i0 + 1;
        if (i0 < 0 || i0 >= qlen) nv = 0;
        else if (nv > qlen - i0) nv = (int)(qlen - i0);
        // a tile spans at most TD_TILE + 1 entries when every entry has
        // edges; a column segment leaves entries with none in it between the
        // tile's owners, and a tile spanning more than LDS holds finds each
        // edge's entry by binary search in the global scan instead
        const bool staged = nv <= TD_TILE + 1;
        const int ns = staged ? nv : 0;
        for (int j = threadIdx.x; j < ns; j += BLK) {
            int32_t u = q[i0 + j];
            int64_t sc = scan[i0 + j];
            int64_t rel = sc - e0;
            s_start[j] = rel < 0 ? 0 : (int32_t)rel;
            // column segment: the row's entries from segpos (its first
            // entry inside the segment) on
            s_base[j] = (int64_t)off[u] + (segpos ? (int64_t)segpos[i0 + j] : 0) - sc;
            s_u[j] = u;
        }
        __syncthreads();
        // the thread's EPT edges move through each stage together so their
        // loads and atomics are in flight at the same time
        int32_t vv[EPT], uu[EPT];
        bool cand[EPT];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int p = k * BLK + threadIdx.x;
            const int64_t e = e0 + p;
            cand[k] = e < e1 && nv > 0;
            vv[k] = 0;
            uu[k] = 0;
            if (cand[k]) {
                int64_t pos;
                if (staged) {
                    int lo = 0, hi = nv - 1;   // last staged vertex starting at or before p
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (s_start[mid] <= p) lo = mid; else hi = mid - 1;
                    }
                    uu[k] = s_u[lo];
                    pos = s_base[lo] + e;
                } else {
                    // last entry whose edges start at or before e (entries
                    // without edges share their successor's start, so the
                    // last one with that start is the owner)
                    int64_t lo = i0, hi = i0 + nv - 1;
                    while (lo < hi) {
                        const int64_t mid = (lo + hi + 1) >> 1;
                        if (scan[mid] <= e) lo = mid; else hi = mid - 1;
                    }
                    const int32_t u = q[lo];
                    uu[k] = u;
                    pos = (int64_t)off[u] + (segpos ? (int64_t)segpos[lo] : 0) + (e - scan[lo]);
                }
                if (pos < 0 || pos >= nnz) pos = 0;   // unreachable for a consistent scan
                // streamed once: non-temporal, so the columns do not push the
                // visited bitmap's lines out of the L2
                vv[k] = __builtin_nontemporal_load(&cols[pos]);
            }
        }
        // one probe of the visited bitmap per edge; ANY modes claim on that
        // same bitmap, MIN mode keeps it frozen for the level and claims on
        // a separate bitmap (all frontier neighbours must reach atomicMin)
        uint64_t vw[EPT];
#pragma unroll
        for (int k = 0; k < EPT; ++k) vw[k] = cand[k] ? visited[vv[k] >> 6] : ~0ull;
        bool won[EPT];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t v = vv[k];
            const uint64_t bit = 1ull << (v & 63);
            won[k] = false;
            if (!(vw[k] & bit)) {
                if (MODE == CLAIM_MIN) {
                    // every frontier neighbour offers itself; the smallest id stays
                    atomicMin((unsigned int*)&parent[v], (unsigned int)uu[k]);
                    const uint64_t old = atomicOr((unsigned long long*)&claim[v >> 6], (unsigned long long)bit);
                    won[k] = !(old & bit);
                } else if (MODE == CLAIM_CAS) {
                    won[k] = atomicCAS(&parent[v], -1, uu[k]) == -1;
                    if (won[k]) atomicOr((unsigned long long*)&visited[v >> 6], (unsigned long long)bit);
                } else if (MODE == CLAIM_BENIGN) {
                    // benign race (Section 5.2): no test, the last parent
                    // written stays; the bit is set by an atomic whose old
                    // value is not waited for, so later probes skip v
                    won[k] = true;
                    __builtin_nontemporal_store(uu[k], &parent[v]);
                    __hip_atomic_fetch_or((unsigned long long*)&visited[v >> 6], (unsigned long long)bit,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    const uint64_t old = atomicOr((unsigned long long*)&visited[v >> 6], (unsigned long long)bit);
                    won[k] = !(old & bit);
                    // scattered single entries: non-temporal stores (see below)
                    if (won[k]) __builtin_nontemporal_store(uu[k], &parent[v]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int32_t v = vv[k];
            int64_t dv = 0;
            if (won[k]) {
                // a winner's entries are scattered single words: stored
                // non-temporally, they cost less than partial lines left dirty
                // in the L2 for a later write-back.  Without `depth` the
                // level's depths are written later, with whole lines (the
                // next level is the sweep that writes the outputs) or from
                // the next frontier's queue.
                if (depth) __builtin_nontemporal_store(next_depth, &depth[v]);
                dv = (int64_t)off[v + 1] - (int64_t)off[v];
                my_n += 1;
                my_m += (uint64_t)dv;
            }
            // vertices without out-edges are discovered but never expanded.
            // The benign race queues nothing: a child may be taken by several
            // threads, so its copies could outnumber the queue's n entries;
            // the next frontier comes from the level's merge instead (exact)
            const bool push = MODE != CLAIM_BENIGN && won[k] && dv > 0;
            const uint64_t wm = __ballot(push);
            if (wm) {
                const int leader = __ffsll((unsigned long long)wm) - 1;
                int b = 0;
                if (lane == leader) b = atomicAdd(&s_cnt, __popcll(wm));
                b = __shfl(b, leader, WAVE);
                if (push) s_out[b + __popcll(wm & lanemask_lt())] = v;
            }
        }
        __syncthreads();
        const int cnt = s_cnt;
        if (cnt > TD_TILE || t + gridDim.x >= ntiles) {
            if (threadIdx.x == 0 && cnt > 0)
                s_qbase = atomicAdd((unsigned long long*)&slot[S_QLEN], (unsigned long long)cnt);
            __syncthreads();
            for (int j = threadIdx.x; j < cnt; j += BLK) qnext[s_qbase + j] = s_out[j];
            __syncthreads();
            if (threadIdx.x == 0) s_cnt = 0;
        }
        __syncthreads();
    }
    uint64_t* ln = slot_line(slot);
    block_add3<BLK / WAVE>(my_n, my_m, 0, &ln[S_NNEXT], &ln[S_MNEXT], nullptr);
}

template <typename OffT>
void launch_td_expand(const Launch& L, int mode, const OffT* off, const int32_t* cols, int64_t nnz,
                      const int32_t* q, const uint64_t* qlen_dev, int64_t qlen_host, const int64_t* scan,
                      const int32_t* tile_start, int64_t total, int32_t* parent, int32_t* depth,
                      uint64_t* visited, uint64_t* claim, int32_t* qnext, uint64_t* slot, uint64_t* zslot,
                      int32_t next_depth, const int64_t* total_dev, const int32_t* segpos, int block) {
    // with total_dev the edge count is read on the device and `total` only
    // bounds the grid
    const int64_t ntiles = (total + TD_TILE - 1) / TD_TILE;
    const int g = grid_for(ntiles, 1, L.grid_cap);
#define BFS_EXPAND(M, B)                                                                                 \
    hipLaunchKernelGGL((k_td_expand<OffT, M, B>), dim3(g), dim3(B), 0, L.stream, off, cols, q, qlen_dev, \
                       qlen_host, scan, tile_start, total_dev, total, nnz, parent, depth, visited, claim,  \
                       qnext, slot, zslot, next_depth, segpos)
#define BFS_EXPAND_B(M)                          \
    do {                                         \
        if (block == 128) BFS_EXPAND(M, 128);    \
        else if (block == 512) BFS_EXPAND(M, 512); \
        else BFS_EXPAND(M, TD_BLOCK);            \
    } while (0)
    if (mode == CLAIM_MIN) BFS_EXPAND_B(CLAIM_MIN);
    else if (mode == CLAIM_CAS) BFS_EXPAND_B(CLAIM_CAS);
    else if (mode == CLAIM_BENIGN) BFS_EXPAND_B(CLAIM_BENIGN);
    else BFS_EXPAND_B(CLAIM_BITMAP);
#undef BFS_EXPAND_B
#undef BFS_EXPAND
}

// ------------------------------------------------------------------ conversions
__global__ void k_clear_words(uint64_t* __restrict__ w, int64_t nw) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += stride) w[i] = 0;
}

void launch_clear_words(const Launch& L, uint64_t* w, int64_t nw) {
    hipLaunchKernelGGL(k_clear_words, dim3(grid_for(nw, 256, L.grid_cap * 4)), dim3(256), 0, L.stream, w, nw);
}

// frontier bitmap -> queue in vertex order: a prefix sum of the words'
// popcounts gives each word its output position (no shared counter, whose
// same-address atomics would serialise), and the last item stores the length
struct WordBits {
    const uint64_t* b;
    __device__ int64_t operator()(int64_t w) const { return __popcll(b[w]); }
};
struct BitsToQueue {
    const uint64_t* b;
    int32_t* q;
    uint64_t* qlen;
    __device__ void item(int64_t w, int64_t before, int64_t c) const {
        if (!c) return;
        uint64_t x = b[w];
        int64_t p = before;
        while (x) {
            const int bb = __ffsll((unsigned long long)x) - 1;
            x &= x - 1;
            q[p++] = (int32_t)(w * 64 + bb);
        }
    }
    __device__ void last(int64_t, int64_t total) const { *qlen = (uint64_t)total; }
};

int launch_bitmap_to_queue(const Launch& L, const uint64_t* bits, int64_t W, int32_t* q, uint64_t* qlen_ctr,
                           int64_t* partial) {
    return launch_scan(L.stream, WordBits{bits}, (const uint64_t*)nullptr, W, partial, BitsToQueue{bits, q, qlen_ctr});
}

// after a top-down level the bits that became set are the next frontier.
// ANY modes claimed on visited itself: next = visited & ~vprev.  MIN mode
// claimed on `claim`: next = claim, folded into visited and cleared.  Both
// leave vprev == visited for the next level.
__global__ void k_merge_any(const uint64_t* __restrict__ visited, uint64_t* __restrict__ vprev,
                            uint64_t* __restrict__ fnext, int64_t W) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < W; i += stride) {
        const uint64_t v = visited[i], p = vprev[i];
        fnext[i] = v & ~p;
        if (v != p) vprev[i] = v;
    }
}

// Benign-race top-down levels: the same merge, plus the exact size of the
// next frontier (new bits, S_DISTINCT) and its edge count (S_MDISTINCT, the
// degrees of the new vertices), since the expansion counted every copy.
template <typename OffT>
__global__ __launch_bounds__(256) void k_merge_exact(const OffT* __restrict__ off,
                                                     const uint64_t* __restrict__ visited,
                                                     uint64_t* __restrict__ vprev, uint64_t* __restrict__ fnext,
                                                     int64_t W, uint64_t* __restrict__ slot) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint64_t cnt = 0, deg = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < W; i += stride) {
        const uint64_t v = visited[i], p = vprev[i];
        uint64_t x = v & ~p;
        fnext[i] = x;
        cnt += (uint64_t)__popcll(x);
        while (x) {
            const int b = __ffsll((unsigned long long)x) - 1;
            x &= x - 1;
            const int64_t u = i * 64 + b;
            deg += (uint64_t)((int64_t)off[u + 1] - (int64_t)off[u]);
        }
        if (v != p) vprev[i] = v;
    }
    uint64_t* ln = slot_line(slot);
    block_add3<256 / WAVE>(cnt, deg, 0, &ln[S_DISTINCT], &ln[S_MDISTINCT], nullptr);
}

template <typename OffT>
void launch_merge_exact(const Launch& L, const OffT* off, const uint64_t* visited, uint64_t* vprev, uint64_t* fnext,
                        int64_t W, uint64_t* slot) {
    hipLaunchKernelGGL(k_merge_exact<OffT>, dim3(grid_for(W, 256, L.grid_cap * 4)), dim3(256), 0, L.stream, off,
                       visited, vprev, fnext, W, slot);
}

__global__ void k_merge_claim(uint64_t* __restrict__ visited, uint64_t* __restrict__ vprev,
                              uint64_t* __restrict__ claim, uint64_t* __restrict__ fnext, int64_t W) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < W; i += stride) {
        const uint64_t c = claim[i];
        fnext[i] = c;
        if (c) {
            const uint64_t v = visited[i] | c;
            visited[i] = v;
            vprev[i] = v;
            claim[i] = 0;
        }
    }
}

void launch_merge(const Launch& L, bool min_mode, uint64_t* visited, uint64_t* vprev, uint64_t* claim,
                  uint64_t* fnext, int64_t W) {
    if (min_mode)
        hipLaunchKernelGGL(k_merge_claim, dim3(grid_for(W, 256, L.grid_cap * 4)), dim3(256), 0, L.stream, visited,
                           vprev, claim, fnext, W);
    else
        hipLaunchKernelGGL(k_merge_any, dim3(grid_for(W, 256, L.grid_cap * 4)), dim3(256), 0, L.stream, visited,
                           vprev, fnext, W);
}

// ------------------------------------------------------------------ validation
// one wave per row: offsets monotone, ids in range, rows ascending (SORTED),
// and for SYMMETRIC|SORTED every (u,v) has (v,u), found by binary search.
template <typename OffT>
__global__ __launch_bounds__(256) void k_validate_csr(const OffT* __restrict__ off, const int32_t* __restrict__ cols,
                                                      int64_t n, int64_t nnz, uint32_t flags,
                                                      uint32_t* __restrict__ err) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (256 / WAVE);
    uint32_t e = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if ((int64_t)off[0] != 0 || (int64_t)off[n] != nnz) e |= VE_OFFSETS;
    }
    for (int64_t u = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE; u < n; u += nwaves) {
        const int64_t b = (int64_t)off[u], en = (int64_t)off[u + 1];
        if (en < b || b < 0 || en > nnz) { e |= VE_OFFSETS; continue; }
        for (int64_t p = b + lane; p < en; p += WAVE) {
            const int32_t c = cols[p];
            if (c < 0 || (int64_t)c >= n) { e |= VE_RANGE; continue; }
            if ((flags & 2u) && p + 1 < en && cols[p + 1] < c) e |= VE_UNSORTED;
            if ((flags & 3u) == 3u) {
                int64_t lo = (int64_t)off[c], hi = (int64_t)off[c + 1];
                if (lo < 0 || hi > nnz || hi < lo) { e |= VE_OFFSETS; continue; }
                bool ok = false;
                while (lo < hi) {
                    int64_t mid = (lo + hi) >> 1;
                    int32_t x = cols[mid];
                    if (x == (int32_t)u) { ok = true; break; }
                    if (x < (int32_t)u) lo = mid + 1; else hi = mid;
                }
                if (!ok) e |= VE_ASYM;
            }
        }
    }
    if (e) atomicOr(err, e);
}

template <typename OffT>
void launch_validate_csr(const Launch& L, const OffT* off, const int32_t* cols, int64_t n, int64_t nnz,
                         uint32_t flags, uint32_t* err) {
    int g = grid_for(n, 256 / WAVE, L.grid_cap);
    hipLaunchKernelGGL(k_validate_csr<OffT>, dim3(g), dim3(256), 0, L.stream, off, cols, n, nnz, flags, err);
}

// ------------------------------------------------------------------ instantiations
#define BFS_INST(T)                                                                                              \
    template void launch_isolated_mask<T>(const Launch&, const T*, int64_t, int64_t, uint64_t*, uint64_t*);      \
    template int launch_td_scan<T>(const Launch&, const T*, const int32_t*, const uint64_t*, int64_t, int64_t*, \
                                   int32_t*, int64_t*, int64_t*);                                               \
    template void launch_td_expand<T>(const Launch&, int, const T*, const int32_t*, int64_t, const int32_t*,   \
                                      const uint64_t*, int64_t, const int64_t*, const int32_t*, int64_t,        \
                                      int32_t*, int32_t*, uint64_t*, uint64_t*, int32_t*, uint64_t*,            \
                                      uint64_t*, int32_t, const int64_t*, const int32_t*, int);                 \
    template int launch_td_scan_seg<T>(const Launch&, const T*, const int32_t*, const int32_t*, const uint64_t*, \
                                       int64_t, int64_t, int64_t, int64_t*, int32_t*, int64_t*, int32_t*,        \
                                       int64_t*);                                                                 \
    template void launch_validate_csr<T>(const Launch&, const T*, const int32_t*, int64_t, int64_t, uint32_t,  \
                                         uint32_t*);                                                              \
    template void launch_merge_exact<T>(const Launch&, const T*, const uint64_t*, uint64_t*, uint64_t*, int64_t, \
                                        uint64_t*);
BFS_INST(int32_t)
BFS_INST(int64_t)

}  // namespace bfsk
