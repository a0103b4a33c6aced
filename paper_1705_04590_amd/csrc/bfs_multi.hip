// Multi-source BFS: up to 64 searches at once, one bit per source in
// per-vertex uint64 masks (visited, frontier F, next N), gfx950.
//
// A top-down level expands the queue of vertices whose frontier mask is not
// zero over the same edge-balanced tiles as the single-source step; an edge
// (u, v) ORs F[u] & ~visited[v] into N[v] with one 64-bit atomic, and the
// thread that turns N[v] from zero to non-zero queues v.  A resolve pass then
// gives every queued v its parents: it scans v's sorted row and, for each
// bit of N[v], keeps the first neighbour whose frontier mask carries it
// (the minimum-id parent of that source).  A bottom-up level instead sweeps
// every vertex with bits still missing, ORing the frontier masks of its
// sorted neighbours and recording the first supplier of each new bit, until
// all missing bits of currently active sources are found.  Long rows are
// scanned by the whole wave with an exclusive prefix-OR across lanes, which
// names the first supplying lane of every bit.
//
// Results are written per (vertex, source) into a vertex-major scratch
// ([n][64] parents, [n][64] 16-bit levels) exactly once, and a final pass
// transposes them into the caller's source-major parent/depth arrays,
// writing -1 where the visited mask says a source never reached a vertex.
#include "bfs_device.h"

namespace bfsk {

// counter slot words of a multi-source level
enum { M_QLEN = 0, M_NNEXT = 1, M_MNEXT = 2, M_OR = 3, M_MFULL = 4, M_EXAM = 5, M_HUBS = 7, M_MAXDEG = 8 };


// rows longer than this are not scanned by the resolve pass: their parents
// come from the frontier side instead (k_ms_hub_resolve)
constexpr int64_t MS_HUB_ROW = 512;
constexpr int MS_ROWS_BLOCK = 256;
constexpr int MS_STEP = 4;   // row entries a lane loads at once in the supplier scan

// Workgroup totals added once per workgroup to its line of the slot (sums;
// the OR of the new-source bits; the maximum row length `mx`).  Every word is
// spread over the SLOT_SPREAD lines, so no single address takes an atomic
// from each of thousands of workgroups; readers combine the lines
// (dslot_or / dslot_max / sums).
__device__ __forceinline__ void or_reduce_add(uint64_t n, uint64_t m, uint64_t orv, uint64_t mfull, uint64_t exam,
                                              uint64_t* slot, uint64_t mx = 0) {
    __shared__ uint64_t red[6][4];
    n = wave_sum(n); m = wave_sum(m); mfull = wave_sum(mfull); exam = wave_sum(exam);
    for (int d = 32; d >= 1; d >>= 1) {
        orv |= __shfl_xor(orv, d, WAVE);
        mx = max(mx, (uint64_t)__shfl_xor(mx, d, WAVE));
    }
    const int wid = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        red[0][wid] = n; red[1][wid] = m; red[2][wid] = orv; red[3][wid] = mfull; red[4][wid] = exam;
        red[5][wid] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, b = 0, c = 0, e = 0, x = 0, y = 0;
        for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) {
            a += red[0][i]; b += red[1][i]; c |= red[2][i]; e += red[3][i]; x += red[4][i];
            y = max(y, red[5][i]);
        }
        uint64_t* ln = slot_line(slot);
        if (a) atomicAdd((unsigned long long*)&ln[M_NNEXT], (unsigned long long)a);
        if (b) atomicAdd((unsigned long long*)&ln[M_MNEXT], (unsigned long long)b);
        if (c) atomicOr((unsigned long long*)&ln[M_OR], (unsigned long long)c);
        if (e) atomicAdd((unsigned long long*)&ln[M_MFULL], (unsigned long long)e);
        if (x) atomicAdd((unsigned long long*)&ln[M_EXAM], (unsigned long long)x);
        if (y) atomicMax((unsigned long long*)&ln[M_MAXDEG], (unsigned long long)y);
    }
}

// OR / maximum of word w over the lines of a slot
__device__ __forceinline__ uint64_t dslot_or(const uint64_t* slot, int w) {
    uint64_t r = 0;
    for (int j = 0; j < SLOT_SPREAD; ++j) r |= ld_dev(&slot[j * SLOT_LINE + w]);
    return r;
}
__device__ __forceinline__ uint64_t dslot_max(const uint64_t* slot, int w) {
    uint64_t r = 0;
    for (int j = 0; j < SLOT_SPREAD; ++j) r = max(r, ld_dev(&slot[j * SLOT_LINE + w]));
    return r;
}

__device__ __forceinline__ void record(int32_t* __restrict__ par_vm, uint16_t* __restrict__ lvl_vm, int64_t v,
                                       uint64_t bits, int32_t u, uint16_t level) {
    while (bits) {
        const int j = __ffsll((unsigned long long)bits) - 1;
        bits &= bits - 1;
        par_vm[v * 64 + j] = u;
        lvl_vm[v * 64 + j] = level;
    }
}

// ---------------------------------------------------------------- init
template <typename OffT>
__global__ void k_ms_init(int64_t n, uint64_t full, const uint64_t* __restrict__ iso, uint64_t* __restrict__ visited,
                          uint64_t* __restrict__ F, uint64_t* __restrict__ N, uint64_t* __restrict__ counters) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        // vertices without edges are reached by no search but their own
        const bool empty = iso && ((iso[v >> 6] >> (v & 63)) & 1ull);
        visited[v] = empty ? full : 0ull;
        F[v] = 0;
        N[v] = 0;
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < SLOTS * SLOT_WORDS; i += blockDim.x) counters[i] = 0;
}

// one workgroup of 64 threads: thread j seeds source j, the first thread of
// every distinct source vertex queues it, and the level-0 counters are set
template <typename OffT>
__global__ void k_ms_sources(const OffT* __restrict__ off, const int64_t* __restrict__ src, int k,
                             uint64_t* __restrict__ visited, uint64_t* __restrict__ F, int32_t* __restrict__ par_vm,
                             uint16_t* __restrict__ lvl_vm, int32_t* __restrict__ q, uint64_t* __restrict__ slot) {
    const int j = threadIdx.x;
    int64_t s = -1;
    bool first = false;
    if (j < k) {
        s = src[j];
        first = true;
        for (int i = 0; i < j; ++i)
            if (src[i] == s) first = false;
        par_vm[s * 64 + j] = (int32_t)s;
        lvl_vm[s * 64 + j] = 0;
    }
    // all bits of one vertex are set by its first thread (no atomics needed);
    // a source without edges is visited by its own search and expands nothing
    uint64_t bits = 0;
    int64_t d = 0;
    if (first) {
        for (int i = j; i < k; ++i)
            if (src[i] == s) bits |= 1ull << i;
        d = (int64_t)off[s + 1] - (int64_t)off[s];
        visited[s] |= bits;
        if (d > 0) F[s] = bits;
    }
    const uint64_t m = __ballot(first);
    const uint64_t mq = __ballot(first && d > 0);
    if (first && d > 0) {
        q[__popcll(mq & lanemask_lt())] = (int32_t)s;
        atomicAdd((unsigned long long*)&slot[M_MNEXT], (unsigned long long)d);
    }
    if (j == 0) {
        slot[M_QLEN] = (uint64_t)__popcll(mq);
        slot[M_NNEXT] = (uint64_t)__popcll(m);
        slot[M_OR] = k == 64 ? ~0ull : ((1ull << k) - 1);
    }
}

// ---------------------------------------------------------------- top-down
template <typename OffT>
__global__ __launch_bounds__(TD_BLOCK) void k_ms_td_expand(
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, const int32_t* __restrict__ q,
    int64_t qlen, const int64_t* __restrict__ scan, const int32_t* __restrict__ tile_start,
    int64_t total, int64_t nnz, const uint64_t* __restrict__ F, const uint64_t* __restrict__ visited,
    uint64_t* __restrict__ N, int32_t* __restrict__ qnext, uint64_t* __restrict__ slot, uint64_t* __restrict__ zslot) {
    __shared__ int32_t s_start[TD_TILE + 1];
    __shared__ int64_t s_base[TD_TILE + 1];
    __shared__ uint64_t s_f[TD_TILE + 1];
    __shared__ int32_t s_out[TD_TILE];
    __shared__ int s_cnt;
    __shared__ uint64_t s_qbase;
    zero_slot(zslot);
    const int64_t ntiles = (total + TD_TILE - 1) / TD_TILE;
    const int lane = lane_id();
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t e0 = t * TD_TILE;
        const int64_t e1 = (e0 + TD_TILE < total) ? e0 + TD_TILE : total;
        const int i0 = tile_start[t];
        int nv = tile_start[t + 1] - i0 + 1;
        if (nv > TD_TILE + 1) nv = TD_TILE + 1;
        if (i0 < 0 || i0 >= qlen) nv = 0;
        else if (nv > qlen - i0) nv = (int)(qlen - i0);
        for (int j = threadIdx.x; j < nv; j += TD_BLOCK) {
            const int32_t u = q[i0 + j];
            const int64_t sc = scan[i0 + j];
            const int64_t rel = sc - e0;
            s_start[j] = rel < 0 ? 0 : (int32_t)rel;
            s_base[j] = (int64_t)off[u] - sc;
            s_f[j] = F[u];
        }
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        int32_t vv[TD_EPT];
        uint64_t ff[TD_EPT];
#pragma unroll
        for (int k = 0; k < TD_EPT; ++k) {
            const int p = k * TD_BLOCK + threadIdx.x;
            const int64_t e = e0 + p;
            vv[k] = -1;
            ff[k] = 0;
            if (e < e1 && nv > 0) {
                int lo = 0, hi = nv - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_start[mid] <= p) lo = mid; else hi = mid - 1;
                }
                int64_t pos = s_base[lo] + e;
                if (pos < 0 || pos >= nnz) pos = 0;
                vv[k] = cols[pos];
                ff[k] = s_f[lo];
            }
        }
#pragma unroll
        for (int k = 0; k < TD_EPT; ++k) {
            bool push = false;
            if (vv[k] >= 0) {
                const uint64_t x = ff[k] & ~visited[vv[k]];
                if (x) {
                    const uint64_t old = atomicOr((unsigned long long*)&N[vv[k]], (unsigned long long)x);
                    push = old == 0;
                }
            }
            const uint64_t wm = __ballot(push);
            if (wm) {
                const int leader = __ffsll((unsigned long long)wm) - 1;
                int b = 0;
                if (lane == leader) b = atomicAdd(&s_cnt, __popcll(wm));
                b = __shfl(b, leader, WAVE);
                if (push) s_out[b + __popcll(wm & lanemask_lt())] = vv[k];
            }
        }
        __syncthreads();
        const int cnt = s_cnt;
        if (threadIdx.x == 0 && cnt > 0)
            s_qbase = atomicAdd((unsigned long long*)&slot[M_QLEN], (unsigned long long)cnt);
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += TD_BLOCK) qnext[s_qbase + j] = s_out[j];
        __syncthreads();
    }
}

// Scan the sorted row [beg, end) of v for the first supplier of every bit of
// `need` among frontier masks F; serial per lane for `serial` entries, then the
// whole wave on the rows still open.  Returns the bits found; *examined gets
// the entries looked at up to the last needed supplier (or the row length).
// Must be called by all lanes of the wave.
// Top-down on a graph whose rows are all short (at most MS_ROWS_MAX_DEG
// entries): one frontier vertex per thread, no degree scan.  The same claims
// as k_ms_td_expand: the sources of u not yet at v are OR-ed into N[v], and v
// joins the next queue when N[v] was zero.  A block's new vertices collect in
// LDS (at most MS_ROWS_BLOCK * MS_ROWS_MAX_DEG of them) and go to the queue
// with one global atomic per block and step.
template <typename OffT>
__global__ __launch_bounds__(MS_ROWS_BLOCK) void k_ms_td_rows(
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, const int32_t* __restrict__ q, int64_t qlen,
    const uint64_t* __restrict__ F, const uint64_t* __restrict__ visited, uint64_t* __restrict__ N,
    int32_t* __restrict__ qnext, uint64_t* __restrict__ slot, uint64_t* __restrict__ zslot) {
    __shared__ int32_t s_out[MS_ROWS_BLOCK * MS_ROWS_MAX_DEG];
    __shared__ int s_cnt;
    __shared__ uint64_t s_base;
    zero_slot(zslot);
    const int64_t stride = (int64_t)gridDim.x * MS_ROWS_BLOCK;
    for (int64_t i0 = (int64_t)blockIdx.x * MS_ROWS_BLOCK; i0 < qlen; i0 += stride) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        const int64_t i = i0 + threadIdx.x;
        int64_t b = 0, e = 0;
        uint64_t f = 0;
        if (i < qlen) {
            const int32_t u = q[i];
            b = (int64_t)off[u];
            e = (int64_t)off[u + 1];
            f = F[u];
        }
        for (int64_t p = b; p < e; ++p) {
            const int32_t v = cols[p];
            const uint64_t x = f & ~visited[v];
            if (x && atomicOr((unsigned long long*)&N[v], (unsigned long long)x) == 0ull)
                s_out[atomicAdd(&s_cnt, 1)] = v;
        }
        __syncthreads();
        const int cnt = s_cnt;
        if (threadIdx.x == 0 && cnt > 0)
            s_base = atomicAdd((unsigned long long*)&slot[M_QLEN], (unsigned long long)cnt);
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += MS_ROWS_BLOCK) qnext[s_base + j] = s_out[j];
        __syncthreads();
    }
}

__device__ __forceinline__ uint64_t first_suppliers(const int32_t* __restrict__ cols, const uint64_t* __restrict__ F,
                                                    int64_t v, int64_t beg, int64_t end, uint64_t need, int serial,
                                                    int32_t* __restrict__ par_vm, uint16_t* __restrict__ lvl_vm,
                                                    uint16_t level, int64_t* examined) {
    const int lane = lane_id();
    uint64_t found = 0;
    int64_t p = beg;
    const int64_t lim = (end - beg > serial) ? beg + serial : end;
    // MS_STEP entries per step: their column loads, then their mask loads,
    // all independent; then taken in row order, stopping right after the
    // entry that supplies the last needed source
    while (need && p < lim) {
        int32_t u[MS_STEP];
        uint64_t f[MS_STEP];
#pragma unroll
        for (int j = 0; j < MS_STEP; ++j) u[j] = p + j < lim ? cols[p + j] : -1;
#pragma unroll
        for (int j = 0; j < MS_STEP; ++j) f[j] = u[j] >= 0 ? F[u[j]] : 0ull;
#pragma unroll
        for (int j = 0; j < MS_STEP; ++j) {
            if (need && u[j] >= 0) {
                const uint64_t x = f[j] & need;
                if (x) {
                    record(par_vm, lvl_vm, v, x, u[j], level);
                    found |= x;
                    need &= ~x;
                }
                ++p;
            }
        }
    }
    int64_t ex = p - beg;
    uint64_t rem = __ballot(need != 0 && p < end);
    while (rem) {
        const int l = __ffsll((unsigned long long)rem) - 1;
        rem &= rem - 1;
        const int64_t vl = __shfl(v, l, WAVE);
        const int64_t pb = __shfl(p, l, WAVE);
        const int64_t pe = __shfl(end, l, WAVE);
        uint64_t nd = __shfl(need, l, WAVE);
        uint64_t got = 0;
        int64_t last = pb;
        for (int64_t b = pb; b < pe && nd; b += WAVE) {
            const int64_t idx = b + lane;
            int32_t u = 0;
            uint64_t f = 0;
            if (idx < pe) {
                u = cols[idx];
                f = F[u] & nd;
            }
            // exclusive prefix-OR: bits already supplied by lower lanes
            uint64_t incl = f;
            for (int d = 1; d < WAVE; d <<= 1) {
                const uint64_t y = __shfl_up(incl, d, WAVE);
                if (lane >= d) incl |= y;
            }
            uint64_t excl = __shfl_up(incl, 1, WAVE);
            if (lane == 0) excl = 0;
            const uint64_t mine = f & ~excl;
            if (mine) record(par_vm, lvl_vm, vl, mine, u, level);
            const uint64_t all = __shfl(incl, WAVE - 1, WAVE);
            // the chunk position where the last needed bit arrived
            const uint64_t hit = __ballot(mine != 0);
            if (all) last = b + (63 - __clzll((long long)hit)) + 1;
            got |= all;
            nd &= ~all;
            if (!nd) break;
            last = (b + WAVE < pe) ? b + WAVE : pe;
        }
        if (lane == l) {
            found |= got;
            need = nd;
            ex = (nd ? (pe - pb) : (last - pb)) + (pb - beg);
        }
    }
    *examined = ex;
    return found;
}

template <typename OffT>
__global__ __launch_bounds__(256) void k_ms_resolve(const OffT* __restrict__ off, const int32_t* __restrict__ cols,
                                                    const int32_t* __restrict__ q, const uint64_t* __restrict__ qlen_dev,
                                                    const uint64_t* __restrict__ F, uint64_t* __restrict__ N,
                                                    uint64_t* __restrict__ visited, uint64_t full,
                                                    int32_t* __restrict__ par_vm, uint16_t* __restrict__ lvl_vm,
                                                    uint16_t level, int serial, uint64_t* __restrict__ hubmark,
                                                    uint64_t* __restrict__ slot) {
    const int64_t qlen = (int64_t)*qlen_dev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint64_t cn = 0, cm = 0, cor = 0, cfull = 0, cx = 0, cmax = 0;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < qlen; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        int64_t v = 0, beg = 0, end = 0;
        uint64_t need = 0;
        if (i < qlen) {
            v = q[i];
            need = N[v];
            beg = (int64_t)off[v];
            end = (int64_t)off[v + 1];
        }
        // a long row would be scanned by one wave up to its first suppliers,
        // which can lie anywhere in it: such vertices get their parents from
        // the frontier's edges instead (an atomic minimum per new bit)
        uint64_t scan_need = need;
        if (i < qlen && need && end - beg > MS_HUB_ROW) {
            atomicOr((unsigned long long*)&hubmark[v >> 6], 1ull << (v & 63));
            uint64_t b = need;
            while (b) {
                const int j = __ffsll((unsigned long long)b) - 1;
                b &= b - 1;
                par_vm[v * 64 + j] = 0x7fffffff;
                lvl_vm[v * 64 + j] = level;
            }
            atomicAdd((unsigned long long*)&slot[M_HUBS], 1ull);
            scan_need = 0;
        }
        int64_t ex = 0;
        first_suppliers(cols, F, v, beg, end, scan_need, serial, par_vm, lvl_vm, level, &ex);
        if (i < qlen) {
            const uint64_t vis = visited[v] | need;
            visited[v] = vis;
            cn += 1;
            cm += (uint64_t)(end - beg);
            cor |= need;
            cx += (uint64_t)ex;
            if (vis == full) cfull += (uint64_t)(end - beg);
            cmax = max(cmax, (uint64_t)(end - beg));
        }
    }
    // with the longest row of the new frontier (the persistent engine's guard)
    or_reduce_add(cn, cm, cor, cfull, cx, slot, cmax);
}

// ---------------------------------------------------------------- bottom-up
template <typename OffT>
__global__ __launch_bounds__(256) void k_ms_bu_sweep(const OffT* __restrict__ off, const int32_t* __restrict__ cols,
                                                     int64_t n, const uint64_t* __restrict__ F,
                                                     uint64_t* __restrict__ N, uint64_t* __restrict__ visited,
                                                     uint64_t full, const uint64_t* __restrict__ active_dev,
                                                     int32_t* __restrict__ par_vm, uint16_t* __restrict__ lvl_vm,
                                                     uint16_t level, int serial, uint64_t* __restrict__ slot,
                                                     uint64_t* __restrict__ zslot) {
    zero_slot(zslot);
    const uint64_t active = dslot_or(active_dev, 0);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint64_t cn = 0, cm = 0, cor = 0, cfull = 0, cx = 0;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        uint64_t vis = 0, need = 0;
        int64_t beg = 0, end = 0;
        if (v < n) {
            vis = visited[v];
            need = ~vis & active;
            if (need) {
                beg = (int64_t)off[v];
                end = (int64_t)off[v + 1];
            }
        }
        int64_t ex = 0;
        const uint64_t found = first_suppliers(cols, F, v, beg, end, need, serial, par_vm, lvl_vm, level, &ex);
        if (v < n) {
            N[v] = found;
            cx += need ? (uint64_t)ex : 0;
            if (found) {
                const uint64_t nv = vis | found;
                visited[v] = nv;
                cn += 1;
                cm += (uint64_t)(end - beg);
                cor |= found;
                if (nv == full) cfull += (uint64_t)(end - beg);
            }
        }
    }
    or_reduce_add(cn, cm, cor, cfull, cx, slot);
}

// vertices with a non-zero mask -> queue (bottom-up -> top-down).  Each
// workgroup takes chunks of MQ_CHUNK vertices: it counts them, reserves its
// range with one atomic per chunk (one per wave would serialise on the shared
// counter), then writes them in vertex order within the chunk.
constexpr int MQ_STEPS = 16;
constexpr int MQ_CHUNK = 256 * MQ_STEPS;

__global__ __launch_bounds__(256) void k_ms_mask_to_queue(const uint64_t* __restrict__ N, int64_t n,
                                                          int32_t* __restrict__ q, uint64_t* __restrict__ qlen) {
    __shared__ int s_cnt[MQ_STEPS][256 / WAVE];
    __shared__ uint64_t s_base;
    const int lane = lane_id();
    const int wid = threadIdx.x / WAVE;
    for (int64_t c0 = (int64_t)blockIdx.x * MQ_CHUNK; c0 < n; c0 += (int64_t)gridDim.x * MQ_CHUNK) {
        uint64_t on_bits[MQ_STEPS];
        for (int j = 0; j < MQ_STEPS; ++j) {
            const int64_t v = c0 + (int64_t)j * 256 + threadIdx.x;
            const uint64_t m = __ballot(v < n && N[v] != 0);
            on_bits[j] = m;
            if (lane == 0) s_cnt[j][wid] = __popcll(m);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // exclusive prefix over (step, wave) in vertex order
            int tot = 0;
            for (int j = 0; j < MQ_STEPS; ++j)
                for (int i = 0; i < 256 / WAVE; ++i) { const int t = s_cnt[j][i]; s_cnt[j][i] = tot; tot += t; }
            s_base = tot ? atomicAdd((unsigned long long*)qlen, (unsigned long long)tot) : 0;
        }
        __syncthreads();
        for (int j = 0; j < MQ_STEPS; ++j) {
            const uint64_t m = on_bits[j];
            if ((m >> lane) & 1ull)
                q[s_base + s_cnt[j][wid] + __popcll(m & lanemask_lt())] = (int32_t)(c0 + (int64_t)j * 256 + threadIdx.x);
        }
        __syncthreads();
    }
}

// zero the masks of the vertices in a queue (top-down levels keep N sparse)
__global__ void k_ms_clear_queue(const int32_t* __restrict__ q, const uint64_t* __restrict__ qlen_dev,
                                 int64_t qlen_host, uint64_t* __restrict__ M) {
    const int64_t qlen = len_of(qlen_dev, qlen_host);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < qlen; i += stride) M[q[i]] = 0;
}

// ---------------------------------------------------------------- output
// transpose a tile of 64 vertices x 64 sources from the vertex-major scratch
// into source-major outputs; -1 where the source never reached the vertex
__global__ __launch_bounds__(256) void k_ms_output(int64_t n, int k, const int64_t* __restrict__ src,
                                                   const uint64_t* __restrict__ visited,
                                                   const uint64_t* __restrict__ iso,
                                                   const int32_t* __restrict__ par_vm,
                                                   const uint16_t* __restrict__ lvl_vm, int32_t* __restrict__ parent,
                                                   int32_t* __restrict__ depth) {
    __shared__ int32_t s_p[64][65];
    __shared__ int32_t s_d[64][65];
    __shared__ uint64_t s_vis[64];
    __shared__ int64_t s_src[64];
    if (threadIdx.x < 64) s_src[threadIdx.x] = threadIdx.x < k ? src[threadIdx.x] : -1;
    const int64_t ntiles = (n + 63) / 64;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t v0 = t * 64;
        __syncthreads();
        if (threadIdx.x < 64) {
            const int64_t v = v0 + threadIdx.x;
            uint64_t vis = 0;
            if (v < n) {
                vis = visited[v];
                // vertices without edges were pre-marked visited; only their own search reaches them
                if (iso && ((iso[v >> 6] >> (v & 63)) & 1ull)) {
                    vis = 0;
                    for (int j = 0; j < k; ++j)
                        if (s_src[j] == v) vis |= 1ull << j;
                }
            }
            s_vis[threadIdx.x] = vis;
        }
        __syncthreads();
        // read: four threads per vertex, 16 sources each, with 16-byte loads
        // of its rows (only for vertices some source reached)
        {
            const int vi = threadIdx.x >> 2, j0 = (threadIdx.x & 3) * 16;
            const int64_t v = v0 + vi;
            const uint32_t bits = (uint32_t)(s_vis[vi] >> j0) & 0xFFFFu;
            int32_t pv[16];
            uint16_t dv[16];
            if (v < n && bits) {
                const int4* pp = (const int4*)(par_vm + v * 64 + j0);
                const uint4* lp = (const uint4*)(lvl_vm + v * 64 + j0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int4 x = pp[q];
                    pv[4 * q] = x.x; pv[4 * q + 1] = x.y; pv[4 * q + 2] = x.z; pv[4 * q + 3] = x.w;
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint4 x = lp[q];
                    const uint32_t w4[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        dv[8 * q + 2 * r] = (uint16_t)(w4[r] & 0xFFFFu);
                        dv[8 * q + 2 * r + 1] = (uint16_t)(w4[r] >> 16);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const bool on = (bits >> j) & 1u;
                s_p[vi][j0 + j] = on ? pv[j] : -1;
                s_d[vi][j0 + j] = on ? (int32_t)dv[j] : -1;
            }
        }
        __syncthreads();
        // write: for each source, 64 consecutive vertices
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int j = e >> 6, vi = e & 63;
            const int64_t v = v0 + vi;
            if (v < n && j < k) {
                if (parent) parent[(int64_t)j * n + v] = s_p[vi][j];
                depth[(int64_t)j * n + v] = s_d[vi][j];
            }
        }
    }
}

// ---------------------------------------------------------------- persistent engine
// Consecutive top-down levels of a small batched frontier inside one launch
// (the multi-source counterpart of the single-source engine in
// bfs_persist.hip): G resident workgroups, bounded grid barriers between the
// phases of a level, and the Section 4.4 rule applied on the device.  Level:
//   A  expand: workgroup g takes the chunk [g C, (g+1) C) of the frontier
//      queue, spreads its rows' edges over its threads (prefix sum in LDS),
//      and ORs F[u] & ~visited[v] into N[v]; the thread that turns N[v] from
//      zero to non-zero queues v                             -- barrier
//   B  resolve: the new queue is split the same way; each v takes its
//      minimum-id parents by scanning its sorted row for the first supplier
//      of every new bit (rows longer than MS_HUB_ROW are marked instead and
//      get them from the frontier side in B2); visited[v] |= N[v]; counts
//                                                            -- barrier
//   B2 (a long row was marked) every frontier edge into a marked v offers u
//      to each bit of F[u] new at v; the minimum stays; marks cleared
//                                                            -- barrier
//   C  the frontier masks of the old queue are cleared: that array is the
//      next level's N; the level's totals decide whether to go on
//                                                            -- barrier
// Every array a phase reads was written before the barrier that opens the
// phase (writes are released and reads acquired at device scope there).
// The output (par_vm, lvl_vm, visited) is the same as the per-level kernels'.
constexpr int MP_BLOCK = 256;
constexpr int MP_WIN = 1024;   // LDS queue buffer per workgroup

__device__ __forceinline__ bool mp_sync(PersistCtl* ctl, uint32_t G, uint32_t& nbar, long long ticks) {
    const bool ok = grid_sync(ctl, G, nbar++, ticks);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

template <typename OffT>
__global__ __launch_bounds__(MP_BLOCK) void k_ms_persist(
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, int64_t n, uint64_t full, uint64_t* Fa,
    uint64_t* Na, uint64_t* __restrict__ visited, int32_t* qa, int32_t* qb, int32_t* __restrict__ par_vm,
    uint16_t* __restrict__ lvl_vm, uint64_t* __restrict__ hubmark, int serial, MsIn in, MsState* __restrict__ st,
    uint64_t* __restrict__ ctr, PersistCtl* __restrict__ ctl, int64_t* __restrict__ rec, int rec_cap, double alpha,
    int64_t edge_cap, int64_t max_levels, long long roll_ticks, long long bar_ticks, uint64_t* __restrict__ hring) {
    __shared__ int32_t s_u[MP_BLOCK];
    __shared__ int64_t s_row[MP_BLOCK];
    __shared__ uint64_t s_f[MP_BLOCK];
    __shared__ int64_t s_pre[MP_BLOCK + 1];
    __shared__ int64_t s_wsum[MP_BLOCK / WAVE];
    __shared__ int32_t s_win[MP_WIN];
    __shared__ int s_nw;
    __shared__ uint64_t s_base;
    const uint32_t G = gridDim.x, g = blockIdx.x;
    const int tid = threadIdx.x, lane = lane_id();
    if (!roll_call(ctl, G, roll_ticks)) return;   // nothing touched yet

    int64_t qlen = in.qlen, n_f = in.n_f, m_f = in.m_f, m_u = in.m_u;
    int32_t level = (int32_t)in.level;
    uint64_t *F = Fa, *N = Na;
    int32_t *qcur = qa, *qnext = qb;
    int64_t done = 0, reason = ENG_EMPTY, reached = 0, examined = 0;
    uint64_t last_or = 0;
    int64_t maxdeg = in.maxdeg;   // longest row of the current frontier, -1 when not known
    uint32_t nbar = 0;
    bool fail = false;

    // the edges of this workgroup's queue chunk, MP_BLOCK rows at a time:
    // visit(u, v, f) for every edge (u, v), f = F[u]; all threads call it together
    auto for_chunk_edges = [&](int64_t i_beg, int64_t i_end, auto&& visit) {
        for (int64_t c0 = i_beg; c0 < i_end; c0 += MP_BLOCK) {
            const int64_t i = c0 + tid;
            int64_t d = 0;
            if (i < i_end) {
                const int32_t u = ld_dev(&qcur[i]);
                const int64_t b = (int64_t)off[u];
                d = (int64_t)off[u + 1] - b;
                s_u[tid] = u;
                s_row[tid] = b;
                s_f[tid] = ld_dev(&F[u]);
            }
            const int64_t inc = wave_incl_scan(d);
            if (lane == WAVE - 1) s_wsum[tid / WAVE] = inc;
            __syncthreads();
            int64_t before = 0;
            for (int k = 0; k < tid / WAVE; ++k) before += s_wsum[k];
            s_pre[tid] = before + inc - d;
            if (tid == MP_BLOCK - 1) s_pre[MP_BLOCK] = before + inc;
            __syncthreads();
            const int nv = (int)min((int64_t)MP_BLOCK, i_end - c0);
            const int64_t E = s_pre[nv];
            for (int64_t e0 = 0; e0 < E; e0 += MP_BLOCK) {
                const int64_t e = e0 + tid;
                int32_t u = 0, v = -1;
                uint64_t f = 0;
                if (e < E) {
                    int lo = 0, hi = nv - 1;   // last row whose edges start at or before e
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= e) lo = mid; else hi = mid - 1;
                    }
                    u = s_u[lo];
                    v = cols[s_row[lo] + (e - s_pre[lo])];
                    f = s_f[lo];
                }
                visit(u, v, f);
            }
            __syncthreads();
        }
    };

    for (;;) {
        if (done >= max_levels) { reason = ENG_LEVEL_CAP; break; }
        if (done > 0 && (double)m_f * alpha > (double)m_u) { reason = ENG_TO_BU; break; }
        if (m_f > (maxdeg < 0 ? min(edge_cap, MS_ENGINE_FIRST_CAP) : edge_cap) || maxdeg > MS_ENGINE_MAX_DEG) {
            reason = ENG_EDGE_CAP;
            break;
        }
        uint64_t* slot = ctr + (size_t)(done % SLOTS) * SLOT_WORDS;
        const uint16_t next_level = (uint16_t)(level + 1);
        const int64_t C = (qlen + G - 1) / G;
        const int64_t i_beg = min(qlen, (int64_t)g * C), i_end = min(qlen, i_beg + C);
        // ---- A: expand
        if (tid == 0) s_nw = 0;
        __syncthreads();
        for_chunk_edges(i_beg, i_end, [&](int32_t u, int32_t v, uint64_t f) {
            (void)u;
            bool push = false;
            if (v >= 0) {
                const uint64_t x = f & ~ld_dev(&visited[v]);
                if (x) push = atomicOr((unsigned long long*)&N[v], (unsigned long long)x) == 0ull;
            }
            if (push) s_win[atomicAdd(&s_nw, 1)] = v;
            __syncthreads();
            const int nw = s_nw;
            if (nw > MP_WIN - MP_BLOCK) {
                if (tid == 0) s_base = atomicAdd((unsigned long long*)&slot[M_QLEN], (unsigned long long)nw);
                __syncthreads();
                for (int j = tid; j < nw; j += MP_BLOCK) qnext[s_base + j] = s_win[j];
                __syncthreads();
                if (tid == 0) s_nw = 0;
                __syncthreads();
            }
        });
        {
            const int nw = s_nw;
            if (tid == 0 && nw) s_base = atomicAdd((unsigned long long*)&slot[M_QLEN], (unsigned long long)nw);
            __syncthreads();
            for (int j = tid; j < nw; j += MP_BLOCK) qnext[s_base + j] = s_win[j];
        }
        if (!mp_sync(ctl, G, nbar, bar_ticks)) { fail = true; break; }
        // ---- B: resolve the new vertices' parents
        const int64_t nq = (int64_t)ld_dev(&slot[M_QLEN]);
        const int64_t Cq = (nq + G - 1) / G;
        const int64_t r_beg = min(nq, (int64_t)g * Cq), r_end = min(nq, r_beg + Cq);
        uint64_t cn = 0, cm = 0, cor = 0, cfull = 0, cx = 0, cmax = 0;
        for (int64_t c0 = r_beg; c0 < r_end; c0 += MP_BLOCK) {
            const int64_t i = c0 + tid;
            int64_t v = 0, beg = 0, end = 0;
            uint64_t need = 0;
            if (i < r_end) {
                v = ld_dev(&qnext[i]);
                need = ld_dev(&N[v]);
                beg = (int64_t)off[v];
                end = (int64_t)off[v + 1];
            }
            uint64_t scan_need = need;
            if (i < r_end && need && end - beg > MS_HUB_ROW) {
                atomicOr((unsigned long long*)&hubmark[v >> 6], 1ull << (v & 63));
                uint64_t b = need;
                while (b) {
                    const int j = __ffsll((unsigned long long)b) - 1;
                    b &= b - 1;
                    par_vm[v * 64 + j] = 0x7fffffff;
                    lvl_vm[v * 64 + j] = next_level;
                }
                atomicAdd((unsigned long long*)&slot[M_HUBS], 1ull);
                scan_need = 0;
            }
            int64_t ex = 0;
            first_suppliers(cols, F, v, beg, end, scan_need, serial, par_vm, lvl_vm, next_level, &ex);
            if (i < r_end) {
                const uint64_t vis = ld_dev(&visited[v]) | need;
                visited[v] = vis;
                cn += 1;
                cm += (uint64_t)(end - beg);
                cor |= need;
                cx += (uint64_t)ex;
                if (vis == full) cfull += (uint64_t)(end - beg);
                cmax = max(cmax, (uint64_t)(end - beg));
            }
        }
        or_reduce_add(cn, cm, cor, cfull, cx, slot, cmax);
        if (!mp_sync(ctl, G, nbar, bar_ticks)) { fail = true; break; }
        // ---- B2: long rows take their parents from the frontier side
        if (ld_dev(&slot[M_HUBS])) {
            for_chunk_edges(i_beg, i_end, [&](int32_t u, int32_t v, uint64_t f) {
                if (v < 0 || !((ld_dev(&hubmark[v >> 6]) >> (v & 63)) & 1ull)) return;
                uint64_t b = f & ld_dev(&N[v]);
                while (b) {
                    const int j = __ffsll((unsigned long long)b) - 1;
                    b &= b - 1;
                    atomicMin(&par_vm[(int64_t)v * 64 + j], u);
                }
            });
            if (!mp_sync(ctl, G, nbar, bar_ticks)) { fail = true; break; }
            for (int64_t i = r_beg + tid; i < r_end; i += MP_BLOCK) {
                const int32_t v = ld_dev(&qnext[i]);
                atomicAnd((unsigned long long*)&hubmark[v >> 6], ~(1ull << (v & 63)));
            }
        }
        // ---- C: the old frontier masks become the next N (cleared); totals
        for (int64_t i = i_beg + tid; i < i_end; i += MP_BLOCK) F[ld_dev(&qcur[i])] = 0ull;
        int64_t n_next = 0, m_next = 0, mfull = 0, exam = 0;
        for (int j = 0; j < SLOT_SPREAD; ++j) {
            n_next += (int64_t)ld_dev(&slot[j * SLOT_LINE + M_NNEXT]);
            m_next += (int64_t)ld_dev(&slot[j * SLOT_LINE + M_MNEXT]);
            mfull += (int64_t)ld_dev(&slot[j * SLOT_LINE + M_MFULL]);
            exam += (int64_t)ld_dev(&slot[j * SLOT_LINE + M_EXAM]);
        }
        last_or = dslot_or(slot, M_OR);
        maxdeg = (int64_t)dslot_max(slot, M_MAXDEG);
        // the slot of the level after next was last read at the previous level
        if (g == 0) {
            uint64_t* zs = ctr + (size_t)((done + 1) % SLOTS) * SLOT_WORDS;
            for (int j = tid; j < SLOT_WORDS; j += MP_BLOCK) zs[j] = 0;
        }
        if (g == 0 && tid == 0 && done < rec_cap) {
            int64_t* r = rec + done * 5;
            r[0] = n_f; r[1] = m_f; r[2] = m_u; r[3] = n_next; r[4] = m_f + exam;
        }
        if (!mp_sync(ctl, G, nbar, bar_ticks)) { fail = true; break; }
        reached += n_next;
        examined += m_f + exam;
        ++done;
        ++level;
        { uint64_t* t = F; F = N; N = t; }
        { int32_t* t = qcur; qcur = qnext; qnext = t; }
        qlen = nq;
        if (n_next == 0) { n_f = 0; m_f = 0; reason = ENG_EMPTY; break; }
        m_u -= mfull;
        n_f = n_next;
        m_f = m_next;
    }
    if (g == 0) {
        // the host's counter ring continues after the engine: cleared, with
        // the last level's new-source bits where the next level reads them
        __syncthreads();
        for (int j = tid; j < SLOTS * SLOT_WORDS; j += MP_BLOCK) hring[j] = 0;
        __syncthreads();
        if (tid == 0) {
            if (done > 0) hring[(size_t)((level + SLOTS - 1) % SLOTS) * SLOT_WORDS + M_OR] = last_or;
            st->levels_done = done;
            st->reason = fail ? ENG_TIMEOUT : reason;
            st->reached = reached;
            st->examined = examined;
            st->qlen = qlen;
            st->n_f = n_f;
            st->m_f = m_f;
            st->m_u = m_u;
            st->level = level;
            st->swapped = (F != Fa) ? 1 : 0;
            st->maxdeg = maxdeg;
        }
    }
}

template <typename OffT>
int ms_persist_max_groups() {
    int dev = 0, nb = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_ms_persist<OffT>, MP_BLOCK, 0) !=
        hipSuccess || nb < 1)
        return 1;
    return nb * p.multiProcessorCount;
}

template <typename OffT>
void launch_ms_persist(const Launch& L, int groups, const OffT* off, const int32_t* cols, int64_t n, uint64_t full,
                       uint64_t* F, uint64_t* N, uint64_t* visited, int32_t* qa, int32_t* qb, int32_t* par_vm,
                       uint16_t* lvl_vm, uint64_t* hubmark, int serial, MsIn in, MsState* st, uint64_t* ctr,
                       PersistCtl* ctl, int64_t* rec, int rec_cap, double alpha, int64_t edge_cap,
                       int64_t max_levels, uint64_t* hring) {
    // 100 MHz device clock: 2 ms to assemble, 2 s per barrier at most
    const long long roll_ticks = 200000, bar_ticks = 200000000;
    hipLaunchKernelGGL(k_ms_persist<OffT>, dim3(groups), dim3(MP_BLOCK), 0, L.stream, off, cols, n, full, F, N,
                       visited, qa, qb, par_vm, lvl_vm, hubmark, serial, in, st, ctr, ctl, rec, rec_cap, alpha,
                       edge_cap, max_levels, roll_ticks, bar_ticks, hring);
}

// ---------------------------------------------------------------- launchers
template <typename OffT>
void launch_ms_init(const Launch& L, const OffT* off, int64_t n, int k, const int64_t* src, const uint64_t* iso,
                    uint64_t* visited, uint64_t* F, uint64_t* N, int32_t* par_vm, uint16_t* lvl_vm, int32_t* q,
                    uint64_t* counters, uint64_t* slot0) {
    const uint64_t full = k == 64 ? ~0ull : ((1ull << k) - 1);
    hipLaunchKernelGGL(k_ms_init<OffT>, dim3(grid_for(n, 256, L.grid_cap * 4)), dim3(256), 0, L.stream, n, full,
                       iso, visited, F, N, counters);
    hipLaunchKernelGGL(k_ms_sources<OffT>, dim3(1), dim3(64), 0, L.stream, off, src, k, visited, F, par_vm, lvl_vm,
                       q, slot0);
}

// parents of the marked long-row vertices, from the frontier side: every
// frontier edge (u, v) into a marked v offers u to each bit of F[u] that is
// new at v this level; the minimum stays.  Same edge tiles as the expansion.
template <typename OffT>
__global__ __launch_bounds__(TD_BLOCK) void k_ms_hub_resolve(
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, const int32_t* __restrict__ q, int64_t qlen,
    const int64_t* __restrict__ scan, const int32_t* __restrict__ tile_start, int64_t total, int64_t nnz,
    const uint64_t* __restrict__ F, const uint64_t* __restrict__ N, const uint64_t* __restrict__ hubmark,
    int32_t* __restrict__ par_vm, const uint64_t* __restrict__ hubs) {
    if (*hubs == 0) return;
    __shared__ int32_t s_start[TD_TILE + 1];
    __shared__ int64_t s_base[TD_TILE + 1];
    __shared__ int32_t s_u[TD_TILE + 1];
    const int64_t ntiles = (total + TD_TILE - 1) / TD_TILE;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t e0 = t * TD_TILE;
        const int64_t e1 = (e0 + TD_TILE < total) ? e0 + TD_TILE : total;
        const int i0 = tile_start[t];
        int nv = tile_start[t + 1] - i0 + 1;
        if (nv > TD_TILE + 1) nv = TD_TILE + 1;
        if (i0 < 0 || i0 >= qlen) nv = 0;
        else if (nv > qlen - i0) nv = (int)(qlen - i0);
        __syncthreads();
        for (int j = threadIdx.x; j < nv; j += TD_BLOCK) {
            const int32_t u = q[i0 + j];
            const int64_t sc = scan[i0 + j];
            const int64_t rel = sc - e0;
            s_start[j] = rel < 0 ? 0 : (int32_t)rel;
            s_base[j] = (int64_t)off[u] - sc;
            s_u[j] = u;
        }
        __syncthreads();
        for (int k = 0; k < TD_EPT; ++k) {
            const int p = k * TD_BLOCK + threadIdx.x;
            const int64_t e = e0 + p;
            if (e >= e1 || nv == 0) continue;
            int lo = 0, hi = nv - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_start[mid] <= p) lo = mid; else hi = mid - 1;
            }
            int64_t pos = s_base[lo] + e;
            if (pos < 0 || pos >= nnz) continue;
            const int32_t v = cols[pos];
            if (!((hubmark[v >> 6] >> (v & 63)) & 1ull)) continue;
            const int32_t u = s_u[lo];
            uint64_t b = F[u] & N[v];
            while (b) {
                const int j = __ffsll((unsigned long long)b) - 1;
                b &= b - 1;
                atomicMin(&par_vm[(int64_t)v * 64 + j], u);
            }
        }
    }
}

// clear the marks of the queued vertices (every marked vertex is queued)
__global__ void k_ms_hub_clear(const int32_t* __restrict__ q, const uint64_t* __restrict__ qlen_dev,
                               uint64_t* __restrict__ hubmark, const uint64_t* __restrict__ hubs) {
    if (*hubs == 0) return;
    const int64_t qlen = (int64_t)*qlen_dev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < qlen; i += stride) hubmark[q[i] >> 6] = 0;
}

template <typename OffT>
void launch_ms_td(const Launch& L, const OffT* off, const int32_t* cols, int64_t nnz, const int32_t* q, int64_t qlen,
                  int64_t total, int64_t* scan, int32_t* tiles, int64_t* partial, const uint64_t* F, uint64_t* N,
                  uint64_t* visited, uint64_t full, int32_t* qnext, int32_t* par_vm, uint16_t* lvl_vm,
                  uint16_t level, int serial, uint64_t* hubmark, uint64_t* slot, uint64_t* zslot,
                  int64_t max_degree) {
    const int64_t ntiles = (total + TD_TILE - 1) / TD_TILE;
    const int g = grid_for(ntiles, 1, L.grid_cap);
    if (max_degree >= 0 && max_degree <= MS_ROWS_MAX_DEG) {
        hipLaunchKernelGGL(k_ms_td_rows<OffT>, dim3(grid_for(qlen, MS_ROWS_BLOCK, L.grid_cap)), dim3(MS_ROWS_BLOCK),
                           0, L.stream, off, cols, q, qlen, F, visited, N, qnext, slot, zslot);
    } else {
        launch_scan(L.stream, QueueDegree<OffT>{off, q}, (const uint64_t*)nullptr, qlen, partial,
                    TileSink{scan, tiles, nullptr});
        hipLaunchKernelGGL(k_ms_td_expand<OffT>, dim3(g), dim3(TD_BLOCK), 0, L.stream,
                           off, cols, q, qlen, scan, tiles, total, nnz, F, visited, N, qnext, slot, zslot);
    }
    // the next queue's length is in slot[M_QLEN], written by the expand; at
    // most `total` vertices are new
    hipLaunchKernelGGL(k_ms_resolve<OffT>, dim3(grid_for(total, 256, L.grid_cap)), dim3(256), 0, L.stream, off, cols,
                       qnext, (const uint64_t*)&slot[M_QLEN], F, N, visited, full, par_vm, lvl_vm, level, serial,
                       hubmark, slot);
    // rows longer than the hub limit exist: the hub passes (over the degree
    // scan's tiles, which the row-per-thread expand never needs here)
    if (max_degree < 0 || max_degree > MS_HUB_ROW) {
        hipLaunchKernelGGL(k_ms_hub_resolve<OffT>, dim3(g), dim3(TD_BLOCK), 0, L.stream, off, cols, q, qlen, scan,
                           tiles, total, nnz, F, N, hubmark, par_vm, (const uint64_t*)&slot[M_HUBS]);
        hipLaunchKernelGGL(k_ms_hub_clear, dim3(L.grid_cap), dim3(256), 0, L.stream, qnext,
                           (const uint64_t*)&slot[M_QLEN], hubmark, (const uint64_t*)&slot[M_HUBS]);
    }
}

template <typename OffT>
void launch_ms_bu(const Launch& L, const OffT* off, const int32_t* cols, int64_t n, const uint64_t* F, uint64_t* N,
                  uint64_t* visited, uint64_t full, const uint64_t* active_dev, int32_t* par_vm, uint16_t* lvl_vm,
                  uint16_t level, int serial, uint64_t* slot, uint64_t* zslot) {
    hipLaunchKernelGGL(k_ms_bu_sweep<OffT>, dim3(grid_for(n, 256, L.grid_cap)), dim3(256), 0, L.stream, off, cols, n,
                       F, N, visited, full, active_dev, par_vm, lvl_vm, level, serial, slot, zslot);
}

void launch_ms_mask_to_queue(const Launch& L, const uint64_t* N, int64_t n, int32_t* q, uint64_t* qlen) {
    hipLaunchKernelGGL(k_ms_mask_to_queue, dim3(grid_for(n, MQ_CHUNK, L.grid_cap)), dim3(256), 0, L.stream, N, n, q,
                       qlen);
}

void launch_ms_clear_queue(const Launch& L, const int32_t* q, const uint64_t* qlen_dev, int64_t qlen_host,
                           uint64_t* M) {
    hipLaunchKernelGGL(k_ms_clear_queue, dim3(grid_for(qlen_host, 256, L.grid_cap * 4)), dim3(256), 0, L.stream, q,
                       qlen_dev, qlen_host, M);
}

void launch_ms_output(const Launch& L, int64_t n, int k, const int64_t* src, const uint64_t* visited,
                      const uint64_t* iso, const int32_t* par_vm, const uint16_t* lvl_vm, int32_t* parent,
                      int32_t* depth) {
    hipLaunchKernelGGL(k_ms_output, dim3(grid_for((n + 63) / 64, 1, L.grid_cap * 2)), dim3(256), 0, L.stream, n, k,
                       src, visited, iso, par_vm, lvl_vm, parent, depth);
}

#define MS_INST(T)                                                                                                  \
    template void launch_ms_init<T>(const Launch&, const T*, int64_t, int, const int64_t*, const uint64_t*,        \
                                    uint64_t*, uint64_t*, uint64_t*, int32_t*, uint16_t*, int32_t*, uint64_t*,      \
                                    uint64_t*);                                                                    \
    template void launch_ms_td<T>(const Launch&, const T*, const int32_t*, int64_t, const int32_t*, int64_t,       \
                                  int64_t, int64_t*, int32_t*, int64_t*, const uint64_t*, uint64_t*, uint64_t*,    \
                                  uint64_t, int32_t*, int32_t*, uint16_t*, uint16_t, int, uint64_t*, uint64_t*,    \
                                  uint64_t*, int64_t);                                                             \
    template void launch_ms_bu<T>(const Launch&, const T*, const int32_t*, int64_t, const uint64_t*, uint64_t*,    \
                                  uint64_t*, uint64_t, const uint64_t*, int32_t*, uint16_t*, uint16_t, int,        \
                                  uint64_t*, uint64_t*);
MS_INST(int32_t)
MS_INST(int64_t)

#define MP_INST(T)                                                                                                  \
    template int ms_persist_max_groups<T>();                                                                       \
    template void launch_ms_persist<T>(const Launch&, int, const T*, const int32_t*, int64_t, uint64_t, uint64_t*, \
                                       uint64_t*, uint64_t*, int32_t*, int32_t*, int32_t*, uint16_t*, uint64_t*,   \
                                       int, MsIn, MsState*, uint64_t*, PersistCtl*, int64_t*, int, double,         \
                                       int64_t, int64_t, uint64_t*);
MP_INST(int32_t)
MP_INST(int64_t)

}  // namespace bfsk
