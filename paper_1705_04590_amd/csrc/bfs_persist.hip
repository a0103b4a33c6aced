// Persistent top-down engine: G workgroups stay resident and run consecutive
// top-down levels (Alg. 1) with the Section 4.4 rule applied on the device,
// separated by grid-wide barriers instead of kernel launches and host round
// trips.  It serves the levels whose frontier is too small to fill the chip:
// the first levels of every search and the thousands of thin levels of
// high-diameter graphs (grids, paths).  With G = 1 the barriers reduce to
// workgroup barriers.
//
// Level L:
//   * workgroup g expands the contiguous chunk [g*C, (g+1)*C) of the queue
//     (C = ceil(qlen / G)): the chunk's degrees are prefix-summed in LDS and
//     its edges spread evenly over the threads (binary search over the LDS
//     prefix).  Claims are those of the whole-graph top-down step: fetch-or on
//     the visited bitmap (ANY), compare-and-swap on parent[] (CAS), or
//     atomicMin on parent[] plus a claim bitmap (MIN, visited frozen for the
//     level).
//   * winners collect in LDS and go to the next queue with one global atomic
//     per flush: those with out-edges at the front, those without at the back
//     of the buffer (discovered, never expanded).
//   * per-level counts (vertices, their degrees) go to spread counter lines.
//   * barrier; every workgroup reads the totals and takes the same decision
//     (stop when the next frontier is empty, when the rule switches to
//     bottom-up, when it exceeds `edge_cap` edges or falls below
//     `shrink_below` edges, or after `max_levels`).
//   * the new vertices are folded into vprev (and in MIN mode into visited,
//     clearing their claim bits, followed by a second barrier, since the next
//     level filters on visited).  The ANY / CAS fold needs no barrier: it is
//     done for level L by the workgroup that expands the same chunk at L + 1,
//     and for the last level before the kernel exits.
// The bitmaps therefore leave the engine exactly as the per-level kernels
// leave them.  Data that other workgroups wrote during the kernel (queue
// entries, visited words, counters) is read with device-scope atomic loads;
// writers publish with a device-scope fence before the barrier.
//
// Residency: a grid barrier needs every workgroup resident at once.  The
// kernel opens with a roll call whose wait is bounded: if not all G
// workgroups arrive within `roll_ticks` (a busy device), the counter is
// poisoned, every workgroup leaves before touching any search state, and the
// host runs the level with the per-level kernels instead.  Later barriers are
// bounded too; a timeout there sets an error flag (the state is then
// unusable and the call fails) rather than spinning forever.
#include "bfs_device.h"

namespace bfsk {

constexpr int PT_BLOCK = 256;
constexpr int PT_WIN = 1024;             // LDS winner buffer per workgroup
constexpr int PT_TILE = TD_TILE;         // edges per tile of an edge-balanced level
constexpr int PT_BAL_AVG = 16;           // average frontier degree from which levels are edge-balanced

template <typename OffT, int MODE>
__global__ __launch_bounds__(PT_BLOCK) void k_td_persist(
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, int32_t* __restrict__ parent,
    int32_t* __restrict__ depth, uint64_t* __restrict__ visited, uint64_t* __restrict__ vprev,
    uint64_t* __restrict__ claim, int32_t* __restrict__ qa, int32_t* __restrict__ qb, int64_t n, SmallIn in,
    SmallState* __restrict__ st, uint64_t* __restrict__ ctr, PersistCtl* __restrict__ ctl, int64_t* __restrict__ rec,
    int rec_cap, double alpha, int64_t edge_cap, int64_t shrink_below, int64_t max_levels, long long roll_ticks,
    long long bar_ticks, int64_t* __restrict__ gscan, int32_t* __restrict__ gtiles, int64_t* __restrict__ csum) {
    // edge-balanced levels: a tile of PT_TILE edges staged per step
    __shared__ int32_t s_tu[PT_TILE + 1];
    __shared__ int32_t s_ts[PT_TILE + 1];
    __shared__ int64_t s_tb[PT_TILE + 1];
    __shared__ int64_t s_E;
    __shared__ int32_t s_u[PT_BLOCK];
    __shared__ int64_t s_row[PT_BLOCK];
    __shared__ int64_t s_pre[PT_BLOCK + 1];
    __shared__ int64_t s_wsum[PT_BLOCK / WAVE];
    __shared__ int32_t s_win[PT_WIN];
    __shared__ int32_t s_win0[PT_WIN];
    __shared__ int s_nw, s_nw0;
    __shared__ uint64_t s_base, s_base0;

    const uint32_t G = gridDim.x;
    const uint32_t g = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    if (!roll_call(ctl, G, roll_ticks)) return;   // nothing touched yet

    int64_t qlen = in.qlen, n_f = in.n_f, m_f = in.m_f, m_u = in.m_u;
    int64_t nz_cur = 0;                            // winners without edges at the back of qcur
    int32_t level = (int32_t)in.level;
    int32_t* qcur = qa;
    int32_t* qnext = qb;
    int64_t done = 0, reason = ENG_EMPTY, found = 0, examined = 0;
    uint32_t nbar = 0;
    bool fail = false;

    // ANY / CAS: fold a level's winners (the current queue) into vprev
    auto fold_vprev = [&](int64_t nq, int64_t nz) {
        const int64_t c = (nq + G - 1) / G, cz = (nz + G - 1) / G;
        const int64_t a0 = min(nq, (int64_t)g * c), a1 = min(nq, a0 + c);
        for (int64_t i = a0 + tid; i < a1; i += PT_BLOCK) {
            const int32_t v = ld_dev(&qcur[i]);
            atomicOr((unsigned long long*)&vprev[v >> 6], 1ull << (v & 63));
        }
        const int64_t b0 = min(nz, (int64_t)g * cz), b1 = min(nz, b0 + cz);
        for (int64_t i = b0 + tid; i < b1; i += PT_BLOCK) {
            const int32_t v = ld_dev(&qcur[n - 1 - i]);
            atomicOr((unsigned long long*)&vprev[v >> 6], 1ull << (v & 63));
        }
    };

    for (;;) {
        if (done >= max_levels) { reason = ENG_LEVEL_CAP; break; }
        // the host chose top-down for the first level; the rule decides the rest
        if (done > 0 && (double)m_f * alpha > (double)m_u) { reason = ENG_TO_BU; break; }
        if (m_f > edge_cap) { reason = ENG_EDGE_CAP; break; }
        if (m_f < shrink_below) { reason = ENG_SHRINK; break; }
        uint64_t* slot = ctr + (size_t)(done % SLOTS) * SLOT_WORDS;
        if (tid == 0) { s_nw = 0; s_nw0 = 0; }
        uint64_t my_n = 0, my_m = 0;
        const int32_t next_depth = level + 1;
        const int64_t C = (qlen + G - 1) / G;
        const int64_t i_beg = min(qlen, (int64_t)g * C), i_end = min(qlen, i_beg + C);
        if (MODE != CLAIM_MIN && done > 0) fold_vprev(0, nz_cur);   // back part of the previous winners
        __syncthreads();
        // one edge per thread: the claim, the winner's outputs and its place
        // in the LDS winner buffers, flushed to the next queue when another
        // step could overflow them (all threads call this together)
        auto edge_step = [&](bool valid, int32_t u, int32_t v) {
            bool won = false;
            if (valid) {
                const uint64_t bit = 1ull << (v & 63);
                const uint64_t vw = ld_dev(&visited[v >> 6]);
                if (!(vw & bit)) {
                    if (MODE == CLAIM_MIN) {
                        atomicMin((unsigned int*)&parent[v], (unsigned int)u);
                        won = !(atomicOr((unsigned long long*)&claim[v >> 6], (unsigned long long)bit) & bit);
                    } else if (MODE == CLAIM_CAS) {
                        won = atomicCAS(&parent[v], -1, u) == -1;
                        if (won) atomicOr((unsigned long long*)&visited[v >> 6], (unsigned long long)bit);
                    } else {
                        won = !(atomicOr((unsigned long long*)&visited[v >> 6], (unsigned long long)bit) & bit);
                        if (won) parent[v] = u;
                    }
                }
            }
            if (won) {
                depth[v] = next_depth;
                const int64_t dv = (int64_t)off[v + 1] - (int64_t)off[v];
                my_n += 1;
                my_m += (uint64_t)dv;
                if (dv > 0) s_win[atomicAdd(&s_nw, 1)] = v;
                else s_win0[atomicAdd(&s_nw0, 1)] = v;
            }
            __syncthreads();
            const int nw = s_nw, nw0 = s_nw0;
            if (nw > PT_WIN - PT_BLOCK || nw0 > PT_WIN - PT_BLOCK) {
                if (tid == 0) {
                    s_base = nw ? atomicAdd((unsigned long long*)&slot[0], (unsigned long long)nw) : 0;
                    s_base0 = nw0 ? atomicAdd((unsigned long long*)&slot[4], (unsigned long long)nw0) : 0;
                }
                __syncthreads();
                for (int j = tid; j < nw; j += PT_BLOCK) qnext[s_base + j] = s_win[j];
                for (int j = tid; j < nw0; j += PT_BLOCK) qnext[n - 1 - (int64_t)(s_base0 + j)] = s_win0[j];
                __syncthreads();
                if (tid == 0) { s_nw = 0; s_nw0 = 0; }
                __syncthreads();
            }
        };
        // a frontier of high average degree (hub rows) is split by edges over
        // all workgroups: a grid-wide degree prefix sum and a tile table
        // first, two barriers; otherwise each workgroup expands the rows of
        // its own queue chunk
        const bool bal = G > 1 && m_f >= (int64_t)PT_BAL_AVG * qlen;
        if (!bal) {
            for (int64_t c0 = i_beg; c0 < i_end; c0 += PT_BLOCK) {
                const int64_t i = c0 + tid;
                int64_t d = 0;
                if (i < i_end) {
                    const int32_t u = ld_dev(&qcur[i]);
                    if (MODE != CLAIM_MIN && done > 0) atomicOr((unsigned long long*)&vprev[u >> 6], 1ull << (u & 63));
                    const int64_t b = (int64_t)off[u];
                    d = (int64_t)off[u + 1] - b;
                    s_u[tid] = u;
                    s_row[tid] = b;
                }
                const int64_t inc = wave_incl_scan(d);
                if (lane == WAVE - 1) s_wsum[tid / WAVE] = inc;
                __syncthreads();
                int64_t before = 0;
                for (int k = 0; k < tid / WAVE; ++k) before += s_wsum[k];
                const int64_t ex = before + inc - d;
                s_pre[tid] = ex;
                if (tid == PT_BLOCK - 1) s_pre[PT_BLOCK] = ex + d;
                __syncthreads();
                const int nv = (int)min((int64_t)PT_BLOCK, i_end - c0);
                const int64_t E = s_pre[nv];
                for (int64_t e0 = 0; e0 < E; e0 += PT_BLOCK) {
                    const int64_t e = e0 + tid;
                    int32_t u = 0, v = 0;
                    if (e < E) {
                        int lo = 0, hi = nv - 1;   // last vertex whose edges start at or before e
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (s_pre[mid] <= e) lo = mid; else hi = mid - 1;
                        }
                        u = s_u[lo];
                        v = cols[s_row[lo] + (e - s_pre[lo])];
                    }
                    edge_step(e < E, u, v);
                }
                __syncthreads();
            }
        } else {
            // (1) the chunk's degrees: local exclusive prefix into gscan, total into csum[g]
            int64_t carry = 0;
            for (int64_t c0 = i_beg; c0 < i_end; c0 += PT_BLOCK) {
                const int64_t i = c0 + tid;
                int64_t d = 0;
                if (i < i_end) {
                    const int32_t u = ld_dev(&qcur[i]);
                    if (MODE != CLAIM_MIN && done > 0) atomicOr((unsigned long long*)&vprev[u >> 6], 1ull << (u & 63));
                    d = (int64_t)off[u + 1] - (int64_t)off[u];
                }
                const int64_t inc = wave_incl_scan(d);
                if (lane == WAVE - 1) s_wsum[tid / WAVE] = inc;
                __syncthreads();
                int64_t before = 0, tot = 0;
                for (int k = 0; k < PT_BLOCK / WAVE; ++k) {
                    if (k < tid / WAVE) before += s_wsum[k];
                    tot += s_wsum[k];
                }
                if (i < i_end) gscan[i] = carry + before + inc - d;
                carry += tot;
                __syncthreads();
            }
            if (tid == 0) csum[g] = carry;
            if (!grid_sync(ctl, G, nbar++, bar_ticks)) { fail = true; break; }
            // (2) global offsets; tile t starts in the row of the vertex owning edge t*PT_TILE
            if (tid == 0) {
                int64_t coff = 0, E = 0;
                for (uint32_t h = 0; h < G; ++h) {
                    const int64_t x = ld_dev(&csum[h]);
                    if (h < g) coff += x;
                    E += x;
                }
                s_base = (uint64_t)coff;
                s_E = E;
            }
            __syncthreads();
            const int64_t coff = (int64_t)s_base, E = s_E;
            for (int64_t i = i_beg + tid; i < i_end; i += PT_BLOCK) {
                const int32_t u = ld_dev(&qcur[i]);
                const int64_t d = (int64_t)off[u + 1] - (int64_t)off[u];
                const int64_t b = coff + gscan[i];   // written by this same thread in (1)
                gscan[i] = b;
                for (int64_t t = (b + PT_TILE - 1) / PT_TILE; t * PT_TILE < b + d; ++t) gtiles[t] = (int32_t)i;
            }
            if (!grid_sync(ctl, G, nbar++, bar_ticks)) { fail = true; break; }
            // (3) the tiles, round robin over the workgroups
            const int64_t ntiles = (E + PT_TILE - 1) / PT_TILE;
            for (int64_t t = g; t < ntiles; t += G) {
                const int64_t e_t0 = t * PT_TILE, e_t1 = min(E, e_t0 + PT_TILE);
                const int64_t i0 = ld_dev(&gtiles[t]);
                const int64_t last = t + 1 < ntiles ? (int64_t)ld_dev(&gtiles[t + 1]) : qlen - 1;
                // every queued vertex has an edge, so a tile spans at most
                // PT_TILE + 1 of them; the clamps only guard memory
                int nv = (int)min((int64_t)PT_TILE + 1, last - i0 + 1);
                if (i0 < 0 || i0 >= qlen) nv = 0;
                else if (nv > qlen - i0) nv = (int)(qlen - i0);
                for (int j = tid; j < nv; j += PT_BLOCK) {
                    const int32_t u = ld_dev(&qcur[i0 + j]);
                    const int64_t gs = ld_dev(&gscan[i0 + j]);
                    s_tu[j] = u;
                    s_ts[j] = (int32_t)(gs > e_t0 ? gs - e_t0 : 0);
                    s_tb[j] = (int64_t)off[u] - gs;
                }
                __syncthreads();
                for (int64_t e0 = e_t0; e0 < e_t1; e0 += PT_BLOCK) {
                    const int64_t e = e0 + tid;
                    const bool valid = e < e_t1 && nv > 0;
                    int32_t u = 0, v = 0;
                    if (valid) {
                        const int p = (int)(e - e_t0);
                        int lo = 0, hi = nv - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (s_ts[mid] <= p) lo = mid; else hi = mid - 1;
                        }
                        u = s_tu[lo];
                        v = cols[s_tb[lo] + e];
                    }
                    edge_step(valid, u, v);
                }
                __syncthreads();
            }
        }
        {
            const int nw = s_nw, nw0 = s_nw0;
            if (tid == 0) {
                s_base = nw ? atomicAdd((unsigned long long*)&slot[0], (unsigned long long)nw) : 0;
                s_base0 = nw0 ? atomicAdd((unsigned long long*)&slot[4], (unsigned long long)nw0) : 0;
            }
            __syncthreads();
            for (int j = tid; j < nw; j += PT_BLOCK) qnext[s_base + j] = s_win[j];
            for (int j = tid; j < nw0; j += PT_BLOCK) qnext[n - 1 - (int64_t)(s_base0 + j)] = s_win0[j];
        }
        {
            uint64_t* ln = slot_line(slot);
            block_add3<PT_BLOCK / WAVE>(my_n, my_m, 0, &ln[1], &ln[2], nullptr);
        }
        if (!grid_sync(ctl, G, nbar++, bar_ticks)) { fail = true; break; }
        const int64_t nq = (int64_t)ld_dev(&slot[0]);
        const int64_t nz = (int64_t)ld_dev(&slot[4]);
        int64_t n_next = 0, m_next = 0;
        for (int j = 0; j < SLOT_SPREAD; ++j) {
            n_next += (int64_t)ld_dev(&slot[j * SLOT_LINE + 1]);
            m_next += (int64_t)ld_dev(&slot[j * SLOT_LINE + 2]);
        }
        if (MODE == CLAIM_MIN) {
            // the new vertices join visited before the next level filters on it
            const int64_t c = (nq + G - 1) / G, cz = (nz + G - 1) / G;
            const int64_t a0 = min(nq, (int64_t)g * c), a1 = min(nq, a0 + c);
            const int64_t b0 = min(nz, (int64_t)g * cz), b1 = min(nz, b0 + cz);
            for (int64_t i = a0 + tid; i < a1 + (b1 - b0); i += PT_BLOCK) {
                const int32_t v = i < a1 ? ld_dev(&qnext[i]) : ld_dev(&qnext[n - 1 - (b0 + (i - a1))]);
                const uint64_t bit = 1ull << (v & 63);
                atomicOr((unsigned long long*)&visited[v >> 6], (unsigned long long)bit);
                atomicOr((unsigned long long*)&vprev[v >> 6], (unsigned long long)bit);
                atomicAnd((unsigned long long*)&claim[v >> 6], ~(unsigned long long)bit);
            }
            if (!grid_sync(ctl, G, nbar++, bar_ticks)) { fail = true; break; }
        }
        // the slot used two levels from now was last read before this barrier
        if (g == 0) {
            uint64_t* zs = ctr + (size_t)((done + 2) % SLOTS) * SLOT_WORDS;
            for (int j = tid; j < SLOT_WORDS; j += PT_BLOCK) zs[j] = 0;
        }
        if (g == 0 && tid == 0 && done < rec_cap) {
            int64_t* r = rec + done * 4;
            r[0] = n_f;
            r[1] = m_f;
            r[2] = m_u;
            r[3] = n_next;
        }
        found += n_next;
        examined += m_f;
        ++done;
        ++level;
        int32_t* t = qcur; qcur = qnext; qnext = t;
        qlen = nq;
        nz_cur = nz;
        if (n_next == 0) { n_f = 0; m_f = 0; reason = ENG_EMPTY; break; }
        m_u -= m_next;
        n_f = n_next;
        m_f = m_next;
    }
    if (!fail && MODE != CLAIM_MIN && done > 0) fold_vprev(qlen, nz_cur);
    if (g == 0 && tid == 0) {
        st->levels_done = done;
        st->reason = fail ? ENG_TIMEOUT : reason;
        st->found = found;
        st->examined = examined;
        st->qlen = qlen;
        st->n_f = n_f;
        st->m_f = m_f;
        st->m_u = m_u;
        st->level = level;
        st->cur_is_b = (qcur == qb) ? 1 : 0;
    }
}

template <typename OffT>
int persist_max_groups() {
    int dev = 0, nb = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_td_persist<OffT, CLAIM_MIN>, PT_BLOCK, 0) !=
        hipSuccess || nb < 1)
        return 1;
    return nb * p.multiProcessorCount;
}

template <typename OffT>
void launch_td_persist(const Launch& L, int mode, int groups, const OffT* off, const int32_t* cols, int32_t* parent,
                       int32_t* depth, uint64_t* visited, uint64_t* vprev, uint64_t* claim, int32_t* qa, int32_t* qb,
                       int64_t n, SmallIn in, SmallState* st, uint64_t* ctr, PersistCtl* ctl, int64_t* rec,
                       int rec_cap, double alpha, int64_t edge_cap, int64_t shrink_below, int64_t max_levels,
                       int64_t* gscan, int32_t* gtiles, int64_t* csum) {
    // 100 MHz device clock: 2 ms to assemble, 2 s per barrier at most
    const long long roll_ticks = 200000, bar_ticks = 200000000;
#define BFS_PT(M)                                                                                               \
    hipLaunchKernelGGL((k_td_persist<OffT, M>), dim3(groups), dim3(PT_BLOCK), 0, L.stream, off, cols, parent,   \
                       depth, visited, vprev, claim, qa, qb, n, in, st, ctr, ctl, rec, rec_cap, alpha, edge_cap, \
                       shrink_below, max_levels, roll_ticks, bar_ticks, gscan, gtiles, csum)
    if (mode == CLAIM_MIN) BFS_PT(CLAIM_MIN);
    else if (mode == CLAIM_CAS) BFS_PT(CLAIM_CAS);
    else BFS_PT(CLAIM_BITMAP);
#undef BFS_PT
}

// frontier queue -> bitmap (words cleared first by the caller)
__global__ void k_queue_to_bitmap(const int32_t* __restrict__ q, int64_t qlen, uint64_t* __restrict__ bits) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < qlen; i += stride) {
        const int32_t v = q[i];
        atomicOr((unsigned long long*)&bits[v >> 6], 1ull << (v & 63));
    }
}

void launch_queue_to_bitmap(const Launch& L, const int32_t* q, int64_t qlen, uint64_t* bits) {
    hipLaunchKernelGGL(k_queue_to_bitmap, dim3(grid_for(qlen, 256, L.grid_cap)), dim3(256), 0, L.stream, q, qlen,
                       bits);
}

#define BFS_PT_INST(T)                                                                                           \
    template int persist_max_groups<T>();                                                                        \
    template void launch_td_persist<T>(const Launch&, int, int, const T*, const int32_t*, int32_t*, int32_t*,   \
                                       uint64_t*, uint64_t*, uint64_t*, int32_t*, int32_t*, int64_t, SmallIn,     \
                                       SmallState*, uint64_t*, PersistCtl*, int64_t*, int, double, int64_t,      \
                                       int64_t, int64_t, int64_t*, int32_t*, int64_t*);
BFS_PT_INST(int32_t)
BFS_PT_INST(int64_t)

}  // namespace bfsk
