// Small-frontier engine: one persistent workgroup runs consecutive top-down
// levels (Alg. 1) on the device while the frontier stays small, so searches
// on high-diameter graphs (grids, paths: thousands of levels with a few
// thousand frontier vertices each) pay neither a kernel launch nor a host
// round trip per level.  Between levels the workgroup synchronises with a
// workgroup barrier only; there is no grid-wide barrier.
//
// Each level walks the frontier queue in chunks of SMALL_BLOCK vertices: the
// chunk's degrees are prefix-summed in LDS and its edges are spread evenly
// over the threads (binary search over the LDS prefix).  Claims follow the
// whole-graph top-down step: an atomic fetch-or on the visited bitmap (ANY;
// or a compare-and-swap on parent[], CLAIM_CAS), or atomicMin on parent[]
// with a claim bitmap (MIN).  Winners are appended to the next queue through
// a workgroup counter in LDS.  At the end of a level the new vertices are
// folded into `vprev` (and, in MIN mode, into visited, clearing their claim
// bits), so the bitmaps leave the engine exactly as the per-level kernels
// would have left them.  Vertices without out-edges are discovered but not
// queued; they are collected from the back of the next-queue buffer.  The
// visited bitmap is read with device-scope atomic loads: its bits are set by
// atomics performed in L2, which do not update the compute unit's L1.
//
// The engine applies the direction rule of Section 4.4 itself (a level stays
// top-down while m_f * alpha <= m_u, compared in double precision) and stops
// before a level that would go bottom-up, before a level with more than
// `edge_cap` frontier edges, when the next frontier is empty, or after
// `max_levels` levels.
#include "bfs_device.h"

namespace bfsk {

constexpr int SMALL_BLOCK = 1024;

template <typename OffT, int MODE>
__global__ __launch_bounds__(SMALL_BLOCK) void k_td_small(
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, int32_t* __restrict__ parent,
    int32_t* __restrict__ depth, uint64_t* __restrict__ visited, uint64_t* __restrict__ vprev,
    uint64_t* __restrict__ claim, int32_t* __restrict__ qa, int32_t* __restrict__ qb, int64_t n,
    SmallState* __restrict__ st, int64_t* __restrict__ rec, int rec_cap, double alpha, int64_t edge_cap,
    int64_t max_levels) {
    __shared__ int32_t s_u[SMALL_BLOCK];
    __shared__ int64_t s_row[SMALL_BLOCK];
    __shared__ int64_t s_pre[SMALL_BLOCK + 1];
    __shared__ int64_t s_wsum[SMALL_BLOCK / WAVE];
    __shared__ unsigned long long s_cnt, s_cnt0, s_n, s_m;

    int64_t qlen = st->qlen, n_f = st->n_f, m_f = st->m_f, m_u = st->m_u;
    int32_t level = (int32_t)st->level;
    int32_t* qcur = st->cur_is_b ? qb : qa;
    int32_t* qnext = st->cur_is_b ? qa : qb;
    int64_t done = 0, reason = 0, found = 0, examined = 0;
    const int tid = threadIdx.x;
    const int lane = lane_id();

    for (;;) {
        // exit tests (identical in every thread)
        if (done >= max_levels) { reason = 3; break; }
        if ((double)m_f * alpha > (double)m_u) { reason = 1; break; }
        if (m_f > edge_cap) { reason = 2; break; }
        if (tid == 0) { s_cnt = 0; s_cnt0 = 0; s_n = 0; s_m = 0; }
        __syncthreads();
        const int32_t next_depth = level + 1;
        for (int64_t c0 = 0; c0 < qlen; c0 += SMALL_BLOCK) {
            const int64_t i = c0 + tid;
            int64_t d = 0;
            if (i < qlen) {
                const int32_t u = qcur[i];
                const int64_t b = (int64_t)off[u];
                d = (int64_t)off[u + 1] - b;
                s_u[tid] = u;
                s_row[tid] = b;
            }
            // workgroup exclusive scan of the chunk's degrees
            const int64_t inc = wave_incl_scan(d);
            if (lane == WAVE - 1) s_wsum[tid / WAVE] = inc;
            __syncthreads();
            if (tid < WAVE) {
                int64_t t = tid < SMALL_BLOCK / WAVE ? s_wsum[tid] : 0;
                t = wave_incl_scan(t);
                if (tid < SMALL_BLOCK / WAVE) s_wsum[tid] = t;
            }
            __syncthreads();
            const int64_t ex = (tid >= WAVE ? s_wsum[tid / WAVE - 1] : 0) + inc - d;
            s_pre[tid] = ex;
            if (tid == SMALL_BLOCK - 1) s_pre[SMALL_BLOCK] = ex + d;
            __syncthreads();
            const int64_t nv = (qlen - c0 < SMALL_BLOCK) ? qlen - c0 : SMALL_BLOCK;
            const int64_t E = s_pre[nv];
            for (int64_t e = tid; e < E; e += SMALL_BLOCK) {
                int lo = 0, hi = (int)nv - 1;   // last vertex whose edges start at or before e
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_pre[mid] <= e) lo = mid; else hi = mid - 1;
                }
                const int32_t u = s_u[lo];
                const int32_t v = cols[s_row[lo] + (e - s_pre[lo])];
                const uint64_t bit = 1ull << (v & 63);
                bool won = false;
                const uint64_t vw = __hip_atomic_load(&visited[v >> 6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
                if (won) {
                    depth[v] = next_depth;
                    const int64_t dv = (int64_t)off[v + 1] - (int64_t)off[v];
                    atomicAdd(&s_n, 1ull);
                    atomicAdd(&s_m, (unsigned long long)dv);
                    // vertices without out-edges are discovered, never expanded:
                    // they go to the back of the buffer, queued vertices to the front
                    if (dv > 0) qnext[atomicAdd(&s_cnt, 1ull)] = v;
                    else qnext[n - 1 - (int64_t)atomicAdd(&s_cnt0, 1ull)] = v;
                }
            }
            __syncthreads();
        }
        // fold this level's discoveries into vprev (and visited / claim in MIN mode)
        const int64_t nq = (int64_t)s_cnt, nz = (int64_t)s_cnt0;
        for (int64_t i = tid; i < nq + nz; i += SMALL_BLOCK) {
            const int32_t v = i < nq ? qnext[i] : qnext[n - 1 - (i - nq)];
            const uint64_t bit = 1ull << (v & 63);
            atomicOr((unsigned long long*)&vprev[v >> 6], (unsigned long long)bit);
            if (MODE == CLAIM_MIN) {
                atomicOr((unsigned long long*)&visited[v >> 6], (unsigned long long)bit);
                atomicAnd((unsigned long long*)&claim[v >> 6], ~(unsigned long long)bit);
            }
        }
        // the fold's atomics return nothing and may still be in flight: wait for
        // them before the barrier, since the next level filters on visited
        __threadfence();
        const int64_t n_next = (int64_t)s_n, m_next = (int64_t)s_m;
        found += n_next;
        examined += m_f;
        if (tid == 0 && done < rec_cap) {
            int64_t* r = rec + done * 4;
            r[0] = n_f;
            r[1] = m_f;
            r[2] = m_u;
            r[3] = n_next;
        }
        ++done;
        ++level;
        __syncthreads();   // everyone has read s_cnt / s_n / s_m before they are reset
        int32_t* t = qcur; qcur = qnext; qnext = t;
        qlen = nq;
        if (n_next == 0) { n_f = 0; m_f = 0; reason = 0; break; }
        m_u -= m_next;
        n_f = n_next;
        m_f = m_next;
    }
    if (tid == 0) {
        st->levels_done = done;
        st->reason = reason;
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
void launch_td_small(const Launch& L, int mode, const OffT* off, const int32_t* cols, int32_t* parent,
                     int32_t* depth, uint64_t* visited, uint64_t* vprev, uint64_t* claim, int32_t* qa, int32_t* qb,
                     int64_t n, SmallState* st, int64_t* rec, int rec_cap, double alpha, int64_t edge_cap,
                     int64_t max_levels) {
#define BFS_SMALL(M)                                                                                              \
    hipLaunchKernelGGL((k_td_small<OffT, M>), dim3(1), dim3(SMALL_BLOCK), 0, L.stream, off, cols, parent, depth, \
                       visited, vprev, claim, qa, qb, n, st, rec, rec_cap, alpha, edge_cap, max_levels)
    if (mode == CLAIM_MIN) BFS_SMALL(CLAIM_MIN);
    else if (mode == CLAIM_CAS) BFS_SMALL(CLAIM_CAS);
    else BFS_SMALL(CLAIM_BITMAP);
#undef BFS_SMALL
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

template void launch_td_small<int32_t>(const Launch&, int, const int32_t*, const int32_t*, int32_t*, int32_t*,
                                       uint64_t*, uint64_t*, uint64_t*, int32_t*, int32_t*, int64_t, SmallState*,
                                       int64_t*, int, double, int64_t, int64_t);
template void launch_td_small<int64_t>(const Launch&, int, const int64_t*, const int32_t*, int32_t*, int32_t*,
                                       uint64_t*, uint64_t*, uint64_t*, int32_t*, int32_t*, int64_t, SmallState*,
                                       int64_t*, int, double, int64_t, int64_t);

}  // namespace bfsk
