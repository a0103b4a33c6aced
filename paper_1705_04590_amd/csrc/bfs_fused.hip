// Fused search for small graphs: every level of one search, in both
// directions, inside one launch of G resident workgroups (Alg. 1 top-down
// levels, Alg. 2 bottom-up levels, the Section 4.4 rule applied on the
// device between them).  A small graph's levels are too short to fill the
// chip, so a host round trip and a handful of launches per level cost more
// than the level's work; here a level costs one grid barrier.
//
// Both frontiers are bitmaps (n/64 words each).  Level d:
//   * top-down: each wave takes frontier words; a frontier vertex with a
//     short row expands it alone, long rows are expanded by the whole wave.
//     Claims: fetch-or on the visited bitmap (any parent), or atomicMin on
//     parent[] with the next-frontier bitmap as the claim bitmap and visited
//     frozen for the level (minimum parent; folded in after the level).
//   * bottom-up: each wave takes 64-vertex words of the visited bitmap; a lane
//     scans its unvisited vertex's row for the first frontier entry, alone
//     for `serial` entries and then with the whole wave, 64 entries at a time
//     (row order, so the first hit is the smallest parent on sorted rows).
//     The wave owns its word, so its new bits go to visited and the next
//     frontier with one atomic each.
//   * per-level counts (new vertices, their degrees, entries examined) go to
//     spread counter lines; one grid barrier; every workgroup reads the
//     totals and takes the same decision.
// Three frontier bitmaps rotate (frontier, next, previous): the previous
// frontier is cleared during a level, when nobody reads it, and is the next
// level's target, so a level needs one barrier.  Minimum-parent claims of a
// top-down level enter visited during the level after, whose probes test
// visited | frontier meanwhile.
// Data other workgroups read during the kernel is written with device-scope
// atomics (or atomic stores).  Its plain loads follow a grid barrier, whose
// acquire invalidates the caches, and read words that the current level
// does not change (the frontier), that only their owner changes (a
// bottom-up wave's visited words), or whose stale copies only cost an
// atomic that returns the truth (top-down probes of visited).  The kernel opens with
// the same bounded roll call as the other persistent engines: if the
// workgroups cannot all be resident, nothing is touched and the host runs
// the search level by level instead.
#include "bfs_device.h"

namespace bfsk {

constexpr int FU_BLOCK = 256;
constexpr int FU_WAVES = FU_BLOCK / WAVE;
constexpr int FU_SHORT = 32;   // top-down rows up to this long are expanded by one lane
constexpr int FU_DIR_TD = 1, FU_DIR_BU = 2;   // direction policy: 0 the Section 4.4 rule, 1 / 2 forced

__device__ __forceinline__ bool test_bit(const uint64_t* bits, int32_t v) {
    return (bits[v >> 6] >> (v & 63)) & 1ull;
}

template <typename OffT, int MIN>
__global__ __launch_bounds__(FU_BLOCK) void k_search_fused(
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, const uint64_t* __restrict__ iso, int64_t n,
    int64_t W, int64_t nnz, int64_t src, int32_t* __restrict__ parent, int32_t* __restrict__ depth,
    uint64_t* __restrict__ visited, uint64_t* b0, uint64_t* b1, uint64_t* b2, int dir, double alpha, double beta,
    int serial, FusedState* __restrict__ st, uint64_t* __restrict__ ctr, PersistCtl* __restrict__ ctl,
    int64_t* __restrict__ rec, int rec_cap, long long roll_ticks, long long bar_ticks) {
    __shared__ int64_t s_tot[3];
    const uint32_t G = gridDim.x, g = blockIdx.x;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / WAVE;
    if (!roll_call(ctl, G, roll_ticks)) return;   // nothing touched yet

    const int64_t gw = (int64_t)g * FU_WAVES + wid, nw = (int64_t)G * FU_WAVES;
    const int64_t gt = (int64_t)g * FU_BLOCK + tid, nt = (int64_t)G * FU_BLOCK;
    // minimum parents: parent[] also takes atomics from other workgroups, so
    // its plain writes must not linger in this workgroup's cache
    auto put_parent = [&](int64_t v, int32_t p) {
        if (MIN) __hip_atomic_store(&parent[v], p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else parent[v] = p;
    };
    auto put_word = [](uint64_t* a, int64_t w, uint64_t x) {
        __hip_atomic_store(&a[w], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // outputs -1 except the source; isolated vertices and the ids >= n of the
    // last word start visited (the isolated bitmap holds both)
    for (int64_t v = gt; v < n; v += nt) {
        put_parent(v, v == src ? (int32_t)src : -1);
        depth[v] = v == src ? 0 : -1;
    }
    for (int64_t w = gt; w < W; w += nt) {
        const uint64_t sb = w == (src >> 6) ? 1ull << (src & 63) : 0ull;
        put_word(visited, w, iso[w] | sb);
        put_word(b0, w, sb);
        put_word(b1, w, 0ull);
        put_word(b2, w, 0ull);
    }
    uint32_t nbar = 0;
    bool fail = !grid_sync(ctl, G, nbar++, bar_ticks);

    const int64_t deg_s = (int64_t)off[src + 1] - (int64_t)off[src];
    int64_t n_f = 1, m_f = deg_s, m_u = nnz - deg_s, unvisited = n - 1, reached = 1, examined = 0;
    int64_t level = 0, done = 0, reason = ENG_EMPTY;
    int cur = dir == FU_DIR_BU ? 1 : 0;
    // F the frontier, N the next frontier (clear), Z the previous frontier,
    // cleared during this level (it is the target of the level after)
    uint64_t *F = b0, *N = b1, *Z = b2;
    while (!fail) {
        if (dir == FU_DIR_TD) cur = 0;
        else if (dir == FU_DIR_BU) cur = 1;
        else if (cur == 0) { if ((double)m_f * alpha > (double)m_u) cur = 1; }
        else { if ((double)n_f * beta < (double)n) cur = 0; }
        uint64_t* slot = ctr + (size_t)(level % SLOTS) * SLOT_WORDS;
        // the slot of the next level was last read two levels ago
        if (g == 0) {
            uint64_t* zs = ctr + (size_t)((level + 1) % SLOTS) * SLOT_WORDS;
            for (int j = tid; j < SLOT_WORDS; j += FU_BLOCK) put_word(zs, j, 0ull);
        }
        // nobody reads the previous frontier during this level; minimum-parent
        // claims of the last level (the frontier) join visited now, and this
        // level's probes test visited | F meanwhile
        for (int64_t w = gt; w < W; w += nt) {
            put_word(Z, w, 0ull);
            if (MIN) {
                const uint64_t f = F[w];
                if (f) atomicOr((unsigned long long*)&visited[w], (unsigned long long)f);
            }
        }
        const int32_t nd = (int32_t)(level + 1);
        uint64_t cn = 0, cm = 0, cx = 0;
        if (cur == 0) {
            auto claim = [&](int32_t u, int32_t v) {
                const uint64_t bit = 1ull << (v & 63);
                uint64_t seen = visited[v >> 6];
                if (MIN) seen |= F[v >> 6];
                if (seen & bit) return;
                bool won;
                if (MIN) {
                    atomicMin((unsigned int*)&parent[v], (unsigned int)u);
                    won = !(atomicOr((unsigned long long*)&N[v >> 6], (unsigned long long)bit) & bit);
                } else {
                    won = !(atomicOr((unsigned long long*)&visited[v >> 6], (unsigned long long)bit) & bit);
                    if (won) {
                        parent[v] = u;
                        atomicOr((unsigned long long*)&N[v >> 6], (unsigned long long)bit);
                    }
                }
                if (won) {
                    depth[v] = nd;
                    cn += 1;
                    cm += (uint64_t)((int64_t)off[v + 1] - (int64_t)off[v]);
                }
            };
            for (int64_t w = gw; w < W; w += nw) {
                const uint64_t fw = F[w];
                if (!fw) continue;
                const bool inF = (fw >> lane) & 1ull;
                const int32_t u = (int32_t)(w * WAVE + lane);
                int64_t b = 0, e = 0;
                if (inF) {
                    b = (int64_t)off[u];
                    e = (int64_t)off[u + 1];
                }
                if (inF && e - b <= FU_SHORT)
                    for (int64_t p = b; p < e; ++p) claim(u, cols[p]);
                uint64_t longm = __ballot(inF && e - b > FU_SHORT);
                while (longm) {
                    const int j = __ffsll((unsigned long long)longm) - 1;
                    longm &= longm - 1;
                    const int64_t rb = __shfl(b, j, WAVE), re = __shfl(e, j, WAVE);
                    const int32_t uj = (int32_t)(w * WAVE + j);
                    for (int64_t p = rb + lane; p < re; p += WAVE) claim(uj, cols[p]);
                }
            }
        } else {
            for (int64_t w = gw; w < W; w += nw) {
                uint64_t vw = visited[w];
                if (MIN) vw |= F[w];
                if (vw == ~0ull) continue;
                const int32_t v = (int32_t)(w * WAVE + lane);
                const bool act = !((vw >> lane) & 1ull);
                int64_t b = 0, e = 0, pos = -1;
                int32_t par = -1;
                if (act) {
                    b = (int64_t)off[v];
                    e = (int64_t)off[v + 1];
                    const int64_t ps = e < b + serial ? e : b + serial;
                    for (int64_t p = b; p < ps; ++p) {
                        const int32_t c = cols[p];
                        if (test_bit(F, c)) { par = c; pos = p - b; break; }
                    }
                }
                // rows longer than `serial` without a hit: the wave scans them
                // together, in row order
                uint64_t pend = __ballot(act && par < 0 && e - b > serial);
                while (pend) {
                    const int j = __ffsll((unsigned long long)pend) - 1;
                    pend &= pend - 1;
                    const int64_t bj = __shfl(b, j, WAVE), ej = __shfl(e, j, WAVE);
                    int32_t hc = -1;
                    int64_t hp = -1;
                    for (int64_t q0 = bj + serial; q0 < ej; q0 += WAVE) {
                        const int64_t q = q0 + lane;
                        int32_t c = -1;
                        bool h = false;
                        if (q < ej) {
                            c = cols[q];
                            h = test_bit(F, c);
                        }
                        const uint64_t hm = __ballot(h);
                        if (hm) {
                            const int k = __ffsll((unsigned long long)hm) - 1;
                            hc = __shfl(c, k, WAVE);
                            hp = q0 + k - bj;
                            break;
                        }
                    }
                    if (lane == j && hc >= 0) { par = hc; pos = hp; }
                }
                const bool found = par >= 0;
                const uint64_t nb = __ballot(found);
                if (found) {
                    put_parent(v, par);
                    depth[v] = nd;
                    cn += 1;
                    cm += (uint64_t)(e - b);
                    cx += (uint64_t)(pos + 1);
                } else if (act) {
                    cx += (uint64_t)(e - b);   // the whole row was examined
                }
                if (lane == 0 && nb) {
                    atomicOr((unsigned long long*)&N[w], (unsigned long long)nb);
                    atomicOr((unsigned long long*)&visited[w], (unsigned long long)nb);
                }
            }
        }
        // the record's fields known before the barrier
        const int64_t rec_nf = n_f, rec_mf = m_f, rec_mu = m_u, rec_unv = unvisited;
        if (g == 0 && tid == 0 && done < rec_cap) {
            int64_t* r = rec + done * 6;
            r[0] = cur; r[1] = rec_nf; r[2] = rec_mf; r[3] = rec_mu; r[4] = rec_unv;
        }
        uint64_t* ln = slot_line(slot);
        block_add3<FU_WAVES>(cn, cm, cx, &ln[S_NNEXT], &ln[S_MNEXT], &ln[S_EXAMINED]);
        if (!grid_sync(ctl, G, nbar++, bar_ticks)) { fail = true; break; }
        // the level's totals, read once per workgroup; the next level's state
        // is derived from them (and from the copies the record took) at once
        if (tid == 0) {
            int64_t a = 0, bb = 0, c = 0;
            for (int j = 0; j < SLOT_SPREAD; ++j) {
                a += (int64_t)ld_dev(&slot[j * SLOT_LINE + S_NNEXT]);
                bb += (int64_t)ld_dev(&slot[j * SLOT_LINE + S_MNEXT]);
                c += (int64_t)ld_dev(&slot[j * SLOT_LINE + S_EXAMINED]);
            }
            s_tot[0] = a; s_tot[1] = bb; s_tot[2] = c;
            if (g == 0 && done < rec_cap) rec[done * 6 + 5] = cur == 0 ? rec_mf : c;
        }
        __syncthreads();
        const int64_t n_next = s_tot[0], m_next = s_tot[1], x = s_tot[2];
        examined += cur == 0 ? rec_mf : x;
        ++done;
        ++level;
        if (n_next == 0) { reason = ENG_EMPTY; break; }
        reached += n_next;
        unvisited = rec_unv - n_next;
        m_u = rec_mu - m_next;
        n_f = n_next;
        m_f = m_next;
        { uint64_t* t = Z; Z = F; F = N; N = t; }
    }
    if (g == 0 && tid == 0) {
        st->levels_done = done;
        st->reason = fail ? ENG_TIMEOUT : reason;
        st->reached = reached;
        st->examined = examined;
        st->level = level;
    }
}

template <typename OffT>
int fused_max_groups() {
    int dev = 0, nb = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_search_fused<OffT, 1>, FU_BLOCK, 0) !=
            hipSuccess ||
        nb < 1)
        return 1;
    return nb * p.multiProcessorCount;
}

template <typename OffT>
void launch_search_fused(const Launch& L, bool min_parent, int groups, const OffT* off, const int32_t* cols,
                         const uint64_t* iso, int64_t n, int64_t nnz, int64_t src, int32_t* parent, int32_t* depth,
                         uint64_t* visited, uint64_t* b0, uint64_t* b1, uint64_t* b2, int dir, double alpha,
                         double beta, int serial, FusedState* st, uint64_t* ctr, PersistCtl* ctl, int64_t* rec,
                         int rec_cap) {
    // 100 MHz device clock: 2 ms to assemble, 2 s per barrier at most
    const long long roll_ticks = 200000, bar_ticks = 200000000;
    const int64_t W = (n + 63) / 64;
#define BFS_FU(M)                                                                                              \
    hipLaunchKernelGGL((k_search_fused<OffT, M>), dim3(groups), dim3(FU_BLOCK), 0, L.stream, off, cols, iso, n, \
                       W, nnz, src, parent, depth, visited, b0, b1, b2, dir, alpha, beta, serial, st, ctr, ctl,   \
                       rec, rec_cap, roll_ticks, bar_ticks)
    if (min_parent) BFS_FU(1);
    else BFS_FU(0);
#undef BFS_FU
}

#define BFS_FU_INST(T)                                                                                          \
    template int fused_max_groups<T>();                                                                         \
    template void launch_search_fused<T>(const Launch&, bool, int, const T*, const int32_t*, const uint64_t*,  \
                                         int64_t, int64_t, int64_t, int32_t*, int32_t*, uint64_t*, uint64_t*,  \
                                         uint64_t*, uint64_t*, int, double, double, int, FusedState*, uint64_t*, \
                                         PersistCtl*, int64_t*, int);
BFS_FU_INST(int32_t)
BFS_FU_INST(int64_t)

}  // namespace bfsk
