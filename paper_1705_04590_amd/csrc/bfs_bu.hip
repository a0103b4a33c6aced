// Bottom-up step (Alg. 2): every unvisited vertex scans its row in stored
// (ascending) order against the frontier bitmap and stops at the first hit,
// which becomes its parent.  With sorted rows the first hit is the smallest
// frontier neighbour, so this step also yields minimum-id parents.
//
// On a large level the step is bound by the rate of random probes into the
// frontier bitmap (n/8 bytes: larger than one XCD's L2 at scale 26) and by
// chains of dependent accesses (row head -> probe -> offsets -> columns ->
// probe), so the layout keeps both short:
//   * row heads, one 16-byte record per vertex {deg, c0, c1, c2}: the degree
//     and the first three entries of the row (unused slots -1).  Most
//     vertices of a large bottom-up level meet a frontier neighbour among
//     their first three entries; only the others read offsets and columns.
//     The heads of the next 64 vertices are loaded while the current 64 probe.
//   * the visited bitmap is read a group of GW consecutive words at a time
//     (one word per lane); the unvisited vertices of the group are compacted
//     in LDS, in vertex order, and processed 64 at a time, one per lane, so
//     sparse levels do not spend a wave per nearly-full word.
//   * rows that continue past their head are scanned four entries per step
//     (four column loads, then four probes, all independent), up to
//     `serial_len` entries; rows still open after that are finished by the
//     whole wave, one row at a time, 64 entries per step.  The first hit in
//     row order is kept in every case.
//   * visited words are streamed with non-temporal loads so they do not push
//     the frontier bitmap out of L2.
//   * next-frontier bits of the group collect in LDS (atomic or on 64-bit
//     LDS words) and each word of nbits / visited / vprev is written once by
//     its lane: no global atomics.
#include "bfs_device.h"

namespace bfsk {

constexpr int BU_WIN = 512;   // compacted-list window per wave (entries)
constexpr int FILL_GW = BU_WIN / WAVE;   // words per group of a sweep that writes the fill
constexpr int BU_PB = 2;   // rounds of 64 heads whose loads and probes are in flight together

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool bit_of(uint64_t word, int32_t c) { return (word >> (c & 63)) & 1ull; }

__device__ __forceinline__ uint64_t stream_load(const uint64_t* p) { return __builtin_nontemporal_load(p); }
// a head record read once per level: marked non-temporal, so the streamed
// records do not push the frontier bitmap's lines out of the L2
__device__ __forceinline__ int4 stream_load4(const int4* p) {
    typedef int v4 __attribute__((ext_vector_type(4)));
    const v4 x = __builtin_nontemporal_load((const v4*)p);
    return make_int4(x.x, x.y, x.z, x.w);
}

// HUB = 0: `head` holds each row's first three entries (row order, as the
// minimum-id parent needs).  HUB = 1 (any-parent searches): it holds the three
// neighbours of highest degree; a vertex of a large bottom-up level finds its
// frontier among them far more often (the frontier of that level is made of
// high-degree vertices), so fewer probes are made; a miss then scans the whole
// row from its start.
//
// HUB = 3: HUB = 2's probes only, as the pre-pass of a heavy top-down level
// (no row scans; only visited is updated, see the level's merge).
//
// HUB = 2 (any-parent searches on graphs with hub ranks): the head holds the
// two neighbours of highest degree and, packed in its last word, their ranks
// among the graph's hubs (0xFFFF: not a hub).  The frontier bits of all hubs
// (HUB_BITS bits, gathered once per level into `hb`) are copied to LDS when
// the workgroup starts, so a probe of a hub neighbour reads LDS, not the
// frontier bitmap in memory.
//
// FILL = 1 (first bottom-up level of a search whose outputs were left
// uninitialised): every output entry of the group's vertices that were not
// visited before this level is written here, once: hits get their parent
// and depth, isolated and still unreached vertices -1.  The hits are not
// stored as they are found; each entry's result goes to its slot of the
// compacted list in LDS (the slot of its head index, consumed one round
// earlier), and after the group one pass per 64-vertex word writes the
// word's entries with 64 consecutive stores, so each output line is written
// by one instruction instead of once by the scattered hit stores and again
// by a fill pass.  With frontier_depth the frontier's vertices, reached by
// the top-down level before, which left their depth unwritten, get it there
// too.  Groups are then at most FILL_GW words, so the whole group
// fits one list window.
// SEG = 1 (column-blocked sweep): the rows are not scanned past their head
// here; a vertex that still needs its row is appended to the pending list
// `pend` (vertex id, row position to resume at), and the sub-steps that
// follow (k_bu_segment) scan those rows one column segment at a time.
template <typename OffT, int HUB, int FILL, int SEG, int BLK>
__device__ __forceinline__ void bu_sweep_body(
    const int4* __restrict__ head, const uint64_t* __restrict__ iso, const uint32_t* __restrict__ nbase,
    const OffT* __restrict__ off, const int32_t* __restrict__ cols,
    const uint64_t* __restrict__ fbits, const uint64_t* __restrict__ hb, uint64_t* __restrict__ nbits,
    uint64_t* __restrict__ visited, uint64_t* __restrict__ vprev, int32_t* __restrict__ parent,
    int32_t* __restrict__ depth, int64_t W, int GW,
    int32_t next_depth, int serial_len, uint64_t* __restrict__ slot, uint64_t* __restrict__ zslot, int64_t n,
    int64_t src, uint64_t* __restrict__ pend, int frontier_depth) {
    __shared__ int32_t s_list[BLK / WAVE][BU_WIN];
    __shared__ int32_t s_hidx[BLK / WAVE][BU_WIN];
    __shared__ unsigned long long s_nb[BLK / WAVE][WAVE];
    __shared__ uint64_t s_hb[HUB >= 2 ? HUB_BITS / 64 : 1];
    // list index of each compacted row still to scan (window-relative)
    __shared__ int16_t s_mx[BLK / WAVE][SEG || HUB == 3 ? 1 : BU_WIN];
    if (HUB >= 2) {
        for (int i = threadIdx.x; i < HUB_BITS / 64; i += BLK) s_hb[i] = hb[i];
        __syncthreads();
    }
    zero_slot(zslot);
    const int lane = lane_id();
    const int wid = threadIdx.x / WAVE;
    int32_t* list = s_list[wid];
    int32_t* hlist = s_hidx[wid];
    unsigned long long* nbw = s_nb[wid];
    const int64_t G = (W + GW - 1) / GW;
    const int64_t nwaves = (int64_t)gridDim.x * (BLK / WAVE);
    uint64_t my_n = 0, my_m = 0, my_x = 0;
    int64_t w0 = 0;
    // v found its parent at row position pos
    auto found = [&](int32_t v, int32_t par, int32_t pos, int32_t deg) {
        if (!FILL) {
            // scattered single entries: non-temporal stores, which cost less
            // than partial lines left dirty in the L2 for a later write-back
            __builtin_nontemporal_store(par, &parent[v]);
            __builtin_nontemporal_store(next_depth, &depth[v]);
        }
        atomicOr(&nbw[(v >> 6) - w0], 1ull << (v & 63));
        my_n += 1;
        my_m += (uint64_t)deg;
        my_x += (uint64_t)(pos + 1);
    };
    for (int64_t gi = (int64_t)blockIdx.x * (BLK / WAVE) + wid; gi < G; gi += nwaves) {
        w0 = gi * GW;
        const int64_t w = w0 + lane;
        const bool mine = lane < GW && w < W;
        const uint64_t wv = mine ? stream_load(&visited[w]) : ~0ull;
        // head records exist for vertices with edges only: index = rank among them
        const uint64_t hasrow = mine ? ~stream_load(&iso[w]) : 0ull;
        // frontier vertices whose depth the fill writes (frontier_depth)
        const uint64_t fdw = FILL && frontier_depth && mine ? fbits[w] : 0ull;
        const uint32_t hbase = mine ? nbase[w] : 0u;
        const int cnt = __popcll(~wv);
        const int incl = wave_incl_scan(cnt);
        const int tot = __shfl(incl, WAVE - 1, WAVE);
        nbw[lane] = 0;
        for (int lo = 0; lo < tot; lo += BU_WIN) {
            const int hi = min(lo + BU_WIN, tot);
            const int nw = hi - lo;
            // this lane's unvisited vertices with list index in [lo, hi)
            int idx = incl - cnt;
            if (cnt && idx < hi && idx + cnt > lo) {
                uint64_t x = ~wv;
                for (; idx < lo; ++idx) x &= x - 1;
                for (; x && idx < hi; ++idx) {
                    const int b = __ffsll((unsigned long long)x) - 1;
                    x &= x - 1;
                    list[idx - lo] = (int32_t)(w * WAVE + b);
                    hlist[idx - lo] = (int32_t)(hbase + (uint32_t)__popcll(hasrow & ((1ull << b) - 1ull)));
                }
            }
            wave_lds_sync();
            int nmiss = 0;   // rows compacted for the second pass (wave-uniform)
            // heads are taken BU_PB rounds of 64 at a time: their loads, then
            // their probes, are all in flight together, and the rounds are
            // then settled in order
            for (int r0 = 0; r0 < nw; r0 += BU_PB * WAVE) {
                int32_t vb[BU_PB];
                int4 hb[BU_PB];
#pragma unroll
                for (int j = 0; j < BU_PB; ++j) {
                    const int idx = r0 + j * WAVE + lane;
                    vb[j] = 0;
                    hb[j] = make_int4(0, -1, -1, -1);
                    if (idx < nw) {
                        vb[j] = list[idx];
                        hb[j] = stream_load4(&head[hlist[idx]]);
                    }
                }
                // entries the head probes; with HUB = 2 its last word holds ranks
                constexpr int32_t nprobe = HUB >= 2 ? 2 : 3;
                // the first probe of every round (and with HUB = 2 the second
                // too) before any is tested
                uint64_t fa[BU_PB], fb[BU_PB];
#pragma unroll
                for (int j = 0; j < BU_PB; ++j) {
                    const int4 h = hb[j];
                    const int deg = h.x;
                    if (HUB >= 2) {
                        const uint32_t q0 = (uint32_t)h.w & 0xFFFFu, q1 = (uint32_t)h.w >> 16;
                        fa[j] = deg > 0 ? (q0 != 0xFFFFu ? s_hb[q0 >> 6] : fbits[h.y >> 6]) : 0ull;
                        fb[j] = deg > 1 ? (q1 != 0xFFFFu ? s_hb[q1 >> 6] : fbits[h.z >> 6]) : 0ull;
                    } else {
                        fa[j] = deg > 0 ? fbits[h.y >> 6] : 0ull;
                        fb[j] = 0ull;
                    }
                }
#pragma unroll
                for (int j = 0; j < BU_PB; ++j) {
                const int r = r0 + j * WAVE;
                const bool act = r + lane < nw;
                const int32_t v = vb[j];
                const int4 h = hb[j];
                const int deg = act ? h.x : 0;
                int32_t par = -1;
                int32_t pos = 0;   // position of the hit in the row
                if (HUB >= 2) {
                    const uint32_t q0 = (uint32_t)h.w & 0xFFFFu, q1 = (uint32_t)h.w >> 16;
                    if (deg > 0 && bit_of(fa[j], q0 != 0xFFFFu ? (int32_t)q0 : h.y)) { par = h.y; pos = 0; }
                    else if (deg > 1 && bit_of(fb[j], q1 != 0xFFFFu ? (int32_t)q1 : h.z)) { par = h.z; pos = 1; }
                } else {
                    if (deg > 0 && bit_of(fa[j], h.y)) { par = h.y; pos = 0; }
                    else if (deg > 1 && bit_of(fbits[h.z >> 6], h.z)) { par = h.z; pos = 1; }
                    else if (deg > 2 && bit_of(fbits[h.w >> 6], h.w)) { par = h.w; pos = 2; }
                }
                // continuation: positions relative to the row start (rows hold < 2^31 entries);
                // `pos` counts the head probes too when the head is not a row prefix
                constexpr int32_t skip = HUB ? 0 : 3, pbase = HUB ? nprobe : 0;
                // the head did not settle v and its row goes on
                const bool cont = HUB != 3 && act && par < 0 && deg > nprobe;
                if (SEG) {
                    // the row goes to the pending list of the first sub-step
                    const uint64_t pm = __ballot(cont);
                    if (pm) {
                        const int leader = __ffsll((unsigned long long)pm) - 1;
                        uint64_t b = 0;
                        if (lane == leader)
                            b = atomicAdd((unsigned long long*)&slot[S_PEND0], (unsigned long long)__popcll(pm));
                        b = __shfl(b, leader, WAVE);
                        if (cont) pend[b + __popcll(pm & lanemask_lt())] = (uint64_t)(uint32_t)v | ((uint64_t)skip << 32);
                    }
                    if (cont) my_x += (uint64_t)(HUB ? nprobe : 3);   // the head; the sub-steps count the rest
                    else if (par >= 0) found(v, par, pos, deg);
                    else if (act) my_x += (uint64_t)(deg > nprobe ? pbase + deg : deg);
                    if (FILL && act) hlist[r + lane] = par;
                    continue;
                }
                // rows to scan are compacted to the front of the list (slots
                // whose vertices were already loaded) and scanned after the
                // window's heads, 64 at a time: a round of heads no longer
                // waits for the one lane whose row needs a chain of loads
                const uint64_t cm = __ballot(cont);
                if (cont) {
                    const int k = nmiss + __popcll(cm & lanemask_lt());
                    list[k] = v;
                    s_mx[wid][k] = (int16_t)(r + lane);
                }
                nmiss += __popcll(cm);
                if (!cont) {
                    if (par >= 0) found(v, par, pos, deg);
                    else if (act) my_x += (uint64_t)(deg > nprobe ? pbase + deg : deg);
                    // the entry's result replaces its head index (read already)
                    if (FILL && act) hlist[r + lane] = par;
                }
                }
            }
            wave_lds_sync();
            for (int r = 0; r < nmiss; r += WAVE) {
                constexpr int32_t nprobe = HUB >= 2 ? 2 : 3;
                constexpr int32_t skip = HUB ? 0 : 3, pbase = HUB ? nprobe : 0;
                const bool act = r + lane < nmiss;
                const int32_t v = act ? list[r + lane] : 0;
                const int idx = act ? (int)s_mx[wid][r + lane] : 0;
                int64_t beg = 0;
                int32_t deg = 0;
                if (act) {
                    beg = (int64_t)off[v];
                    deg = (int32_t)((int64_t)off[v + 1] - beg);
                }
                int32_t par = -1;
                int32_t pos = 0;   // position of the hit in the row
                int32_t rp = deg;   // next entry to scan; deg when nothing is left
                if (act) {
                    const int32_t lim = deg - skip > serial_len ? skip + serial_len : deg;
                    const int32_t* row = cols + beg;
                    for (rp = skip; rp < lim; rp += 4) {
                        // four entries at once: loads first, then probes
                        const int32_t c0 = row[rp];
                        const int32_t c1 = rp + 1 < lim ? row[rp + 1] : -1;
                        const int32_t c2 = rp + 2 < lim ? row[rp + 2] : -1;
                        const int32_t c3 = rp + 3 < lim ? row[rp + 3] : -1;
                        const uint64_t f0 = fbits[c0 >> 6];
                        const uint64_t f1 = c1 >= 0 ? fbits[c1 >> 6] : 0ull;
                        const uint64_t f2 = c2 >= 0 ? fbits[c2 >> 6] : 0ull;
                        const uint64_t f3 = c3 >= 0 ? fbits[c3 >> 6] : 0ull;
                        if (bit_of(f0, c0)) { par = c0; break; }
                        if (c1 >= 0 && bit_of(f1, c1)) { par = c1; rp += 1; break; }
                        if (c2 >= 0 && bit_of(f2, c2)) { par = c2; rp += 2; break; }
                        if (c3 >= 0 && bit_of(f3, c3)) { par = c3; rp += 3; break; }
                    }
                    if (par >= 0) pos = pbase + rp;
                    else if (rp > lim) rp = lim;
                }
                uint64_t rem = __ballot(act && par < 0 && rp < deg);
                while (rem) {
                    const int l = __ffsll((unsigned long long)rem) - 1;
                    rem &= rem - 1;
                    const int32_t* row = cols + __shfl(beg, l, WAVE);
                    const int32_t pb = __shfl(rp, l, WAVE);
                    const int32_t pe = __shfl(deg, l, WAVE);
                    int32_t got = -1, gotpos = pe;
                    for (int32_t b = pb; b < pe; b += WAVE) {
                        const int32_t i = b + lane;
                        bool hit = false;
                        int32_t c = 0;
                        if (i < pe) {
                            c = row[i];
                            hit = bit_of(fbits[c >> 6], c);
                        }
                        const uint64_t hm = __ballot(hit);
                        if (hm) {
                            const int f = __ffsll((unsigned long long)hm) - 1;
                            got = __shfl(c, f, WAVE);
                            gotpos = b + f;
                            break;
                        }
                    }
                    if (lane == l) {
                        par = got;
                        if (got >= 0) pos = pbase + gotpos;
                    }
                }
                if (par >= 0) found(v, par, pos, deg);
                else if (act) my_x += (uint64_t)(pbase + deg);
                if (FILL && act) hlist[idx] = par;
            }
            wave_lds_sync();
        }
        const uint64_t nb = nbw[lane];
        if (mine) {
            if (HUB == 3) {
                // pre-pass of a top-down level: only visited changes; the
                // level's merge finds these vertices as new (visited & ~vprev)
                if (nb) visited[w] = wv | nb;
            } else {
                nbits[w] = nb;
                if (nb) {
                    visited[w] = wv | nb;
                    vprev[w] = wv | nb;
                }
            }
        }
        if (FILL) {
            // word j of the group, one entry per lane: vertices unvisited at
            // the start of the level take their list slot's result (parent
            // or -1); isolated vertices take -1; vertices visited earlier
            // keep what their level wrote.  Ids >= n and the source excluded.
            const int first = incl - cnt;   // list index of this lane's word's first unvisited vertex
            for (int j = 0; j < GW; ++j) {
                const int64_t wj = w0 + j;
                if (wj >= W) break;
                const uint64_t unv = ~__shfl(wv, j, WAVE);
                uint64_t iso_j = ~__shfl(hasrow, j, WAVE);
                const uint64_t fd_j = __shfl(fdw, j, WAVE);
                const int base = __shfl(first, j, WAVE);
                if (wj == W - 1 && (n & 63)) iso_j &= (1ull << (n & 63)) - 1ull;
                if (wj == (src >> 6)) iso_j &= ~(1ull << (src & 63));
                const uint64_t bit = 1ull << lane;
                const int64_t v = wj * WAVE + lane;
                if (unv & bit) {
                    const int32_t par = hlist[base + __popcll(unv & lanemask_lt())];
                    parent[v] = par;
                    depth[v] = par >= 0 ? next_depth : -1;
                } else if (iso_j & bit) {
                    parent[v] = -1;
                    depth[v] = -1;
                } else if (fd_j & bit) {
                    depth[v] = next_depth - 1;
                }
            }
        }
        wave_lds_sync();
    }
    uint64_t* ln = slot_line(slot);
    block_add3<BLK / WAVE>(my_n, my_m, my_x, &ln[S_NNEXT], &ln[S_MNEXT], &ln[S_EXAMINED]);
}

#define BFS_SWEEP_PARAMS                                                                                          \
    const int4* __restrict__ head, const uint64_t* __restrict__ iso, const uint32_t* __restrict__ nbase,          \
        const OffT* __restrict__ off, const int32_t* __restrict__ cols, const uint64_t* __restrict__ fbits,        \
        const uint64_t* __restrict__ hb, uint64_t* __restrict__ nbits, uint64_t* __restrict__ visited,             \
        uint64_t* __restrict__ vprev, int32_t* __restrict__ parent, int32_t* __restrict__ depth, int64_t W, int GW, \
        int32_t next_depth, int serial_len, uint64_t* __restrict__ slot, uint64_t* __restrict__ zslot, int64_t n,  \
        int64_t src, uint64_t* __restrict__ pend, int frontier_depth
#define BFS_SWEEP_ARGS                                                                                            \
    head, iso, nbase, off, cols, fbits, hb, nbits, visited, vprev, parent, depth, W, GW, next_depth, serial_len,   \
        slot, zslot, n, src, pend, frontier_depth

// the bottom-up step
// (BLK threads per workgroup, one 64-lane wave per group of words)
template <typename OffT, int HUB, int FILL, int SEG, int BLK>
__global__ __launch_bounds__(BLK, 5) void k_bu_sweep(BFS_SWEEP_PARAMS) {
    bu_sweep_body<OffT, HUB, FILL, SEG, BLK>(BFS_SWEEP_ARGS);
}

// ---------------------------------------------------------- first sweep
// The first bottom-up level of a search whose outputs were left unwritten
// (FILL = 1 of k_bu_sweep), laid out one lane per vertex: a wave takes
// BF_WORDS consecutive 64-vertex words at once, with no compacted lists, so
// the loads of all its vertices' heads, and then all their probes, are in
// flight together.  A lane's vertex: reached earlier (the source among
// them) -> nothing written, except the depth of a frontier vertex when the
// top-down level before left it (frontier_depth); isolated -> -1; otherwise
// its head is probed (HUB as in k_bu_sweep), and its parent and depth, or -1,
// are written with its word: lanes write consecutive entries, so each output
// line is written once, whole but for entries of vertices reached earlier.  A vertex whose row goes
// on past an unsettled head (about one in a hundred on a large level) joins
// its wave's waiting list, and the list's rows are scanned a full wave (64)
// at a time (k_bu_sweep's second pass), so a step does not wait for one
// lane's chain of offset, column and probe loads.  A hit found there is
// written over the entry's -1.  Counts and bitmaps as k_bu_sweep.
// HUB = 3 is the hub pre-pass of a heavy top-down level that writes the
// outputs (k_td_hub_prepass's probes): no rows are scanned and only visited
// changes.
constexpr int BF_WORDS = 8;

// lane j's value of x (j the same in every lane), as a wave-uniform value
__device__ __forceinline__ uint64_t read_lane64(uint64_t x, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// v's row, entries [from, deg) at cols + beg: the first frontier entry. A lane
// with `need` scans alone for `serial_len` entries, four loads at a time; the
// rows left are then scanned by the whole wave, one at a time (every lane of
// the wave calls this).  Returns the entry (-1 if none); *at = its position.
__device__ __forceinline__ int32_t row_first_hit(const int32_t* __restrict__ cols, const uint64_t* __restrict__ fbits,
                                                 int64_t beg, int32_t deg, int32_t from, bool need, int serial_len,
                                                 int32_t* at) {
    const int lane = lane_id();
    int32_t par = -1, rp = deg;
    if (need) {
        const int32_t lim = deg - from > serial_len ? from + serial_len : deg;
        const int32_t* row = cols + beg;
        for (rp = from; rp < lim; rp += 4) {
            const int32_t c0 = row[rp];
            const int32_t c1 = rp + 1 < lim ? row[rp + 1] : -1;
            const int32_t c2 = rp + 2 < lim ? row[rp + 2] : -1;
            const int32_t c3 = rp + 3 < lim ? row[rp + 3] : -1;
            const uint64_t f0 = fbits[c0 >> 6];
            const uint64_t f1 = c1 >= 0 ? fbits[c1 >> 6] : 0ull;
            const uint64_t f2 = c2 >= 0 ? fbits[c2 >> 6] : 0ull;
            const uint64_t f3 = c3 >= 0 ? fbits[c3 >> 6] : 0ull;
            if (bit_of(f0, c0)) { par = c0; break; }
            if (c1 >= 0 && bit_of(f1, c1)) { par = c1; rp += 1; break; }
            if (c2 >= 0 && bit_of(f2, c2)) { par = c2; rp += 2; break; }
            if (c3 >= 0 && bit_of(f3, c3)) { par = c3; rp += 3; break; }
        }
        if (par < 0 && rp > lim) rp = lim;
    }
    uint64_t rem = __ballot(need && par < 0 && rp < deg);
    while (rem) {
        const int l = __ffsll((unsigned long long)rem) - 1;
        rem &= rem - 1;
        const int32_t* row = cols + __shfl(beg, l, WAVE);
        const int32_t pb = __shfl(rp, l, WAVE);
        const int32_t pe = __shfl(deg, l, WAVE);
        int32_t got = -1, gotpos = pe;
        for (int32_t b = pb; b < pe; b += WAVE) {
            const int32_t i = b + lane;
            bool hit = false;
            int32_t c = 0;
            if (i < pe) {
                c = row[i];
                hit = bit_of(fbits[c >> 6], c);
            }
            const uint64_t hm = __ballot(hit);
            if (hm) {
                const int f = __ffsll((unsigned long long)hm) - 1;
                got = __shfl(c, f, WAVE);
                gotpos = b + f;
                break;
            }
        }
        if (lane == l) {
            par = got;
            rp = gotpos;
        }
    }
    *at = rp;
    return par;
}

template <typename OffT, int HUB>
__global__ __launch_bounds__(BU_BLOCK) void k_bu_fill(
    const int4* __restrict__ head, const uint64_t* __restrict__ iso, const uint32_t* __restrict__ nbase,
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, const uint64_t* __restrict__ fbits,
    const uint64_t* __restrict__ hb, uint64_t* __restrict__ nbits, uint64_t* __restrict__ visited,
    uint64_t* __restrict__ vprev, int32_t* __restrict__ parent, int32_t* __restrict__ depth, int64_t W,
    int32_t next_depth, int serial_len, uint64_t* __restrict__ slot, uint64_t* __restrict__ zslot, int64_t n,
    int64_t src, int frontier_depth) {
    __shared__ uint64_t s_hb[HUB >= 2 ? HUB_BITS / 64 : 1];
    // vertices whose head did not settle them, waiting for their row scan
    __shared__ int32_t s_miss[BU_BLOCK / WAVE][WAVE * (BF_WORDS + 1)];
    if (HUB >= 2) {
        for (int i = threadIdx.x; i < HUB_BITS / 64; i += BU_BLOCK) s_hb[i] = hb[i];
        __syncthreads();
    }
    zero_slot(zslot);
    const int lane = lane_id();
    const uint64_t lbit = 1ull << lane;
    int32_t* miss = s_miss[threadIdx.x / WAVE];
    int nmiss = 0;   // wave-uniform
    const int64_t G = (W + BF_WORDS - 1) / BF_WORDS;
    const int64_t nwaves = (int64_t)gridDim.x * (BU_BLOCK / WAVE);
    uint64_t my_n = 0, my_m = 0, my_x = 0;
    // HUB = 3: the hub pre-pass of a heavy top-down level
    constexpr bool PRE = HUB == 3;
    // entries the head probes; with HUB >= 2 its last word holds hub ranks
    constexpr int32_t nprobe = HUB >= 2 ? 2 : 3;
    // a row scan starts past the head when the head is the row's prefix;
    // positions count the head's probes too when it is not
    constexpr int32_t skip = HUB ? 0 : 3, pbase = HUB ? nprobe : 0;
    // the row scans of `cnt` (<= 64) waiting vertices from list index i0, one per lane.
    // Their entries hold -1 already (written with their word); a hit
    // overwrites them and sets the vertex's bits with atomics.  The release
    // fence first completes this wave's earlier stores to the same words and
    // entries.
    auto drain = [&](int i0, int cnt) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        const bool a = lane < cnt;
        const int32_t v = a ? miss[i0 + lane] : 0;
        int64_t beg = 0;
        int32_t deg = 0;
        if (a) {
            beg = (int64_t)off[v];
            deg = (int32_t)((int64_t)off[v + 1] - beg);
        }
        int32_t at = 0;
        const int32_t got = row_first_hit(cols, fbits, beg, deg, skip, a, serial_len, &at);
        if (a) {
            if (got >= 0) {
                my_n += 1;
                my_m += (uint64_t)deg;
                my_x += (uint64_t)(pbase + at + 1);
                __builtin_nontemporal_store(got, &parent[v]);
                __builtin_nontemporal_store(next_depth, &depth[v]);
                const unsigned long long bit = 1ull << (v & 63);
                atomicOr((unsigned long long*)&nbits[v >> 6], bit);
                atomicOr((unsigned long long*)&visited[v >> 6], bit);
                atomicOr((unsigned long long*)&vprev[v >> 6], bit);
            } else {
                my_x += (uint64_t)(pbase + deg);
            }
        }
    };
    // lane j < BF_WORDS holds word j of the wave's current step; the next
    // step's words are loaded while the current one is processed
    int64_t gi = (int64_t)blockIdx.x * (BU_BLOCK / WAVE) + threadIdx.x / WAVE;
    uint64_t cv = ~0ull, ci = ~0ull, cf = 0ull;
    uint32_t cb = 0;
    if (gi < G && lane < BF_WORDS && gi * BF_WORDS + lane < W) {
        const int64_t w = gi * BF_WORDS + lane;
        cv = stream_load(&visited[w]);
        ci = stream_load(&iso[w]);
        cb = nbase[w];
        if (frontier_depth) cf = fbits[w];
    }
    for (; gi < G; gi += nwaves) {
        const int64_t w0 = gi * BF_WORDS;
        uint64_t vw[BF_WORDS], iw[BF_WORDS], fw[BF_WORDS];
        uint32_t base[BF_WORDS];
#pragma unroll
        for (int j = 0; j < BF_WORDS; ++j) {
            vw[j] = read_lane64(cv, j);
            iw[j] = read_lane64(ci, j);
            fw[j] = read_lane64(cf, j);
            base[j] = (uint32_t)__builtin_amdgcn_readlane((int)cb, j);
        }
        {
            const int64_t gn = gi + nwaves;
            cv = ~0ull;
            ci = ~0ull;
            cf = 0ull;
            cb = 0;
            if (gn < G && lane < BF_WORDS && gn * BF_WORDS + lane < W) {
                const int64_t w = gn * BF_WORDS + lane;
                cv = stream_load(&visited[w]);
                ci = stream_load(&iso[w]);
                cb = nbase[w];
                if (frontier_depth) cf = fbits[w];
            }
        }
        // this lane's vertices: unvisited with edges load their heads
        bool act[BF_WORDS];
        int4 h[BF_WORDS];
#pragma unroll
        for (int j = 0; j < BF_WORDS; ++j) {
            act[j] = !((vw[j] | iw[j]) & lbit);
            h[j] = make_int4(0, -1, -1, -1);
            if (act[j]) h[j] = stream_load4(&head[base[j] + (uint32_t)__popcll(~iw[j] & (lbit - 1ull))]);
        }
        uint64_t fa[BF_WORDS], fb[BF_WORDS];
#pragma unroll
        for (int j = 0; j < BF_WORDS; ++j) {
            const int deg = h[j].x;
            if (HUB >= 2) {
                const uint32_t q0 = (uint32_t)h[j].w & 0xFFFFu, q1 = (uint32_t)h[j].w >> 16;
                fa[j] = deg > 0 ? (q0 != 0xFFFFu ? s_hb[q0 >> 6] : fbits[h[j].y >> 6]) : 0ull;
                fb[j] = deg > 1 ? (q1 != 0xFFFFu ? s_hb[q1 >> 6] : fbits[h[j].z >> 6]) : 0ull;
            } else {
                fa[j] = deg > 0 ? fbits[h[j].y >> 6] : 0ull;
                fb[j] = 0ull;
            }
        }
#pragma unroll
        for (int j = 0; j < BF_WORDS; ++j) {
            const int64_t w = w0 + j;
            const int64_t v = w * WAVE + lane;
            const int32_t deg = h[j].x;
            int32_t par = -1, pos = 0;
            if (HUB >= 2) {
                const uint32_t q0 = (uint32_t)h[j].w & 0xFFFFu, q1 = (uint32_t)h[j].w >> 16;
                if (deg > 0 && bit_of(fa[j], q0 != 0xFFFFu ? (int32_t)q0 : h[j].y)) { par = h[j].y; pos = 0; }
                else if (deg > 1 && bit_of(fb[j], q1 != 0xFFFFu ? (int32_t)q1 : h[j].z)) { par = h[j].z; pos = 1; }
            } else {
                if (deg > 0 && bit_of(fa[j], h[j].y)) { par = h[j].y; pos = 0; }
                else if (deg > 1 && bit_of(fbits[h[j].z >> 6], h[j].z)) { par = h[j].z; pos = 1; }
                else if (deg > 2 && bit_of(fbits[h[j].w >> 6], h[j].w)) { par = h[j].w; pos = 2; }
            }
            const bool found = par >= 0;
            // the head did not settle v and its row goes on: the scan waits
            // (the pre-pass scans no rows)
            const bool cont = !PRE && act[j] && !found && deg > nprobe;
            const uint64_t cm = __ballot(cont);
            if (cont) miss[nmiss + __popcll(cm & lanemask_lt())] = (int32_t)v;
            nmiss += __popcll(cm);
            if (found) {
                my_n += 1;
                my_m += (uint64_t)deg;
                my_x += (uint64_t)(pos + 1);
            } else if (act[j] && !cont) {
                my_x += (uint64_t)(deg > nprobe ? pbase + deg : deg);
            }
            // every entry of a vertex not reached before this level, once
            // (isolated vertices are marked visited when a search starts)
            const bool unreached = !(vw[j] & lbit) || ((iw[j] & lbit) && v != src);
            if (v < n && unreached) {
                parent[v] = found ? par : -1;
                depth[v] = found ? next_depth : -1;
            } else if (fw[j] & lbit) {
                // reached by the top-down level before, which left its depth
                depth[v] = next_depth - 1;
            }
            const uint64_t nb = __ballot(found);
            if (PRE) {
                // the level's merge finds the hits as new (visited & ~vprev)
                if (lane == 0 && w < W && nb) visited[w] = vw[j] | nb;
            } else if (lane == 0 && w < W) {
                nbits[w] = nb;
                if (nb) {
                    visited[w] = vw[j] | nb;
                    vprev[w] = vw[j] | nb;
                }
            }
        }
        // full waves of waiting rows are scanned; the rest move to the front
        if (nmiss >= WAVE) {
            wave_lds_sync();
            int done = 0;
            for (; nmiss - done >= WAVE; done += WAVE) drain(done, WAVE);
            const int rest = nmiss - done;
            int32_t keep = lane < rest ? miss[done + lane] : 0;
            wave_lds_sync();
            if (lane < rest) miss[lane] = keep;
            nmiss = rest;
        }
    }
    if (nmiss) {
        wave_lds_sync();
        drain(0, nmiss);
    }
    uint64_t* ln = slot_line(slot);
    block_add3<BU_BLOCK / WAVE>(my_n, my_m, my_x, &ln[S_NNEXT], &ln[S_MNEXT], &ln[S_EXAMINED]);
}

// the hub pre-pass of a heavy top-down level (a kernel of its own name, so
// profiles keep it apart from the bottom-up step)
template <typename OffT, int FILL>
__global__ __launch_bounds__(BU_BLOCK) void k_td_hub_prepass(BFS_SWEEP_PARAMS) {
    bu_sweep_body<OffT, 3, FILL, 0, BU_BLOCK>(BFS_SWEEP_ARGS);
}

// ------------------------------------------------------------ column segments
// One sub-step of a column-blocked bottom-up level (Alg. 4's sub-steps with
// the completed mask, inside one device): every pending row (vertex v, row
// position p) is scanned from p over its entries below `seg_end` only, in
// row order, probing the frontier bitmap's words of this segment (an
// L2-sized slice when the segments are chosen so).  The first frontier entry
// found is v's parent: the rows are sorted and the segments ascend, so it is
// the first frontier entry of the whole row.  A row that reaches an entry
// >= seg_end without a hit goes, with that position, to the pending list of
// the next sub-step; the last sub-step has seg_end = n.  Found vertices set
// their bits of nbits / visited / vprev with atomics (the words are shared
// between waves here) and write their outputs.
template <typename OffT>
__global__ __launch_bounds__(BU_BLOCK) void k_bu_segment(
    const OffT* __restrict__ off, const int32_t* __restrict__ cols, const uint64_t* __restrict__ fbits,
    const uint64_t* __restrict__ pin, const uint64_t* __restrict__ cin, uint64_t* __restrict__ pout,
    uint64_t* __restrict__ cout, int64_t seg_end, int32_t* __restrict__ parent, int32_t* __restrict__ depth,
    uint64_t* __restrict__ nbits, uint64_t* __restrict__ visited, uint64_t* __restrict__ vprev,
    int32_t next_depth, int serial_len, uint64_t* __restrict__ slot) {
    const int lane = lane_id();
    const int64_t count = (int64_t)*cin;
    const int64_t nwaves = (int64_t)gridDim.x * (BU_BLOCK / WAVE);
    const int32_t lim_id = seg_end < 2147483647LL ? (int32_t)seg_end : 2147483647;
    uint64_t my_n = 0, my_m = 0, my_x = 0;
    const int64_t wi = (int64_t)blockIdx.x * (BU_BLOCK / WAVE) + threadIdx.x / WAVE;
    for (int64_t i0 = wi * WAVE; i0 < count; i0 += nwaves * WAVE) {
        const int64_t i = i0 + lane;
        const bool act = i < count;
        int32_t v = 0, rp = 0, deg = 0;
        int64_t beg = 0;
        if (act) {
            const uint64_t e = pin[i];
            v = (int32_t)(uint32_t)e;
            rp = (int32_t)(e >> 32);
            beg = (int64_t)off[v];
            deg = (int32_t)((int64_t)off[v + 1] - beg);
        }
        const int32_t rp0 = rp;
        int32_t par = -1;
        bool stop = false;   // reached an entry of a later segment
        const int32_t* row = cols + beg;
        if (act) {
            const int32_t lim = deg - rp > serial_len ? rp + serial_len : deg;
            for (; rp < lim; rp += 4) {
                const int32_t c0 = row[rp];
                const int32_t c1 = rp + 1 < lim ? row[rp + 1] : lim_id;
                const int32_t c2 = rp + 2 < lim ? row[rp + 2] : lim_id;
                const int32_t c3 = rp + 3 < lim ? row[rp + 3] : lim_id;
                const uint64_t f0 = c0 < lim_id ? fbits[c0 >> 6] : 0ull;
                const uint64_t f1 = c1 < lim_id ? fbits[c1 >> 6] : 0ull;
                const uint64_t f2 = c2 < lim_id ? fbits[c2 >> 6] : 0ull;
                const uint64_t f3 = c3 < lim_id ? fbits[c3 >> 6] : 0ull;
                if (c0 >= lim_id) { stop = true; break; }
                if (bit_of(f0, c0)) { par = c0; break; }
                if (rp + 1 >= lim) { rp += 1; break; }
                if (c1 >= lim_id) { rp += 1; stop = true; break; }
                if (bit_of(f1, c1)) { par = c1; rp += 1; break; }
                if (rp + 2 >= lim) { rp += 2; break; }
                if (c2 >= lim_id) { rp += 2; stop = true; break; }
                if (bit_of(f2, c2)) { par = c2; rp += 2; break; }
                if (rp + 3 >= lim) { rp += 3; break; }
                if (c3 >= lim_id) { rp += 3; stop = true; break; }
                if (bit_of(f3, c3)) { par = c3; rp += 3; break; }
            }
            if (rp > lim) rp = lim;
        }
        // rows still open after serial_len entries: the whole wave, 64 at a time
        uint64_t rem = __ballot(act && par < 0 && !stop && rp < deg);
        while (rem) {
            const int l = __ffsll((unsigned long long)rem) - 1;
            rem &= rem - 1;
            const int32_t* lrow = cols + __shfl(beg, l, WAVE);
            const int32_t pb = __shfl(rp, l, WAVE);
            const int32_t pe = __shfl(deg, l, WAVE);
            int32_t got = -1, at = pe;
            bool out = false;
            for (int32_t b = pb; b < pe; b += WAVE) {
                const int32_t x = b + lane;
                int32_t c = lim_id;
                bool hit = false;
                if (x < pe) {
                    c = lrow[x];
                    hit = c < lim_id && bit_of(fbits[c >> 6], c);
                }
                const uint64_t hm = __ballot(hit);
                const uint64_t om = __ballot(x < pe && c >= lim_id);
                if (hm | om) {
                    const int fh = hm ? __ffsll((unsigned long long)hm) - 1 : WAVE;
                    const int fo = om ? __ffsll((unsigned long long)om) - 1 : WAVE;
                    if (fh < fo) {
                        got = __shfl(c, fh, WAVE);
                        at = b + fh;
                    } else {
                        out = true;
                        at = b + fo;
                    }
                    break;
                }
            }
            if (lane == l) {
                par = got;
                stop = out;
                rp = at;
            }
        }
        if (act) {
            if (par >= 0) {
                __builtin_nontemporal_store(par, &parent[v]);
                __builtin_nontemporal_store(next_depth, &depth[v]);
                const unsigned long long bit = 1ull << (v & 63);
                __hip_atomic_fetch_or((unsigned long long*)&nbits[v >> 6], bit, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_or((unsigned long long*)&visited[v >> 6], bit, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_or((unsigned long long*)&vprev[v >> 6], bit, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                my_n += 1;
                my_m += (uint64_t)deg;
                my_x += (uint64_t)(rp - rp0 + 1);
            } else {
                my_x += (uint64_t)(rp - rp0);   // up to the segment's end or the row's
            }
        }
        const bool again = act && par < 0 && stop;
        const uint64_t am = __ballot(again);
        if (am) {
            const int leader = __ffsll((unsigned long long)am) - 1;
            uint64_t b = 0;
            if (lane == leader) b = atomicAdd((unsigned long long*)cout, (unsigned long long)__popcll(am));
            b = __shfl(b, leader, WAVE);
            if (again) pout[b + __popcll(am & lanemask_lt())] = (uint64_t)(uint32_t)v | ((uint64_t)rp << 32);
        }
    }
    uint64_t* ln = slot_line(slot);
    block_add3<BU_BLOCK / WAVE>(my_n, my_m, my_x, &ln[S_NNEXT], &ln[S_MNEXT], &ln[S_EXAMINED]);
}
#undef BFS_SWEEP_PARAMS
#undef BFS_SWEEP_ARGS

// words per group: 64 when that still gives every wave of the grid several
// groups, fewer on small graphs so the sweep spreads over the whole chip
static int group_words(int64_t W, int waves) {
    int gw = WAVE;
    while (gw > 1 && (W + gw - 1) / gw < 2 * (int64_t)waves) gw >>= 1;
    return gw;
}

template <typename OffT>
void launch_bu_sweep(const Launch& L, const int4* head, int hub, const uint64_t* iso, const uint32_t* nbase,
                     const OffT* off, const int32_t* cols, const uint64_t* fbits, const uint64_t* hb, uint64_t* nbits,
                     uint64_t* visited, uint64_t* vprev, int32_t* parent, int32_t* depth, int64_t W,
                     int32_t next_depth, int serial_len, uint64_t* slot, uint64_t* zslot, bool fill, int64_t n,
                     int64_t src, uint64_t* pend, int block, int group_cap, bool frontier_depth) {
    // the column-blocked sweep and the pre-pass keep the default shape
    const int blk = (hub == 3 || pend || (block != 128 && block != 512)) ? BU_BLOCK : block;
    int gw = group_words(W, L.grid_cap * (blk / WAVE));
    if (group_cap > 0 && gw > group_cap) gw = group_cap;
    if (fill && gw > FILL_GW) gw = FILL_GW;
    const int64_t G = (W + gw - 1) / gw;
    const int g = grid_for(G, blk / WAVE, L.grid_cap);
#define BFS_SWEEP(H, F, S, B)                                                                                     \
    hipLaunchKernelGGL((k_bu_sweep<OffT, H, F, S, B>), dim3(g), dim3(B), 0, L.stream, head, iso, nbase, off,       \
                       cols, fbits, hb, nbits, visited, vprev, parent, depth, W, gw, next_depth, serial_len, slot,  \
                       zslot, n, src, pend, (int)frontier_depth)
#define BFS_PREPASS(F)                                                                                              \
    hipLaunchKernelGGL((k_td_hub_prepass<OffT, F>), dim3(g), dim3(BU_BLOCK), 0, L.stream, head, iso, nbase, off,    \
                       cols, fbits, hb, nbits, visited, vprev, parent, depth, W, gw, next_depth, serial_len, slot,     \
                       zslot, n, src, pend, (int)frontier_depth)
#define BFS_SWEEP_H(F, S, B)                 \
    if (hub == 2) BFS_SWEEP(2, F, S, B);     \
    else if (hub == 1) BFS_SWEEP(1, F, S, B); \
    else BFS_SWEEP(0, F, S, B);
#define BFS_SWEEP_HB(F)                                   \
    if (blk == 128) { BFS_SWEEP_H(F, 0, 128) }            \
    else if (blk == 512) { BFS_SWEEP_H(F, 0, 512) }       \
    else { BFS_SWEEP_H(F, 0, BU_BLOCK) }
    if (fill && hub != 0 && !pend) {
        // the first sweep of a search that writes the outputs (or the hub
        // pre-pass that writes them), with heads of high-degree neighbours:
        // one lane per vertex.  Heads that are row prefixes (HUB = 0) leave
        // far more rows to scan (about one vertex in five on a large level),
        // and k_bu_sweep's compacted lists do better.
        const int gf = grid_for((W + BF_WORDS - 1) / BF_WORDS, BU_BLOCK / WAVE, L.grid_cap);
#define BFS_FILL1(H)                                                                                             \
    hipLaunchKernelGGL((k_bu_fill<OffT, H>), dim3(gf), dim3(BU_BLOCK), 0, L.stream, head, iso, nbase, off, cols, \
                       fbits, hb, nbits, visited, vprev, parent, depth, W, next_depth, serial_len, slot, zslot, n,   \
                       src, (int)frontier_depth)
        if (hub == 3) BFS_FILL1(3);
        else if (hub == 2) BFS_FILL1(2);
        else BFS_FILL1(1);
#undef BFS_FILL1
        return;
    }
    if (hub == 3) {
        if (fill) BFS_PREPASS(1);
        else BFS_PREPASS(0);
    } else if (pend) {
        if (fill) { BFS_SWEEP_H(1, 1, BU_BLOCK) }
        else { BFS_SWEEP_H(0, 1, BU_BLOCK) }
    } else {
        if (fill) { BFS_SWEEP_HB(1) }
        else { BFS_SWEEP_HB(0) }
    }
#undef BFS_SWEEP_HB
#undef BFS_SWEEP_H
#undef BFS_SWEEP
#undef BFS_PREPASS
}

template <typename OffT>
void launch_bu_segment(const Launch& L, const OffT* off, const int32_t* cols, const uint64_t* fbits,
                       const uint64_t* pin, const uint64_t* cin, uint64_t* pout, uint64_t* cout, int64_t seg_end,
                       int32_t* parent, int32_t* depth, uint64_t* nbits, uint64_t* visited, uint64_t* vprev,
                       int32_t next_depth, int serial_len, uint64_t* slot) {
    hipLaunchKernelGGL(k_bu_segment<OffT>, dim3(L.grid_cap), dim3(BU_BLOCK), 0, L.stream, off, cols, fbits, pin, cin,
                       pout, cout, seg_end, parent, depth, nbits, visited, vprev, next_depth, serial_len, slot);
}

// ------------------------------------------------------------------ row heads
// index of vertex v's head record: its rank among the vertices with edges
__device__ __forceinline__ int64_t head_index(const uint64_t* iso, const uint32_t* nbase, int64_t v) {
    return (int64_t)nbase[v >> 6] + __popcll(~iso[v >> 6] & ((1ull << (v & 63)) - 1ull));
}

template <typename OffT>
__global__ void k_row_heads(const OffT* __restrict__ off, const int32_t* __restrict__ cols, int64_t n,
                            const uint64_t* __restrict__ iso, const uint32_t* __restrict__ nbase,
                            int4* __restrict__ head) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int64_t b = (int64_t)off[v];
        const int64_t d = (int64_t)off[v + 1] - b;
        if (d == 0) continue;
        int4 h;
        h.x = (int32_t)d;
        h.y = d > 0 ? cols[b] : -1;
        h.z = d > 1 ? cols[b + 1] : -1;
        h.w = d > 2 ? cols[b + 2] : -1;
        head[head_index(iso, nbase, v)] = h;
    }
}

template <typename OffT>
void launch_row_heads(const Launch& L, const OffT* off, const int32_t* cols, int64_t n, const uint64_t* iso,
                      const uint32_t* nbase, int4* head) {
    hipLaunchKernelGGL(k_row_heads<OffT>, dim3(grid_for(n, 256, L.grid_cap)), dim3(256), 0, L.stream, off, cols, n,
                       iso, nbase, head);
}

// nbase[w] = vertices with edges in words [0, w)
struct RowsInWord {
    const uint64_t* iso;
    __device__ int64_t operator()(int64_t w) const { return __popcll(~iso[w]); }
};
struct BaseSink {
    uint32_t* nbase;
    __device__ void item(int64_t w, int64_t before, int64_t) const { nbase[w] = (uint32_t)before; }
    __device__ void last(int64_t, int64_t) const {}
};

void launch_head_index(const Launch& L, const uint64_t* iso, int64_t W, uint32_t* nbase, int64_t* partial) {
    launch_scan(L.stream, RowsInWord{iso}, (const uint64_t*)nullptr, W, partial, BaseSink{nbase});
}

// hub heads: {deg, the three neighbours of highest degree (ties: smaller id)}
// chosen among the first HUB_SCAN entries of the row; degrees come from the
// row heads
constexpr int HUB_SCAN = 64;

__device__ __forceinline__ bool hub_before(int32_t da, int32_t a, int32_t db, int32_t b) {
    return da > db || (da == db && a < b);
}

template <typename OffT>
__global__ void k_hub_heads(const OffT* __restrict__ off, const int32_t* __restrict__ cols, int64_t n,
                            const uint64_t* __restrict__ iso, const uint32_t* __restrict__ nbase,
                            int4* __restrict__ hub) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int64_t b = (int64_t)off[v];
        const int64_t d = (int64_t)off[v + 1] - b;
        if (d == 0) continue;
        const int64_t m = d < HUB_SCAN ? d : HUB_SCAN;
        int32_t c0 = -1, c1 = -1, c2 = -1, d0 = -1, d1 = -1, d2 = -1;
        for (int64_t i = 0; i < m; ++i) {
            const int32_t c = cols[b + i];
            const int32_t dc = (int32_t)((int64_t)off[c + 1] - (int64_t)off[c]);
            if (hub_before(dc, c, d0, c0) || c0 < 0) {
                c2 = c1; d2 = d1; c1 = c0; d1 = d0; c0 = c; d0 = dc;
            } else if (hub_before(dc, c, d1, c1) || c1 < 0) {
                c2 = c1; d2 = d1; c1 = c; d1 = dc;
            } else if (hub_before(dc, c, d2, c2) || c2 < 0) {
                c2 = c; d2 = dc;
            }
        }
        hub[head_index(iso, nbase, v)] = make_int4((int32_t)d, c0, c1, c2);
    }
}

template <typename OffT>
void launch_hub_heads(const Launch& L, const OffT* off, const int32_t* cols, int64_t n, const uint64_t* iso,
                      const uint32_t* nbase, int4* hub) {
    hipLaunchKernelGGL(k_hub_heads<OffT>, dim3(grid_for(n, 256, L.grid_cap)), dim3(256), 0, L.stream, off, cols, n,
                       iso, nbase, hub);
}

// ------------------------------------------------------------------ hub ranks
// The hubs are the vertices of degree >= a threshold chosen so that at most
// HUB_BITS - 1 of them exist; rank = position among the hubs in id order.
// small degrees (most vertices) are counted in LDS first: same-address
// global atomics would serialise
constexpr int HIST_LDS = 2048;

template <typename OffT>
__global__ __launch_bounds__(256) void k_deg_hist(const OffT* __restrict__ off, int64_t n,
                                                  uint32_t* __restrict__ hist, int nbins) {
    __shared__ uint32_t s_h[HIST_LDS];
    for (int i = threadIdx.x; i < HIST_LDS; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int64_t d = (int64_t)off[v + 1] - (int64_t)off[v];
        if (d <= 0) continue;
        const int64_t b = d < nbins - 1 ? d : nbins - 1;
        if (b < HIST_LDS) atomicAdd(&s_h[b], 1u);
        else atomicAdd(&hist[b], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HIST_LDS && i < nbins; i += blockDim.x)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

template <typename OffT>
__global__ void k_hub_mask(const OffT* __restrict__ off, int64_t n, int64_t W, int64_t thr,
                           uint64_t* __restrict__ mask) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < W; w += stride) {
        uint64_t m = 0;
        for (int b = 0; b < 64; ++b) {
            const int64_t v = w * 64 + b;
            if (v < n && (int64_t)off[v + 1] - (int64_t)off[v] >= thr) m |= 1ull << b;
        }
        mask[w] = m;
    }
}

struct PopcWord {
    const uint64_t* m;
    __device__ int64_t operator()(int64_t w) const { return __popcll(m[w]); }
};

__global__ void k_hub_ids(const uint64_t* __restrict__ mask, const uint32_t* __restrict__ hbase, int64_t W,
                          int32_t* __restrict__ hubid) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < W; w += stride) {
        uint64_t m = mask[w];
        uint32_t r = hbase[w];
        while (m) {
            const int b = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            hubid[r++] = (int32_t)(w * 64 + b);
        }
    }
}

// {deg, c0, c1, ranks} from the hub heads {deg, c0, c1, c2}
__global__ void k_hub_rank_heads(const int4* __restrict__ hub, int64_t nrec, const uint64_t* __restrict__ mask,
                                 const uint32_t* __restrict__ hbase, int4* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrec; i += stride) {
        const int4 h = hub[i];
        uint32_t rk[2] = {0xFFFFu, 0xFFFFu};
        const int32_t c[2] = {h.y, h.z};
        for (int j = 0; j < 2; ++j) {
            if (c[j] < 0) continue;
            const uint64_t mw = mask[c[j] >> 6];
            const uint64_t bit = 1ull << (c[j] & 63);
            if (mw & bit) rk[j] = hbase[c[j] >> 6] + (uint32_t)__popcll(mw & (bit - 1ull));
        }
        out[i] = make_int4(h.x, h.y, h.z, (int32_t)(rk[0] | (rk[1] << 16)));
    }
}

template <typename OffT>
void launch_deg_hist(const Launch& L, const OffT* off, int64_t n, uint32_t* hist, int nbins) {
    hipLaunchKernelGGL(k_deg_hist<OffT>, dim3(grid_for(n, 256, 1024)), dim3(256), 0, L.stream, off, n, hist, nbins);
}

template <typename OffT>
void launch_hub_ranks(const Launch& L, const OffT* off, int64_t n, int64_t thr, const int4* hub, int64_t nrec,
                      uint64_t* mask, uint32_t* hbase, int64_t* partial, int32_t* hubid, int4* out) {
    const int64_t W = (n + 63) / 64;
    hipLaunchKernelGGL(k_hub_mask<OffT>, dim3(grid_for(W, 256, L.grid_cap)), dim3(256), 0, L.stream, off, n, W, thr,
                       mask);
    launch_scan(L.stream, PopcWord{mask}, (const uint64_t*)nullptr, W, partial, BaseSink{hbase});
    hipLaunchKernelGGL(k_hub_ids, dim3(grid_for(W, 256, L.grid_cap)), dim3(256), 0, L.stream, mask, hbase, W, hubid);
    hipLaunchKernelGGL(k_hub_rank_heads, dim3(grid_for(nrec, 256, L.grid_cap)), dim3(256), 0, L.stream, hub, nrec,
                       mask, hbase, out);
}

// frontier bits of the hubs, in rank order (one wave per output word)
__global__ void k_hub_gather(const uint64_t* __restrict__ fbits, const int32_t* __restrict__ hubid, int nhub,
                             uint64_t* __restrict__ hb) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    bool on = false;
    if (r < nhub) {
        const int32_t v = hubid[r];
        on = (fbits[v >> 6] >> (v & 63)) & 1ull;
    }
    const uint64_t m = __ballot(on);
    if (lane_id() == 0 && r < HUB_BITS) hb[r >> 6] = m;
}

void launch_hub_gather(const Launch& L, const uint64_t* fbits, const int32_t* hubid, int nhub, uint64_t* hb) {
    hipLaunchKernelGGL(k_hub_gather, dim3(HUB_BITS / 256), dim3(256), 0, L.stream, fbits, hubid, nhub, hb);
}

#define BFS_BU_INST(T)                                                                                           \
    template void launch_bu_sweep<T>(const Launch&, const int4*, int, const uint64_t*, const uint32_t*,          \
                                     const T*, const int32_t*, const uint64_t*, const uint64_t*, uint64_t*,      \
                                     uint64_t*, uint64_t*, int32_t*, int32_t*, int64_t, int32_t, int, uint64_t*, \
                                     uint64_t*, bool, int64_t, int64_t, uint64_t*, int, int, bool);              \
    template void launch_bu_segment<T>(const Launch&, const T*, const int32_t*, const uint64_t*, const uint64_t*, \
                                       const uint64_t*, uint64_t*, uint64_t*, int64_t, int32_t*, int32_t*,       \
                                       uint64_t*, uint64_t*, uint64_t*, int32_t, int, uint64_t*);                \
    template void launch_deg_hist<T>(const Launch&, const T*, int64_t, uint32_t*, int);                          \
    template void launch_hub_ranks<T>(const Launch&, const T*, int64_t, int64_t, const int4*, int64_t,          \
                                      uint64_t*, uint32_t*, int64_t*, int32_t*, int4*);                         \
    template void launch_row_heads<T>(const Launch&, const T*, const int32_t*, int64_t, const uint64_t*,        \
                                      const uint32_t*, int4*);                                                   \
    template void launch_hub_heads<T>(const Launch&, const T*, const int32_t*, int64_t, const uint64_t*,        \
                                      const uint32_t*, int4*);
BFS_BU_INST(int32_t)
BFS_BU_INST(int64_t)

}  // namespace bfsk
