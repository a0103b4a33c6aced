// Local discovery on one hypersparse DCSC block A_ij of a p_r x p_c 2D
// decomposition (Eq. 1, Section 5.1), gfx950.
//
// Top-down (Alg. 3, the sparse-matrix sparse-vector product on the
// (select2nd, min) semiring of Section 4.2, with a sparse accumulator as in
// Section 5.2):
//   0. (dense frontiers, more than 1/32 of the columns, sorted block with its
//      row-compressed copy) the result is computed from the row side instead:
//      a first-hit sweep of every row against a bitmap of F, the pull form of
//      the same product, with no accumulator and no atomics
//   1. every frontier column is looked up in JC (binary search; for frontiers
//      where |F| log2 nzc > nzc one pass over JC against a column bitmap of F
//      instead); the JC indices found are compacted into a queue
//   2. a prefix sum over their column lengths splits all their entries into
//      fixed tiles (the same edge-balanced tiling as the whole-graph
//      top-down step)
//   3. each entry (r, k) offers col_base + k to row r: the accumulator keeps
//      the minimum (stored complemented, so the atomic is a max and the
//      all-zero state means "empty"), and an occupied bitmap marks r
//   4. an ordered compaction over the occupied bitmap emits (row, parent)
//      pairs in ascending row order and resets exactly the accumulator
//      entries and bitmap words it read, leaving the workspace zeroed.
// Bottom-up (Alg. 4, one sub-step of local discovery) over the row-compressed
// copy of the block:
//   1. the JR entries of rows [row_lo, row_hi) are found by binary search
//   2. one wave takes 64 consecutive non-empty rows; a row not yet completed
//      scans its ascending columns against the frontier bitmap, serially for
//      `serial_len` entries and then 64 at a time with the whole wave, and
//      stops at the first hit; found rows set their completed bit
//   3. an ordered compaction over the per-wave ballots emits (row, parent)
//      pairs in ascending row order.
// Both paths run entirely on the device: lengths and totals never travel to
// the host, so the calls are asynchronous on their stream.
#include <cmath>

#include "bfs_device.h"

namespace bfsk {

// ---------------------------------------------------------------- top-down
__global__ __launch_bounds__(256) void k_blk_find(const int32_t* __restrict__ jc, int64_t nzc,
                                                  const int32_t* __restrict__ F, int64_t nf,
                                                  int32_t* __restrict__ q, uint64_t* __restrict__ qlen) {
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < nf; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        int32_t h = -1;
        if (i < nf) {
            const int32_t c = F[i];
            int64_t lo = 0, hi = nzc;   // first JC entry >= c
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (jc[mid] < c) lo = mid + 1; else hi = mid;
            }
            if (lo < nzc && jc[lo] == c) h = (int32_t)lo;
        }
        const uint64_t m = __ballot(h >= 0);
        if (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            uint64_t b = 0;
            if (lane == leader) b = atomicAdd((unsigned long long*)qlen, (unsigned long long)__popcll(m));
            b = __shfl(b, leader, WAVE);
            if (h >= 0) q[b + __popcll(m & lanemask_lt())] = h;
        }
    }
}

__global__ __launch_bounds__(TD_BLOCK) void k_blk_expand(
    const int64_t* __restrict__ cp, const int32_t* __restrict__ jc, const int32_t* __restrict__ ir,
    const int32_t* __restrict__ q, const uint64_t* __restrict__ qlen_dev, const int64_t* __restrict__ scan,
    const int32_t* __restrict__ tile_start, const int64_t* __restrict__ total_dev, int64_t nnz, int64_t nrows,
    int64_t col_base, uint32_t* __restrict__ spa, uint64_t* __restrict__ occ, const uint64_t* __restrict__ skip) {
    __shared__ int32_t s_start[TD_TILE + 1];
    __shared__ int64_t s_base[TD_TILE + 1];
    __shared__ uint32_t s_par[TD_TILE + 1];
    if (*skip) return;   // the sorted union already wrote the output
    const int64_t qlen = (int64_t)*qlen_dev;
    const int64_t total = *total_dev;
    const int64_t ntiles = (total + TD_TILE - 1) / TD_TILE;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t e0 = t * TD_TILE;
        const int64_t e1 = (e0 + TD_TILE < total) ? e0 + TD_TILE : total;
        const int i0 = tile_start[t];
        int nv = tile_start[t + 1] - i0 + 1;
        if (nv > TD_TILE + 1) nv = TD_TILE + 1;
        if (i0 < 0 || i0 >= qlen) nv = 0;
        else if (nv > qlen - i0) nv = (int)(qlen - i0);
        for (int j = threadIdx.x; j < nv; j += TD_BLOCK) {
            const int32_t h = q[i0 + j];
            const int64_t sc = scan[i0 + j];
            const int64_t rel = sc - e0;
            s_start[j] = rel < 0 ? 0 : (int32_t)rel;
            s_base[j] = cp[h] - sc;
            s_par[j] = (uint32_t)(col_base + jc[h]);
        }
        __syncthreads();
        int32_t rr[TD_EPT];
        uint32_t pp[TD_EPT];
#pragma unroll
        for (int k = 0; k < TD_EPT; ++k) {
            const int p = k * TD_BLOCK + threadIdx.x;
            const int64_t e = e0 + p;
            rr[k] = -1;
            pp[k] = 0;
            if (e < e1 && nv > 0) {
                int lo = 0, hi = nv - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_start[mid] <= p) lo = mid; else hi = mid - 1;
                }
                int64_t pos = s_base[lo] + e;
                if (pos < 0 || pos >= nnz) pos = 0;
                rr[k] = ir[pos];
                pp[k] = s_par[lo];
            }
        }
#pragma unroll
        for (int k = 0; k < TD_EPT; ++k) {
            const int32_t r = rr[k];
            if (r >= 0 && r < nrows) {
                // min over parents == max over complements; 0 stays "empty"
                atomicMax(&spa[r], ~pp[k]);
                atomicOr((unsigned long long*)&occ[r >> 6], 1ull << (r & 63));
            }
        }
        __syncthreads();
    }
}

struct WordPopc {
    const uint64_t* w;
    __device__ int64_t operator()(int64_t i) const { return __popcll(w[i]); }
};

// occupied words of the accumulator; none when the sorted union ran instead
struct OccPopc {
    const uint64_t* w;
    const uint64_t* skip;
    __device__ int64_t operator()(int64_t i) const { return *skip ? 0 : __popcll(w[i]); }
};

// emits the rows of occupied word i in ascending order and clears what it read
struct SpaEmit {
    uint64_t* occ;
    uint32_t* spa;
    int32_t* out_rows;
    int32_t* out_parents;
    int64_t* nout;
    const uint64_t* skip;
    __device__ void item(int64_t i, int64_t before, int64_t d) const {
        if (!d) return;
        uint64_t x = occ[i];
        int64_t pos = before;
        while (x) {
            const int b = __ffsll((unsigned long long)x) - 1;
            x &= x - 1;
            const int64_t r = i * 64 + b;
            out_rows[pos] = (int32_t)r;
            out_parents[pos] = (int32_t)~spa[r];
            spa[r] = 0;
            ++pos;
        }
        occ[i] = 0;
    }
    __device__ void last(int64_t, int64_t total) const {
        if (!*skip) *nout = total;
    }
};

// ---------------------------------------------------------------- sorted union
// Hypersparse frontiers (Section 5.2 weighs a sparse accumulator against a
// heap-based union of the frontier columns; for very few columns the
// accumulator's ordered pass over all nrows/64 occupied words dominates).
// One workgroup gathers the entries (r, col_base + k) of the frontier
// columns into LDS as 64-bit keys r << 32 | parent, sorts them (bitonic),
// and keeps the first key of every row: rows come out ascending, each with
// its smallest parent, the same pairs the accumulator gives.  When the
// columns hold more than SORT_CAP entries it writes nothing and leaves
// `skip` at 0, and the accumulator path that follows does the work.
constexpr int SORT_CAP = 8192;
constexpr int SORT_BLOCK = 1024;

__global__ __launch_bounds__(SORT_BLOCK) void k_blk_sorted_union(
    const int64_t* __restrict__ cp, const int32_t* __restrict__ jc, const int32_t* __restrict__ ir,
    const int32_t* __restrict__ q, const uint64_t* __restrict__ qlen_dev, const int64_t* __restrict__ scan,
    const int64_t* __restrict__ total_dev, int64_t col_base, int32_t* __restrict__ out_rows,
    int32_t* __restrict__ out_parents, int64_t* __restrict__ nout, uint64_t* __restrict__ skip) {
    __shared__ uint64_t key[SORT_CAP];
    __shared__ int32_t s_cnt[SORT_BLOCK];
    const int tid = threadIdx.x;
    const int64_t total = *total_dev;
    const int64_t qlen = (int64_t)*qlen_dev;
    if (total > SORT_CAP) return;   // skip stays 0: the accumulator runs
    int np = 2;
    while (np < total) np <<= 1;
    for (int e = tid; e < np; e += SORT_BLOCK) {
        uint64_t k = ~0ull;
        if (e < total) {
            // the queue entry owning edge e: last i with scan[i] <= e
            int64_t lo = 0, hi = qlen - 1;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (scan[mid] <= e) lo = mid; else hi = mid - 1;
            }
            const int32_t h = q[lo];
            const int32_t r = ir[cp[h] + (e - scan[lo])];
            k = ((uint64_t)(uint32_t)r << 32) | (uint32_t)(col_base + jc[h]);
        }
        key[e] = k;
    }
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < np / 2; t += SORT_BLOCK) {
                const int i = 2 * t - (t & (stride - 1));   // lower index of the pair
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const uint64_t a = key[i], b = key[j];
                if ((a > b) == up) { key[i] = b; key[j] = a; }
            }
            __syncthreads();
        }
    }
    // first key of every row, compacted in order: each thread takes a run of
    // consecutive keys, counts its row starts, and a block prefix places them
    const int per = (np + SORT_BLOCK - 1) / SORT_BLOCK;
    const int a0 = tid * per, a1 = min(a0 + per, (int)total);
    int c = 0;
    for (int i = a0; i < a1; ++i)
        if (i == 0 || (key[i] >> 32) != (key[i - 1] >> 32)) ++c;
    s_cnt[tid] = c;
    __syncthreads();
    for (int d = 1; d < SORT_BLOCK; d <<= 1) {
        const int x = tid >= d ? s_cnt[tid - d] : 0;
        __syncthreads();
        s_cnt[tid] += x;
        __syncthreads();
    }
    int pos = s_cnt[tid] - c;
    for (int i = a0; i < a1; ++i) {
        if (i == 0 || (key[i] >> 32) != (key[i - 1] >> 32)) {
            out_rows[pos] = (int32_t)(key[i] >> 32);
            out_parents[pos] = (int32_t)(uint32_t)key[i];
            ++pos;
        }
    }
    if (tid == SORT_BLOCK - 1) {
        *nout = s_cnt[SORT_BLOCK - 1];
        *skip = 1;
    }
}

// ---------------------------------------------------------------- bottom-up
// range[0] = first JR index with row >= row_lo, range[1] = first with row >=
// row_hi, range[2] = number of 64-entry chunks in between
__global__ void k_blk_range(const int32_t* __restrict__ jr, int64_t nzr, int64_t row_lo, int64_t row_hi,
                            uint64_t* __restrict__ range) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t bound[2];
    for (int k = 0; k < 2; ++k) {
        const int64_t key = k == 0 ? row_lo : row_hi;
        int64_t lo = 0, hi = nzr;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)jr[mid] < key) lo = mid + 1; else hi = mid;
        }
        bound[k] = lo;
    }
    range[0] = (uint64_t)bound[0];
    range[1] = (uint64_t)bound[1];
    range[2] = (uint64_t)((bound[1] - bound[0] + 63) / 64);
}

// COMP = 1: rows with their completed bit set are skipped and found rows set
// it (Alg. 4).  COMP = 0: every row is scanned and `completed` is unused (the
// pull form of the top-down step, see launch_block_td).
template <int COMP>
__global__ __launch_bounds__(BU_BLOCK) void k_blk_bu(
    const int32_t* __restrict__ jr, const int64_t* __restrict__ rp, const int32_t* __restrict__ ic,
    const uint64_t* __restrict__ range, const uint64_t* __restrict__ fbits, uint64_t* __restrict__ completed,
    int64_t col_base, int64_t ncols, int serial_len, int32_t* __restrict__ bpar, uint64_t* __restrict__ bmask) {
    const int lane = lane_id();
    const int64_t a = (int64_t)range[0], b = (int64_t)range[1];
    const int64_t nchunks = (int64_t)range[2];
    const int64_t nwaves = (int64_t)gridDim.x * (BU_BLOCK / WAVE);
    for (int64_t c = (int64_t)blockIdx.x * (BU_BLOCK / WAVE) + threadIdx.x / WAVE; c < nchunks; c += nwaves) {
        const int64_t t = a + c * WAVE + lane;
        bool active = t < b;
        int32_t r = 0;
        int64_t beg = 0, end = 0;
        if (active) {
            r = jr[t];
            if (COMP) active = !((completed[r >> 6] >> (r & 63)) & 1ull);
        }
        if (active) {
            beg = rp[t];
            end = rp[t + 1];
        }
        int64_t p = beg;
        const int64_t lim = (end - beg > serial_len) ? beg + serial_len : end;
        int32_t par = -1;
        while (p < lim) {
            const int32_t col = ic[p];
            if (col >= 0 && col < ncols && ((fbits[col >> 6] >> (col & 63)) & 1ull)) { par = col; break; }
            ++p;
        }
        uint64_t rem = __ballot(active && par < 0 && p < end);
        while (rem) {
            const int l = __ffsll((unsigned long long)rem) - 1;
            rem &= rem - 1;
            const int64_t pb = __shfl(p, l, WAVE);
            const int64_t pe = __shfl(end, l, WAVE);
            int32_t got = -1;
            for (int64_t x = pb; x < pe; x += WAVE) {
                const int64_t idx = x + lane;
                bool hit = false;
                int32_t col = 0;
                if (idx < pe) {
                    col = ic[idx];
                    hit = col >= 0 && col < ncols && ((fbits[col >> 6] >> (col & 63)) & 1ull);
                }
                const uint64_t hm = __ballot(hit);
                if (hm) {
                    got = __shfl(col, __ffsll((unsigned long long)hm) - 1, WAVE);
                    break;
                }
            }
            if (lane == l) par = got;
        }
        const bool found = par >= 0;
        const uint64_t fm = __ballot(found);
        if (lane == 0) bmask[c] = fm;
        if (found) {
            bpar[c * WAVE + lane] = (int32_t)(col_base + par);
            if (COMP) atomicOr((unsigned long long*)&completed[r >> 6], 1ull << (r & 63));
        }
    }
}

struct ChunkEmit {
    const uint64_t* bmask;
    const int32_t* bpar;
    const int32_t* jr;
    const uint64_t* range;
    int32_t* out_rows;
    int32_t* out_parents;
    int64_t* nout;
    __device__ void item(int64_t c, int64_t before, int64_t d) const {
        if (!d) return;
        const int64_t a = (int64_t)range[0];
        uint64_t x = bmask[c];
        int64_t pos = before;
        while (x) {
            const int k = __ffsll((unsigned long long)x) - 1;
            x &= x - 1;
            out_rows[pos] = jr[a + c * WAVE + k];
            out_parents[pos] = bpar[c * WAVE + k];
            ++pos;
        }
    }
    __device__ void last(int64_t, int64_t total) const { *nout = total; }
};

// Dense frontiers: when |F| binary searches would cost more than one pass
// over JC (|F| log2 nzc > nzc), F is marked in a column bitmap and JC is
// scanned once; the found JC indices come out of an ordered compaction.
__global__ void k_blk_mark(const int32_t* __restrict__ F, int64_t nf, uint64_t* __restrict__ fmark, int clear) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += stride) {
        const int32_t c = F[i];
        if (clear) fmark[c >> 6] = 0;
        else atomicOr((unsigned long long*)&fmark[c >> 6], 1ull << (c & 63));
    }
}

struct JcInFrontier {
    const int32_t* jc;
    const uint64_t* fmark;
    __device__ int64_t operator()(int64_t i) const {
        const int32_t c = jc[i];
        return (int64_t)((fmark[c >> 6] >> (c & 63)) & 1ull);
    }
};

struct JcIndexSink {
    int32_t* q;
    uint64_t* qlen;
    __device__ void item(int64_t i, int64_t before, int64_t d) const {
        if (d) q[before] = (int32_t)i;
    }
    __device__ void last(int64_t, int64_t total) const { *qlen = (uint64_t)total; }
};

// ---------------------------------------------------------------- launchers
void launch_block_td(const Launch& L, const BlockArgs& B, const int32_t* F, int64_t nf, int32_t* out_rows,
                     int32_t* out_parents, int64_t* nout, const BlockWs& W) {
    // A dense frontier (more than 1/32 of the columns): the same result from
    // the row side.  Each row's minimum frontier column is the first frontier
    // column of its ascending row, so a first-hit sweep of the row-compressed
    // copy against a bitmap of F gives the (row, parent) pairs in row order
    // with no accumulator and no atomics.
    if (B.jr && B.sorted && B.nzr > 0 && nf * 32 > B.ncols) {
        const int gm = grid_for(nf, 256, L.grid_cap);
        hipLaunchKernelGGL(k_blk_mark, dim3(gm), dim3(256), 0, L.stream, F, nf, W.fmark, 0);
        hipLaunchKernelGGL(k_blk_range, dim3(1), dim3(1), 0, L.stream, B.jr, B.nzr, (int64_t)0, B.nrows, W.range);
        const int64_t chunks_max = (B.nzr + WAVE - 1) / WAVE;
        hipLaunchKernelGGL(k_blk_bu<0>, dim3(grid_for(chunks_max, BU_BLOCK / WAVE, L.grid_cap)), dim3(BU_BLOCK), 0,
                           L.stream, B.jr, B.rp, B.ic, W.range, W.fmark, nullptr, B.col_base, B.ncols, 16, W.bpar,
                           W.bmask);
        launch_scan(L.stream, WordPopc{W.bmask}, W.range + 2, chunks_max, W.partial,
                    ChunkEmit{W.bmask, W.bpar, B.jr, W.range, out_rows, out_parents, nout});
        hipLaunchKernelGGL(k_blk_mark, dim3(gm), dim3(256), 0, L.stream, F, nf, W.fmark, 1);
        return;
    }
    const double lg = B.nzc > 1 ? std::log2((double)B.nzc) : 1.0;
    if (B.nzc > 0 && (double)nf * lg > (double)B.nzc) {
        const int gm = grid_for(nf, 256, L.grid_cap);
        hipLaunchKernelGGL(k_blk_mark, dim3(gm), dim3(256), 0, L.stream, F, nf, W.fmark, 0);
        launch_scan(L.stream, JcInFrontier{B.jc, W.fmark}, (const uint64_t*)nullptr, B.nzc, W.partial,
                    JcIndexSink{W.q, W.qlen});
        hipLaunchKernelGGL(k_blk_mark, dim3(gm), dim3(256), 0, L.stream, F, nf, W.fmark, 1);
    } else {
        hipLaunchKernelGGL(k_blk_find, dim3(grid_for(nf, 256, L.grid_cap)), dim3(256), 0, L.stream, B.jc, B.nzc, F,
                           nf, W.q, W.qlen);
    }
    const int64_t qmax = nf < B.nzc ? nf : B.nzc;
    launch_scan(L.stream, QueueDegree<int64_t>{B.cp, W.q}, W.qlen, qmax, W.partial,
                TileSink{W.scan, W.tiles, W.total});
    // the sorted union when asked for (bfs_block_set_union 1): it takes the
    // call unless the frontier's columns hold more than SORT_CAP entries
    // (then it leaves the skip word at 0 and the accumulator runs).  Not the
    // default: measured on one 2^27 x 2^27 block at |F| = 1342, the
    // accumulator's call took 0.042 ms and the sorted union's 0.078 ms, the
    // accumulator's ordered pass over nrows/64 words being only a few us
    const bool sorted_union = B.sort_union == 1;
    if (sorted_union)
        hipLaunchKernelGGL(k_blk_sorted_union, dim3(1), dim3(SORT_BLOCK), 0, L.stream, B.cp, B.jc, B.ir, W.q, W.qlen,
                           W.scan, W.total, B.col_base, out_rows, out_parents, nout, W.skip);
    const int64_t tiles_max = (B.nnz + TD_TILE - 1) / TD_TILE;
    hipLaunchKernelGGL(k_blk_expand, dim3(grid_for(tiles_max, 1, L.grid_cap)), dim3(TD_BLOCK), 0, L.stream, B.cp,
                       B.jc, B.ir, W.q, W.qlen, W.scan, W.tiles, W.total, B.nnz, B.nrows, B.col_base, W.spa,
                       W.occ, W.skip);
    const int64_t wr = (B.nrows + 63) / 64;
    launch_scan(L.stream, OccPopc{W.occ, W.skip}, (const uint64_t*)nullptr, wr, W.partial,
                SpaEmit{W.occ, W.spa, out_rows, out_parents, nout, W.skip});
}

void launch_block_bu(const Launch& L, const BlockArgs& B, const uint64_t* fbits, uint64_t* completed,
                     int64_t row_lo, int64_t row_hi, int serial_len, int32_t* out_rows, int32_t* out_parents,
                     int64_t* nout, const BlockWs& W) {
    hipLaunchKernelGGL(k_blk_range, dim3(1), dim3(1), 0, L.stream, B.jr, B.nzr, row_lo, row_hi, W.range);
    const int64_t chunks_max = (B.nzr + WAVE - 1) / WAVE;
    hipLaunchKernelGGL(k_blk_bu<1>, dim3(grid_for(chunks_max, BU_BLOCK / WAVE, L.grid_cap)), dim3(BU_BLOCK), 0,
                       L.stream, B.jr, B.rp, B.ic, W.range, fbits, completed, B.col_base, B.ncols, serial_len,
                       W.bpar, W.bmask);
    launch_scan(L.stream, WordPopc{W.bmask}, W.range + 2, chunks_max, W.partial,
                ChunkEmit{W.bmask, W.bpar, B.jr, W.range, out_rows, out_parents, nout});
}

// ---------------------------------------------------------------- validation
// one wave per non-empty major (column of the DCSC, row of the DCSR): ids of
// majors ascending and in range, pointers monotone, minors in range and
// (SORTED) ascending inside each major
__global__ __launch_bounds__(256) void k_validate_dcs(const int32_t* __restrict__ j, const int64_t* __restrict__ p,
                                                      const int32_t* __restrict__ minor, int64_t nz, int64_t nmajor,
                                                      int64_t nminor, int64_t nnz, uint32_t sorted,
                                                      uint32_t* __restrict__ err) {
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (256 / WAVE);
    uint32_t e = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && (p[0] != 0 || p[nz] != nnz)) e |= VE_OFFSETS;
    for (int64_t k = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE; k < nz; k += nwaves) {
        const int32_t id = j[k];
        if (id < 0 || id >= nmajor || (k > 0 && j[k - 1] >= id)) e |= VE_RANGE;
        const int64_t b = p[k], en = p[k + 1];
        if (b < 0 || en > nnz || en <= b) { e |= VE_OFFSETS; continue; }
        for (int64_t x = b + lane; x < en; x += WAVE) {
            const int32_t m = minor[x];
            if (m < 0 || m >= nminor) e |= VE_RANGE;
            if (sorted && x + 1 < en && minor[x + 1] < m) e |= VE_UNSORTED;
        }
    }
    if (e) atomicOr(err, e);
}

void launch_validate_dcs(const Launch& L, const int32_t* j, const int64_t* p, const int32_t* minor, int64_t nz,
                         int64_t nmajor, int64_t nminor, int64_t nnz, bool sorted, uint32_t* err) {
    hipLaunchKernelGGL(k_validate_dcs, dim3(grid_for(nz, 256 / WAVE, L.grid_cap)), dim3(256), 0, L.stream, j, p,
                       minor, nz, nmajor, nminor, nnz, (uint32_t)sorted, err);
}

}  // namespace bfsk
