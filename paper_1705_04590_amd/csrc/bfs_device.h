// Device helpers shared by the libbfs kernels (gfx950, wave64): wave and
// workgroup reductions, and a three-phase device-wide exclusive scan whose
// value source and per-item action are functors.
#pragma once
#include "bfs_internal.h"

namespace bfsk {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, WAVE);
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    for (int d = 1; d < WAVE; d <<= 1) {
        T y = __shfl_up(x, d, WAVE);
        if (lane_id() >= d) x += y;
    }
    return x;
}

// this workgroup's line of a counter slot
__device__ __forceinline__ uint64_t* slot_line(uint64_t* slot) {
    return slot + (blockIdx.x % SLOT_SPREAD) * SLOT_LINE;
}

// workgroup 0 clears a whole counter slot
__device__ __forceinline__ void zero_slot(uint64_t* zslot) {
    if (blockIdx.x == 0 && zslot)
        for (int i = threadIdx.x; i < SLOT_WORDS; i += blockDim.x) zslot[i] = 0;
}

// Sum of (a, b, c) over the workgroup, added once to three counters.
template <int NWAVES>
__device__ __forceinline__ void block_add3(uint64_t a, uint64_t b, uint64_t c, uint64_t* ca, uint64_t* cb,
                                           uint64_t* cc) {
    __shared__ uint64_t red[3][NWAVES];
    a = wave_sum(a); b = wave_sum(b); c = wave_sum(c);
    int wid = threadIdx.x / WAVE;
    if (lane_id() == 0) { red[0][wid] = a; red[1][wid] = b; red[2][wid] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t x = 0, y = 0, z = 0;
        for (int i = 0; i < NWAVES; ++i) { x += red[0][i]; y += red[1][i]; z += red[2][i]; }
        if (x && ca) atomicAdd((unsigned long long*)ca, (unsigned long long)x);
        if (y && cb) atomicAdd((unsigned long long*)cb, (unsigned long long)y);
        if (z && cc) atomicAdd((unsigned long long*)cc, (unsigned long long)z);
    }
}

static inline int grid_for(int64_t items, int per_block, int cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

__device__ __forceinline__ int64_t len_of(const uint64_t* len_dev, int64_t len_host) {
    return len_dev ? (int64_t)*len_dev : len_host;
}

// ---------------------------------------------------------------- generic scan
// Value functor V: `int64_t operator()(int64_t i) const`, i < len.
// Sink functor S: `void item(int64_t i, int64_t before, int64_t value) const`
// for every item, and `void last(int64_t len, int64_t total) const` once.
// The length comes from len_dev when it is not NULL (len_host is then an
// upper bound that sizes the grid).

template <typename V>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_partials_g(V val, const uint64_t* __restrict__ len_dev,
                                                                 int64_t len_host, int64_t* __restrict__ partial) {
    __shared__ int64_t red[SCAN_BLOCK / WAVE];
    const int64_t len = len_of(len_dev, len_host);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int64_t s = 0;
    for (int k = 0; k < SCAN_IPT; ++k)
        if (base + k < len) s += val(base + k);
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int i = 0; i < SCAN_BLOCK / WAVE; ++i) t += red[i];
        partial[blockIdx.x] = t;
    }
}

// exclusive scan of partial[0..nb) in place; partial[nb] receives the total
template <int UNUSED = 0>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_top_g(int64_t* __restrict__ partial, int64_t nb) {
    __shared__ int64_t wsum[SCAN_BLOCK / WAVE];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += SCAN_BLOCK) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t x = i < nb ? partial[i] : 0;
        const int64_t inc = wave_incl_scan(x);
        const int wid = threadIdx.x / WAVE;
        if (lane_id() == WAVE - 1) wsum[wid] = inc;
        __syncthreads();
        if (wid == 0) {
            int64_t t = lane_id() < SCAN_BLOCK / WAVE ? wsum[lane_id()] : 0;
            t = wave_incl_scan(t);
            if (lane_id() < SCAN_BLOCK / WAVE) wsum[lane_id()] = t;
        }
        __syncthreads();
        const int64_t before = (wid ? wsum[wid - 1] : 0) + carry;
        if (i < nb) partial[i] = before + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) carry += wsum[SCAN_BLOCK / WAVE - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[nb] = carry;
}

template <typename V, typename S>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply_g(V val, const uint64_t* __restrict__ len_dev,
                                                              int64_t len_host, const int64_t* __restrict__ partial,
                                                              int64_t nb, S sink) {
    __shared__ int64_t wsum[SCAN_BLOCK / WAVE];
    const int64_t len = len_of(len_dev, len_host);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int64_t d[SCAN_IPT];
    int64_t s = 0;
    for (int k = 0; k < SCAN_IPT; ++k) {
        d[k] = (base + k < len) ? val(base + k) : 0;
        s += d[k];
    }
    const int64_t inc = wave_incl_scan(s);
    const int wid = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) wsum[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int64_t t = lane_id() < SCAN_BLOCK / WAVE ? wsum[lane_id()] : 0;
        t = wave_incl_scan(t);
        if (lane_id() < SCAN_BLOCK / WAVE) wsum[lane_id()] = t;
    }
    __syncthreads();
    const int64_t block_off = (nb > 1) ? partial[blockIdx.x] : 0;
    int64_t run = block_off + (wid ? wsum[wid - 1] : 0) + inc - s;
    for (int k = 0; k < SCAN_IPT; ++k) {
        const int64_t i = base + k;
        if (i >= len) break;
        sink.item(i, run, d[k]);
        run += d[k];
    }
    if (len > 0 && base <= len - 1 && len - 1 < base + SCAN_IPT) {
        // the thread holding the last item knows the grand total
        sink.last(len, run);
    } else if (len == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        sink.last(0, 0);
    }
}

// Launches the scan; returns the number of kernels launched.  partial needs
// ceil(len_host / SCAN_TILE) + 2 int64.
template <typename V, typename S>
int launch_scan(hipStream_t stream, V val, const uint64_t* len_dev, int64_t len_host, int64_t* partial, S sink) {
    const int64_t nb = (len_host + SCAN_TILE - 1) / SCAN_TILE;
    int launches = 1;
    if (nb > 1) {
        hipLaunchKernelGGL((k_scan_partials_g<V>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, stream, val, len_dev,
                           len_host, partial);
        hipLaunchKernelGGL((k_scan_top_g<0>), dim3(1), dim3(SCAN_BLOCK), 0, stream, partial, nb);
        launches += 2;
    }
    hipLaunchKernelGGL((k_scan_apply_g<V, S>), dim3((unsigned)(nb > 0 ? nb : 1)), dim3(SCAN_BLOCK), 0, stream, val,
                       len_dev, len_host, partial, nb, sink);
    return launches;
}

// ---------------------------------------------------------------- scan pieces
// degree of queue entry i in a compressed structure with pointers `off`
template <typename OffT>
struct QueueDegree {
    const OffT* off;
    const int32_t* q;
    __device__ int64_t operator()(int64_t i) const {
        const int32_t u = q[i];
        return (int64_t)off[u + 1] - (int64_t)off[u];
    }
};

// scan[i] = edges before queue entry i; tile_start[t] = queue index owning
// edge t*TD_TILE; tile_start[ntiles] = len-1; scan[len] = *total_out = total.
struct TileSink {
    int64_t* scan;
    int32_t* tile_start;
    int64_t* total_out;   // may be NULL
    __device__ void item(int64_t i, int64_t before, int64_t d) const {
        scan[i] = before;
        if (d > 0) {
            const int64_t t0 = (before + TD_TILE - 1) / TD_TILE;
            const int64_t t1 = (before + d - 1) / TD_TILE;
            for (int64_t t = t0; t <= t1; ++t) tile_start[t] = (int32_t)i;
        }
    }
    __device__ void last(int64_t len, int64_t total) const {
        scan[len] = total;
        tile_start[(total + TD_TILE - 1) / TD_TILE] = (int32_t)(len - 1);
        if (total_out) *total_out = total;
    }
};

// ---------------------------------------------------------------- persistent kernels
// Residency check and grid barrier of the persistent engines (see
// bfs_persist.hip): every workgroup of the grid must be resident at once.
constexpr uint32_t ROLL_POISON = 1u << 30;

template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Roll call: true when all G workgroups arrived before the deadline (then all
// of them see true), false when the count was poisoned (then all see false).
__device__ __forceinline__ bool roll_call(PersistCtl* ctl, uint32_t G, long long ticks) {
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        const uint32_t old = atomicAdd(&ctl->roll, 1u);
        int ok = -1;
        if (old & ROLL_POISON) ok = 0;
        const long long t0 = wall_clock64();
        while (ok < 0) {
            const uint32_t c = ld_dev(&ctl->roll);
            if (c & ROLL_POISON) { ok = 0; break; }
            if (c >= G) { ok = 1; break; }
            if (wall_clock64() - t0 > ticks) {
                // poison only a count that is still short; if the last
                // workgroup arrived meanwhile the exchange fails and the
                // next read sees G
                if (atomicCAS(&ctl->roll, c, c | ROLL_POISON) == c) ok = 0;
            } else {
                __builtin_amdgcn_s_sleep(2);
            }
        }
        s_ok = ok;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return s_ok == 1;
}

// Grid barrier number `k` (0, 1, 2, ...): false on timeout (error flag set).
// Every wave first waits for its own memory operations to complete (the
// workgroup barrier alone does not wait for global stores and atomics whose
// results are unused), so thread 0's release covers the whole workgroup.
__device__ __forceinline__ bool grid_sync(PersistCtl* ctl, uint32_t G, uint32_t k, long long ticks) {
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (G == 1) return true;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        atomicAdd(&ctl->bar, 1u);
        const uint32_t target = G * (k + 1);
        const long long t0 = wall_clock64();
        int ok = 1;
        while (ld_dev(&ctl->bar) < target) {
            if (ld_dev(&ctl->err) || wall_clock64() - t0 > ticks) {
                atomicOr(&ctl->err, 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        s_ok = ok;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return s_ok != 0;
}

}  // namespace bfsk
