// graphgen_gpu.hip -- the Kronecker 2D-block generator of graphgen.c, on the
// GPU: the same counter-based draws (SplitMix64 output function keyed by seed
// and draw index), the same seeded relabelling bijection and the same cleanup
// (self-loops dropped, both orientations of every draw, duplicates removed,
// entries sorted inside each column and each row).  It exists for blocks of
// graphs too large to enumerate on the host: one 8x8 block of a scale-30
// graph takes 1.7e10 draws.  Like graphgen.c it holds no search arithmetic.
//
// Output: the block's DCSC (jc, cp, ir) and DCSR (jr, rp, ic) forms in device
// memory owned by an opaque handle, copied out with ggg_block_copy.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <stdint.h>
#include <string.h>

namespace {

__host__ __device__ inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t rnd(uint64_t key, uint64_t i) { return sm64_mix(key + (i + 1) * 0x9e3779b97f4a7c15ULL); }
inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return sm64_mix(seed * 0x2545f4914f6cdd1dULL + stream * 0x9e3779b97f4a7c15ULL + 0x5851f42d4c957f2dULL);
}

struct Kron {
    int scale, permute;
    uint32_t tA, tAB, tABC;
    uint64_t key, mask, m[3], c[3];
    int r[3];
};

Kron kron_make(int scale, uint64_t seed, double a, double b, double c, int permute) {
    Kron k;
    memset(&k, 0, sizeof(k));
    k.scale = scale;
    k.permute = permute;
    k.tA = (uint32_t)(a * 4294967296.0);
    k.tAB = (uint32_t)((a + b) * 4294967296.0);
    k.tABC = (uint32_t)((a + b + c) * 4294967296.0);
    k.key = stream_key(seed, 1);
    k.mask = (scale >= 64) ? ~0ULL : ((1ULL << scale) - 1);
    const uint64_t pkey = stream_key(seed, 7);
    for (int j = 0; j < 3; ++j) {
        k.m[j] = (rnd(pkey, 2 * j) | 1ULL) & k.mask;
        if (k.m[j] == 0) k.m[j] = 1;
        k.c[j] = rnd(pkey, 2 * j + 1) & k.mask;
        const int r = scale / 2 + j - 1;
        k.r[j] = r < 1 ? 1 : r;
    }
    return k;
}

__device__ inline uint64_t perm_apply(const Kron& k, uint64_t x) {
    for (int j = 0; j < 3; ++j) {
        x = (x * k.m[j] + k.c[j]) & k.mask;
        x ^= (x >> k.r[j]);
    }
    return x;
}

__device__ inline void kron_draw(const Kron& k, uint64_t i, uint64_t* u, uint64_t* v) {
    uint64_t su = 0, sv = 0;
    const uint64_t base = i * (uint64_t)((k.scale + 1) / 2);
    for (int lvl = 0; lvl < k.scale; lvl += 2) {
        const uint64_t r = rnd(k.key, base + (uint64_t)(lvl / 2));
        for (int h = 0; h < 2 && lvl + h < k.scale; ++h) {
            const uint32_t x = (uint32_t)(h ? (r >> 32) : r);
            const uint64_t rb = (uint64_t)(x >= k.tAB);
            const uint64_t cb = (uint64_t)((x >= k.tA) & (x < k.tAB)) | (uint64_t)(x >= k.tABC);
            su |= rb << (lvl + h);
            sv |= cb << (lvl + h);
        }
    }
    if (k.permute) {
        su = perm_apply(k, su);
        sv = perm_apply(k, sv);
    }
    *u = su;
    *v = sv;
}

struct Box {
    int64_t r0, R, c0, C;
    __device__ bool in(uint64_t a, uint64_t b) const {
        return (int64_t)a >= r0 && (int64_t)a < r0 + R && (int64_t)b >= c0 && (int64_t)b < c0 + C;
    }
};

// pass 1: entries that fall in the block, both orientations of every non-loop draw
__global__ void k_count(Kron k, Box bx, uint64_t m, unsigned long long* total) {
    unsigned long long cnt = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        uint64_t u, v;
        kron_draw(k, i, &u, &v);
        if (u == v) continue;
        cnt += bx.in(u, v);
        cnt += bx.in(v, u);
    }
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(total, cnt);
}

// pass 2: the same entries as keys (column << 32 | row), block-local ids
__global__ void k_fill(Kron k, Box bx, uint64_t m, uint64_t* keys, unsigned long long* pos, uint64_t cap) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < m; i0 += stride) {
        const uint64_t i = i0 + threadIdx.x;
        uint64_t key0 = 0, key1 = 0;
        int nk = 0;
        if (i < m) {
            uint64_t u, v;
            kron_draw(k, i, &u, &v);
            if (u != v) {
                if (bx.in(u, v)) key0 = ((uint64_t)(v - bx.c0) << 32) | (uint64_t)(u - bx.r0), nk = 1;
                if (bx.in(v, u)) {
                    const uint64_t kk = ((uint64_t)(u - bx.c0) << 32) | (uint64_t)(v - bx.r0);
                    if (nk) key1 = kk; else key0 = kk;
                    ++nk;
                }
            }
        }
        // wave-wide append: exclusive prefix of nk
        int incl = nk;
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d, 64);
            if (lane >= d) incl += y;
        }
        const int tot = __shfl(incl, 63, 64);
        unsigned long long base = 0;
        if (lane == 63 && tot) base = atomicAdd(pos, (unsigned long long)tot);
        base = __shfl(base, 63, 64);
        const uint64_t p = base + (uint64_t)(incl - nk);
        if (nk > 0 && p < cap) keys[p] = key0;
        if (nk > 1 && p + 1 < cap) keys[p + 1] = key1;
    }
}

__global__ void k_split(const uint64_t* __restrict__ keys, int64_t n, int32_t* __restrict__ major,
                        int32_t* __restrict__ minor) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        major[e] = (int32_t)(keys[e] >> 32);
        minor[e] = (int32_t)(keys[e] & 0xffffffffULL);
    }
}

__global__ void k_swap_halves(const uint64_t* __restrict__ in, int64_t n, uint64_t* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        out[e] = (in[e] << 32) | (in[e] >> 32);
}

__global__ void k_last(int64_t* p, int64_t nz, int64_t nnz) { p[nz] = nnz; }

struct Block {
    int64_t nnz = 0, nzc = 0, nzr = 0;
    int32_t *jc = nullptr, *ir = nullptr, *jr = nullptr, *ic = nullptr;
    int64_t *cp = nullptr, *rp = nullptr;
};

#define CK(x)                              \
    do {                                   \
        if ((x) != hipSuccess) goto fail;  \
    } while (0)

// sorted unique keys (major << 32 | minor) -> compressed form (j, p, i)
int compress(const uint64_t* keys, int64_t nnz, int32_t** j_out, int64_t** p_out, int32_t** i_out, int64_t* nz_out,
             hipStream_t s) {
    int32_t *major = nullptr, *minor = nullptr, *uniq = nullptr, *cnt = nullptr;
    int64_t* d_nz = nullptr;
    int64_t* pp = nullptr;
    void* tmp = nullptr;
    size_t tb = 0, tb2 = 0;
    int64_t nz = 0;
    const int G = 4096;
    CK(hipMalloc(&major, sizeof(int32_t) * (nnz + 1)));
    CK(hipMalloc(&minor, sizeof(int32_t) * (nnz + 1)));
    CK(hipMalloc(&uniq, sizeof(int32_t) * (nnz + 1)));
    CK(hipMalloc(&cnt, sizeof(int32_t) * (nnz + 1)));
    CK(hipMalloc(&d_nz, sizeof(int64_t)));
    if (nnz > 0) hipLaunchKernelGGL(k_split, dim3(G), dim3(256), 0, s, keys, nnz, major, minor);
    CK(hipGetLastError());
    CK(hipcub::DeviceRunLengthEncode::Encode(nullptr, tb, major, uniq, cnt, d_nz, (int)nnz, s));
    CK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, cnt, (int64_t*)nullptr, (int)nnz, s));
    CK(hipMalloc(&tmp, tb > tb2 ? tb : tb2));
    CK(hipcub::DeviceRunLengthEncode::Encode(tmp, tb, major, uniq, cnt, d_nz, (int)nnz, s));
    CK(hipMemcpyAsync(&nz, d_nz, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    CK(hipMalloc(&pp, sizeof(int64_t) * (nz + 1)));
    if (nz > 0) CK(hipcub::DeviceScan::ExclusiveSum(tmp, tb2, cnt, pp, (int)nz, s));
    hipLaunchKernelGGL(k_last, dim3(1), dim3(1), 0, s, pp, nz, nnz);
    CK(hipGetLastError());
    CK(hipStreamSynchronize(s));
    (void)hipFree(major);
    (void)hipFree(cnt);
    (void)hipFree(tmp);
    (void)hipFree(d_nz);
    *j_out = uniq;
    *p_out = pp;
    *i_out = minor;
    *nz_out = nz;
    return 0;
fail:
    (void)hipFree(major); (void)hipFree(minor); (void)hipFree(uniq); (void)hipFree(cnt);
    (void)hipFree(d_nz); (void)hipFree(pp); (void)hipFree(tmp);
    return 3;
}

void block_free(Block* b) {
    if (!b) return;
    (void)hipFree(b->jc); (void)hipFree(b->ir); (void)hipFree(b->jr); (void)hipFree(b->ic);
    (void)hipFree(b->cp); (void)hipFree(b->rp);
    delete b;
}

}  // namespace

extern "C" {

// Block A[r0:r0+R, c0:c0+C] of the Kronecker graph (scale, edgefactor, seed,
// initiator a,b,c, relabelled when permute != 0), built on the current device.
// Returns 0 and a handle, 1 for bad arguments, 2 when the raw entry count
// exceeds 2^31-1 (the sort's index type), 3 for a HIP error.
int ggg_kron_block(int scale, int64_t edgefactor, uint64_t seed, double a, double b, double c, int permute,
                   int64_t r0, int64_t R, int64_t c0, int64_t C, void** handle, int64_t* nnz, int64_t* nzc,
                   int64_t* nzr) {
    if (!handle || scale < 1 || scale > 40) return 1;
    *handle = nullptr;
    const int64_t n = (int64_t)1 << scale;
    if (r0 < 0 || c0 < 0 || R < 1 || C < 1 || r0 + R > n || c0 + C > n || R > 2147483647LL || C > 2147483647LL)
        return 1;
    const Kron k = kron_make(scale, seed, a, b, c, permute);
    const Box bx{r0, R, c0, C};
    const uint64_t m = (uint64_t)edgefactor << scale;
    hipStream_t s = nullptr;
    unsigned long long* d_ctr = nullptr;
    unsigned long long raw = 0;
    uint64_t *keys = nullptr, *sorted = nullptr, *uniq = nullptr, *swapped = nullptr;
    int64_t* d_nu = nullptr;
    int64_t nu = 0;
    void* tmp = nullptr;
    size_t tb = 0, tb2 = 0;
    Block* blk = nullptr;
    const int G = 8192;
    CK(hipStreamCreate(&s));
    CK(hipMalloc(&d_ctr, 2 * sizeof(unsigned long long)));
    CK(hipMemsetAsync(d_ctr, 0, 2 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_count, dim3(G), dim3(256), 0, s, k, bx, m, d_ctr);
    CK(hipGetLastError());
    CK(hipMemcpyAsync(&raw, d_ctr, sizeof(raw), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (raw > 2147483647ULL) {
        (void)hipFree(d_ctr);
        (void)hipStreamDestroy(s);
        return 2;
    }
    CK(hipMalloc(&keys, sizeof(uint64_t) * (raw + 1)));
    CK(hipMalloc(&sorted, sizeof(uint64_t) * (raw + 1)));
    hipLaunchKernelGGL(k_fill, dim3(G), dim3(256), 0, s, k, bx, m, keys, d_ctr + 1, (uint64_t)raw);
    CK(hipGetLastError());
    // sort, drop duplicates: column-major keys
    CK(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, keys, sorted, (int)raw, 0, 64, s));
    CK(hipMalloc(&d_nu, sizeof(int64_t)));
    CK(hipcub::DeviceSelect::Unique(nullptr, tb2, sorted, keys, d_nu, (int)raw, s));
    CK(hipMalloc(&tmp, tb > tb2 ? tb : tb2));
    CK(hipcub::DeviceRadixSort::SortKeys(tmp, tb, keys, sorted, (int)raw, 0, 64, s));
    CK(hipcub::DeviceSelect::Unique(tmp, tb2, sorted, keys, d_nu, (int)raw, s));
    CK(hipMemcpyAsync(&nu, d_nu, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    uniq = keys;
    blk = new Block();
    blk->nnz = nu;
    if (compress(uniq, nu, &blk->jc, &blk->cp, &blk->ir, &blk->nzc, s)) goto fail;
    // row-major keys: swap halves, sort again
    swapped = sorted;
    hipLaunchKernelGGL(k_swap_halves, dim3(G), dim3(256), 0, s, uniq, nu, swapped);
    CK(hipGetLastError());
    CK(hipcub::DeviceRadixSort::SortKeys(tmp, tb, swapped, uniq, (int)nu, 0, 64, s));
    if (compress(uniq, nu, &blk->jr, &blk->rp, &blk->ic, &blk->nzr, s)) goto fail;
    CK(hipStreamSynchronize(s));
    (void)hipFree(keys); (void)hipFree(sorted); (void)hipFree(tmp); (void)hipFree(d_nu); (void)hipFree(d_ctr);
    (void)hipStreamDestroy(s);
    *handle = blk;
    *nnz = blk->nnz;
    *nzc = blk->nzc;
    *nzr = blk->nzr;
    return 0;
fail:
    (void)hipFree(keys); (void)hipFree(sorted); (void)hipFree(tmp); (void)hipFree(d_nu); (void)hipFree(d_ctr);
    block_free(blk);
    if (s) (void)hipStreamDestroy(s);
    return 3;
}

// copy the block into caller-owned device arrays (sizes from ggg_kron_block)
int ggg_block_copy(void* handle, int32_t* jc, int64_t* cp, int32_t* ir, int32_t* jr, int64_t* rp, int32_t* ic) {
    Block* b = (Block*)handle;
    if (!b) return 1;
    if (hipMemcpy(jc, b->jc, sizeof(int32_t) * b->nzc, hipMemcpyDeviceToDevice) != hipSuccess) return 3;
    if (hipMemcpy(cp, b->cp, sizeof(int64_t) * (b->nzc + 1), hipMemcpyDeviceToDevice) != hipSuccess) return 3;
    if (hipMemcpy(ir, b->ir, sizeof(int32_t) * b->nnz, hipMemcpyDeviceToDevice) != hipSuccess) return 3;
    if (hipMemcpy(jr, b->jr, sizeof(int32_t) * b->nzr, hipMemcpyDeviceToDevice) != hipSuccess) return 3;
    if (hipMemcpy(rp, b->rp, sizeof(int64_t) * (b->nzr + 1), hipMemcpyDeviceToDevice) != hipSuccess) return 3;
    if (hipMemcpy(ic, b->ic, sizeof(int32_t) * b->nnz, hipMemcpyDeviceToDevice) != hipSuccess) return 3;
    return 0;
}

void ggg_block_free(void* handle) { block_free((Block*)handle); }

}  // extern "C"
