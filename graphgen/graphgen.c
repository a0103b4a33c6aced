/*
 * graphgen.c -- seeded synthetic graph generators and CSR/DCSC builders.
 *
 * This module produces the INPUTS that both the GPU library and the CPU
 * oracle consume.  It holds none of the search's arithmetic: no frontier,
 * no parent, no depth, no level.  It only draws edges, relabels vertices,
 * and lays the cleaned edge set out as sorted adjacency arrays.
 *
 * Workloads (the paper's section on data sets):
 *   - R-MAT / Kronecker graphs with initiator (a,b,c,d) = (.57,.19,.19,.05)
 *     and edgefactor 16, 2^scale vertices.  Each of the ef*2^scale draws picks
 *     one quadrant per bit level; no noise is added.
 *   - Erdos-Renyi G(n, M): M uniform endpoint pairs.
 *   - 2D grids with 4-neighbour connectivity, row-major ids.
 * Cleanup for all of them: self-loops dropped, edges symmetrised, duplicate
 * entries removed, every adjacency row sorted ascending.
 *
 * Randomness is counter based: value i of stream `key` is
 * splitmix64_mix(key + (i+1) * 0x9e3779b97f4a7c15), the output function of
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).  Every draw is a pure
 * function of (seed, index), so the output is independent of thread count.
 *
 * Vertex relabelling for Kronecker graphs is a seeded bijection on
 * scale-bit integers built from invertible steps (odd multiply mod 2^scale,
 * add, xor-shift right), three rounds.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GG_OK 0
#define GG_E_ARG 1
#define GG_E_NOMEM 2

/* ---------------------------------------------------------------- RNG */
static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static inline uint64_t rnd(uint64_t key, uint64_t i) {
    return sm64_mix(key + (i + 1) * 0x9e3779b97f4a7c15ULL);
}
/* independent stream keys derived from the user seed */
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return sm64_mix(seed * 0x2545f4914f6cdd1dULL + stream * 0x9e3779b97f4a7c15ULL + 0x5851f42d4c957f2dULL);
}

uint64_t gg_rand64(uint64_t seed, uint64_t stream, uint64_t i) {
    return rnd(stream_key(seed, stream), i);
}

/* ---------------------------------------------------------------- relabel */
typedef struct { uint64_t mask, m[3], c[3]; int r[3]; } perm_t;

static perm_t perm_make(int scale, uint64_t seed) {
    perm_t p;
    p.mask = (scale >= 64) ? ~0ULL : ((1ULL << scale) - 1);
    uint64_t key = stream_key(seed, 7);
    for (int k = 0; k < 3; ++k) {
        p.m[k] = (rnd(key, 2 * k) | 1ULL) & p.mask;
        if (p.m[k] == 0) p.m[k] = 1;
        p.c[k] = rnd(key, 2 * k + 1) & p.mask;
        int r = scale / 2 + (int)k - 1;
        p.r[k] = r < 1 ? 1 : r;
    }
    return p;
}
static inline uint64_t perm_apply(const perm_t* p, uint64_t x) {
    for (int k = 0; k < 3; ++k) {
        x = (x * p->m[k] + p->c[k]) & p->mask;
        x ^= (x >> p->r[k]);
    }
    return x;
}

uint64_t gg_kron_relabel(int scale, uint64_t seed, uint64_t x) {
    perm_t p = perm_make(scale, seed);
    return perm_apply(&p, x);
}

/* ---------------------------------------------------------------- Kronecker draw */
typedef struct {
    int scale;
    uint32_t tA, tAB, tABC;
    uint64_t key;
    int permute;
    perm_t perm;
} kron_t;

static kron_t kron_make(int scale, uint64_t seed, double a, double b, double c, int permute) {
    kron_t k;
    k.scale = scale;
    k.tA = (uint32_t)(a * 4294967296.0);
    k.tAB = (uint32_t)((a + b) * 4294967296.0);
    k.tABC = (uint32_t)((a + b + c) * 4294967296.0);
    k.key = stream_key(seed, 1);
    k.permute = permute;
    k.perm = perm_make(scale, seed);
    return k;
}

/* draw i -> (u, v): one quadrant per bit level, two levels per 64-bit word */
static inline void kron_draw(const kron_t* k, uint64_t i, uint64_t* u, uint64_t* v) {
    uint64_t su = 0, sv = 0;
    uint64_t base = i * (uint64_t)((k->scale + 1) / 2);
    for (int lvl = 0; lvl < k->scale; lvl += 2) {
        uint64_t r = rnd(k->key, base + (uint64_t)(lvl / 2));
        for (int h = 0; h < 2 && lvl + h < k->scale; ++h) {
            uint32_t x = (uint32_t)(h ? (r >> 32) : r);
            /* quadrant: [0,tA) -> (0,0), [tA,tAB) -> (0,1), [tAB,tABC) -> (1,0), else (1,1) */
            uint64_t rb = (uint64_t)(x >= k->tAB);
            uint64_t cb = (uint64_t)((x >= k->tA) & (x < k->tAB)) | (uint64_t)(x >= k->tABC);
            su |= rb << (lvl + h);
            sv |= cb << (lvl + h);
        }
    }
    if (k->permute) {
        su = perm_apply(&k->perm, su);
        sv = perm_apply(&k->perm, sv);
    }
    *u = su; *v = sv;
}

/* raw draws [start, start+count) -- for tests that start from the edge list */
int gg_kron_edges(int scale, int64_t edgefactor, uint64_t seed, double a, double b, double c,
                  int permute, int64_t start, int64_t count, int64_t* src, int64_t* dst) {
    if (scale < 1 || scale > 40 || count < 0 || start < 0) return GG_E_ARG;
    kron_t k = kron_make(scale, seed, a, b, c, permute);
    (void)edgefactor;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        uint64_t u, v;
        kron_draw(&k, (uint64_t)(start + i), &u, &v);
        src[i] = (int64_t)u; dst[i] = (int64_t)v;
    }
    return GG_OK;
}

/* ---------------------------------------------------------------- generic builder */
/* An edge source yields undirected draws (u, v); the builder drops u == v,
 * inserts both (u,v) and (v,u), sorts each row and removes duplicates.     */
typedef struct {
    int kind;               /* 0 kron, 1 er, 2 explicit list */
    int64_t m;              /* number of draws */
    kron_t kron;
    uint64_t er_key; int64_t er_n;
    const int64_t* es; const int64_t* ed;
    const int32_t* es32; const int32_t* ed32;
    int symmetrize;
    int keep_loops;         /* block compression: row and column spaces differ */
} esrc_t;

static inline void esrc_get(const esrc_t* s, int64_t i, uint64_t* u, uint64_t* v) {
    if (s->kind == 0) { kron_draw(&s->kron, (uint64_t)i, u, v); return; }
    if (s->kind == 1) {
        uint64_t r0 = rnd(s->er_key, 2 * (uint64_t)i), r1 = rnd(s->er_key, 2 * (uint64_t)i + 1);
        *u = (uint64_t)(((unsigned __int128)r0 * (uint64_t)s->er_n) >> 64);
        *v = (uint64_t)(((unsigned __int128)r1 * (uint64_t)s->er_n) >> 64);
        return;
    }
    if (s->kind == 3) { *u = (uint64_t)(uint32_t)s->es32[i]; *v = (uint64_t)(uint32_t)s->ed32[i]; return; }
    *u = (uint64_t)s->es[i]; *v = (uint64_t)s->ed[i];
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static void sort_i32(int32_t* a, int64_t len) {
    if (len < 2) return;
    if (len <= 32) {   /* insertion sort for the common short row */
        for (int64_t i = 1; i < len; ++i) {
            int32_t x = a[i]; int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
            a[j + 1] = x;
        }
        return;
    }
    qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
}

/* exclusive prefix sum of cnt[0..n) into off[0..n], parallel in blocks */
static void prefix_sum(int64_t n, const int64_t* cnt, int64_t* off) {
    int nt = omp_get_max_threads();
    int64_t* part = (int64_t*)calloc((size_t)nt + 1, sizeof(int64_t));
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num(), T = omp_get_num_threads();
        int64_t lo = n * t / T, hi = n * (t + 1) / T, s = 0;
        for (int64_t i = lo; i < hi; ++i) s += cnt[i];
        part[t + 1] = s;
#pragma omp barrier
#pragma omp single
        for (int k = 1; k <= T; ++k) part[k] += part[k - 1];
        s = part[t];
        for (int64_t i = lo; i < hi; ++i) { off[i] = s; s += cnt[i]; }
        if (t == T - 1) off[n] = s;
    }
    free(part);
}

/* Bucketed CSR build without shared counters (Kronecker hubs would make a
 * per-vertex atomic count contend).  Entries are packed as (row<<32 | col).
 *   1. every thread counts its draws per row bucket (2^shift rows each)
 *   2. draws are regenerated and scattered into their bucket's range
 *   3. each bucket is counting-sorted by row; every row is sorted and
 *      deduplicated; rows are then copied into the final cols array.      */
static int build_csr(const esrc_t* s, int64_t n, int64_t** off_out, int32_t** cols_out, int64_t* nnz_out) {
    int shift = 0;
    while (shift < 40 && (((int64_t)1 << shift) < n)) ++shift;   /* 2^shift >= n */
    int bshift = shift > 16 ? shift - 16 : 0;                        /* <= 65536 rows per bucket */
    int rshift = shift - bshift;                                     /* bucket = row >> rshift */
    int64_t B = (int64_t)1 << bshift;
    int64_t rows_per_b = (int64_t)1 << rshift;
    int T = omp_get_max_threads();
    int64_t* bc = (int64_t*)calloc((size_t)(B * T + 1), sizeof(int64_t));
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!bc || !deg) { free(bc); free(deg); return GG_E_NOMEM; }
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int64_t lo = s->m * t / T, hi = s->m * (t + 1) / T;
        int64_t* my = bc + (int64_t)t * B;
        for (int64_t i = lo; i < hi; ++i) {
            uint64_t u, v; esrc_get(s, i, &u, &v);
            if (u == v && !s->keep_loops) continue;
            my[u >> rshift]++;
            if (s->symmetrize) my[v >> rshift]++;
        }
    }
    /* positions ordered by (bucket, thread) so each bucket is contiguous */
    int64_t* bstart = (int64_t*)malloc(((size_t)B + 1) * sizeof(int64_t));
    int64_t* pos = (int64_t*)malloc((size_t)(B * T) * sizeof(int64_t));
    if (!bstart || !pos) { free(bc); free(deg); free(bstart); free(pos); return GG_E_NOMEM; }
    int64_t run = 0;
    for (int64_t b = 0; b < B; ++b) {
        bstart[b] = run;
        for (int t = 0; t < T; ++t) { pos[(int64_t)t * B + b] = run; run += bc[(int64_t)t * B + b]; }
    }
    bstart[B] = run;
    int64_t total = run;
    uint64_t* ent = (uint64_t*)malloc(((size_t)total + 1) * sizeof(uint64_t));
    if (!ent) { free(bc); free(deg); free(bstart); free(pos); return GG_E_NOMEM; }
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int64_t lo = s->m * t / T, hi = s->m * (t + 1) / T;
        int64_t* my = pos + (int64_t)t * B;
        for (int64_t i = lo; i < hi; ++i) {
            uint64_t u, v; esrc_get(s, i, &u, &v);
            if (u == v && !s->keep_loops) continue;
            ent[my[u >> rshift]++] = (u << 32) | v;
            if (s->symmetrize) ent[my[v >> rshift]++] = (v << 32) | u;
        }
    }
    free(pos); free(bc);
    /* per bucket: counting sort by row into int32 cols stored over the
     * bucket's own entry range (reinterpreted), then sort + dedup rows.   */
#pragma omp parallel num_threads(T)
    {
        int64_t* rc = (int64_t*)malloc(((size_t)rows_per_b + 1) * sizeof(int64_t));
        int64_t* rp = (int64_t*)malloc(((size_t)rows_per_b + 1) * sizeof(int64_t));
        int32_t* tmp = NULL; int64_t tmpcap = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t b = 0; b < B; ++b) {
            int64_t e0 = bstart[b], e1 = bstart[b + 1], len = e1 - e0;
            int64_t r0 = b << rshift;
            int64_t nr = rows_per_b;
            if (r0 >= n) continue;
            if (r0 + nr > n) nr = n - r0;
            if (len > tmpcap) { free(tmp); tmpcap = len; tmp = (int32_t*)malloc((size_t)tmpcap * sizeof(int32_t)); }
            memset(rc, 0, ((size_t)nr + 1) * sizeof(int64_t));
            for (int64_t e = e0; e < e1; ++e) rc[(int64_t)(ent[e] >> 32) - r0]++;
            int64_t acc = 0;
            for (int64_t r = 0; r < nr; ++r) { rp[r] = acc; acc += rc[r]; }
            rp[nr] = acc;
            for (int64_t r = 0; r < nr; ++r) rc[r] = rp[r];
            for (int64_t e = e0; e < e1; ++e) {
                int64_t r = (int64_t)(ent[e] >> 32) - r0;
                tmp[rc[r]++] = (int32_t)(ent[e] & 0xffffffffULL);
            }
            /* rows sorted + deduplicated, written back compacted as int32
             * into the start of this bucket's (8-byte) entry range          */
            int32_t* outc = (int32_t*)(ent + e0);
            int64_t w = 0;
            for (int64_t r = 0; r < nr; ++r) {
                int32_t* a = tmp + rp[r];
                int64_t l = rp[r + 1] - rp[r];
                sort_i32(a, l);
                int64_t w0 = w;
                for (int64_t j = 0; j < l; ++j)
                    if (w == w0 || a[j] != outc[w - 1]) outc[w++] = a[j];
                deg[r0 + r] = w - w0;
            }
        }
        free(rc); free(rp); free(tmp);
    }
    int64_t* off = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!off) { free(deg); free(bstart); free(ent); return GG_E_NOMEM; }
    prefix_sum(n, deg, off);
    int64_t nnz = off[n];
    int32_t* cols = (int32_t*)malloc(((size_t)nnz + 1) * sizeof(int32_t));
    if (!cols) { free(deg); free(bstart); free(ent); free(off); return GG_E_NOMEM; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < B; ++b) {
        int64_t r0 = b << rshift;
        if (r0 >= n) continue;
        int64_t r1 = r0 + rows_per_b < n ? r0 + rows_per_b : n;
        memcpy(cols + off[r0], (int32_t*)(ent + bstart[b]), (size_t)(off[r1] - off[r0]) * sizeof(int32_t));
    }
    free(deg); free(bstart); free(ent);
    *off_out = off; *cols_out = cols; *nnz_out = nnz;
    return GG_OK;
}

void gg_free(void* p) { free(p); }

int gg_kronecker_csr(int scale, int64_t edgefactor, uint64_t seed, double a, double b, double c,
                     int permute, int64_t* n_out, int64_t* nnz_out, int64_t** off_out, int32_t** cols_out) {
    if (scale < 1 || scale > 31 || edgefactor < 0) return GG_E_ARG;
    esrc_t s; memset(&s, 0, sizeof(s));
    s.kind = 0; s.m = edgefactor << scale; s.symmetrize = 1;
    s.kron = kron_make(scale, seed, a, b, c, permute);
    int64_t n = (int64_t)1 << scale;
    *n_out = n;
    return build_csr(&s, n, off_out, cols_out, nnz_out);
}

int gg_er_csr(int64_t n, int64_t m_draws, uint64_t seed, int64_t* nnz_out,
              int64_t** off_out, int32_t** cols_out) {
    if (n < 1 || n > 2147483647LL || m_draws < 0) return GG_E_ARG;
    esrc_t s; memset(&s, 0, sizeof(s));
    s.kind = 1; s.m = m_draws; s.symmetrize = 1;
    s.er_key = stream_key(seed, 2); s.er_n = n;
    return build_csr(&s, n, off_out, cols_out, nnz_out);
}

int gg_edges_csr(int64_t n, int64_t m, const int64_t* src, const int64_t* dst, int symmetrize,
                 int64_t* nnz_out, int64_t** off_out, int32_t** cols_out) {
    if (n < 0 || n > 2147483647LL || m < 0) return GG_E_ARG;
    for (int64_t i = 0; i < m; ++i)
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return GG_E_ARG;
    esrc_t s; memset(&s, 0, sizeof(s));
    s.kind = 2; s.m = m; s.es = src; s.ed = dst; s.symmetrize = symmetrize;
    return build_csr(&s, n, off_out, cols_out, nnz_out);
}

int gg_grid2d_csr(int64_t H, int64_t W, int64_t* nnz_out, int64_t** off_out, int32_t** cols_out) {
    if (H < 1 || W < 1 || H * W > 2147483647LL) return GG_E_ARG;
    int64_t n = H * W;
    int64_t* off = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!off) return GG_E_NOMEM;
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t r = v / W, c = v % W;
        off[v + 1] = off[v] + (r > 0) + (c > 0) + (c < W - 1) + (r < H - 1);
    }
    int32_t* cols = (int32_t*)malloc(((size_t)off[n] + 1) * sizeof(int32_t));
    if (!cols) { free(off); return GG_E_NOMEM; }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
        int64_t r = v / W, c = v % W, p = off[v];
        if (r > 0) cols[p++] = (int32_t)(v - W);
        if (c > 0) cols[p++] = (int32_t)(v - 1);
        if (c < W - 1) cols[p++] = (int32_t)(v + 1);
        if (r < H - 1) cols[p++] = (int32_t)(v + W);
    }
    *nnz_out = off[n]; *off_out = off; *cols_out = cols;
    return GG_OK;
}

/* ---------------------------------------------------------------- 2D blocks */
/* One block A[r0:r0+R, c0:c0+C] of a symmetric CSR graph as two compressed
 * forms with block-local ids:
 *   DCSC (column-major): jc[nzc] column ids, cp[nzc+1], ir[nnz] row ids
 *   DCSR (row-major)   : jr[nzr] row ids,    rp[nzr+1], ic[nnz] column ids
 * Entries inside each column (row) are sorted ascending.                    */
typedef struct {
    int64_t nnz, nzc, nzr;
    int32_t *jc, *ir, *jr, *ic;
    int64_t *cp, *rp;
} gg_block;

static int build_csr(const esrc_t* s, int64_t n, int64_t** off_out, int32_t** cols_out, int64_t* nnz_out);

/* COO (major, minor) -> doubly compressed form: j[nz] non-empty majors,
 * p[nz+1] pointers, i[nnz] sorted, deduplicated minors.                   */
static int compress_major(int64_t nmajor, int64_t nnz, const int32_t* maj, const int32_t* mnr,
                          int64_t* nz_out, int32_t** j_out, int64_t** p_out, int32_t** i_out,
                          int64_t* nnz_out) {
    esrc_t s; memset(&s, 0, sizeof(s));
    s.kind = 3; s.m = nnz; s.es32 = maj; s.ed32 = mnr; s.symmetrize = 0; s.keep_loops = 1;
    int64_t* off; int32_t* minor; int64_t dnnz;
    int rc = build_csr(&s, nmajor, &off, &minor, &dnnz);
    if (rc) return rc;
    int64_t nz = 0;
    for (int64_t j = 0; j < nmajor; ++j) nz += (off[j + 1] > off[j]);
    int32_t* jj = (int32_t*)malloc(((size_t)nz + 1) * sizeof(int32_t));
    int64_t* pp = (int64_t*)malloc(((size_t)nz + 1) * sizeof(int64_t));
    if (!jj || !pp) { free(off); free(minor); free(jj); free(pp); return GG_E_NOMEM; }
    int64_t k = 0;
    for (int64_t j = 0; j < nmajor; ++j)
        if (off[j + 1] > off[j]) { jj[k] = (int32_t)j; pp[k] = off[j]; ++k; }
    pp[nz] = dnnz;
    free(off);
    *nz_out = nz; *j_out = jj; *p_out = pp; *i_out = minor; *nnz_out = dnnz;
    return GG_OK;
}

static int block_from_coo(int64_t R, int64_t C, int64_t nnz, int32_t* rr, int32_t* cc, gg_block* out) {
    memset(out, 0, sizeof(*out));
    int64_t n1, n2;
    int rc = compress_major(C, nnz, cc, rr, &out->nzc, &out->jc, &out->cp, &out->ir, &n1);
    if (rc) return rc;
    rc = compress_major(R, nnz, rr, cc, &out->nzr, &out->jr, &out->rp, &out->ic, &n2);
    out->nnz = n1;
    return rc ? rc : (n1 == n2 ? GG_OK : GG_E_ARG);
}

/* block from a plain (row, col) entry list with block-local ids */
int gg_coo_block(int64_t R, int64_t C, int64_t nnz, const int32_t* rows, const int32_t* cols, gg_block* out) {
    if (R < 1 || C < 1 || nnz < 0) return GG_E_ARG;
    for (int64_t e = 0; e < nnz; ++e)
        if (rows[e] < 0 || rows[e] >= R || cols[e] < 0 || cols[e] >= C) return GG_E_ARG;
    int32_t* rr = (int32_t*)malloc(((size_t)nnz + 1) * sizeof(int32_t));
    int32_t* cc = (int32_t*)malloc(((size_t)nnz + 1) * sizeof(int32_t));
    if (!rr || !cc) { free(rr); free(cc); return GG_E_NOMEM; }
    memcpy(rr, rows, (size_t)nnz * sizeof(int32_t));
    memcpy(cc, cols, (size_t)nnz * sizeof(int32_t));
    int rc = block_from_coo(R, C, nnz, rr, cc, out);
    free(rr); free(cc);
    return rc;
}

/* block of an existing CSR graph (entries are already deduplicated) */
int gg_csr_block(int64_t n, const int64_t* off, const int32_t* cols, int64_t r0, int64_t R,
                 int64_t c0, int64_t C, gg_block* out) {
    if (r0 < 0 || c0 < 0 || R < 1 || C < 1 || r0 + R > n || c0 + C > n) return GG_E_ARG;
    int64_t nnz = 0;
    for (int64_t r = r0; r < r0 + R; ++r)
        for (int64_t p = off[r]; p < off[r + 1]; ++p)
            nnz += (cols[p] >= c0 && cols[p] < c0 + C);
    int32_t* rr = (int32_t*)malloc(((size_t)nnz + 1) * sizeof(int32_t));
    int32_t* cc = (int32_t*)malloc(((size_t)nnz + 1) * sizeof(int32_t));
    if (!rr || !cc) { free(rr); free(cc); return GG_E_NOMEM; }
    int64_t k = 0;
    for (int64_t r = r0; r < r0 + R; ++r)
        for (int64_t p = off[r]; p < off[r + 1]; ++p)
            if (cols[p] >= c0 && cols[p] < c0 + C) { rr[k] = (int32_t)(r - r0); cc[k] = (int32_t)(cols[p] - c0); ++k; }
    int rc = block_from_coo(R, C, nnz, rr, cc, out);
    free(rr); free(cc);
    return rc;
}

/* block of a Kronecker graph, straight from the draws (for graphs too large
 * to hold whole): entries (u,v) and (v,u) of every non-loop draw that fall
 * in the block, deduplicated.                                              */
int gg_kron_block(int scale, int64_t edgefactor, uint64_t seed, double a, double b, double c,
                  int permute, int64_t r0, int64_t R, int64_t c0, int64_t C, gg_block* out) {
    if (scale < 1 || scale > 40) return GG_E_ARG;
    int64_t n = (int64_t)1 << scale;
    if (r0 < 0 || c0 < 0 || R < 1 || C < 1 || r0 + R > n || c0 + C > n || R > 2147483647LL || C > 2147483647LL)
        return GG_E_ARG;
    kron_t k = kron_make(scale, seed, a, b, c, permute);
    int64_t m = edgefactor << scale;
    int nt = omp_get_max_threads();
    int64_t* tcount = (int64_t*)calloc((size_t)nt + 1, sizeof(int64_t));
    /* pass 1: count per thread (static schedule => same ranges in pass 2) */
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num(), T = omp_get_num_threads();
        int64_t lo = m * t / T, hi = m * (t + 1) / T, cnt = 0;
        for (int64_t i = lo; i < hi; ++i) {
            uint64_t u, v; kron_draw(&k, (uint64_t)i, &u, &v);
            if (u == v) continue;
            cnt += ((int64_t)u >= r0 && (int64_t)u < r0 + R && (int64_t)v >= c0 && (int64_t)v < c0 + C);
            cnt += ((int64_t)v >= r0 && (int64_t)v < r0 + R && (int64_t)u >= c0 && (int64_t)u < c0 + C);
        }
        tcount[t + 1] = cnt;
    }
    for (int t = 1; t <= nt; ++t) tcount[t] += tcount[t - 1];
    int64_t raw = tcount[nt];
    int32_t* rr = (int32_t*)malloc(((size_t)raw + 1) * sizeof(int32_t));
    int32_t* cc = (int32_t*)malloc(((size_t)raw + 1) * sizeof(int32_t));
    if (!rr || !cc) { free(rr); free(cc); free(tcount); return GG_E_NOMEM; }
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num(), T = omp_get_num_threads();
        int64_t lo = m * t / T, hi = m * (t + 1) / T, w = tcount[t];
        for (int64_t i = lo; i < hi; ++i) {
            uint64_t u, v; kron_draw(&k, (uint64_t)i, &u, &v);
            if (u == v) continue;
            if ((int64_t)u >= r0 && (int64_t)u < r0 + R && (int64_t)v >= c0 && (int64_t)v < c0 + C) {
                rr[w] = (int32_t)((int64_t)u - r0); cc[w] = (int32_t)((int64_t)v - c0); ++w;
            }
            if ((int64_t)v >= r0 && (int64_t)v < r0 + R && (int64_t)u >= c0 && (int64_t)u < c0 + C) {
                rr[w] = (int32_t)((int64_t)v - r0); cc[w] = (int32_t)((int64_t)u - c0); ++w;
            }
        }
    }
    free(tcount);
    /* duplicates are removed by the compression */
    int rc = block_from_coo(R, C, raw, rr, cc, out);
    free(rr); free(cc);
    return rc;
}

void gg_block_free(gg_block* b) {
    free(b->jc); free(b->cp); free(b->ir); free(b->jr); free(b->rp); free(b->ic);
    memset(b, 0, sizeof(*b));
}
