/*
 * bfs_oracle.c -- plain, serial, obviously-correct CPU reference for the
 * breadth-first search computed by the GPU library.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the GPU path.
 *
 * What it computes (Buluc, Beamer, Madduri, Asanovic, Patterson,
 * "Distributed-Memory Breadth-First Search on Massive Graphs"):
 *   - oracle_bfs: the serial level-synchronous top-down search of Alg. 1
 *     (Section 2) with one FIFO queue, plus a depth (hop count) array.
 *     parent[s] = s; unreachable vertices keep parent = depth = -1.
 *   - oracle_bfs_bottom_up: the serial bottom-up search of Alg. 2: every
 *     unvisited vertex scans its neighbours in stored order and takes the
 *     first one in the frontier, then stops.
 *   - oracle_min_parent: the unique "minimum-id" parent: for each reached
 *     v != s, the smallest u with an edge u->v and depth[u] = depth[v]-1.
 *     Section 2 allows any such u as the parent; Section 4.2 describes the
 *     top-down local discovery as a sparse matrix-sparse vector product on
 *     the semiring whose multiply returns its second operand and whose add
 *     returns the minimum, which selects exactly this parent.
 *   - oracle_validate: the BFS-tree invariants, checked with no search of
 *     its own (depth[s] = 0, parent chain made of real edges one level
 *     apart, no edge from a reached vertex skips a level or leaves the
 *     reached set).
 *   - oracle_level_stats / oracle_direction_schedule /
 *     oracle_bu_scan_lengths: the per-level frontier size and edge counts
 *     the direction-optimizing heuristic of Section 4.4 reads, the
 *     top-down / bottom-up decision it makes, and the number of adjacency
 *     entries a first-hit bottom-up scan examines.
 *   - oracle_block_td / oracle_block_bu: one processor's local discovery on
 *     its block A_ij of the 2D decomposition (Eq. 1): the (select2nd, min)
 *     product of Alg. 3 and one sub-step of the first-hit search of Alg. 4,
 *     both written from the block's plain list of (row, column) entries.
 *
 * Graph input everywhere: CSR with int64 offsets[n+1] and int32 cols[nnz].
 * All functions return 0 on success and a positive code on bad input.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG 1
#define OR_E_NOMEM 2

static int check_csr(int64_t n, const int64_t* off, const int32_t* cols) {
    if (n < 0) return OR_E_ARG;
    if (off[0] != 0) return OR_E_ARG;
    for (int64_t v = 0; v < n; ++v)
        if (off[v + 1] < off[v]) return OR_E_ARG;
    for (int64_t p = 0; p < off[n]; ++p)
        if (cols[p] < 0 || (int64_t)cols[p] >= n) return OR_E_ARG;
    return OR_OK;
}

/* Alg. 1 with a FIFO queue.  The queue holds every vertex once, in the
 * order it was first reached, so levels are contiguous in it.            */
int oracle_bfs(int64_t n, const int64_t* off, const int32_t* cols, int64_t s,
               int32_t* parent, int32_t* depth) {
    if (check_csr(n, off, cols) != OR_OK || s < 0 || s >= n) return OR_E_ARG;
    int32_t* queue = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!queue) return OR_E_NOMEM;
    for (int64_t v = 0; v < n; ++v) { parent[v] = -1; depth[v] = -1; }
    parent[s] = (int32_t)s;
    depth[s] = 0;
    int64_t head = 0, tail = 0;
    queue[tail++] = (int32_t)s;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t p = off[u]; p < off[u + 1]; ++p) {
            int32_t v = cols[p];
            if (parent[v] == -1) {
                parent[v] = u;
                depth[v] = depth[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return OR_OK;
}

/* Alg. 2: level by level, every vertex without a parent scans its own
 * adjacency row in stored order and adopts the first frontier member.
 * The frontier of a level is the set of vertices discovered in the
 * previous level; `next` collects this level's discoveries.             */
int oracle_bfs_bottom_up(int64_t n, const int64_t* off, const int32_t* cols, int64_t s,
                         int32_t* parent, int32_t* depth) {
    if (check_csr(n, off, cols) != OR_OK || s < 0 || s >= n) return OR_E_ARG;
    unsigned char* frontier = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    unsigned char* next = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!frontier || !next) { free(frontier); free(next); return OR_E_NOMEM; }
    for (int64_t v = 0; v < n; ++v) { parent[v] = -1; depth[v] = -1; }
    parent[s] = (int32_t)s;
    depth[s] = 0;
    frontier[s] = 1;
    int64_t frontier_size = 1;
    int32_t level = 0;
    while (frontier_size > 0) {
        int64_t found = 0;
        for (int64_t u = 0; u < n; ++u) {
            if (parent[u] != -1) continue;
            for (int64_t p = off[u]; p < off[u + 1]; ++p) {
                int32_t v = cols[p];
                if (frontier[v]) {
                    parent[u] = v;
                    depth[u] = level + 1;
                    next[u] = 1;
                    ++found;
                    break;
                }
            }
        }
        unsigned char* t = frontier; frontier = next; next = t;
        memset(next, 0, (size_t)n);
        frontier_size = found;
        ++level;
    }
    free(frontier); free(next);
    return OR_OK;
}

/* min-id parent from the definition: scan every edge u->v once. */
int oracle_min_parent(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* depth,
                      int32_t* parent_min) {
    if (check_csr(n, off, cols) != OR_OK) return OR_E_ARG;
    for (int64_t v = 0; v < n; ++v) parent_min[v] = -1;
    for (int64_t u = 0; u < n; ++u) {
        if (depth[u] < 0) continue;
        for (int64_t p = off[u]; p < off[u + 1]; ++p) {
            int32_t v = cols[p];
            if (depth[v] == depth[u] + 1 && (parent_min[v] == -1 || parent_min[v] > (int32_t)u))
                parent_min[v] = (int32_t)u;
        }
    }
    for (int64_t v = 0; v < n; ++v)
        if (depth[v] == 0) parent_min[v] = (int32_t)v;
    return OR_OK;
}

/* Validator error codes (0 = valid). */
#define V_SOURCE 1        /* depth[s] != 0 or parent[s] != s              */
#define V_PAIRING 2       /* exactly one of parent[v], depth[v] is -1      */
#define V_RANGE 3         /* parent or depth outside its legal range      */
#define V_ROOT 4          /* a vertex other than s has depth 0            */
#define V_NOT_EDGE 5      /* (parent[v], v) is not an edge                */
#define V_PARENT_LEVEL 6  /* depth[parent[v]] != depth[v] - 1             */
#define V_LEAK 7          /* edge u->v, u reached, v not reached          */
#define V_SKIP 8          /* edge u->v, u reached, depth[v] > depth[u]+1  */

/* Checks the BFS-tree invariants; *bad_vertex receives the first vertex
 * that violates one.  Together the invariants force depth to equal the
 * hop distance from s: edges from reached vertices never skip a level, so
 * depth <= distance along any shortest path; parent chains are real paths
 * of length depth, so distance <= depth.  One pass over the edges marks
 * every v whose claimed parent edge (parent[v], v) exists.               */
int oracle_validate(int64_t n, const int64_t* off, const int32_t* cols, int64_t s,
                    const int32_t* parent, const int32_t* depth, int64_t* bad_vertex) {
    *bad_vertex = -1;
    if (check_csr(n, off, cols) != OR_OK || s < 0 || s >= n) return -OR_E_ARG;
    if (depth[s] != 0 || parent[s] != (int32_t)s) { *bad_vertex = s; return V_SOURCE; }
    for (int64_t v = 0; v < n; ++v) {
        if ((parent[v] == -1) != (depth[v] == -1)) { *bad_vertex = v; return V_PAIRING; }
        if (parent[v] < -1 || (int64_t)parent[v] >= n || depth[v] < -1 || (int64_t)depth[v] >= n) {
            *bad_vertex = v; return V_RANGE;
        }
        if (depth[v] == 0 && v != s) { *bad_vertex = v; return V_ROOT; }
    }
    for (int64_t v = 0; v < n; ++v) {
        if (depth[v] <= 0) continue;
        if (depth[parent[v]] != depth[v] - 1) { *bad_vertex = v; return V_PARENT_LEVEL; }
    }
    unsigned char* edge_ok = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!edge_ok) return -OR_E_NOMEM;
    int code = 0;
    for (int64_t u = 0; u < n && !code; ++u) {
        if (depth[u] < 0) continue;
        for (int64_t p = off[u]; p < off[u + 1]; ++p) {
            int32_t v = cols[p];
            if (depth[v] < 0) { *bad_vertex = v; code = V_LEAK; break; }
            if (depth[v] > depth[u] + 1) { *bad_vertex = v; code = V_SKIP; break; }
            if (parent[v] == (int32_t)u) edge_ok[v] = 1;
        }
    }
    for (int64_t v = 0; v < n && !code; ++v)
        if (depth[v] > 0 && !edge_ok[v]) { *bad_vertex = v; code = V_NOT_EDGE; }
    free(edge_ok);
    return code;
}

/* Per level d of a finished search (depth array):
 *   n_f[d] = |L_d|, m_f[d] = sum of out-degrees over L_d,
 *   m_u[d] = sum of out-degrees over vertices not in L_0..L_d
 *            (the unexplored edges when level d is expanded).
 * Returns the number of levels (max depth + 1) in *nlevels; arrays must
 * hold cap entries.                                                       */
int oracle_level_stats(int64_t n, const int64_t* off, const int32_t* depth, int64_t cap,
                       int64_t* n_f, int64_t* m_f, int64_t* m_u, int64_t* nlevels) {
    int32_t maxd = -1;
    for (int64_t v = 0; v < n; ++v) if (depth[v] > maxd) maxd = depth[v];
    *nlevels = (int64_t)maxd + 1;
    if (*nlevels > cap) return OR_E_ARG;
    int64_t total = off[n];
    for (int64_t d = 0; d < *nlevels; ++d) { n_f[d] = 0; m_f[d] = 0; }
    for (int64_t v = 0; v < n; ++v)
        if (depth[v] >= 0) { n_f[depth[v]] += 1; m_f[depth[v]] += off[v + 1] - off[v]; }
    int64_t seen = 0;
    for (int64_t d = 0; d < *nlevels; ++d) { seen += m_f[d]; m_u[d] = total - seen; }
    return OR_OK;
}

/* The direction choice of Section 4.4 with the thresholds alpha, beta:
 * top-down first; while top-down, switch to bottom-up when the frontier's
 * edges exceed the unexplored edges divided by alpha; while bottom-up,
 * switch back when the frontier holds fewer than n/beta vertices.  Both
 * comparisons are made in double precision as m_f*alpha > m_u and
 * n_f*beta < n.  dir[d] = 0 (top-down) or 1 (bottom-up) for the
 * expansion of level d; mode 1 forces top-down, mode 2 bottom-up.       */
int oracle_direction_schedule(int64_t n, int64_t nlevels, const int64_t* n_f, const int64_t* m_f,
                              const int64_t* m_u, double alpha, double beta, int mode, int32_t* dir) {
    int32_t cur = 0;
    for (int64_t d = 0; d < nlevels; ++d) {
        if (mode == 1) cur = 0;
        else if (mode == 2) cur = 1;
        else if (cur == 0) { if ((double)m_f[d] * alpha > (double)m_u[d]) cur = 1; }
        else { if ((double)n_f[d] * beta < (double)n) cur = 0; }
        dir[d] = cur;
    }
    return OR_OK;
}

/* Adjacency entries examined by a first-hit bottom-up expansion of level
 * d: every vertex without a parent yet (depth -1 or > d) scans its row in
 * stored order until it meets a member of L_d (counted inclusive) or
 * reaches the end of the row.                                            */
int oracle_bu_scan_lengths(int64_t n, const int64_t* off, const int32_t* cols, const int32_t* depth,
                           int32_t d, int64_t* scanned, int64_t* unvisited) {
    int64_t tot = 0, un = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (depth[v] >= 0 && depth[v] <= d) continue;
        ++un;
        for (int64_t p = off[v]; p < off[v + 1]; ++p) {
            ++tot;
            if (depth[cols[p]] == d) break;
        }
    }
    *scanned = tot; *unvisited = un;
    return OR_OK;
}

/* ------------------------------------------------------------ 2D blocks */
/* A block is given as its plain entry list (rows[e], cols[e]) with
 * block-local ids, rows in [0, nrows) and columns in [0, ncols).  Rows are
 * children, columns candidate parents; a parent's global id is
 * col_base + local column.                                               */

/* Alg. 3, local discovery: t(r) = min over frontier columns k of
 * col_base + k for every entry (r, k).  Output sorted by row.            */
int oracle_block_td(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* erow, const int32_t* ecol,
                    int64_t col_base, int64_t nf, const int32_t* fcols,
                    int32_t* out_rows, int32_t* out_parents, int64_t* nout) {
    unsigned char* inf = (unsigned char*)calloc((size_t)(ncols > 0 ? ncols : 1), 1);
    int64_t* best = (int64_t*)malloc((size_t)(nrows > 0 ? nrows : 1) * sizeof(int64_t));
    if (!inf || !best) { free(inf); free(best); return OR_E_NOMEM; }
    for (int64_t i = 0; i < nf; ++i) {
        if (fcols[i] < 0 || fcols[i] >= ncols) { free(inf); free(best); return OR_E_ARG; }
        inf[fcols[i]] = 1;
    }
    for (int64_t r = 0; r < nrows; ++r) best[r] = INT64_MAX;
    for (int64_t e = 0; e < nnz; ++e) {
        if (erow[e] < 0 || erow[e] >= nrows || ecol[e] < 0 || ecol[e] >= ncols) {
            free(inf); free(best); return OR_E_ARG;
        }
        if (inf[ecol[e]] && col_base + ecol[e] < best[erow[e]]) best[erow[e]] = col_base + ecol[e];
    }
    int64_t k = 0;
    for (int64_t r = 0; r < nrows; ++r)
        if (best[r] != INT64_MAX) { out_rows[k] = (int32_t)r; out_parents[k] = (int32_t)best[r]; ++k; }
    *nout = k;
    free(inf); free(best);
    return OR_OK;
}

/* Alg. 4, one sub-step of local discovery over rows [row_lo, row_hi):
 * a row r not yet completed takes the smallest frontier column among its
 * entries (the first hit of a scan in ascending column order), emits
 * (r, col_base + column) and is marked completed.  fbits holds the
 * frontier over columns, completed holds rows; bit i of word w is id
 * 64*w + i.  Output sorted by row.                                       */
int oracle_block_bu(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* erow, const int32_t* ecol,
                    int64_t col_base, const uint64_t* fbits, uint64_t* completed, int64_t row_lo,
                    int64_t row_hi, int32_t* out_rows, int32_t* out_parents, int64_t* nout) {
    if (row_lo < 0 || row_hi > nrows || row_lo > row_hi) return OR_E_ARG;
    int64_t* best = (int64_t*)malloc((size_t)(nrows > 0 ? nrows : 1) * sizeof(int64_t));
    if (!best) return OR_E_NOMEM;
    for (int64_t r = 0; r < nrows; ++r) best[r] = INT64_MAX;
    for (int64_t e = 0; e < nnz; ++e) {
        int64_t r = erow[e], c = ecol[e];
        if (r < 0 || r >= nrows || c < 0 || c >= ncols) { free(best); return OR_E_ARG; }
        if (r < row_lo || r >= row_hi) continue;
        if ((completed[r >> 6] >> (r & 63)) & 1ULL) continue;
        if (!((fbits[c >> 6] >> (c & 63)) & 1ULL)) continue;
        if (c < best[r]) best[r] = c;
    }
    int64_t k = 0;
    for (int64_t r = row_lo; r < row_hi; ++r)
        if (best[r] != INT64_MAX) {
            out_rows[k] = (int32_t)r;
            out_parents[k] = (int32_t)(col_base + best[r]);
            completed[r >> 6] |= 1ULL << (r & 63);
            ++k;
        }
    *nout = k;
    free(best);
    return OR_OK;
}
