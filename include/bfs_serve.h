/*
 * bfs_serve.h -- C ABI of the libbfs query server: breadth-first-search
 * queries on graphs kept resident on one MI355X, served with continuous
 * same-graph batching.
 *
 * A query is (graph, source).  Queries are queued per graph as they arrive.
 * Whenever a worker slot is free, the server picks the graph whose oldest
 * waiting query arrived first, takes up to `max_batch` of that graph's
 * waiting queries and runs them as one multi-source search (bfs_run_multi,
 * one bit per query in per-vertex uint64 masks); a batch of one query runs
 * the single-source search (bfs_run, minimum-id parents).  Each slot has its own
 * HIP stream and host thread, so batches of different slots run on the
 * device at the same time.  A batch is admitted only when its workspace and
 * outputs fit in what is left of the server's device-memory budget (one
 * pool allocated at create time); otherwise it waits until running batches
 * free memory.  Queries arriving while batches run join the next batch of
 * their graph.  Results are the minimum-id parents and depths, identical to
 * bfs_run with BFS_PARENT_MIN; they stay in device memory unless the query
 * gave host buffers.
 *
 * Latency of a query = time from its arrival (bfs_server_submit) to the
 * completion of its batch on the device (and of its copy to host, when
 * requested).  All calls are thread safe.
 */
#ifndef BFS_SERVE_H
#define BFS_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "bfs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfs_server bfs_server;

typedef struct {
    int32_t slots;          /* batches in flight at once (worker threads/streams), >= 1 */
    int32_t max_batch;      /* queries per batch, 1..64                                  */
    int32_t want_parent;    /* nonzero: compute parents as well as depths               */
    int32_t reserved0;
    size_t hbm_budget;      /* device bytes for batch workspaces and outputs             */
    double batch_wait_us;   /* a slot waits this long for more same-graph queries when
                               its batch is not full (0 = dispatch at once)              */
    bfs_opts opts;          /* search options (dir, alpha, beta, tuning knobs)           */
} bfs_server_opts;

typedef struct {
    int64_t submitted, completed, batches;
    int64_t max_inflight;        /* most batches seen running at once                   */
    double mean_batch;           /* queries per batch                                   */
    double p50_us, p99_us, mean_us, max_us;   /* latency over completed queries           */
    double first_arrival_s, last_completion_s; /* seconds on the server's clock          */
    double queries_per_s;        /* completed / (last completion - first arrival)        */
    int64_t device_max_overlap;  /* most batches whose spans on the device overlap: a
                                    batch's span runs from a HIP event recorded on its
                                    slot's stream before its first kernel to one after
                                    its last                                           */
} bfs_server_stats;

/* Fill *o with defaults: 4 slots, batches of 64, depths only, 8 GiB budget,
 * no batch wait, bfs_opts_default search options. */
void bfs_server_opts_default(bfs_server_opts* o);

/* Create a server and allocate its device pool (o->hbm_budget bytes) on the
 * current device.  BFS_E_INVALID_ARG for bad options, BFS_E_HIP when the pool
 * cannot be allocated. */
bfs_status bfs_server_create(const bfs_server_opts* o, bfs_server** out);

/* Register a resident graph (a CSR handle created SYMMETRIC and SORTED; the
 * caller keeps it alive until bfs_server_destroy).  *graph_id receives its id. */
bfs_status bfs_server_add_graph(bfs_server* s, bfs_graph* g, int32_t* graph_id);

/* Submit one query now.  request_id is returned in the results.  h_depth
 * (and h_parent when parents are computed) may be host buffers of the
 * graph's n entries that receive the result; NULL keeps it on the device
 * only.  BFS_E_BUDGET if one batch of this graph can never fit the budget. */
bfs_status bfs_server_submit(bfs_server* s, int32_t graph_id, int64_t source, int64_t request_id, int32_t* h_depth,
                             int32_t* h_parent);

/* Submit n queries at arrival times arrival_us[i] (microseconds after the
 * call; ascending) from a server-side thread, and return at once. */
bfs_status bfs_server_replay(bfs_server* s, int64_t n, const double* arrival_us, const int32_t* graph_ids,
                             const int64_t* sources, const int64_t* request_ids);

/* Block until every submitted query has completed (including a replay). */
bfs_status bfs_server_drain(bfs_server* s);

bfs_status bfs_server_stats_get(bfs_server* s, bfs_server_stats* out);

/* Per-query records of completed queries, in completion order: request id,
 * latency (microseconds), the batch size it ran in and the batch sequence
 * number.  Copies up to cap records; *count receives the number copied. */
bfs_status bfs_server_records(bfs_server* s, int64_t* request_ids, double* latency_us, int32_t* batch_size,
                              int64_t* batch_seq, int64_t cap, int64_t* count);

/* Stop the workers (after draining) and free the pool. */
void bfs_server_destroy(bfs_server* s);

#ifdef __cplusplus
}
#endif

#endif /* BFS_SERVE_H */
