// Query server (include/bfs_serve.h): resident graphs, device-memory budget
// admission, continuous same-graph batching onto multi-source searches, one
// host thread + HIP stream per slot so batches overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/bfs_serve.h"

#include "bfs_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    int64_t id;
    int32_t graph;
    int64_t src;
    double t_arr;   // seconds on the server clock
    int32_t* h_depth;
    int32_t* h_parent;
};

struct Rec {
    int64_t id;
    double lat_us;
    int32_t bsize;
    int64_t bseq;
};

// first-fit allocator over one device allocation, 256-byte granules
struct Pool {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length

    void init(char* b, size_t n) {
        base = b;
        size = n;
        free_.clear();
        free_[0] = n;
    }
    static size_t round(size_t x) { return (x + 255) / 256 * 256; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t roff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round(bytes);
        auto it = free_.emplace(off, bytes).first;
        // merge with the next and previous free ranges
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

struct bfs_server {
    bfs_server_opts o{};
    int device = 0;
    Clock::time_point t0;
    std::vector<bfs_graph*> graphs;
    std::vector<int64_t> graph_n;
    std::vector<std::deque<Req>> pending;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    Pool pool;
    std::vector<std::thread> workers;
    std::vector<std::thread> replayers;
    int replays_running = 0;
    bool stop = false;
    int64_t submitted = 0, completed = 0, failed = 0, batches = 0, inflight = 0, max_inflight = 0;
    double first_arrival = -1.0, last_completion = 0.0;
    std::vector<Rec> recs;
    // every batch's span on the device: HIP events recorded on its slot's
    // stream before its first and after its last kernel, in ms after `ref_ev`
    // (recorded once when the server starts)
    hipEvent_t ref_ev = nullptr;
    std::vector<std::pair<double, double>> dev_spans;
    bfs_status first_error = BFS_OK;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    // workspace of a multi-source search (its layout does not depend on k)
    // a batch of one runs the single-source search (bfs_run), larger batches
    // the multi-source one; both give minimum-id parents
    size_t ws_for(int32_t gid, int k) const { return bfs_workspace_bytes(graphs[gid], k == 1 ? 1 : 2); }

    size_t batch_bytes(int32_t gid, int k) const {
        const int64_t n = graph_n[gid];
        const size_t ws = ws_for(gid, k);
        const size_t outs = (size_t)k * (size_t)n * sizeof(int32_t) * ((o.want_parent || k == 1) ? 2 : 1);
        return Pool::round(ws) + Pool::round(outs);
    }

    // picks the next batch under the lock; false when the server stops
    bool next_batch(std::unique_lock<std::mutex>& lk, std::vector<Req>& batch, int32_t* gid_out, size_t* off,
                    size_t* bytes, int64_t* seq) {
        for (;;) {
            if (stop) return false;
            // the graph whose oldest waiting query arrived first
            int32_t gid = -1;
            double oldest = 0;
            for (size_t g = 0; g < pending.size(); ++g)
                if (!pending[g].empty() && (gid < 0 || pending[g].front().t_arr < oldest)) {
                    gid = (int32_t)g;
                    oldest = pending[g].front().t_arr;
                }
            if (gid < 0) {
                cv_work.wait(lk);
                continue;
            }
            int k = (int)std::min<size_t>((size_t)o.max_batch, pending[gid].size());
            if (k < o.max_batch && o.batch_wait_us > 0) {
                const double waited = (now() - oldest) * 1e6;
                if (waited < o.batch_wait_us) {
                    cv_work.wait_for(lk, std::chrono::microseconds((int64_t)(o.batch_wait_us - waited) + 1));
                    continue;
                }
            }
            // admission by the memory budget: with nothing running, shrink the
            // batch until it fits (one query always fits, see submit)
            bool ok = pool.alloc(batch_bytes(gid, k), off);
            while (!ok && inflight == 0 && k > 1) {
                k = (k + 1) / 2;
                ok = pool.alloc(batch_bytes(gid, k), off);
            }
            if (!ok) {
                cv_work.wait(lk);   // wait until a running batch frees memory
                continue;
            }
            *bytes = batch_bytes(gid, k);
            batch.assign(pending[gid].begin(), pending[gid].begin() + k);
            pending[gid].erase(pending[gid].begin(), pending[gid].begin() + k);
            *seq = batches++;
            ++inflight;
            max_inflight = std::max(max_inflight, inflight);
            *gid_out = gid;
            return true;
        }
    }

    void worker() {
        (void)hipSetDevice(device);
        hipStream_t stream = nullptr;
        if (hipStreamCreate(&stream) != hipSuccess) return;
        hipEvent_t ev_a = nullptr, ev_b = nullptr;
        if (hipEventCreate(&ev_a) != hipSuccess || hipEventCreate(&ev_b) != hipSuccess) {
            if (ev_a) (void)hipEventDestroy(ev_a);
            (void)hipStreamDestroy(stream);
            return;
        }
        std::vector<Req> batch;
        std::vector<int64_t> srcs;
        for (;;) {
            int32_t gid = -1;
            size_t off = 0, bytes = 0;
            int64_t seq = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                if (!next_batch(lk, batch, &gid, &off, &bytes, &seq)) break;
            }
            // ---- run the batch on this slot's stream
            const int k = (int)batch.size();
            const int64_t n = graph_n[gid];
            char* chunk = pool.base + off;
            const size_t ws_bytes = ws_for(gid, k);
            int32_t* depth = (int32_t*)(chunk + Pool::round(ws_bytes));
            int32_t* parent = (o.want_parent || k == 1) ? depth + (size_t)k * (size_t)n : nullptr;
            bfs_status st;
            const bool span_a = hipEventRecord(ev_a, stream) == hipSuccess;
            if (k == 1) {
                bfs_opts so = o.opts;
                so.parent_mode = BFS_PARENT_MIN;
                st = bfs_run(graphs[gid], batch[0].src, &so, parent, depth, chunk, ws_bytes, stream, nullptr);
            } else {
                srcs.resize(k);
                for (int j = 0; j < k; ++j) srcs[j] = batch[j].src;
                st = bfs_run_multi(graphs[gid], srcs.data(), k, &o.opts, parent, depth, chunk, ws_bytes, stream,
                                   nullptr);
            }
            const bool span_b = span_a && hipEventRecord(ev_b, stream) == hipSuccess;
            // the batch's memory goes back to the pool only once every kernel
            // that touches it has finished
            if (hipStreamSynchronize(stream) != hipSuccess && st == BFS_OK) st = BFS_E_HIP;
            float ms_a = 0.f, ms_b = 0.f;
            const bool span = st == BFS_OK && span_b && hipEventElapsedTime(&ms_a, ref_ev, ev_a) == hipSuccess &&
                              hipEventElapsedTime(&ms_b, ref_ev, ev_b) == hipSuccess;
            if (st == BFS_OK) {
                bool copied = false;
                for (int j = 0; j < k; ++j) {
                    if (batch[j].h_depth) {
                        (void)hipMemcpyAsync(batch[j].h_depth, depth + (size_t)j * n, sizeof(int32_t) * n,
                                             hipMemcpyDeviceToHost, stream);
                        copied = true;
                    }
                    if (parent && batch[j].h_parent) {
                        (void)hipMemcpyAsync(batch[j].h_parent, parent + (size_t)j * n, sizeof(int32_t) * n,
                                             hipMemcpyDeviceToHost, stream);
                        copied = true;
                    }
                }
                if (copied && hipStreamSynchronize(stream) != hipSuccess) st = BFS_E_HIP;
            }
            const double t_done = now();
            {
                std::lock_guard<std::mutex> lk(mu);
                for (int j = 0; j < k; ++j)
                    recs.push_back({batch[j].id, st == BFS_OK ? (t_done - batch[j].t_arr) * 1e6 : -1.0, k, seq});
                completed += k;
                if (st != BFS_OK) {
                    failed += k;
                    if (first_error == BFS_OK) first_error = st;
                }
                --inflight;
                if (span) dev_spans.emplace_back((double)ms_a, (double)ms_b);
                last_completion = std::max(last_completion, t_done);
                pool.release(off, bytes);
            }
            batch.clear();
            cv_work.notify_all();
            cv_done.notify_all();
        }
        (void)hipEventDestroy(ev_a);
        (void)hipEventDestroy(ev_b);
        (void)hipStreamDestroy(stream);
    }

    void submit_locked(int32_t gid, int64_t src, int64_t id, int32_t* hd, int32_t* hp) {
        const double t = now();
        pending[gid].push_back({id, gid, src, t, hd, hp});
        ++submitted;
        if (first_arrival < 0) first_arrival = t;
    }
};

extern "C" {

void bfs_server_opts_default(bfs_server_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->slots = 4;
    o->max_batch = 64;
    o->want_parent = 0;
    o->hbm_budget = (size_t)8 << 30;
    o->batch_wait_us = 0.0;
    bfs_opts_default(&o->opts);
}

bfs_status bfs_server_create(const bfs_server_opts* o, bfs_server** out) {
    if (!o || !out) return BFS_E_INVALID_ARG;
    *out = nullptr;
    if (o->slots < 1 || o->slots > 64 || o->max_batch < 1 || o->max_batch > 64 || o->hbm_budget < 4096 ||
        o->batch_wait_us < 0)
        return BFS_E_INVALID_ARG;
    bfs_server* s = new (std::nothrow) bfs_server();
    if (!s) return BFS_E_NO_MEMORY;
    s->o = *o;
    s->t0 = Clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return BFS_E_HIP;
    }
    void* base = nullptr;
    const hipError_t e = hipMalloc(&base, o->hbm_budget);
    if (e != hipSuccess) {
        char msg[160];
        size_t fr = 0, tot = 0;
        (void)hipMemGetInfo(&fr, &tot);
        snprintf(msg, sizeof(msg), "server pool of %zu bytes: %s (%zu of %zu bytes free)", (size_t)o->hbm_budget,
                 hipGetErrorString(e), fr, tot);
        bfsk::set_last_error(msg);
        delete s;
        return BFS_E_HIP;
    }
    s->pool.init((char*)base, o->hbm_budget);
    if (hipEventCreate(&s->ref_ev) != hipSuccess || hipEventRecord(s->ref_ev, nullptr) != hipSuccess ||
        hipEventSynchronize(s->ref_ev) != hipSuccess) {
        bfsk::set_last_error("server reference event");
        if (s->ref_ev) (void)hipEventDestroy(s->ref_ev);
        (void)hipFree(base);
        delete s;
        return BFS_E_HIP;
    }
    for (int i = 0; i < o->slots; ++i) s->workers.emplace_back([s] { s->worker(); });
    *out = s;
    return BFS_OK;
}

bfs_status bfs_server_add_graph(bfs_server* s, bfs_graph* g, int32_t* graph_id) {
    if (!s || !g || !graph_id) return BFS_E_INVALID_ARG;
    // bfs_workspace_bytes(g, 2) is nonzero only for CSR graphs
    if (bfs_workspace_bytes(g, 2) == 0) return BFS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *graph_id = (int32_t)s->graphs.size();
    s->graphs.push_back(g);
    s->graph_n.push_back(bfsk::graph_vertices(g));
    s->pending.emplace_back();
    return BFS_OK;
}

bfs_status bfs_server_submit(bfs_server* s, int32_t graph_id, int64_t source, int64_t request_id, int32_t* h_depth,
                             int32_t* h_parent) {
    if (!s) return BFS_E_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return BFS_E_INVALID_ARG;
        if (source < 0 || source >= s->graph_n[graph_id]) return BFS_E_OUT_OF_RANGE;
        if (s->batch_bytes(graph_id, 1) > s->pool.size) return BFS_E_BUDGET;
        s->submit_locked(graph_id, source, request_id, h_depth, h_parent);
    }
    s->cv_work.notify_one();
    return BFS_OK;
}

bfs_status bfs_server_replay(bfs_server* s, int64_t n, const double* arrival_us, const int32_t* graph_ids,
                             const int64_t* sources, const int64_t* request_ids) {
    if (!s || n < 0 || (n > 0 && (!arrival_us || !graph_ids || !sources || !request_ids))) return BFS_E_INVALID_ARG;
    std::vector<double> t(arrival_us, arrival_us + n);
    std::vector<int32_t> gids(graph_ids, graph_ids + n);
    std::vector<int64_t> src(sources, sources + n), ids(request_ids, request_ids + n);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (int64_t i = 0; i < n; ++i) {
            if (gids[i] < 0 || gids[i] >= (int32_t)s->graphs.size()) return BFS_E_INVALID_ARG;
            if (src[i] < 0 || src[i] >= s->graph_n[gids[i]]) return BFS_E_OUT_OF_RANGE;
            if (s->batch_bytes(gids[i], 1) > s->pool.size) return BFS_E_BUDGET;
            if (i && t[i] < t[i - 1]) return BFS_E_INVALID_ARG;
        }
        ++s->replays_running;
    }
    const Clock::time_point start = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    s->replayers.emplace_back([s, start, t = std::move(t), gids = std::move(gids), src = std::move(src),
                               ids = std::move(ids)] {
        for (size_t i = 0; i < t.size(); ++i) {
            std::this_thread::sleep_until(start + std::chrono::duration_cast<Clock::duration>(
                                                      std::chrono::duration<double, std::micro>(t[i])));
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->submit_locked(gids[i], src[i], ids[i], nullptr, nullptr);
            }
            s->cv_work.notify_one();
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            --s->replays_running;
        }
        s->cv_done.notify_all();
    });
    return BFS_OK;
}

bfs_status bfs_server_drain(bfs_server* s) {
    if (!s) return BFS_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [s] { return s->replays_running == 0 && s->completed >= s->submitted; });
    return s->first_error;
}

bfs_status bfs_server_stats_get(bfs_server* s, bfs_server_stats* out) {
    if (!s || !out) return BFS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->batches = s->batches;
    out->max_inflight = s->max_inflight;
    std::vector<double> lat;
    lat.reserve(s->recs.size());
    for (const Rec& r : s->recs)
        if (r.lat_us >= 0) lat.push_back(r.lat_us);
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            const double pos = p * (double)(lat.size() - 1);
            const size_t i = (size_t)pos;
            const double f = pos - (double)i;
            return i + 1 < lat.size() ? lat[i] * (1 - f) + lat[i + 1] * f : lat[i];
        };
        out->p50_us = pct(0.50);
        out->p99_us = pct(0.99);
        double sum = 0;
        for (double x : lat) sum += x;
        out->mean_us = sum / (double)lat.size();
        out->max_us = lat.back();
    }
    out->mean_batch = s->batches ? (double)s->completed / (double)s->batches : 0.0;
    out->first_arrival_s = s->first_arrival;
    out->last_completion_s = s->last_completion;
    const double span = s->last_completion - s->first_arrival;
    out->queries_per_s = span > 0 ? (double)(s->completed - s->failed) / span : 0.0;
    // most device spans open at one time (a span that ends where another
    // starts does not overlap it)
    std::vector<std::pair<double, int>> ends;
    ends.reserve(2 * s->dev_spans.size());
    for (const auto& sp : s->dev_spans) {
        ends.emplace_back(sp.first, 1);
        ends.emplace_back(sp.second, -1);
    }
    std::sort(ends.begin(), ends.end());
    int64_t open = 0;
    for (const auto& e : ends) {
        open += e.second;
        out->device_max_overlap = std::max(out->device_max_overlap, open);
    }
    return BFS_OK;
}

bfs_status bfs_server_records(bfs_server* s, int64_t* request_ids, double* latency_us, int32_t* batch_size,
                              int64_t* batch_seq, int64_t cap, int64_t* count) {
    if (!s || !count || cap < 0) return BFS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t m = std::min<int64_t>(cap, (int64_t)s->recs.size());
    for (int64_t i = 0; i < m; ++i) {
        if (request_ids) request_ids[i] = s->recs[i].id;
        if (latency_us) latency_us[i] = s->recs[i].lat_us;
        if (batch_size) batch_size[i] = s->recs[i].bsize;
        if (batch_seq) batch_seq[i] = s->recs[i].bseq;
    }
    *count = m;
    return BFS_OK;
}

void bfs_server_destroy(bfs_server* s) {
    if (!s) return;
    (void)bfs_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& t : s->replayers) t.join();
    if (s->ref_ev) (void)hipEventDestroy(s->ref_ev);
    if (s->pool.base) {
        const hipError_t e = hipFree(s->pool.base);
        if (e != hipSuccess) {
            char msg[128];
            snprintf(msg, sizeof(msg), "server pool release: %s", hipGetErrorString(e));
            bfsk::set_last_error(msg);
        }
    }
    delete s;
}

}  // extern "C"
