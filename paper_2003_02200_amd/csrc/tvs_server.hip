// tvs_server.hip -- a viewshed request server with continuous batching.
//
// Grids are uploaded once and stay resident. Clients submit total-viewshed and singular
// requests from any thread; one scheduler thread owns the device work:
//  - total requests are admitted in arrival order while their device memory (output maps plus
//    scratch) fits the HBM budget. Whenever one of two group slots is free, the waiting totals
//    (same sector count and precision, up to a group limit) leave together as one batch on the
//    slot's stream: per sector chunk, one gather + sweep launch per size bucket with one workgroup
//    per (request, sector, skewed row) item, so that singular work started later interleaves with
//    it, and one back-projection launch; requests that arrive while both groups run gather into the
//    next group. Totals the batched sweep does not take (float Kahan sums, the lane-per-target
//    sweep, the full walk, rows longer than the LDS) run alone on the next of several streams,
//    overlapping with the rest;
//  - singular requests that are waiting are launched together: one multi-query ray-scan launch
//    (every line of sight of every query, one wavefront each) and one per-query area sum, up to a
//    batch limit, as soon as the previous singular batch has finished;
//  - completion is read from events recorded after each piece of work; latency runs from
//    submission to the scheduler seeing that event.
// Results do not depend on what else runs: every kernel writes its own outputs and accumulates
// in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/libtvs.h"
#include "tvs_geom.h"
#include "tvs_host.h"
#include "tvs_internal.h"

using namespace tvs;
using namespace tvs::host;

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Grid {
    float *d = nullptr;
    float *dT = nullptr;  // its transpose (cols x rows): batched sweeps read it for the 45..135 deg axes
    int rows = 0, cols = 0;
    double spacing = 0.0;
};

enum Kind { KIND_TOTAL = 1, KIND_SINGULAR = 2 };
enum State { ST_PENDING, ST_RUNNING, ST_DONE };

struct Request {
    uint64_t ticket = 0;
    int kind = 0;
    int dem = 0;
    double h0 = 0.0, R = 0.0;
    int n = 0;
    int pi = 0, pj = 0;
    uint32_t flags = 0;
    State state = ST_PENDING;
    int status = TVS_OK;
    Clock::time_point t_submit, t_start, t_done;
    double area = 0.0;
    double *d_out = nullptr;  // total: the map (server-owned until released)
    size_t bytes = 0;          // budget held while running
    int stream = -1;
    hipEvent_t ev = nullptr;
    int batch = -1;            // singular: its batch slot
};

// One launched group of total requests (a batch over their grids) and its pinned staging.
struct TotGroup {
    bool busy = false;
    std::vector<Request *> reqs;
    hipEvent_t ev = nullptr;
    int stream = 0;     // index into the server's streams
    PinnedStaging stage;
    size_t bytes = 0;   // budget held: the maps and the batch's scratch
};

// One launched group of singular queries and its staging memory.
struct SingBatch {
    bool busy = false;
    std::vector<Request *> reqs;
    hipEvent_t ev = nullptr;
    size_t cap_secs = 0, cap_q = 0;
    SingSec *h_secs = nullptr;    // pinned staging
    SingQuery *h_q = nullptr;
    double *h_area = nullptr;
    char *d_mem = nullptr;        // device tables, rays and areas
    SingSec *d_secs = nullptr;
    SingQuery *d_q = nullptr;
    uint32_t *d_rays = nullptr;
    double *d_area = nullptr;
};

}  // namespace

struct tvs_server {
    int dev = 0;
    size_t budget = 0, used = 0, peak = 0;
    int nstreams = 4;
    int max_batch = 64;
    int max_total_batch = 16;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    hipStream_t sing_stream = nullptr;
    std::vector<Grid> grids;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> q_total, q_sing;
    std::vector<Request *> running;
    std::unordered_map<uint64_t, Request *> reqs;
    uint64_t next_ticket = 1;
    SingBatch sb[2];
    TotGroup tg[2];
    std::vector<void *> retired_host;  // outgrown pinned staging, freed at the end
    int64_t n_done = 0, n_batches = 0, n_batched = 0, max_running = 0, n_tbatches = 0, n_tbatched = 0;
    bool stop = false;
    int fatal = TVS_OK;
    std::thread worker;
};

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device memory of a total request: its map and the launch sequence's scratch (capped at a
// quarter of the budget, so that several requests can run side by side).
size_t total_bytes(const tvs_server *s, const Grid &g, const Request *r) {
    const size_t cap = std::max(s->budget / 4, (size_t)64 << 20);  // launch_cap
    return align256((size_t)g.rows * g.cols * sizeof(double)) +
           total_scratch_bytes(g.rows, g.cols, g.spacing, r->n, r->R, r->flags, cap);
}

// Sizes a singular slot's staging for `secs` sectors and `nq` queries. The server sizes both slots
// at its start for a full batch of 180-sector queries; a later growth never waits for the device:
// the old pinned buffers are kept until the server ends (freeing pinned memory waits for every
// stream) and the device tables move through the slot's stream-ordered pool.
int grow_batch(tvs_server *s, SingBatch &b, size_t secs, size_t nq) {
    if (secs <= b.cap_secs && nq <= b.cap_q) return TVS_OK;
    secs = std::max(secs, b.cap_secs * 2);
    nq = std::max(nq, b.cap_q * 2);
    for (void *p : {(void *)b.h_secs, (void *)b.h_q, (void *)b.h_area})
        if (p) s->retired_host.push_back(p);
    if (b.d_mem) (void)hipFreeAsync(b.d_mem, s->sing_stream);
    b.h_secs = nullptr;
    b.h_q = nullptr;
    b.h_area = nullptr;
    b.d_mem = nullptr;
    b.cap_secs = b.cap_q = 0;
    HIPCHK(hipHostMalloc((void **)&b.h_secs, secs * sizeof(SingSec), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&b.h_q, nq * sizeof(SingQuery), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&b.h_area, nq * sizeof(double), hipHostMallocDefault));
    const size_t a = align256(secs * sizeof(SingSec)), q = align256(nq * sizeof(SingQuery)),
                 rays = align256(2 * secs * sizeof(uint32_t)), ar = align256(nq * sizeof(double));
    HIPCHK(hipMallocAsync((void **)&b.d_mem, a + q + rays + ar, s->sing_stream));
    b.d_secs = (SingSec *)b.d_mem;
    b.d_q = (SingQuery *)(b.d_mem + a);
    b.d_rays = (uint32_t *)(b.d_mem + a + q);
    b.d_area = (double *)(b.d_mem + a + q + rays);
    b.cap_secs = secs;
    b.cap_q = nq;
    return TVS_OK;
}

// Launches the waiting singular queries that share the front query's precision (caller holds mu).
int launch_singular_batch(tvs_server *s, SingBatch &b) {
    const uint32_t pmask = TVS_FLAG_SLOPE_F32 | TVS_FLAG_SLOPE_F64 | TVS_FLAG_SLOPE_EXACT;
    const uint32_t key = s->q_sing.front()->flags & pmask;
    b.reqs.clear();
    size_t secs = 0;
    for (auto it = s->q_sing.begin(); it != s->q_sing.end() && (int)b.reqs.size() < s->max_batch;) {
        if (((*it)->flags & pmask) == key) {
            secs += (*it)->n;
            b.reqs.push_back(*it);
            it = s->q_sing.erase(it);
        } else {
            ++it;
        }
    }
    if (int rc = grow_batch(s, b, secs, b.reqs.size())) return rc;
    size_t k0 = 0;
    for (size_t qi = 0; qi < b.reqs.size(); ++qi) {
        Request *r = b.reqs[qi];
        const Grid &g = s->grids[r->dem];
        SingQuery &Q = b.h_q[qi];
        memset(&Q, 0, sizeof(Q));
        Q.dem = g.d;
        Q.H = g.rows;
        Q.W = g.cols;
        Q.pov_i = r->pi;
        Q.pov_j = r->pj;
        Q.sec0 = (int32_t)k0;
        Q.nsec = r->n;
        Q.h0 = r->h0;
        Q.h0f = (float)r->h0;
        for (int k = 0; k < r->n; ++k, ++k0) {
            const Sector p = plan_sector(k, r->n, g.rows, g.cols, g.spacing, r->R);
            SingSec &S = b.h_secs[k0];
            memset(&S, 0, sizeof(S));
            S.s.T = p.T;
            S.s.scale = p.scale;
            S.s.clip = p.clip;
            S.s.kase = p.kase;
            S.s.K = p.K;
            S.s.t0 = p.t0;
            S.s.nrows = p.nrows;
            S.query = (int32_t)qi;
        }
        r->state = ST_RUNNING;
        r->t_start = Clock::now();
        r->batch = (int)(&b - s->sb);
    }
    const int nq = (int)b.reqs.size();
    const bool f64 = (key & TVS_FLAG_SLOPE_F32) == 0;
    const bool rcp = (key & (TVS_FLAG_SLOPE_EXACT | TVS_FLAG_SLOPE_F64)) == 0;
    hipStream_t st = s->sing_stream;
    HIPCHK(hipMemcpyAsync(b.d_secs, b.h_secs, secs * sizeof(SingSec), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b.d_q, b.h_q, nq * sizeof(SingQuery), hipMemcpyHostToDevice, st));
    HIPCHK(launch_singular_multi(b.d_secs, (int)secs, b.d_q, nq, b.d_rays, b.d_area, f64, rcp, st));
    HIPCHK(hipMemcpyAsync(b.h_area, b.d_area, nq * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(b.ev, st));
    b.busy = true;
    s->n_batches += 1;
    s->n_batched += nq;
    return TVS_OK;
}

void finish(tvs_server *s, Request *r, int status) {
    r->status = status;
    r->state = ST_DONE;
    r->t_done = Clock::now();
    s->n_done += 1;
}

// Scratch cap of one launch sequence: a quarter of the budget, so that several run side by side.
size_t launch_cap(const tvs_server *s) { return std::max(s->budget / 4, (size_t)64 << 20); }

// Total requests the batched sweep takes: the default early exit, double or float decisions, rows
// that fit the LDS.
bool batchable(const tvs_server *s, const Request *r) {
    const uint32_t pmask = TVS_FLAG_SLOPE_F32 | TVS_FLAG_SLOPE_F64 | TVS_FLAG_SLOPE_EXACT;
    if (r->flags & ~pmask) return false;
    const Grid &g = s->grids[r->dem];
    return batch_rows_fit(std::max(g.rows, g.cols), (r->flags & TVS_FLAG_SLOPE_F32) == 0);
}

tvs_tile tile_of(const tvs_server *s, const Request *r) {
    const Grid &g = s->grids[r->dem];
    tvs_tile t;
    t.d_dem = g.d;
    t.d_out = r->d_out;
    t.rows = g.rows;
    t.cols = g.cols;
    t.spacing = g.spacing;
    t.obs_height = r->h0;
    t.max_dist = r->R;
    return t;
}

// Launches the group's requests as one batch on the slot's stream (caller holds mu); the maps are
// taken stream-ordered there.
int launch_total_group(tvs_server *s, TotGroup &G) {
    hipStream_t st = s->streams[G.stream];
    std::vector<tvs_tile> tiles;
    std::vector<const float *> demT;
    for (Request *r : G.reqs) {
        const Grid &g = s->grids[r->dem];
        r->state = ST_RUNNING;
        r->t_start = Clock::now();
        r->stream = G.stream;
        if (hipMallocAsync((void **)&r->d_out, (size_t)g.rows * g.cols * sizeof(double), st) != hipSuccess) {
            (void)hipGetLastError();
            r->d_out = nullptr;
            return fail(TVS_ENOMEM, "map of %d x %d not available", g.rows, g.cols);
        }
        tiles.push_back(tile_of(s, r));
        demT.push_back(g.dT);
    }
    int chunks = 0;
    if (int rc = batch_enqueue(tiles.data(), demT.data(), (int)tiles.size(), G.reqs[0]->n, G.reqs[0]->flags, st,
                               launch_cap(s), G.stage, &chunks))
        return rc;
    HIPCHK(hipEventRecord(G.ev, st));
    G.busy = true;
    s->n_tbatches += 1;
    s->n_tbatched += (int64_t)G.reqs.size();
    return TVS_OK;
}

void scheduler(tvs_server *s) {
    (void)hipSetDevice(s->dev);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        bool progress = false;
        // completions
        for (size_t x = 0; x < s->running.size();) {
            Request *r = s->running[x];
            const hipError_t q = hipEventQuery(r->ev);
            if (q == hipErrorNotReady) {
                ++x;
                continue;
            }
            s->used -= r->bytes;
            r->bytes = 0;
            finish(s, r, q == hipSuccess ? r->status : TVS_EDEVICE);
            s->running.erase(s->running.begin() + x);
            progress = true;
        }
        for (TotGroup &G : s->tg) {
            if (!G.busy) continue;
            const hipError_t q = hipEventQuery(G.ev);
            if (q == hipErrorNotReady) continue;
            for (Request *r : G.reqs) finish(s, r, q == hipSuccess ? TVS_OK : TVS_EDEVICE);
            s->used -= G.bytes;
            G.bytes = 0;
            G.reqs.clear();
            G.busy = false;
            progress = true;
        }
        for (SingBatch &b : s->sb) {
            if (!b.busy) continue;
            const hipError_t q = hipEventQuery(b.ev);
            if (q == hipErrorNotReady) continue;
            for (size_t qi = 0; qi < b.reqs.size(); ++qi) {
                b.reqs[qi]->area = b.h_area[qi];
                finish(s, b.reqs[qi], q == hipSuccess ? TVS_OK : TVS_EDEVICE);
            }
            b.reqs.clear();
            b.busy = false;
            progress = true;
        }
        if (progress) s->cv_done.notify_all();
        if (s->stop && s->q_total.empty() && s->q_sing.empty() && s->running.empty() && !s->sb[0].busy &&
            !s->sb[1].busy && !s->tg[0].busy && !s->tg[1].busy)
            break;
        // admission of total requests, in arrival order
        while (!s->q_total.empty()) {
            Request *r = s->q_total.front();
            const bool idle = s->running.empty() && !s->tg[0].busy && !s->tg[1].busy;
            if (batchable(s, r)) {
                // a free group slot takes the waiting totals of the front request's sector count and
                // precision, in arrival order, while their maps and the batch's scratch fit the budget
                TotGroup *G = !s->tg[0].busy ? &s->tg[0] : !s->tg[1].busy ? &s->tg[1] : nullptr;
                if (!G) break;  // both groups run: arrivals gather into the next one
                BatchSize sum;
                size_t maps = 0, need = 0;
                auto it = s->q_total.begin();
                while (it != s->q_total.end() && (int)G->reqs.size() < s->max_total_batch) {
                    Request *x = *it;
                    if (!batchable(s, x) || x->n != r->n || x->flags != r->flags) break;
                    const Grid &gx = s->grids[x->dem];
                    BatchSize with = sum;
                    with.add(batch_tile_size(tile_of(s, x), x->n));
                    const size_t mx = maps + align256((size_t)gx.rows * gx.cols * sizeof(double));
                    const size_t nx = mx + batch_scratch_bytes(with, launch_cap(s));
                    if ((!G->reqs.empty() || !idle) && s->used + nx > s->budget) break;  // wait for memory
                    sum = with;
                    maps = mx;
                    need = nx;
                    G->reqs.push_back(x);
                    it = s->q_total.erase(it);
                }
                if (G->reqs.empty()) break;
                const int rc = launch_total_group(s, *G);
                if (rc != TVS_OK) {
                    for (Request *x : G->reqs) finish(s, x, rc);
                    G->reqs.clear();
                    G->busy = false;
                    progress = true;
                    continue;
                }
                G->bytes = need;
                s->used += need;
                s->peak = std::max(s->peak, s->used);
                const int64_t nrun = (int64_t)(s->running.size() + s->tg[0].reqs.size() + s->tg[1].reqs.size());
                s->max_running = std::max(s->max_running, nrun);
                progress = true;
                continue;
            }
            const Grid &g = s->grids[r->dem];
            const size_t need = total_bytes(s, g, r);
            if (!idle && s->used + need > s->budget) break;  // wait for memory
            s->q_total.pop_front();
            const int si = s->next_stream;
            s->next_stream = (s->next_stream + 1) % s->nstreams;
            hipStream_t st = s->streams[si];
            r->stream = si;
            r->t_start = Clock::now();
            r->state = ST_RUNNING;
            int rc = TVS_OK;
            if (hipMallocAsync((void **)&r->d_out, (size_t)g.rows * g.cols * sizeof(double), st) != hipSuccess) {
                (void)hipGetLastError();
                r->d_out = nullptr;
                rc = fail(TVS_ENOMEM, "map of %d x %d not available", g.rows, g.cols);
            }
            if (rc == TVS_OK)
                rc = total_on_stream(g.d, g.rows, g.cols, g.spacing, r->h0, r->n, r->R, r->d_out, r->flags, st,
                                     launch_cap(s));
            if (rc == TVS_OK && hipEventRecord(r->ev, st) != hipSuccess) rc = TVS_EDEVICE;
            if (rc != TVS_OK) {
                finish(s, r, rc);
                progress = true;
                continue;
            }
            r->bytes = need;
            s->used += need;
            s->peak = std::max(s->peak, s->used);
            s->running.push_back(r);
            const int64_t nrun = (int64_t)(s->running.size() + s->tg[0].reqs.size() + s->tg[1].reqs.size());
            s->max_running = std::max(s->max_running, nrun);
            progress = true;
        }
        // singular queries that are waiting: up to two batches in flight (double-buffered
        // staging); while both are busy, arrivals gather into the next, larger batch
        if (!s->q_sing.empty()) {
            for (SingBatch &b : s->sb) {
                if (b.busy || s->q_sing.empty()) continue;
                const int rc = launch_singular_batch(s, b);
                if (rc != TVS_OK) {
                    for (Request *r : b.reqs) finish(s, r, rc);
                    b.reqs.clear();
                    b.busy = false;
                }
                progress = true;
            }
        }
        if (progress) {
            s->cv_done.notify_all();
            continue;
        }
        const bool busy = !s->running.empty() || s->sb[0].busy || s->sb[1].busy || s->tg[0].busy || s->tg[1].busy;
        // poll device work every 50 us; sleep until a submission when idle
        s->cv_work.wait_for(lk, busy ? std::chrono::microseconds(50) : std::chrono::milliseconds(50));
    }
}

int check_request(tvs_server *s, int dem, double h0, int n, double R, uint32_t flags, bool total) {
    if (dem < 0 || dem >= (int)s->grids.size()) return fail(TVS_EINVAL, "unknown grid id %d", dem);
    const Grid &g = s->grids[dem];
    if (int rc = check_scalars(g.rows, g.cols, g.spacing, h0, n, R)) return rc;
    const uint32_t ok = TVS_FLAG_SLOPE_F32 | TVS_FLAG_SLOPE_F64 | TVS_FLAG_SLOPE_EXACT |
                        (total ? TVS_FLAG_NO_PRUNE | TVS_FLAG_SWEEP_SCAN | TVS_FLAG_ACC_KAHAN32 : 0u);
    if (flags & ~ok) return fail(TVS_EINVAL, "unsupported flags 0x%x for this request", flags);
    if ((flags & TVS_FLAG_SLOPE_F32) && (flags & TVS_FLAG_SLOPE_F64))
        return fail(TVS_EINVAL, "TVS_FLAG_SLOPE_F32 and TVS_FLAG_SLOPE_F64 exclude each other");
    if (total && (flags & TVS_FLAG_SWEEP_SCAN) &&
        sweep_lds_bytes(std::max(g.rows, g.cols), (flags & TVS_FLAG_SLOPE_F32) == 0) + 64 > (size_t)lds_limit(s->dev))
        return fail(TVS_ERANGE, "grid %d x %d: the lane-per-target sweep holds whole rows in LDS", g.rows, g.cols);
    return TVS_OK;
}

}  // namespace

extern "C" {

int tvs_server_create(const tvs_server_config *cfg, tvs_server **out) {
    g_err[0] = 0;
    if (!out) return fail(TVS_EINVAL, "null out");
    tvs_server_config c{};
    if (cfg) c = *cfg;
    if (c.streams < 0 || c.streams > 16 || c.max_singular_batch < 0 || c.hbm_budget_bytes < 0 ||
        c.max_total_batch < 0)
        return fail(TVS_EINVAL,
                    "streams in [0, 16], max_singular_batch >= 0, max_total_batch >= 0, hbm_budget_bytes >= 0");
    tvs_server *s = new (std::nothrow) tvs_server;
    if (!s) return fail(TVS_ENOMEM, "host memory for the server");
    auto bail = [&](int rc) {
        for (SingBatch &b : s->sb) {
            if (b.ev) (void)hipEventDestroy(b.ev);
            for (void *p : {(void *)b.h_secs, (void *)b.h_q, (void *)b.h_area})
                if (p) (void)hipHostFree(p);
            if (b.d_mem) (void)hipFreeAsync(b.d_mem, s->sing_stream);
        }
        for (void *p : s->retired_host) (void)hipHostFree(p);
        for (TotGroup &G : s->tg) {
            if (G.ev) (void)hipEventDestroy(G.ev);
            if (G.stage.p) (void)hipHostFree(G.stage.p);
        }
        if (s->sing_stream) (void)hipStreamSynchronize(s->sing_stream);
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        if (s->sing_stream) (void)hipStreamDestroy(s->sing_stream);
        delete s;
        return rc;
    };
    if (hipGetDevice(&s->dev) != hipSuccess) return bail(fail(TVS_EDEVICE, "no current HIP device"));
    size_t freeb = 0, totalb = 0;
    (void)hipMemGetInfo(&freeb, &totalb);
    s->budget = c.hbm_budget_bytes > 0 ? (size_t)c.hbm_budget_bytes : freeb / 2;
    s->nstreams = c.streams > 0 ? c.streams : 4;
    s->max_batch = c.max_singular_batch > 0 ? c.max_singular_batch : 64;
    s->max_total_batch = c.max_total_batch > 0 ? c.max_total_batch : 16;
    pool_keep_memory(s->dev);
    // the singular stream first: streams beyond the hardware queues share one, and the first created
    // is the least likely to share with a long total
    if (hipStreamCreateWithFlags(&s->sing_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(TVS_EDEVICE, "stream creation failed"));
    for (int x = 0; x < s->nstreams; ++x) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(TVS_EDEVICE, "stream creation failed"));
        s->streams.push_back(st);
    }
    for (SingBatch &b : s->sb)
        if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess)
            return bail(fail(TVS_EDEVICE, "event creation failed"));
    for (int x = 0; x < 2; ++x) {
        TotGroup &G = s->tg[x];
        G.stream = x % s->nstreams;
        if (hipEventCreateWithFlags(&G.ev, hipEventDisableTiming) != hipSuccess)
            return bail(fail(TVS_EDEVICE, "event creation failed"));
    }
    // Staging sized up front (a full batch of 180-sector singular queries; 8 MB of work lists per
    // group of totals), so that serving seldom grows it.
    for (SingBatch &b : s->sb)
        if (int rc = grow_batch(s, b, (size_t)s->max_batch * 180, (size_t)s->max_batch)) return bail(rc);
    for (TotGroup &G : s->tg) {
        const size_t want = (size_t)8 << 20;
        if (hipHostMalloc(&G.stage.p, want, hipHostMallocDefault) != hipSuccess) {
            G.stage.p = nullptr;
            return bail(fail(TVS_ENOMEM, "pinned staging of %zu bytes", want));
        }
        G.stage.cap = want;
    }
    s->worker = std::thread(scheduler, s);
    *out = s;
    return TVS_OK;
}

int tvs_server_add_grid(tvs_server *s, const float *dem, int32_t rows, int32_t cols, double spacing,
                        int32_t *out_id) {
    g_err[0] = 0;
    if (!s || !dem || !out_id) return fail(TVS_EINVAL, "null server, dem or out_id");
    if (int rc = check_scalars(rows, cols, spacing, 0.0, 1, INFINITY)) return rc;
    if (int rc = check_host_dem(dem, rows, cols)) return rc;
    Grid g;
    g.rows = rows;
    g.cols = cols;
    g.spacing = spacing;
    const size_t bytes = (size_t)rows * cols * sizeof(float);
    if (hipMalloc((void **)&g.d, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TVS_ENOMEM, "grid of %d x %d not available", rows, cols);
    }
    if (hipMemcpy(g.d, dem, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(g.d);
        return fail(TVS_EDEVICE, "grid upload failed");
    }
    if (hipMalloc((void **)&g.dT, bytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(g.d);
        return fail(TVS_ENOMEM, "transposed grid of %d x %d not available", cols, rows);
    }
    if (launch_transpose(g.d, g.dT, rows, cols, nullptr) != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
        (void)hipFree(g.d);
        (void)hipFree(g.dT);
        return fail(TVS_EDEVICE, "grid transposition failed");
    }
    std::lock_guard<std::mutex> lk(s->mu);
    *out_id = (int32_t)s->grids.size();
    s->grids.push_back(g);
    return TVS_OK;
}

static int submit(tvs_server *s, Request *r, uint64_t *out_ticket) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        delete r;
        return fail(TVS_EINVAL, "the server is shutting down");
    }
    if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
        delete r;
        return fail(TVS_EDEVICE, "event creation failed");
    }
    r->ticket = s->next_ticket++;
    r->t_submit = Clock::now();
    s->reqs[r->ticket] = r;
    (r->kind == KIND_TOTAL ? s->q_total : s->q_sing).push_back(r);
    *out_ticket = r->ticket;
    s->cv_work.notify_one();
    return TVS_OK;
}

int tvs_server_submit_total(tvs_server *s, int32_t grid_id, double obs_height, int32_t n_sectors, double max_dist,
                            uint32_t flags, uint64_t *out_ticket) {
    g_err[0] = 0;
    if (!s || !out_ticket) return fail(TVS_EINVAL, "null server or out_ticket");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (int rc = check_request(s, grid_id, obs_height, n_sectors, max_dist, flags, true)) return rc;
    }
    Request *r = new (std::nothrow) Request;
    if (!r) return fail(TVS_ENOMEM, "host memory");
    r->kind = KIND_TOTAL;
    r->dem = grid_id;
    r->h0 = obs_height;
    r->n = n_sectors;
    r->R = max_dist;
    r->flags = flags;
    return submit(s, r, out_ticket);
}

int tvs_server_submit_singular(tvs_server *s, int32_t grid_id, double obs_height, int32_t n_sectors,
                               double max_dist, int32_t pov_row, int32_t pov_col, uint32_t flags,
                               uint64_t *out_ticket) {
    g_err[0] = 0;
    if (!s || !out_ticket) return fail(TVS_EINVAL, "null server or out_ticket");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (int rc = check_request(s, grid_id, obs_height, n_sectors, max_dist, flags, false)) return rc;
        const Grid &g = s->grids[grid_id];
        if (pov_row < 0 || pov_row >= g.rows || pov_col < 0 || pov_col >= g.cols)
            return fail(TVS_EINVAL, "POV (%d, %d) outside the %d x %d grid", pov_row, pov_col, g.rows, g.cols);
    }
    Request *r = new (std::nothrow) Request;
    if (!r) return fail(TVS_ENOMEM, "host memory");
    r->kind = KIND_SINGULAR;
    r->dem = grid_id;
    r->h0 = obs_height;
    r->n = n_sectors;
    r->R = max_dist;
    r->pi = pov_row;
    r->pj = pov_col;
    r->flags = flags;
    return submit(s, r, out_ticket);
}

int tvs_server_wait(tvs_server *s, uint64_t ticket, double timeout_ms, tvs_request_result *res) {
    g_err[0] = 0;
    if (!s || !res) return fail(TVS_EINVAL, "null server or result");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(TVS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    auto done = [&] { return r->state == ST_DONE; };
    if (timeout_ms < 0) s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), done))
        return fail(TVS_ETIMEDOUT, "request %llu not finished", (unsigned long long)ticket);
    memset(res, 0, sizeof(*res));
    res->status = r->status;
    res->kind = r->kind;
    res->area_m2 = r->area;
    res->latency_ms = ms_since(r->t_submit, r->t_done);
    res->queue_ms = ms_since(r->t_submit, r->t_start);
    res->rows = s->grids[r->dem].rows;
    res->cols = s->grids[r->dem].cols;
    return TVS_OK;
}

int tvs_server_copy_map(tvs_server *s, uint64_t ticket, double *out, void *hip_stream) {
    g_err[0] = 0;
    if (!s || !out) return fail(TVS_EINVAL, "null server or out");
    double *src = nullptr;
    size_t bytes = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(TVS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        Request *r = it->second;
        if (r->kind != KIND_TOTAL || r->state != ST_DONE || r->status != TVS_OK || !r->d_out)
            return fail(TVS_EINVAL, "ticket %llu holds no finished map", (unsigned long long)ticket);
        src = r->d_out;
        bytes = (size_t)s->grids[r->dem].rows * s->grids[r->dem].cols * sizeof(double);
    }
    HIPCHK(hipMemcpyAsync(out, src, bytes, hipMemcpyDefault, (hipStream_t)hip_stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)hip_stream));
    return TVS_OK;
}

int tvs_server_release(tvs_server *s, uint64_t ticket) {
    g_err[0] = 0;
    if (!s) return fail(TVS_EINVAL, "null server");
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(TVS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        if (it->second->state != ST_DONE) return fail(TVS_EINVAL, "request %llu still running",
                                                      (unsigned long long)ticket);
        r = it->second;
        s->reqs.erase(it);
    }
    if (r->d_out) (void)hipFreeAsync(r->d_out, s->streams[std::max(r->stream, 0)]);
    if (r->ev) (void)hipEventDestroy(r->ev);
    delete r;
    return TVS_OK;
}

int tvs_server_get_stats(tvs_server *s, tvs_server_stats *st) {
    g_err[0] = 0;
    if (!s || !st) return fail(TVS_EINVAL, "null server or stats");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(st, 0, sizeof(*st));
    st->grids = (int32_t)s->grids.size();
    st->pending = (int32_t)(s->q_total.size() + s->q_sing.size());
    st->running = (int32_t)s->running.size() + (int32_t)(s->sb[0].reqs.size() + s->sb[1].reqs.size()) +
                  (int32_t)(s->tg[0].reqs.size() + s->tg[1].reqs.size());
    st->completed = s->n_done;
    st->singular_batches = s->n_batches;
    st->singular_batched = s->n_batched;
    st->max_concurrent_totals = s->max_running;
    st->budget_bytes = (int64_t)s->budget;
    st->bytes_in_use = (int64_t)s->used;
    st->peak_bytes = (int64_t)s->peak;
    st->total_batches = s->n_tbatches;
    st->total_batched = s->n_tbatched;
    return TVS_OK;
}

int tvs_server_destroy(tvs_server *s) {
    g_err[0] = 0;
    if (!s) return TVS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipDeviceSynchronize();
    for (auto &kv : s->reqs) {
        Request *r = kv.second;
        if (r->d_out) (void)hipFreeAsync(r->d_out, s->streams[std::max(r->stream, 0)]);
        if (r->ev) (void)hipEventDestroy(r->ev);
        delete r;
    }
    for (TotGroup &G : s->tg) {
        if (G.ev) (void)hipEventDestroy(G.ev);
        if (G.stage.p) (void)hipHostFree(G.stage.p);
        for (void *p : G.stage.retired) (void)hipHostFree(p);
    }
    for (SingBatch &b : s->sb) {
        if (b.ev) (void)hipEventDestroy(b.ev);
        if (b.h_secs) (void)hipHostFree(b.h_secs);
        if (b.h_q) (void)hipHostFree(b.h_q);
        if (b.h_area) (void)hipHostFree(b.h_area);
        if (b.d_mem) (void)hipFreeAsync(b.d_mem, s->sing_stream);
    }
    for (void *p : s->retired_host) (void)hipHostFree(p);
    if (s->sing_stream) (void)hipStreamSynchronize(s->sing_stream);
    for (Grid &g : s->grids) {
        (void)hipFree(g.d);
        (void)hipFree(g.dT);
    }
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (s->sing_stream) (void)hipStreamDestroy(s->sing_stream);
    delete s;
    return TVS_OK;
}

}  // extern "C"
