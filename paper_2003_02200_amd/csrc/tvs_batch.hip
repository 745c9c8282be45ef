// tvs_batch.hip -- total viewsheds of many independent DEM tiles of uneven size as one batch.
//
// Each tile is its own total viewshed (Section 4.1 steps 1a-1d); the tiles share the sector
// count. Per chunk of sectors, sweep launches walk the list of every (tile, sector, skewed row)
// item of every tile -- gathering each skewed row straight from its tile's DEM or its transposed
// copy (the relocation fused into the sweep) -- and one back-projection launch covers all tiles. The whole pass is captured once into a HIP graph and replayed; the work lists live in
// device memory and a replay only resets the item counters (with a fill kernel). Tiles are grouped
// into buckets by the size classes of their longest side and their longest line of sight; each
// bucket has its own sweep launch per chunk, sized for its rows, and its own launch shape (waves
// per workgroup; persistent workgroups per CU, or one workgroup per item), picked by timing
// candidates on a sample of the bucket's items and remembered per device and library build.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <new>
#include <vector>

#include "../../include/libtvs.h"
#include "tvs_geom.h"
#include "tvs_host.h"
#include "tvs_internal.h"

using namespace tvs;
using namespace tvs::host;

namespace {

struct ChunkPlan {
    int k0, k1;       // sectors [k0, k1)
    size_t ent_off;   // first BatchEnt of the chunk (tile t, sector k0 + x at ent_off + t * nsec + x)
    size_t tile_off;  // first BatchTile of the chunk
    size_t item_off;  // first work item of the chunk
    int nitems;       // (tile, sector, skewed row) items
    int nblocks;      // back-projection blocks over every tile
    size_t vbytes;    // skewed viewshed rows of every tile and sector of the chunk
    std::vector<int> bucket_items;  // per bucket: its items (they follow each other in bucket order)
};

struct Shape {
    int waves;   // wavefronts per workgroup of the sweep
    int per_cu;  // persistent workgroups per CU; 0: one workgroup per item
};

constexpr Shape kDefaultShape{4, 8};
const Shape kCandidates[] = {{2, 4}, {2, 8}, {2, 16}, {4, 2}, {4, 4}, {4, 8}, {8, 1},
                             {8, 2}, {8, 4}, {2, 0}, {4, 0}, {8, 0}};

// Tiles whose longest side and longest line of sight (capped at the side) fall in the same ceil(log2)
// classes: one sweep launch per chunk, sized for their rows, with one launch shape.
struct Bucket {
    int side_b, rho_b;  // size classes
    int maxWx, maxK;    // longest side and line of sight of its tiles
    int ntiles;
    Shape shape;
    bool tuned;
};

int cu_count(int dev) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    return v;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Skewed row index of the i-th row taken from a sector: middle-out, long rows first.
int middle_out(int i, int nrows) {
    const int c = (nrows - 1) >> 1;
    return (i & 1) ? c + ((i + 1) >> 1) : c - (i >> 1);
}

}  // namespace

struct tvs_batch {
    int dev = 0;
    int ntiles = 0, n = 0;
    uint32_t flags = 0;
    bool f64 = true, rcp = true, count = false;
    std::vector<tvs_tile> tiles;
    std::vector<std::vector<Sector>> sectors;  // per tile
    std::vector<const float *> demT;           // per tile: its transposed grid (empty: none)
    bool transpose = false;                    // the pass transposes the tiles into demT first
    bool persistent = true;                    // persistent sweep (else one workgroup per item)
    std::vector<ChunkPlan> chunks;
    std::vector<Bucket> buckets;
    std::vector<int> tile_bucket;  // per tile
    int maxWx = 0, tabN = 0, maxK = 0;
    bool counted = false;
    int64_t evals = 0, pairs = 0;
    size_t dbytes = 0;
    char *dmem = nullptr;
    float2 *tab32 = nullptr;
    double2 *tab64 = nullptr;
    unsigned int *counters = nullptr;
    unsigned long long *work = nullptr;
    BatchEnt *ent = nullptr;
    BatchTile *btiles = nullptr;
    uint32_t *items = nullptr;
    uint32_t *V = nullptr;
    int cus = 256;
    bool tuned = false;
    double tune_ms = 0.0;
    int launches = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~tvs_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) {
            (void)hipStreamSynchronize(cap);
            (void)hipStreamDestroy(cap);
        }
        if (dmem) {
            (void)hipDeviceSynchronize();
            (void)hipFree(dmem);
        }
    }
};

namespace {

int check_tiles(const tvs_tile *tiles, int ntiles, int n) {
    if (!tiles || ntiles < 1) return fail(TVS_EINVAL, "a batch needs at least one tile");
    for (int t = 0; t < ntiles; ++t) {
        const tvs_tile &T = tiles[t];
        if (!T.d_dem || !T.d_out) return fail(TVS_EINVAL, "tile %d: null d_dem or d_out", t);
        if (int rc = check_scalars(T.rows, T.cols, T.spacing, T.obs_height, n, T.max_dist)) {
            char msg[512];
            snprintf(msg, sizeof(msg), "tile %d: %s", t, g_err);
            return fail(rc, "%s", msg);
        }
    }
    return TVS_OK;
}

int check_batch_flags(uint32_t flags) {
    const uint32_t known = TVS_FLAG_SLOPE_F64 | TVS_FLAG_SLOPE_EXACT | TVS_FLAG_SLOPE_F32 | TVS_FLAG_COUNT_EVALS |
                           TVS_FLAG_AUTOTUNE | TVS_FLAG_COMPACT;
    if (flags & ~known)
        return fail(TVS_EINVAL, "unsupported flags 0x%x for a batch (the batched sweep always uses the early exit)",
                    flags);
    if ((flags & TVS_FLAG_SLOPE_F32) && (flags & TVS_FLAG_SLOPE_F64))
        return fail(TVS_EINVAL, "TVS_FLAG_SLOPE_F32 and TVS_FLAG_SLOPE_F64 exclude each other");
    return TVS_OK;
}

// Buckets of the batch's tiles (largest side first), each with its cached shape or the default.
void plan_buckets(tvs_batch *b) {
    std::map<std::pair<int, int>, int> idx;
    std::vector<std::pair<int, int>> keys(b->ntiles);
    for (int t = 0; t < b->ntiles; ++t) {
        const tvs_tile &T = b->tiles[t];
        const int side = std::max(T.rows, T.cols);
        int k = 0;
        for (const Sector &s : b->sectors[t]) k = std::max(k, std::min(s.K, std::max(s.Hx, s.Wx)));
        keys[t] = std::make_pair(-ceil_log2(side), ceil_log2(k + 1));
        idx[keys[t]] = 0;
    }
    for (auto &kv : idx) {
        kv.second = (int)b->buckets.size();
        Bucket bk{-kv.first.first, kv.first.second, 0, 0, 0, kDefaultShape, false};
        int a = 0, c = 0;
        if (tune_lookup(TuneKey{0, (int)b->f64, (int)b->rcp, bk.side_b, bk.rho_b}, a, c)) {
            bk.shape = Shape{a, c};
            bk.tuned = true;
        }
        b->buckets.push_back(bk);
    }
    b->tile_bucket.resize(b->ntiles);
    for (int t = 0; t < b->ntiles; ++t) {
        const int x = idx[keys[t]];
        b->tile_bucket[t] = x;
        Bucket &bk = b->buckets[x];
        const tvs_tile &T = b->tiles[t];
        bk.maxWx = std::max(bk.maxWx, std::max(T.rows, T.cols));
        for (const Sector &s : b->sectors[t]) bk.maxK = std::max(bk.maxK, std::min(s.K, std::max(s.Hx, s.Wx)));
        bk.ntiles += 1;
    }
}

// Sector groups of the batch: every tile's sectors [k0, k1) together, within the scratch budget
// and the item format (entries of a chunk < 2^16).
int plan_chunks(tvs_batch *b, size_t budget) {
    std::vector<int> pitch(b->ntiles);
    for (int t = 0; t < b->ntiles; ++t) pitch[t] = pitch_of(b->tiles[t].rows, b->tiles[t].cols);
    int k = 0;
    while (k < b->n) {
        ChunkPlan c{};
        c.k0 = c.k1 = k;
        while (c.k1 < b->n && (int64_t)b->ntiles * (c.k1 - c.k0 + 1) < 65536) {
            size_t add = 0;
            for (int t = 0; t < b->ntiles; ++t) add += (size_t)b->sectors[t][c.k1].prows * pitch[t] * 4;
            if (c.k1 > c.k0 && c.vbytes + add > budget) break;
            c.vbytes += add;
            ++c.k1;
        }
        if (c.k1 == c.k0) return fail(TVS_ENOMEM, "a batch of %d tiles is too large for one sector", b->ntiles);
        b->chunks.push_back(c);
        k = c.k1;
    }
    return TVS_OK;
}

// Device tables of every chunk: entries, back-projection tiles and work items.
void build_tables(tvs_batch *b, std::vector<BatchEnt> &ent, std::vector<BatchTile> &bt,
                  std::vector<uint32_t> &items) {
    std::vector<int> order(b->ntiles);
    for (int t = 0; t < b->ntiles; ++t) order[t] = t;
    // largest tiles first: their long rows start early, short rows fill the tail
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return (int64_t)b->tiles[x].rows * b->tiles[x].cols > (int64_t)b->tiles[y].rows * b->tiles[y].cols;
    });
    for (ChunkPlan &c : b->chunks) {
        const int nsec = c.k1 - c.k0;
        c.ent_off = ent.size();
        c.tile_off = bt.size();
        c.item_off = items.size();
        int64_t off = 0;
        int blk = 0;
        for (int t = 0; t < b->ntiles; ++t) {
            const tvs_tile &T = b->tiles[t];
            const int pitch = pitch_of(T.rows, T.cols);
            for (int x = 0; x < nsec; ++x) {
                const Sector &s = b->sectors[t][c.k0 + x];
                BatchEnt e;
                memset(&e, 0, sizeof(e));
                e.s.T = s.T;
                e.s.scale = s.scale;
                e.s.clip = s.clip;
                e.s.off = off;
                e.s.kase = s.kase;
                e.s.K = s.K;
                e.s.t0 = s.t0;
                e.s.nrows = s.nrows;
                e.s.wrap = s.wrap;
                e.s.winv = s.wrap ? 1.0f / (float)s.wrap : 0.0f;
                e.dem = T.d_dem;
                e.demT = b->demT.empty() ? nullptr : b->demT[t];
                e.H = T.rows;
                e.W = T.cols;
                e.pitch = pitch;
                e.h0 = T.obs_height;
                e.h0f = (float)T.obs_height;
                ent.push_back(e);
                off += (int64_t)s.prows * pitch;
            }
            BatchTile q;
            memset(&q, 0, sizeof(q));
            q.out = T.d_out;
            q.H = T.rows;
            q.W = T.cols;
            q.ent0 = t * nsec;
            q.bx = (T.cols + BATCH_BLOCK - 1) / BATCH_BLOCK;
            q.blk0 = blk;
            blk += q.bx * ((T.rows + BATCH_BLOCK - 1) / BATCH_BLOCK);
            bt.push_back(q);
        }
        c.nblocks = blk;
        c.bucket_items.assign(b->buckets.size(), 0);
        for (size_t bk = 0; bk < b->buckets.size(); ++bk) {
            const size_t before = items.size();
            for (int t : order) {
                if (b->tile_bucket[t] != (int)bk) continue;
                for (int x = 0; x < nsec; ++x) {
                    const int nr = b->sectors[t][c.k0 + x].nrows;
                    const uint32_t e = (uint32_t)(t * nsec + x);
                    for (int i = 0; i < nr; ++i) items.push_back((e << 16) | (uint32_t)middle_out(i, nr));
                }
            }
            c.bucket_items[bk] = (int)(items.size() - before);
        }
        c.nitems = (int)(items.size() - c.item_off);
    }
}

hipError_t enqueue_pass(tvs_batch *b, hipStream_t st) {
    hipError_t e;
    const size_t nb = b->buckets.size();
    if ((e = launch_divtab(b->tab32, b->tab64, b->tabN, st)) != hipSuccess) return e;
    if ((e = launch_fill_u32(b->counters, (int64_t)(b->chunks.size() * nb), 0u, st)) != hipSuccess) return e;
    b->launches = 2;
    if (b->transpose)
        for (int t = 0; t < b->ntiles; ++t) {
            const tvs_tile &T = b->tiles[t];
            if ((e = launch_transpose(T.d_dem, const_cast<float *>(b->demT[t]), T.rows, T.cols, st)) != hipSuccess)
                return e;
            ++b->launches;
        }
    if (b->count) {
        if ((e = launch_fill_u32((uint32_t *)b->work, 128, 0u, st)) != hipSuccess) return e;
        ++b->launches;
    }
    for (size_t ci = 0; ci < b->chunks.size(); ++ci) {
        const ChunkPlan &c = b->chunks[ci];
        size_t off = c.item_off;
        for (size_t bk = 0; bk < nb; ++bk) {
            const int cnt = c.bucket_items[bk];
            if (cnt == 0) continue;
            const Bucket &B = b->buckets[bk];
            const bool pers = b->persistent && B.shape.per_cu > 0;
            if ((e = launch_sweep_batch(b->ent + c.ent_off, b->items + off, cnt,
                                        pers ? b->counters + ci * nb + bk : nullptr, b->V, b->tab32, b->tab64,
                                        b->f64, b->rcp, B.shape.waves, pers ? b->cus * B.shape.per_cu : 1, B.maxWx,
                                        B.maxK, b->count ? b->work : nullptr, st)) != hipSuccess)
                return e;
            off += (size_t)cnt;
            ++b->launches;
        }
        if ((e = launch_backproj_batch(b->btiles + c.tile_off, b->ntiles, c.nblocks, b->ent + c.ent_off,
                                       c.k1 - c.k0, b->V, ci == 0, st)) != hipSuccess)
            return e;
        ++b->launches;
    }
    return hipSuccess;
}

// Times every candidate shape on a strided sample of each bucket's items in the first chunk (an
// eager pass first builds the reciprocal tables), keeps the fastest per bucket and remembers it.
int autotune(tvs_batch *b) {
    const ChunkPlan &c = b->chunks[0];
    std::vector<uint32_t> all((size_t)c.nitems);
    HIPCHK(hipMemcpy(all.data(), b->items + c.item_off, all.size() * 4, hipMemcpyDeviceToHost));
    uint32_t *d_sample = nullptr;
    HIPCHK(hipMalloc((void **)&d_sample, (size_t)16384 * 4 + 256));
    unsigned int *d_ctr = (unsigned int *)((char *)d_sample + (size_t)16384 * 4);
    const auto t0 = std::chrono::steady_clock::now();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = TVS_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        launch_divtab(b->tab32, b->tab64, b->tabN, b->cap) != hipSuccess)
        rc = fail(TVS_EDEVICE, "autotune set-up failed: %s", hipGetErrorString(hipGetLastError()));
    size_t off = 0;
    for (size_t bk = 0; bk < b->buckets.size() && rc == TVS_OK; ++bk) {
        Bucket &B = b->buckets[bk];
        const int cnt = c.bucket_items[bk];
        const size_t first = off;
        off += (size_t)cnt;
        if (cnt == 0) continue;
        const int stride = std::max(1, (cnt + 16383) / 16384);
        std::vector<uint32_t> sample;
        for (int i = 0; i < cnt; i += stride) sample.push_back(all[first + i]);
        if (hipMemcpy(d_sample, sample.data(), sample.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(TVS_EDEVICE, "autotune upload failed");
            break;
        }
        float best = 1e30f;
        Shape pick = B.shape;
        for (const Shape &sh : kCandidates) {
            float ms = 0.f;
            for (int rep = 0; rep < 2 && rc == TVS_OK; ++rep) {  // the first run warms the caches
                const bool pers = sh.per_cu > 0;
                if (launch_sweep_batch(nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, b->f64, b->rcp,
                                       sh.waves, 0, B.maxWx, B.maxK, nullptr, b->cap) != hipSuccess ||
                    launch_fill_u32(d_ctr, 1, 0u, b->cap) != hipSuccess || hipEventRecord(e0, b->cap) != hipSuccess ||
                    launch_sweep_batch(b->ent + c.ent_off, d_sample, (int)sample.size(), pers ? d_ctr : nullptr, b->V,
                                       b->tab32, b->tab64, b->f64, b->rcp, sh.waves, pers ? b->cus * sh.per_cu : 1,
                                       B.maxWx, B.maxK, nullptr, b->cap) != hipSuccess ||
                    hipEventRecord(e1, b->cap) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    rc = fail(TVS_EDEVICE, "autotune run failed: %s", hipGetErrorString(hipGetLastError()));
            }
            if (rc != TVS_OK) break;
            if (ms < best) {
                best = ms;
                pick = sh;
            }
        }
        if (rc != TVS_OK) break;
        B.shape = pick;
        B.tuned = true;
        tune_store(TuneKey{0, (int)b->f64, (int)b->rcp, B.side_b, B.rho_b}, pick.waves, pick.per_cu);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(b->cap);
    (void)hipFree(d_sample);
    if (rc != TVS_OK) return rc;
    b->tuned = true;
    b->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return TVS_OK;
}

int create(const tvs_tile *tiles, int ntiles, int n, uint32_t flags, tvs_batch *b) {
    b->ntiles = ntiles;
    b->n = n;
    b->flags = flags;
    b->f64 = (flags & TVS_FLAG_SLOPE_F32) == 0;
    b->rcp = (flags & (TVS_FLAG_SLOPE_EXACT | TVS_FLAG_SLOPE_F64)) == 0;
    b->count = (flags & TVS_FLAG_COUNT_EVALS) != 0;
    b->tiles.assign(tiles, tiles + ntiles);
    HIPCHK(hipGetDevice(&b->dev));
    for (int t = 0; t < ntiles; ++t) {
        const tvs_tile &T = tiles[t];
        std::vector<Sector> S;
        S.reserve(n);
        for (int k = 0; k < n; ++k) {
            S.push_back(plan_sector(k, n, T.rows, T.cols, T.spacing, T.max_dist));
            if (flags & TVS_FLAG_COMPACT) compact_layout(S.back());
        }
        for (const Sector &s : S) b->maxK = std::max(b->maxK, std::min(s.K, std::max(s.Hx, s.Wx)));
        b->sectors.push_back(std::move(S));
        b->maxWx = std::max(b->maxWx, std::max(T.rows, T.cols));
    }
    b->tabN = b->maxWx;
    if (sweep_lds_bytes(b->maxWx, b->f64) + 64 > (size_t)lds_limit(b->dev))
        return fail(TVS_ERANGE, "a skewed row of %d %s samples does not fit the workgroup LDS", b->maxWx,
                    b->f64 ? "double" : "float");
    b->cus = cu_count(b->dev);
    plan_buckets(b);
    if (int rc = plan_chunks(b, scratch_budget())) return rc;
    std::vector<BatchEnt> ent;
    std::vector<BatchTile> bt;
    std::vector<uint32_t> items;
    build_tables(b, ent, bt, items);
    size_t maxV = 0;
    for (const ChunkPlan &c : b->chunks) maxV = std::max(maxV, c.vbytes);
    const size_t nch = b->chunks.size();
    const size_t sz_tab32 = align256((size_t)b->tabN * sizeof(float2));
    const size_t sz_tab64 = align256((size_t)b->tabN * sizeof(double2));
    const size_t sz_ctr = align256(nch * b->buckets.size() * sizeof(unsigned int));
    const size_t sz_work = align256(64 * sizeof(unsigned long long));
    const size_t sz_ent = align256(ent.size() * sizeof(BatchEnt));
    const size_t sz_bt = align256(bt.size() * sizeof(BatchTile));
    const size_t sz_items = align256(items.size() * sizeof(uint32_t));
    size_t sz_demT = 0;
    if (n >= 2)  // sectors of the 45..135 deg axes read the tiles' transposed grids
        for (int t = 0; t < ntiles; ++t) sz_demT += align256((size_t)tiles[t].rows * tiles[t].cols * sizeof(float));
    b->dbytes = sz_tab32 + sz_tab64 + sz_ctr + sz_work + sz_ent + sz_bt + sz_items + sz_demT + align256(maxV);
    if (hipMalloc((void **)&b->dmem, b->dbytes) != hipSuccess) {
        (void)hipGetLastError();
        b->dmem = nullptr;
        return fail(TVS_ENOMEM, "batch device memory of %zu bytes not available", b->dbytes);
    }
    char *p = b->dmem;
    b->tab32 = (float2 *)p; p += sz_tab32;
    b->tab64 = (double2 *)p; p += sz_tab64;
    b->counters = (unsigned int *)p; p += sz_ctr;
    b->work = (unsigned long long *)p; p += sz_work;
    b->ent = (BatchEnt *)p; p += sz_ent;
    b->btiles = (BatchTile *)p; p += sz_bt;
    b->items = (uint32_t *)p; p += sz_items;
    if (sz_demT) {
        b->transpose = true;
        for (int t = 0; t < ntiles; ++t) {
            b->demT.push_back((const float *)p);
            p += align256((size_t)tiles[t].rows * tiles[t].cols * sizeof(float));
        }
        for (const ChunkPlan &c : b->chunks)  // tile t's sectors of chunk c follow its ent_off + t * nsec
            for (int t = 0; t < ntiles; ++t)
                for (int x = 0; x < c.k1 - c.k0; ++x) ent[c.ent_off + (size_t)t * (c.k1 - c.k0) + x].demT = b->demT[t];
    }
    b->V = (uint32_t *)p;
    HIPCHK(hipMemcpy(b->ent, ent.data(), ent.size() * sizeof(BatchEnt), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->btiles, bt.data(), bt.size() * sizeof(BatchTile), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->items, items.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(b->work, 0, 64 * sizeof(unsigned long long)));
    HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));

    if (flags & TVS_FLAG_AUTOTUNE) {
        if (int rc = autotune(b)) return rc;
    } else {
        for (const Bucket &B : b->buckets) b->tuned |= B.tuned;  // shapes remembered from earlier timing
    }
    // raise the sweeps' LDS limits before capture (no attribute calls inside a graph)
    for (const Bucket &B : b->buckets)
        HIPCHK(launch_sweep_batch(nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, b->f64, b->rcp,
                                  B.shape.waves, 0, B.maxWx, B.maxK, nullptr, b->cap));
    HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const hipError_t le = enqueue_pass(b, b->cap);
    const hipError_t ce = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess) return fail(TVS_EDEVICE, "batch capture: %s", hipGetErrorString(le));
    if (ce != hipSuccess) return fail(TVS_EDEVICE, "batch capture: %s", hipGetErrorString(ce));
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return TVS_OK;
}

}  // namespace

namespace tvs {
namespace host {

bool batch_rows_fit(int maxWx, bool f64) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    return sweep_lds_bytes(maxWx, f64) + 64 <= (size_t)lds_limit(dev);
}

// A batch enqueued once on a stream, without a graph (the request server's groups of total requests):
// the same plan, work lists and launches as a captured batch pass. The work lists go through the
// caller's pinned staging buffer (grown here; the caller keeps it untouched until the stream has
// passed this work), the device memory is taken and returned stream-ordered on `st`.
int batch_enqueue(const tvs_tile *tiles, const float *const *demT, int ntiles, int n, uint32_t flags, hipStream_t st,
                  size_t budget, PinnedStaging &stage, int *out_chunks) {
    tvs_batch b;
    b.persistent = false;  // other work (the server's singular launches) interleaves with its workgroups
    if (demT) b.demT.assign(demT, demT + ntiles);
    b.ntiles = ntiles;
    b.n = n;
    b.flags = flags;
    b.f64 = (flags & TVS_FLAG_SLOPE_F32) == 0;
    b.rcp = (flags & (TVS_FLAG_SLOPE_EXACT | TVS_FLAG_SLOPE_F64)) == 0;
    b.tiles.assign(tiles, tiles + ntiles);
    HIPCHK(hipGetDevice(&b.dev));
    for (int t = 0; t < ntiles; ++t) {
        const tvs_tile &T = tiles[t];
        std::vector<Sector> S;
        S.reserve(n);
        for (int k = 0; k < n; ++k) S.push_back(plan_sector(k, n, T.rows, T.cols, T.spacing, T.max_dist));
        for (const Sector &x : S) b.maxK = std::max(b.maxK, std::min(x.K, std::max(x.Hx, x.Wx)));
        b.sectors.push_back(std::move(S));
        b.maxWx = std::max(b.maxWx, std::max(T.rows, T.cols));
    }
    b.tabN = b.maxWx;
    if (!batch_rows_fit(b.maxWx, b.f64))
        return fail(TVS_ERANGE, "a skewed row of %d samples does not fit the workgroup LDS", b.maxWx);
    b.cus = cu_count(b.dev);
    plan_buckets(&b);
    if (int rc = plan_chunks(&b, budget)) return rc;
    std::vector<BatchEnt> ent;
    std::vector<BatchTile> bt;
    std::vector<uint32_t> items;
    build_tables(&b, ent, bt, items);
    size_t maxV = 0;
    for (const ChunkPlan &c : b.chunks) maxV = std::max(maxV, c.vbytes);
    const size_t nch = b.chunks.size();
    const size_t sz_ent = align256(ent.size() * sizeof(BatchEnt)), sz_bt = align256(bt.size() * sizeof(BatchTile)),
                 sz_items = align256(items.size() * sizeof(uint32_t));
    const size_t sz_tab32 = align256((size_t)b.tabN * sizeof(float2)), sz_tab64 = align256((size_t)b.tabN * sizeof(double2)),
                 sz_ctr = align256(nch * b.buckets.size() * sizeof(unsigned int));
    const size_t host_bytes = sz_ent + sz_bt + sz_items;
    if (stage.cap < host_bytes) {
        const size_t want = std::max(host_bytes, (size_t)2 * stage.cap);
        if (stage.p) stage.retired.push_back(stage.p);
        stage.p = nullptr;
        stage.cap = 0;
        HIPCHK(hipHostMalloc(&stage.p, want, hipHostMallocDefault));
        stage.cap = want;
    }
    char *h = (char *)stage.p;
    memcpy(h, ent.data(), ent.size() * sizeof(BatchEnt));
    memcpy(h + sz_ent, bt.data(), bt.size() * sizeof(BatchTile));
    memcpy(h + sz_ent + sz_bt, items.data(), items.size() * sizeof(uint32_t));
    const size_t dev_bytes = host_bytes + sz_tab32 + sz_tab64 + sz_ctr + align256(maxV);
    char *d = nullptr;
    if (hipMallocAsync((void **)&d, dev_bytes, st) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TVS_ENOMEM, "batch device memory of %zu bytes not available", dev_bytes);
    }
    b.ent = (BatchEnt *)d;
    b.btiles = (BatchTile *)(d + sz_ent);
    b.items = (uint32_t *)(d + sz_ent + sz_bt);
    b.tab32 = (float2 *)(d + host_bytes);
    b.tab64 = (double2 *)(d + host_bytes + sz_tab32);
    b.counters = (unsigned int *)(d + host_bytes + sz_tab32 + sz_tab64);
    b.V = (uint32_t *)(d + host_bytes + sz_tab32 + sz_tab64 + sz_ctr);
    b.work = nullptr;
    hipError_t e = hipMemcpyAsync(d, h, host_bytes, hipMemcpyHostToDevice, st);
    for (const Bucket &B : b.buckets)
        if (e == hipSuccess)
            e = launch_sweep_batch(nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, b.f64, b.rcp, B.shape.waves,
                                   0, B.maxWx, B.maxK, nullptr, st);
    if (e == hipSuccess) e = enqueue_pass(&b, st);
    const hipError_t fe = hipFreeAsync(d, st);
    if (e != hipSuccess) return fail(TVS_EDEVICE, "batch launch: %s", hipGetErrorString(e));
    if (fe != hipSuccess) return fail(TVS_EDEVICE, "batch scratch release: %s", hipGetErrorString(fe));
    if (out_chunks) *out_chunks = (int)nch;
    return TVS_OK;
}

// One tile's share of batch_enqueue's device memory: its skewed viewshed rows over all sectors and its
// work items and entries.
BatchSize batch_tile_size(const tvs_tile &T, int n) {
    BatchSize z;
    z.maxWx = std::max(T.rows, T.cols);
    const int pitch = pitch_of(T.rows, T.cols);
    size_t nrows = 0;
    for (int k = 0; k < n; ++k) {
        const Sector s = plan_sector(k, n, T.rows, T.cols, T.spacing, T.max_dist);
        z.vbytes += (size_t)s.prows * pitch * 4;
        nrows += (size_t)s.nrows;
    }
    z.tables = (size_t)n * (sizeof(BatchEnt) + 256) + sizeof(BatchTile) + nrows * sizeof(uint32_t);
    return z;
}

// Device memory batch_enqueue takes for tiles of these summed sizes (beyond their maps), an upper bound.
size_t batch_scratch_bytes(const BatchSize &sum, size_t budget) {
    return sum.tables + (size_t)sum.maxWx * 24 + 64 * 256 + std::min(sum.vbytes, std::max(budget, (size_t)1));
}

}  // namespace host
}  // namespace tvs

extern "C" {

int tvs_batch_create(const tvs_tile *tiles, int32_t ntiles, int32_t n_sectors, uint32_t flags,
                     tvs_batch **out_batch) {
    g_err[0] = 0;
    if (!out_batch) return fail(TVS_EINVAL, "null out_batch");
    if (n_sectors < 1 || n_sectors > TVS_MAX_SECTORS)
        return fail(TVS_EINVAL, "n_sectors must be in [1, %d]", TVS_MAX_SECTORS);
    if (int rc = check_batch_flags(flags)) return rc;
    if (int rc = check_tiles(tiles, ntiles, n_sectors)) return rc;
    tvs_batch *b = new (std::nothrow) tvs_batch;
    if (!b) return fail(TVS_ENOMEM, "host memory for the batch plan");
    const int rc = create(tiles, ntiles, n_sectors, flags, b);
    if (rc != TVS_OK) {
        delete b;
        return rc;
    }
    *out_batch = b;
    return TVS_OK;
}

int tvs_batch_run(tvs_batch *batch, void *hip_stream) {
    g_err[0] = 0;
    if (!batch || !batch->exec) return fail(TVS_EINVAL, "null or unbuilt batch");
    HIPCHK(hipGraphLaunch(batch->exec, (hipStream_t)hip_stream));
    return TVS_OK;
}

int tvs_batch_get_info(const tvs_batch *batch, tvs_batch_info *info) {
    g_err[0] = 0;
    if (!batch || !info) return fail(TVS_EINVAL, "null batch or info");
    tvs_batch *b = const_cast<tvs_batch *>(batch);
    if (!b->counted) {
        for (int t = 0; t < b->ntiles; ++t)
            for (const Sector &s : b->sectors[t]) count_sector(s, b->evals, b->pairs);
        b->counted = true;
    }
    memset(info, 0, sizeof(*info));
    info->tiles = b->ntiles;
    info->chunks = (int32_t)b->chunks.size();
    info->kernel_launches = b->launches;
    info->waves_per_group = b->buckets[0].shape.waves;  // the bucket of the largest tiles
    info->groups = b->buckets[0].shape.per_cu ? b->cus * b->buckets[0].shape.per_cu : 0;
    info->buckets = (int32_t)b->buckets.size();
    info->tuned = b->tuned ? 1 : 0;
    info->los_evals = b->evals;
    info->pov_sector_pairs = b->pairs;
    info->scratch_bytes = (int64_t)b->dbytes;
    info->tune_ms = b->tune_ms;
    if (b->count) {
        unsigned long long h[64];
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(h, b->work, sizeof(h), hipMemcpyDeviceToHost));
        for (int x = 0; x < 64; ++x) info->sweep_evals_done += (int64_t)h[x];
    }
    return TVS_OK;
}

int tvs_batch_get_bucket(const tvs_batch *batch, int32_t i, tvs_batch_bucket *out) {
    g_err[0] = 0;
    if (!batch || !out) return fail(TVS_EINVAL, "null batch or out");
    if (i < 0 || i >= (int)batch->buckets.size())
        return fail(TVS_EINVAL, "bucket %d outside [0, %d)", i, (int)batch->buckets.size());
    const Bucket &B = batch->buckets[i];
    memset(out, 0, sizeof(*out));
    out->side_class = B.side_b;
    out->reach_class = B.rho_b;
    out->tiles = B.ntiles;
    out->longest_side = B.maxWx;
    out->longest_reach = B.maxK;
    out->waves_per_group = B.shape.waves;
    out->groups_per_cu = B.shape.per_cu;
    out->tuned = B.tuned ? 1 : 0;
    for (const ChunkPlan &c : batch->chunks) out->items += c.bucket_items[i];
    return TVS_OK;
}

int tvs_batch_destroy(tvs_batch *batch) {
    g_err[0] = 0;
    delete batch;
    return TVS_OK;
}

}  // extern "C"
