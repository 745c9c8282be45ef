// tvs_api.hip -- C ABI of libtvs: validation, the per-sector plan, scratch management and the
// launch sequence of the sDEM total viewshed (Section 4.1 steps 1a-1d with the three kernels
// of Section 4.2) and of the singular viewshed (Alg. 1).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cstring>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/libtvs.h"
#include "tvs_geom.h"
#include "tvs_internal.h"
#include "tvs_host.h"

using namespace tvs;

namespace tvs {
namespace host {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

// Sector k of n (Section 3.1 axes; base-frame cases of the kernels' 0..45 deg range).
Sector plan_sector(int k, int n, int H, int W, double dx, double R) {
    Sector s;
    long long num, den;
    if (4LL * k <= n) {
        s.kase = 0; num = k; den = n;
    } else if (4LL * k <= 2LL * n) {
        s.kase = 1; num = n - 2LL * k; den = 2LL * n;
    } else if (4LL * k < 3LL * n) {
        s.kase = 2; num = 2LL * k - n; den = 2LL * n;
    } else {
        s.kase = 3; num = n - k; den = n;
    }
    frame_dims(s.kase, H, W, s.Hx, s.Wx);
    const double sp = (M_PI * (double)num) / (double)den;
    if (num == 0) s.T = 0.0;
    else if (4 * num == den) s.T = 1.0;
    else s.T = tan(sp);
    const double c = cos(sp);
    s.c = c;
    s.scale = (M_PI / (2.0 * (double)n)) * (dx * dx) / (c * c);
    s.K = TVS_K_UNBOUNDED;
    s.clip = 0.0;
    if (isinf(R)) {
        s.rho = INFINITY;
    } else {
        s.rho = (R * c) / dx;
        const double kk = ceil(s.rho) - 1.0;
        if (kk < (double)TVS_K_UNBOUNDED) {
            s.K = (int)kk;
            s.clip = s.rho * s.rho - (double)s.K * (double)s.K;
        }
    }
    int dmax;
    double rmax;
    col_offset(s.T, s.Wx - 1, dmax, rmax);
    s.t0 = -dmax - 1;
    s.nrows = s.Hx - s.t0;
    s.wrap = 0;
    s.prows = s.nrows;
    return s;
}

// Skewed row t holds the samples of the columns with -1 < t + y_j < Hx (Section 3.1, Algorithm 6),
// row t + Hx + 1 those with -1 - t - Hx - 1 < y_j < -1 - t: disjoint column ranges. Rows congruent
// modulo Hx + 1 therefore share one stored row, and the rows t0 .. Hx - 1 fit Hx + 1 rows.
void compact_layout(Sector &s) {
    s.wrap = s.Hx + 1;
    s.prows = std::min(s.nrows, s.wrap);
}

// Elevations and the observer height must be finite, and either 0 or at least 2^-60 m in
// magnitude. The second rule keeps every quantity of the sweep a multiple of 2^-83, so no slope
// underflows to a signed zero (the kernels read strict comparisons from sign bits).

bool magnitude_ok(double v) { return v == 0.0 || fabs(v) >= TVS_MIN_MAGNITUDE; }

int check_scalars(int rows, int cols, double dx, double h0, int n, double R) {
    if (rows < 1 || cols < 1) return fail(TVS_EINVAL, "rows and cols must be >= 1 (got %d x %d)", rows, cols);
    if (rows > TVS_MAX_SIDE || cols > TVS_MAX_SIDE)
        return fail(TVS_ERANGE, "grid %d x %d exceeds the %d-cell side limit", rows, cols, TVS_MAX_SIDE);
    if (!(dx > 0.0) || !isfinite(dx)) return fail(TVS_EINVAL, "spacing must be finite and > 0");
    if (!isfinite(h0) || !magnitude_ok(h0)) return fail(TVS_EINVAL, "obs_height must be finite, and 0 or >= 2^-60 m");
    if (n < 1 || n > TVS_MAX_SECTORS) return fail(TVS_EINVAL, "n_sectors must be in [1, %d]", TVS_MAX_SECTORS);
    if (isnan(R) || !(R > 0.0)) return fail(TVS_EINVAL, "max_dist must be > 0 (INFINITY allowed)");
    return TVS_OK;
}

int check_host_dem(const float *dem, int rows, int cols) {
    const int64_t N = (int64_t)rows * cols;
    // a vectorisable pass on the bit patterns first: a non-finite value has exponent field 255; a
    // nonzero magnitude below 2^-60 has a biased exponent below 127 - 60
    uint32_t bad = 0;
    for (int64_t x = 0; x < N; ++x) {
        uint32_t u;
        memcpy(&u, dem + x, sizeof(u));
        const uint32_t e = (u >> 23) & 0xFFu;
        bad |= (uint32_t)(e == 0xFFu) | ((uint32_t)(e < 67u) & (uint32_t)((u & 0x7FFFFFFFu) != 0u));
    }
    if (!bad) return TVS_OK;
    for (int64_t x = 0; x < N; ++x)
        if (!isfinite(dem[x]) || !magnitude_ok(dem[x]))
            return fail(TVS_EINVAL, "elevation %g at cell (%lld, %lld) is not finite, or is nonzero below 2^-60 m",
                        (double)dem[x], (long long)(x / cols), (long long)(x % cols));
    return TVS_OK;
}

int check_flags(uint32_t flags, bool accumulation) {
    const uint32_t known = TVS_FLAG_SLOPE_F64 | TVS_FLAG_SWEEP_SCAN | TVS_FLAG_SLOPE_EXACT | TVS_FLAG_NO_PRUNE |
                           TVS_FLAG_SLOPE_F32 | TVS_FLAG_RELOCATE |
                           (accumulation ? TVS_FLAG_ACC_KAHAN32 | TVS_FLAG_COUNT_EVALS | TVS_FLAG_COMPACT |
                                               TVS_FLAG_AUTOTUNE
                                         : 0u);
    if (flags & ~known) return fail(TVS_EINVAL, "unsupported flags 0x%x", flags);
    if ((flags & TVS_FLAG_SLOPE_F32) && (flags & TVS_FLAG_SLOPE_F64))
        return fail(TVS_EINVAL, "TVS_FLAG_SLOPE_F32 and TVS_FLAG_SLOPE_F64 exclude each other");
    return TVS_OK;
}

// Sector k's row extents on the host (same predicates as the kernels) -> evals / pairs.
void count_sector(const Sector &s, int64_t &evals, int64_t &pairs) {
    for (int ri = 0; ri < s.nrows; ++ri) {
        const int t = s.t0 + ri;
        const int nt = row_last(s.T, t, s.Hx, s.Wx) - row_first(s.T, t, s.Hx, s.Wx) + 1;
        if (nt <= 0) continue;
        pairs += nt;
        const int64_t K = s.K;
        if (K >= nt - 1) {
            evals += (int64_t)nt * (nt - 1);
        } else {
            evals += 2 * (K * (K - 1) / 2 + (int64_t)(nt - K) * K);
        }
    }
}

int pitch_of(int H, int W) { return ((std::max(H, W) + 63) / 64) * 64; }

size_t scratch_budget() {
    const char *env = getenv("TVS_SCRATCH_MB");
    if (env && *env) return (size_t)atoll(env) << 20;
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) return (size_t)4 << 30;
    return std::min(freeb / 2, (size_t)16 << 30);
}

void pool_keep_memory(int dev) {
    static std::atomic<bool> done[64];  // calls come from any thread (the request server's included)
    if (dev < 0 || dev >= 64 || done[dev].load(std::memory_order_acquire)) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    done[dev].store(true, std::memory_order_release);
}

int lds_limit(int dev) {
    int v = 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || v <= 0) {
        v = 65536;
        (void)hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    }
    return v;
}

}  // namespace host
}  // namespace tvs

using namespace tvs::host;

namespace {

// Groups of consecutive sectors: at most TVS_CHUNK each, scratch within the budget.
struct Chunk {
    int k0, k1;        // [k0, k1)
    size_t bytes;      // skewed buffers of the chunk
    int maxRows, maxWx;
};

std::vector<Chunk> make_chunks(const std::vector<Sector> &S, size_t elem, int pitch, size_t budget) {
    std::vector<Chunk> out;
    int k = 0;
    const int n = (int)S.size();
    // as few chunks as TVS_CHUNK allows, of even size (180 sectors: 3 x 60, not 72 + 72 + 36)
    const int per = n > 0 ? (n + (n + TVS_CHUNK - 1) / TVS_CHUNK - 1) / ((n + TVS_CHUNK - 1) / TVS_CHUNK) : 1;
    while (k < n) {
        Chunk c{k, k, 0, 0, 0};
        while (c.k1 < n && c.k1 - c.k0 < per) {
            const size_t b = (size_t)S[c.k1].prows * pitch * (elem + sizeof(uint32_t));
            if (c.k1 > c.k0 && c.bytes + b > budget) break;
            c.bytes += b;
            c.maxRows = std::max(c.maxRows, S[c.k1].nrows);
            c.maxWx = std::max(c.maxWx, S[c.k1].Wx);
            ++c.k1;
        }
        out.push_back(c);
        k = c.k1;
    }
    return out;
}

ChunkArgs chunk_args(const std::vector<Sector> &S, const Chunk &c, int H, int W, int pitch, double h0) {
    ChunkArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nsec = c.k1 - c.k0;
    a.H = H;
    a.W = W;
    a.pitch = pitch;
    a.h0 = h0;
    a.h0f = (float)h0;
    a.k_base = c.k0;
    int64_t off = 0;
    for (int x = 0; x < a.nsec; ++x) {
        const Sector &s = S[c.k0 + x];
        SecDev &d = a.s[x];
        d.T = s.T;
        d.scale = s.scale;
        d.clip = s.clip;
        d.off = off;
        d.kase = s.kase;
        d.K = s.K;
        d.t0 = s.t0;
        d.nrows = s.nrows;
        d.wrap = s.wrap;
        d.winv = s.wrap ? 1.0f / (float)s.wrap : 0.0f;
        off += (int64_t)s.prows * pitch;
    }
    return a;
}

// Stream-ordered device scratch, released when the stream reaches the free.
struct Scratch {
    void *p = nullptr;
    hipStream_t st = nullptr;
    ~Scratch() {
        if (p) (void)hipFreeAsync(p, st);
    }
};

// Timing of launches with events on the call's stream (only when stats are requested).
struct Timer {
    bool on = false;
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;  // 0 reloc, 1 sweep, 2 backproj
    ~Timer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipError_t mark() {
        if (!on) return hipSuccess;
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ev.push_back(e);
        return hipEventRecord(e, st);
    }
    hipError_t begin(int k) {
        if (on) kind.push_back(k);
        return mark();
    }
};

// Waves per workgroup of the lane-per-POV sweep for this call: with TVS_FLAG_AUTOTUNE, timed on up
// to four sectors spread over the axes (4, 8 and 16 waves; the skewed viewshed buffer is written and
// later overwritten) and remembered; otherwise a remembered choice for the same size class, or 0
// (the launcher's choice from the LDS a row takes). Negative: a failure status.
int sweep_shape(const std::vector<Sector> &S, const std::vector<Chunk> &chunks, int H, int W, int pitch, double h0,
                uint32_t flags, const float *dem, const float *demT, char *scratch, size_t scratch_bytes,
                const float2 *tab32, const double2 *tab64, hipStream_t st, bool fused, bool f64, bool scan, bool rcp,
                bool prune, bool noalloc) {
    if (scan || noalloc || S.empty()) return 0;
    int maxWx = 0, maxK = 0;
    for (const Sector &s : S) {
        maxWx = std::max(maxWx, s.Wx);
        maxK = std::max(maxK, std::min(s.K, s.Wx));
    }
    if (!sweep_row_fits(maxWx, f64)) return 0;
    const TuneKey key{1, (int)f64, (int)rcp, ceil_log2(maxWx), ceil_log2(maxK + 1)};
    int a = 0, b = 0;
    if (!(flags & TVS_FLAG_AUTOTUNE)) return tune_lookup(key, a, b) ? a : 0;
    // a sample of sectors spread over the axes that fits the skewed buffers
    const size_t elem = fused ? 0 : (f64 ? sizeof(double) : sizeof(float));
    std::vector<Sector> smp;
    size_t bytes = 0;
    const int n = (int)S.size();
    for (int i = 0; i < 4; ++i) {
        const Sector &s = S[(size_t)i * n / 4];
        const size_t add = (size_t)s.prows * pitch * (elem + sizeof(uint32_t));
        if (!smp.empty() && (bytes + add > scratch_bytes || smp.size() >= (size_t)TVS_CHUNK)) break;
        if (i > 0 && (size_t)i * n / 4 == (size_t)(i - 1) * n / 4) continue;
        smp.push_back(s);
        bytes += add;
    }
    Chunk c{0, (int)smp.size(), bytes, 0, 0};
    for (const Sector &s : smp) {
        c.maxRows = std::max(c.maxRows, s.nrows);
        c.maxWx = std::max(c.maxWx, s.Wx);
    }
    ChunkArgs ca = chunk_args(smp, c, H, W, pitch, h0);
    const int64_t elems = (int64_t)(bytes / (elem + sizeof(uint32_t)));
    void *skw = fused ? nullptr : scratch;
    uint32_t *V = (uint32_t *)(scratch + (size_t)elems * elem);
    if (!fused) HIPCHK(launch_relocate(ca, c.maxWx, c.maxRows, dem, skw, f64, st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(TVS_EDEVICE, "event creation failed");
    }
    float best = 1e30f;
    int pick = 0;
    int rc = TVS_OK;
    for (int cand : {4, 8, 16}) {
        float ms = 0.f;
        for (int rep = 0; rep < 2 && rc == TVS_OK; ++rep)  // the first run warms the caches
            if (hipEventRecord(e0, st) != hipSuccess ||
                launch_sweep(ca, c.maxWx, dem, demT, skw, V, tab32, tab64, f64, false, rcp, prune, nullptr,
                             st, cand) != hipSuccess ||
                hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = fail(TVS_EDEVICE, "sweep shape timing failed: %s", hipGetErrorString(hipGetLastError()));
        if (rc != TVS_OK) break;
        if (ms < best) {
            best = ms;
            pick = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TVS_OK) return rc;
    tune_store(key, pick, 0);
    return pick;
}

// The total viewshed on the device: one chunk of sectors at a time, sweep (each workgroup gathering
// its skewed row from the grid; with TVS_FLAG_RELOCATE a relocation launch writes skwDEM first) ->
// back-projection, the per-cell sum carried in d_out (double) or in float Kahan scratch.
// With `fixed` non-null the call takes no device memory of its own: every buffer is carved from the
// `fixed_bytes` at `fixed` (the allocation-free entry point's static array), the skewed buffers use
// the compacted layout, and sector chunks are sized to fit; a sector that alone does not fit is
// rejected with TVS_ERANGE before anything is enqueued.
// With check_dem the grid's elevations are checked on the device (entry points that take device grids
// and never read them on the host): a grid that breaks the rule gives a map of NaN.
int run_total(const float *d_dem, int H, int W, double dx, double h0, int n, double R, double *d_out,
              uint32_t flags, tvs_stats *stats, hipStream_t st, int debug_sector, uint32_t *d_debugV,
              int *debug_pitch, size_t budget = 0, void *fixed = nullptr, size_t fixed_bytes = 0,
              bool check_dem = false) {
    const bool f64 = (flags & TVS_FLAG_SLOPE_F32) == 0;
    const bool scan = (flags & TVS_FLAG_SWEEP_SCAN) != 0;
    const bool kahan = (flags & TVS_FLAG_ACC_KAHAN32) != 0;
    const bool rcp = (flags & (TVS_FLAG_SLOPE_EXACT | TVS_FLAG_SLOPE_F64)) == 0;
    const bool prune = (flags & TVS_FLAG_NO_PRUNE) == 0;
    const bool count = (flags & TVS_FLAG_COUNT_EVALS) != 0;
    const bool fused = (flags & TVS_FLAG_RELOCATE) == 0;
    if (count && !stats) return fail(TVS_EINVAL, "TVS_FLAG_COUNT_EVALS needs a stats argument");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (!fixed) pool_keep_memory(dev);
    const int pitch = pitch_of(H, W);
    const size_t elem = f64 ? sizeof(double) : sizeof(float);
    const size_t skwElem = fused ? 0 : elem;  // bytes per sample of skwDEM
    if (scan && !sweep_row_fits(std::max(H, W), f64))
        return fail(TVS_ERANGE, "the lane-per-target sweep holds whole rows: %d %s samples do not fit the workgroup "
                    "LDS (%d bytes)", std::max(H, W), f64 ? "double" : "float", lds_limit(dev));

    std::vector<Sector> S;
    if (debug_sector >= 0) S.push_back(plan_sector(debug_sector, n, H, W, dx, R));  // plain rows, copied out
    else
        for (int k = 0; k < n; ++k) {
            S.push_back(plan_sector(k, n, H, W, dx, R));
            if ((flags & TVS_FLAG_COMPACT) || fixed) compact_layout(S.back());
        }
    // the gathering sweep reads the 45..135 deg frames from the transposed grid
    bool needT = false;
    for (const Sector &s : S) needT |= fused && (s.kase == 1 || s.kase == 2);
    const size_t demTBytes = needT ? (size_t)H * W * sizeof(float) : 0;
    const int tabN = std::max(H, W);  // entries for m = 1 .. max(H, W)
    const size_t tabBytes = (size_t)tabN * (sizeof(float2) + sizeof(double2));
    const size_t kahanBytes = kahan ? (size_t)H * W * 2 * sizeof(float) : 0;
    constexpr int kWorkSlots = 64;  // evaluation counters of the sweep (TVS_FLAG_COUNT_EVALS)
    // every carved piece is rounded up to 256 bytes: at most 7 pieces besides the skewed buffers
    const size_t fixedParts = tabBytes + kahanBytes + demTBytes + 256 * 4 + kWorkSlots * 8 + 256 + 8 * 256;
    if (fixed && fixed_bytes <= fixedParts)
        return fail(TVS_ERANGE, "tables of a %d x %d grid (%zu bytes) exceed the %zu-byte allocation-free scratch",
                    H, W, fixedParts, fixed_bytes);
    const size_t chunkBudget = fixed ? fixed_bytes - fixedParts : budget ? budget : scratch_budget();
    const std::vector<Chunk> chunks = make_chunks(S, skwElem, pitch, chunkBudget);
    size_t maxChunk = 0;
    for (const Chunk &c : chunks) maxChunk = std::max(maxChunk, c.bytes);
    if (fixed && maxChunk > chunkBudget)
        return fail(TVS_ERANGE,
                    "one sector of a %d x %d grid needs %zu bytes of skewed buffers; the allocation-free scratch "
                    "holds %zu",
                    H, W, maxChunk, chunkBudget);
    const size_t total = fixedParts + maxChunk;

    Scratch scr;
    scr.st = st;
    if (fixed) {
        scr.p = nullptr;  // not owned: nothing to free
    } else if (hipMallocAsync(&scr.p, total, st) != hipSuccess) {
        (void)hipGetLastError();
        scr.p = nullptr;
        return fail(TVS_ENOMEM, "device scratch of %zu bytes not available", total);
    }
    char *base = fixed ? (char *)fixed : (char *)scr.p;
    auto carve = [&](size_t b) {
        char *p = base;
        base += (b + 255) & ~(size_t)255;
        return (void *)p;
    };
    float2 *tab32 = (float2 *)carve((size_t)tabN * sizeof(float2));
    double2 *tab64 = (double2 *)carve((size_t)tabN * sizeof(double2));
    float *ksum = kahan ? (float *)carve((size_t)H * W * sizeof(float)) : nullptr;
    float *kc = kahan ? (float *)carve((size_t)H * W * sizeof(float)) : nullptr;
    unsigned long long *work = count ? (unsigned long long *)carve(kWorkSlots * 8) : nullptr;
    float *demT = needT ? (float *)carve(demTBytes) : nullptr;
    uint32_t *bad = (uint32_t *)carve(256);
    char *skwV = (char *)carve(maxChunk);

    Timer tm;
    tm.on = stats != nullptr;
    tm.st = st;
    HIPCHK(launch_divtab(tab32, tab64, tabN, st));
    if (work) HIPCHK(launch_fill_u32((uint32_t *)work, 2 * kWorkSlots, 0u, st));
    const bool check = check_dem && d_out;
    if (check) {
        HIPCHK(launch_fill_u32(bad, 1, 0u, st));
        HIPCHK(launch_check_dem(d_dem, (int64_t)H * W, bad, st));
    }
    if (needT) {
        HIPCHK(tm.begin(0));
        HIPCHK(launch_transpose(d_dem, demT, H, W, st));
        HIPCHK(tm.mark());
    }
    const int nw = sweep_shape(S, chunks, H, W, pitch, h0, flags, d_dem, demT, skwV, maxChunk, tab32, tab64, st,
                               fused, f64, scan, rcp, prune, fixed != nullptr);
    if (nw < 0) return nw;
    int64_t evals = 0, pairs = 0;
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        const Chunk &c = chunks[ci];
        ChunkArgs a = chunk_args(S, c, H, W, pitch, h0);
        const int64_t elems = (int64_t)(c.bytes / (skwElem + sizeof(uint32_t)));
        void *skw = fused ? nullptr : skwV;
        uint32_t *V = (uint32_t *)(skwV + (size_t)elems * skwElem);
        if (d_debugV) HIPCHK(launch_fill_u32(V, elems, 0xFFFFFFFFu, st));
        if (!fused) {
            HIPCHK(tm.begin(0));
            HIPCHK(launch_relocate(a, c.maxWx, c.maxRows, d_dem, skw, f64, st));
            HIPCHK(tm.mark());
        }
        HIPCHK(tm.begin(1));
        HIPCHK(launch_sweep(a, c.maxWx, d_dem, demT, skw, V, tab32, tab64, f64, scan, rcp, prune, work,
                            st, nw));
        HIPCHK(tm.mark());
        if (d_debugV) {
            const Sector &s = S[0];
            HIPCHK(hipMemcpy2DAsync(d_debugV, (size_t)s.Wx * 4, V, (size_t)pitch * 4, (size_t)s.Wx * 4,
                                    (size_t)s.nrows, hipMemcpyDeviceToDevice, st));
            if (debug_pitch) *debug_pitch = pitch;
            continue;
        }
        HIPCHK(tm.begin(2));
        HIPCHK(launch_backproj(a, V, d_out, ksum, kc, ci == 0, ci + 1 == chunks.size(), st));
        HIPCHK(tm.mark());
        if (stats)
            for (int k = c.k0; k < c.k1; ++k) count_sector(S[k], evals, pairs);
    }
    if (check) HIPCHK(launch_poison(d_out, (int64_t)H * W, bad, st));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        if (!tm.ev.empty()) HIPCHK(hipEventSynchronize(tm.ev.back()));
        for (size_t x = 0; x < tm.kind.size(); ++x) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, tm.ev[2 * x], tm.ev[2 * x + 1]));
            if (tm.kind[x] == 0) { stats->reloc_ms += ms; stats->reloc_launches++; }
            else if (tm.kind[x] == 1) { stats->sweep_ms += ms; stats->sweep_launches++; }
            else { stats->backproj_ms += ms; stats->backproj_launches++; }
        }
        stats->chunks = (int32_t)chunks.size();
        stats->los_evals = evals;
        stats->pov_sector_pairs = pairs;
        // relocation: 4 B read + the element written per sample; fused, only the transposition of the grid
        stats->reloc_bytes = fused ? (int64_t)(2 * demTBytes) : pairs * (int64_t)(4 + elem);
        // sweep: the row's elevations read (4 B of grid, or the skwDEM element) + 4 B of ring sums written
        stats->sweep_bytes = pairs * (int64_t)((fused ? 4 : elem) + 4);
        stats->scratch_bytes = (int64_t)total;
        if (work) {
            unsigned long long h[kWorkSlots];
            HIPCHK(hipMemcpyAsync(h, work, sizeof(h), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int x = 0; x < kWorkSlots; ++x) stats->sweep_evals_done += (int64_t)h[x];
        }
    }
    return TVS_OK;
}

int run_singular(const float *d_dem, int H, int W, double dx, double h0, int n, double R, int pi, int pj,
                 uint32_t flags, double *d_area, uint32_t *d_rayV, hipStream_t st) {
    const bool f64 = (flags & TVS_FLAG_SLOPE_F32) == 0;
    const bool rcp = (flags & (TVS_FLAG_SLOPE_EXACT | TVS_FLAG_SLOPE_F64)) == 0;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    pool_keep_memory(dev);
    Scratch scr;
    scr.st = st;
    uint32_t *rayV = d_rayV;
    if (!rayV) {
        if (hipMallocAsync(&scr.p, (size_t)2 * n * sizeof(uint32_t), st) != hipSuccess) {
            (void)hipGetLastError();
            scr.p = nullptr;
            return fail(TVS_ENOMEM, "device scratch for %d lines of sight not available", 2 * n);
        }
        rayV = (uint32_t *)scr.p;
    }
    std::vector<Sector> S;
    for (int k = 0; k < n; ++k) S.push_back(plan_sector(k, n, H, W, dx, R));
    const int pitch = pitch_of(H, W);
    for (int k0 = 0; k0 < n; k0 += TVS_CHUNK) {
        Chunk c{k0, std::min(n, k0 + TVS_CHUNK), 0, 0, 0};
        ChunkArgs a = chunk_args(S, c, H, W, pitch, h0);
        a.pov_i = pi;
        a.pov_j = pj;
        HIPCHK(launch_singular(a, d_dem, rayV, f64, rcp, st));
        HIPCHK(launch_singular_sum(a, rayV, d_area, k0 == 0, st));
    }
    return TVS_OK;
}

// Singular lines of sight of npov POVs on one grid in one launch, then their areas (d_areas,
// nullable) and the visibility mask of POV 0 (d_mask) or the multiple viewshed (d_count). The
// tables are uploaded before return; the kernels are enqueued on st.
int run_multi(const float *d_dem, int H, int W, double dx, double h0, int n, double R, const int32_t *povs,
              int npov, uint32_t flags, double *d_areas, uint8_t *d_mask, uint32_t *d_count, hipStream_t st) {
    const bool f64 = (flags & TVS_FLAG_SLOPE_F32) == 0;
    const bool rcp = (flags & (TVS_FLAG_SLOPE_EXACT | TVS_FLAG_SLOPE_F64)) == 0;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    pool_keep_memory(dev);
    std::vector<Sector> S;
    for (int k = 0; k < n; ++k) S.push_back(plan_sector(k, n, H, W, dx, R));
    std::vector<SingSec> secs((size_t)npov * n);
    std::vector<SingQuery> qs(npov);
    for (int p = 0; p < npov; ++p) {
        SingQuery &Q = qs[p];
        std::memset(&Q, 0, sizeof(Q));
        Q.dem = d_dem;
        Q.H = H;
        Q.W = W;
        Q.pov_i = povs[2 * p];
        Q.pov_j = povs[2 * p + 1];
        Q.sec0 = p * n;
        Q.nsec = n;
        Q.h0 = h0;
        Q.h0f = (float)h0;
        for (int k = 0; k < n; ++k) {
            SingSec &E = secs[(size_t)p * n + k];
            std::memset(&E, 0, sizeof(E));
            E.s.T = S[k].T;
            E.s.scale = S[k].scale;
            E.s.clip = S[k].clip;
            E.s.kase = S[k].kase;
            E.s.K = S[k].K;
            E.s.t0 = S[k].t0;
            E.s.nrows = S[k].nrows;
            E.query = p;
        }
    }
    // half-sector boundary directions (2q + 1) pi / 2n and the sectors' cos s', rho
    std::vector<double> geo(6 * (size_t)n);
    for (int q = 0; q < 2 * n; ++q) {
        const double beta = (M_PI * (double)(2 * q + 1)) / (double)(2 * n);
        geo[q] = cos(beta);
        geo[2 * n + q] = sin(beta);
    }
    for (int k = 0; k < n; ++k) {
        geo[4 * n + k] = S[k].c;
        geo[5 * n + k] = S[k].rho;
    }
    const int L = std::max(H, W);
    const int words = 2 * ((L + 63) / 64 + 1);
    const size_t nr = (size_t)2 * npov * n;
    const bool want_cells = d_mask || d_count;
    auto a256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_secs = a256(secs.size() * sizeof(SingSec)), b_q = a256(qs.size() * sizeof(SingQuery)),
                 b_pov = a256((size_t)2 * npov * sizeof(int32_t)), b_geo = a256(geo.size() * sizeof(double)),
                 b_rays = a256(nr * sizeof(uint32_t)), b_bits = want_cells ? a256(nr * words * sizeof(uint32_t)) : 0,
                 b_ml = want_cells ? a256(nr * sizeof(int32_t)) : 0,
                 b_area = d_areas ? 0 : a256((size_t)npov * sizeof(double));
    Scratch scr;
    scr.st = st;
    if (hipMallocAsync(&scr.p, b_secs + b_q + b_pov + b_geo + b_rays + b_bits + b_ml + b_area, st) != hipSuccess) {
        (void)hipGetLastError();
        scr.p = nullptr;
        return fail(TVS_ENOMEM, "device scratch for %d singular viewsheds not available", npov);
    }
    char *base = (char *)scr.p;
    SingSec *d_secs = (SingSec *)base;
    SingQuery *d_q = (SingQuery *)(base += b_secs);
    int32_t *d_pov = (int32_t *)(base += b_q);
    double *d_geo = (double *)(base += b_pov);
    uint32_t *d_rays = (uint32_t *)(base += b_geo);
    uint32_t *d_bits = want_cells ? (uint32_t *)(base + b_rays) : nullptr;
    int32_t *d_ml = want_cells ? (int32_t *)(base + b_rays + b_bits) : nullptr;
    double *areas = d_areas ? d_areas : (double *)(base + b_rays + b_bits + b_ml);
    HIPCHK(hipMemcpyAsync(d_secs, secs.data(), secs.size() * sizeof(SingSec), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_q, qs.data(), qs.size() * sizeof(SingQuery), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_pov, povs, (size_t)2 * npov * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // the host tables may go out of scope
    HIPCHK(launch_singular_multi(d_secs, npov * n, d_q, npov, d_rays, areas, f64, rcp, st, d_bits, words, d_ml));
    if (want_cells) {
        MaskArgs m;
        std::memset(&m, 0, sizeof(m));
        m.H = H;
        m.W = W;
        m.n = n;
        m.npov = d_mask ? 1 : npov;
        m.pov = d_pov;
        m.cb = d_geo;
        m.sb = d_geo + 2 * n;
        m.ck = d_geo + 4 * n;
        m.rho = d_geo + 5 * n;
        m.bits = d_bits;
        m.mlast = d_ml;
        m.words = words;
        m.mask = d_mask;
        m.count = d_count;
        HIPCHK(launch_mask_multi(m, st));
    }
    return TVS_OK;
}

// Device buffer of the synchronous host entry points: taken from the device's stream-ordered pool on
// the null stream (which keeps freed memory, so repeated calls do not map and unmap it) and returned
// there; the entry points copy with hipMemcpy, ordered on the same stream.
template <typename T>
struct DevBuf {
    T *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFreeAsync(p, nullptr);
    }
    hipError_t alloc(size_t n) {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) pool_keep_memory(dev);
        return hipMallocAsync((void **)&p, n * sizeof(T), nullptr);
    }
};

}  // namespace

namespace tvs {
namespace host {

int total_on_stream(const float *d_dem, int H, int W, double dx, double h0, int n, double R, double *d_out,
                    uint32_t flags, hipStream_t st, size_t budget) {
    return run_total(d_dem, H, W, dx, h0, n, R, d_out, flags, nullptr, st, -1, nullptr, nullptr, budget);
}

size_t total_scratch_bytes(int H, int W, double dx, int n, double R, uint32_t flags, size_t budget) {
    const bool f64 = (flags & TVS_FLAG_SLOPE_F32) == 0;
    const bool fused = (flags & TVS_FLAG_RELOCATE) == 0;
    const size_t elem = fused ? 0 : f64 ? sizeof(double) : sizeof(float);
    std::vector<Sector> S;
    for (int k = 0; k < n; ++k) {
        S.push_back(plan_sector(k, n, H, W, dx, R));
        if (flags & TVS_FLAG_COMPACT) compact_layout(S.back());
    }
    size_t maxChunk = 0;
    for (const Chunk &c : make_chunks(S, elem, pitch_of(H, W), budget ? budget : scratch_budget()))
        maxChunk = std::max(maxChunk, c.bytes);
    const size_t tab = (size_t)std::max(H, W) * (sizeof(float2) + sizeof(double2));
    const size_t kahan = (flags & TVS_FLAG_ACC_KAHAN32) ? (size_t)H * W * 2 * sizeof(float) : 0;
    const size_t demT = (fused && n >= 2) ? (size_t)H * W * sizeof(float) : 0;
    return tab + kahan + demT + 256 * 4 + 64 * 8 + 256 + maxChunk + 8 * 256;
}

}  // namespace host
}  // namespace tvs

// ---------------------------------------------------------------- allocation-free variant
// Device memory of tvs_total_viewshed_noalloc: one copy of this array per device, allocated when
// the library's code object is loaded on the device and held until the process ends. In host code
// the name stands for a host-side symbol, not a device address: host code uses only the address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[TVS_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_noalloc_mu;
void *g_noalloc_base[64];  // per device: this device's address of `scratch`

// Address of the current device's `scratch`, looked up once per device with that device current.
int noalloc_base(void **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(TVS_EDEVICE, "device ordinal %d outside 0..63", dev);
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (!g_noalloc_base[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TVS_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_noalloc_base[dev] = p;
    }
    *out = g_noalloc_base[dev];
    return TVS_OK;
}

}  // namespace

extern "C" {

int tvs_total_viewshed_noalloc(const float *d_dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                               int32_t n_sectors, double max_dist, double *d_out, void *hip_stream) {
    g_err[0] = 0;
    if (!d_dem || !d_out) return fail(TVS_EINVAL, "null dem or out pointer");
    int rc = check_scalars(rows, cols, spacing, obs_height, n_sectors, max_dist);
    if (rc) return rc;
    void *base = nullptr;
    if ((rc = noalloc_base(&base))) return rc;
    return run_total(d_dem, rows, cols, spacing, obs_height, n_sectors, max_dist, d_out, 0u, nullptr,
                     (hipStream_t)hip_stream, -1, nullptr, nullptr, 0, base, TVS_NOALLOC_SCRATCH_BYTES, true);
}

int tvs_abi_version(void) { return TVS_ABI_VERSION; }

const char *tvs_last_error(void) { return g_err; }

int tvs_total_viewshed_ex(const float *d_dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                          int32_t n_sectors, double max_dist, double *d_out, uint32_t flags, tvs_stats *stats,
                          void *hip_stream) {
    g_err[0] = 0;
    if (!d_dem || !d_out) return fail(TVS_EINVAL, "null dem or out pointer");
    int rc = check_scalars(rows, cols, spacing, obs_height, n_sectors, max_dist);
    if (rc) return rc;
    if (int rc2 = check_flags(flags, true)) return rc2;
    return run_total(d_dem, rows, cols, spacing, obs_height, n_sectors, max_dist, d_out, flags, stats,
                     (hipStream_t)hip_stream, -1, nullptr, nullptr, 0, nullptr, 0, true);
}

int tvs_total_viewshed_async(const float *d_dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                             int32_t n_sectors, double max_dist, double *d_out, void *hip_stream) {
    return tvs_total_viewshed_ex(d_dem, rows, cols, spacing, obs_height, n_sectors, max_dist, d_out, 0u, nullptr,
                                 hip_stream);
}

int tvs_total_viewshed(const float *dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                       int32_t n_sectors, double max_dist, double *out) {
    g_err[0] = 0;
    if (!dem || !out) return fail(TVS_EINVAL, "null dem or out pointer");
    int rc = check_scalars(rows, cols, spacing, obs_height, n_sectors, max_dist);
    if (rc) return rc;
    if ((rc = check_host_dem(dem, rows, cols))) return rc;
    const size_t N = (size_t)rows * cols;
    DevBuf<float> d_dem;
    DevBuf<double> d_out;
    if (d_dem.alloc(N) != hipSuccess || d_out.alloc(N) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TVS_ENOMEM, "device buffers for a %d x %d grid not available", rows, cols);
    }
    HIPCHK(hipMemcpy(d_dem.p, dem, N * sizeof(float), hipMemcpyHostToDevice));
    rc = run_total(d_dem.p, rows, cols, spacing, obs_height, n_sectors, max_dist, d_out.p, 0u, nullptr, nullptr,
                   -1, nullptr, nullptr);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(nullptr));
    HIPCHK(hipMemcpy(out, d_out.p, N * sizeof(double), hipMemcpyDeviceToHost));
    return TVS_OK;
}

int tvs_singular_viewshed_ex(const float *d_dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                             int32_t n_sectors, double max_dist, int32_t pov_row, int32_t pov_col, uint32_t flags,
                             double *d_area, uint32_t *d_ray_V, void *hip_stream) {
    g_err[0] = 0;
    if (!d_dem || !d_area) return fail(TVS_EINVAL, "null dem or area pointer");
    int rc = check_scalars(rows, cols, spacing, obs_height, n_sectors, max_dist);
    if (rc) return rc;
    if (pov_row < 0 || pov_row >= rows || pov_col < 0 || pov_col >= cols)
        return fail(TVS_EINVAL, "POV (%d, %d) outside the %d x %d grid", pov_row, pov_col, rows, cols);
    if (flags & ~(TVS_FLAG_SLOPE_F64 | TVS_FLAG_SLOPE_EXACT | TVS_FLAG_SLOPE_F32))
        return fail(TVS_EINVAL, "unsupported flags 0x%x for the singular viewshed", flags);
    if ((flags & TVS_FLAG_SLOPE_F32) && (flags & TVS_FLAG_SLOPE_F64))
        return fail(TVS_EINVAL, "TVS_FLAG_SLOPE_F32 and TVS_FLAG_SLOPE_F64 exclude each other");
    return run_singular(d_dem, rows, cols, spacing, obs_height, n_sectors, max_dist, pov_row, pov_col, flags,
                        d_area, d_ray_V, (hipStream_t)hip_stream);
}

int tvs_singular_viewshed_async(const float *d_dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                                int32_t n_sectors, double max_dist, int32_t pov_row, int32_t pov_col,
                                double *d_area, uint8_t *d_mask, void *hip_stream) {
    if (!d_mask)
        return tvs_singular_viewshed_ex(d_dem, rows, cols, spacing, obs_height, n_sectors, max_dist, pov_row,
                                        pov_col, 0u, d_area, nullptr, hip_stream);
    g_err[0] = 0;
    if (!d_dem || !d_area) return fail(TVS_EINVAL, "null dem or area pointer");
    int rc = check_scalars(rows, cols, spacing, obs_height, n_sectors, max_dist);
    if (rc) return rc;
    if (pov_row < 0 || pov_row >= rows || pov_col < 0 || pov_col >= cols)
        return fail(TVS_EINVAL, "POV (%d, %d) outside the %d x %d grid", pov_row, pov_col, rows, cols);
    const int32_t pov[2] = {pov_row, pov_col};
    return run_multi(d_dem, rows, cols, spacing, obs_height, n_sectors, max_dist, pov, 1, 0u, d_area, d_mask, nullptr,
                     (hipStream_t)hip_stream);
}

int tvs_multiple_viewshed(const float *d_dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                          int32_t n_sectors, double max_dist, const int32_t *povs, int32_t npov, uint32_t flags,
                          uint32_t *d_count, double *d_areas, void *hip_stream) {
    g_err[0] = 0;
    if (!d_dem || !povs || !d_count) return fail(TVS_EINVAL, "null dem, povs or count pointer");
    if (npov < 1 || npov > (1 << 20)) return fail(TVS_EINVAL, "npov must be in [1, 2^20]");
    int rc = check_scalars(rows, cols, spacing, obs_height, n_sectors, max_dist);
    if (rc) return rc;
    for (int p = 0; p < npov; ++p)
        if (povs[2 * p] < 0 || povs[2 * p] >= rows || povs[2 * p + 1] < 0 || povs[2 * p + 1] >= cols)
            return fail(TVS_EINVAL, "POV %d (%d, %d) outside the %d x %d grid", p, povs[2 * p], povs[2 * p + 1], rows,
                        cols);
    if (flags & ~(TVS_FLAG_SLOPE_F64 | TVS_FLAG_SLOPE_EXACT | TVS_FLAG_SLOPE_F32))
        return fail(TVS_EINVAL, "unsupported flags 0x%x for the multiple viewshed", flags);
    if ((flags & TVS_FLAG_SLOPE_F32) && (flags & TVS_FLAG_SLOPE_F64))
        return fail(TVS_EINVAL, "TVS_FLAG_SLOPE_F32 and TVS_FLAG_SLOPE_F64 exclude each other");
    return run_multi(d_dem, rows, cols, spacing, obs_height, n_sectors, max_dist, povs, npov, flags, d_areas, nullptr,
                     d_count, (hipStream_t)hip_stream);
}

int tvs_singular_viewshed(const float *dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                          int32_t n_sectors, double max_dist, int32_t pov_row, int32_t pov_col, double *out_area,
                          uint8_t *out_mask) {
    g_err[0] = 0;
    if (!dem || !out_area) return fail(TVS_EINVAL, "null dem or area pointer");
    int rc = check_scalars(rows, cols, spacing, obs_height, n_sectors, max_dist);
    if (rc) return rc;
    if (pov_row < 0 || pov_row >= rows || pov_col < 0 || pov_col >= cols)
        return fail(TVS_EINVAL, "POV (%d, %d) outside the %d x %d grid", pov_row, pov_col, rows, cols);
    if ((rc = check_host_dem(dem, rows, cols))) return rc;
    const size_t N = (size_t)rows * cols;
    DevBuf<float> d_dem;
    DevBuf<double> d_area;
    DevBuf<uint8_t> d_mask;
    if (d_dem.alloc(N) != hipSuccess || d_area.alloc(1) != hipSuccess || (out_mask && d_mask.alloc(N) != hipSuccess)) {
        (void)hipGetLastError();
        return fail(TVS_ENOMEM, "device buffers for a %d x %d grid not available", rows, cols);
    }
    HIPCHK(hipMemcpy(d_dem.p, dem, N * sizeof(float), hipMemcpyHostToDevice));
    if (out_mask) {
        const int32_t pov[2] = {pov_row, pov_col};
        rc = run_multi(d_dem.p, rows, cols, spacing, obs_height, n_sectors, max_dist, pov, 1, 0u, d_area.p, d_mask.p,
                       nullptr, nullptr);
    } else {
        rc = run_singular(d_dem.p, rows, cols, spacing, obs_height, n_sectors, max_dist, pov_row, pov_col, 0u,
                          d_area.p, nullptr, nullptr);
    }
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(nullptr));
    HIPCHK(hipMemcpy(out_area, d_area.p, sizeof(double), hipMemcpyDeviceToHost));
    if (out_mask) HIPCHK(hipMemcpy(out_mask, d_mask.p, N, hipMemcpyDeviceToHost));
    return TVS_OK;
}

int tvs_sector_shape(int32_t rows, int32_t cols, int32_t n_sectors, int32_t sector, int32_t *out_nrows,
                     int32_t *out_ncols, int32_t *out_t0) {
    g_err[0] = 0;
    if (!out_nrows || !out_ncols || !out_t0) return fail(TVS_EINVAL, "null output pointer");
    int rc = check_scalars(rows, cols, 1.0, 0.0, n_sectors, INFINITY);
    if (rc) return rc;
    if (sector < 0 || sector >= n_sectors) return fail(TVS_EINVAL, "sector %d outside [0, %d)", sector, n_sectors);
    const Sector s = plan_sector(sector, n_sectors, rows, cols, 1.0, INFINITY);
    *out_nrows = s.nrows;
    *out_ncols = s.Wx;
    *out_t0 = s.t0;
    return TVS_OK;
}

int tvs_debug_sector_rays(const float *dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                          int32_t n_sectors, double max_dist, int32_t sector, uint32_t flags, uint32_t *out_V) {
    g_err[0] = 0;
    if (!dem || !out_V) return fail(TVS_EINVAL, "null dem or out_V pointer");
    int rc = check_scalars(rows, cols, spacing, obs_height, n_sectors, max_dist);
    if (rc) return rc;
    if (sector < 0 || sector >= n_sectors) return fail(TVS_EINVAL, "sector %d outside [0, %d)", sector, n_sectors);
    if (int rc2 = check_flags(flags, false)) return rc2;
    if ((rc = check_host_dem(dem, rows, cols))) return rc;
    const Sector s = plan_sector(sector, n_sectors, rows, cols, spacing, max_dist);
    const size_t N = (size_t)rows * cols;
    const size_t NV = (size_t)s.nrows * s.Wx;
    DevBuf<float> d_dem;
    DevBuf<uint32_t> d_V;
    if (d_dem.alloc(N) != hipSuccess || d_V.alloc(NV) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TVS_ENOMEM, "device buffers not available");
    }
    HIPCHK(hipMemcpy(d_dem.p, dem, N * sizeof(float), hipMemcpyHostToDevice));
    int pitch = 0;
    rc = run_total(d_dem.p, rows, cols, spacing, obs_height, n_sectors, max_dist, nullptr, flags, nullptr, nullptr,
                   sector, d_V.p, &pitch);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(nullptr));
    HIPCHK(hipMemcpy(out_V, d_V.p, NV * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return TVS_OK;
}

int tvs_debug_sector_rays_async(const float *d_dem, int32_t rows, int32_t cols, double spacing, double obs_height,
                                int32_t n_sectors, double max_dist, int32_t sector, uint32_t flags, uint32_t *d_out_V,
                                void *hip_stream) {
    g_err[0] = 0;
    if (!d_dem || !d_out_V) return fail(TVS_EINVAL, "null d_dem or d_out_V pointer");
    int rc = check_scalars(rows, cols, spacing, obs_height, n_sectors, max_dist);
    if (rc) return rc;
    if (sector < 0 || sector >= n_sectors) return fail(TVS_EINVAL, "sector %d outside [0, %d)", sector, n_sectors);
    if (int rc2 = check_flags(flags, false)) return rc2;
    int pitch = 0;
    return run_total(d_dem, rows, cols, spacing, obs_height, n_sectors, max_dist, nullptr, flags, nullptr,
                     (hipStream_t)hip_stream, sector, d_out_V, &pitch);
}

int tvs_los_evals(int32_t rows, int32_t cols, double spacing, int32_t n_sectors, double max_dist, int64_t *out_evals,
                  int64_t *out_pairs) {
    g_err[0] = 0;
    if (!out_evals || !out_pairs) return fail(TVS_EINVAL, "null output pointer");
    int rc = check_scalars(rows, cols, spacing, 0.0, n_sectors, max_dist);
    if (rc) return rc;
    int64_t ev = 0, pr = 0;
    for (int k = 0; k < n_sectors; ++k) count_sector(plan_sector(k, n_sectors, rows, cols, spacing, max_dist), ev, pr);
    *out_evals = ev;
    *out_pairs = pr;
    return TVS_OK;
}

int tvs_total_viewshed_tiles(const tvs_tile *tiles, int32_t ntiles, int32_t n_sectors, uint32_t flags,
                             void *hip_stream) {
    g_err[0] = 0;
    if (!tiles || ntiles < 1) return fail(TVS_EINVAL, "at least one tile");
    if (int rc = check_flags(flags, true)) return rc;
    if (flags & TVS_FLAG_COUNT_EVALS) return fail(TVS_EINVAL, "TVS_FLAG_COUNT_EVALS needs a stats argument");
    for (int t = 0; t < ntiles; ++t) {
        const tvs_tile &T = tiles[t];
        if (!T.d_dem || !T.d_out) return fail(TVS_EINVAL, "tile %d: null d_dem or d_out", t);
        if (int rc = check_scalars(T.rows, T.cols, T.spacing, T.obs_height, n_sectors, T.max_dist)) return rc;
    }
    for (int t = 0; t < ntiles; ++t) {
        const tvs_tile &T = tiles[t];
        if (int rc = run_total(T.d_dem, T.rows, T.cols, T.spacing, T.obs_height, n_sectors, T.max_dist, T.d_out,
                               flags, nullptr, (hipStream_t)hip_stream, -1, nullptr, nullptr, 0, nullptr, 0, true))
            return rc;
    }
    return TVS_OK;
}

}  // extern "C"
