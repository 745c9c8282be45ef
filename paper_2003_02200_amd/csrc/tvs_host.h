// tvs_host.h -- host-side helpers shared by the C entry points of libtvs (not part of the C
// ABI): error text, argument checks and the per-sector plan.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/libtvs.h"
#include "tvs_geom.h"

namespace tvs {
namespace host {

// Text of the last failure on the calling thread (tvs_last_error).
extern thread_local char g_err[512];

// Records the message and returns `code`.
int fail(int code, const char *fmt, ...);

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(TVS_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// One sector of the plan (host side).
struct Sector {
    int kase, Hx, Wx;
    double T;      // tan s'
    double c;      // cos s'
    double rho;    // max_dist cos s' / spacing
    int K;         // last target index in range (TVS_K_UNBOUNDED when max_dist never binds)
    double scale;  // (pi / 2n) spacing^2 / cos^2 s'
    double clip;   // rho^2 - K^2
    int t0, nrows;
    int wrap;      // 0: plain layout; Hx + 1: compacted layout (skewed row t in row t mod wrap)
    int prows;     // rows the sector's skewed buffers take: nrows, or Hx + 1 compacted
};

// Switches the sector to the compacted layout of its skewed buffers.
void compact_layout(Sector &s);

// Elevations and the observer height must be finite, and either 0 or at least 2^-60 m in
// magnitude. The second rule keeps every quantity of the sweep a multiple of 2^-83, so no slope
// underflows to a signed zero (the kernels read strict comparisons from sign bits).
constexpr double TVS_MIN_MAGNITUDE = 0x1p-60;

Sector plan_sector(int k, int n, int H, int W, double dx, double R);
bool magnitude_ok(double v);
int check_scalars(int rows, int cols, double dx, double h0, int n, double R);
int check_host_dem(const float *dem, int rows, int cols);
int check_flags(uint32_t flags, bool accumulation);
// Closed-form line-of-sight evaluations and POV-sector pairs of one sector.
void count_sector(const Sector &s, int64_t &evals, int64_t &pairs);
// Row pitch (elements) of a grid's skewed buffers.
int pitch_of(int H, int W);
// Device scratch a call may take: TVS_SCRATCH_MB, else min(free / 2, 16 GiB).
size_t scratch_budget();
// Keeps freed stream-ordered memory in the device's pool (no release between calls).
void pool_keep_memory(int dev);
// Largest LDS a workgroup of this device may request.
int lds_limit(int dev);
// The total viewshed's launch sequence on a stream (tvs_total_viewshed_ex without stats); its
// device scratch is taken stream-ordered and limited to `budget` bytes (0: scratch_budget()).
int total_on_stream(const float *d_dem, int H, int W, double dx, double h0, int n, double R, double *d_out,
                    uint32_t flags, hipStream_t st, size_t budget);
// Device scratch that total_on_stream takes for these arguments.
size_t total_scratch_bytes(int H, int W, double dx, int n, double R, uint32_t flags, size_t budget);

// Launch shapes chosen by timing (tvs_tune.hip): kind 0 the batched sweep (a = waves per
// workgroup, b = workgroups per CU, 0 for one workgroup per item), kind 1 the single-grid sweep
// (a = waves per workgroup); keyed by decision precision and slope form and the ceil(log2) size
// classes of the longest skewed row and of the longest line of sight (+1). Kept per device and
// library build, in memory and in a cache file.
struct TuneKey {
    int kind, f64, rcp, side_b, rho_b;
};
bool tune_lookup(const TuneKey &k, int &a, int &b);
void tune_store(const TuneKey &k, int a, int b);
const char *source_hash();
int ceil_log2(int64_t v);

// Pinned host staging owned by a caller of batch_enqueue (grown there, freed by the owner). A grown
// buffer leaves the old one in `retired` rather than freeing it, because freeing pinned memory waits
// for the whole device; the owner frees both at its end.
struct PinnedStaging {
    void *p = nullptr;
    size_t cap = 0;
    std::vector<void *> retired;
};
// Do the skewed rows of grids with sides up to maxWx fit the batched sweep's LDS?
bool batch_rows_fit(int maxWx, bool f64);
// Total viewsheds of independent tiles as one batch enqueued on `st` (no graph): per sector chunk
// (skewed viewshed rows within `budget` bytes) one fused relocate + sweep launch per bucket of tiles
// with a workgroup per (tile, sector, row) item and one back-projection launch over every tile. `demT` (nullable) holds
// each tile's transposed grid, read for the 45..135 deg axes. Flags: the decision precision and slope
// form (TVS_FLAG_SLOPE_F32, _F64, _EXACT).
int batch_enqueue(const tvs_tile *tiles, const float *const *demT, int ntiles, int n, uint32_t flags, hipStream_t st,
                  size_t budget, PinnedStaging &stage, int *out_chunks);
// Sizes that add up over the tiles of a batch.
struct BatchSize {
    size_t vbytes = 0;  // skewed viewshed rows of every sector
    size_t tables = 0;  // entries, tiles and work items
    int maxWx = 0;      // longest side
    void add(const BatchSize &o) {
        vbytes += o.vbytes;
        tables += o.tables;
        maxWx = maxWx > o.maxWx ? maxWx : o.maxWx;
    }
};
BatchSize batch_tile_size(const tvs_tile &T, int n);
// Device memory batch_enqueue takes for tiles of these summed sizes beyond their maps (an upper bound).
size_t batch_scratch_bytes(const BatchSize &sum, size_t budget);

}  // namespace host
}  // namespace tvs
