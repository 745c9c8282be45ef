/*
 * libtvs.h -- C ABI of libtvs, the MI355X (gfx950) implementation of the sDEM total
 * viewshed (Sanchez-Fernandez, Romero, Bandera, Tabik, "A data relocation approach for
 * terrain surface analysis on multi-GPU systems: a case study on the total viewshed
 * problem").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * dem        Row-major, C-contiguous rows x cols float32 elevations in metres. Row index
 *            grows "south", column index "east". Cells are square, `spacing` metres apart.
 *            Every elevation must be finite (the paper has no no-data concept) and either 0 or
 *            at least 2^-60 m in magnitude (the sweep's sign tests assume no slope underflows).
 * spacing    Grid step in metres, finite and > 0.
 * obs_height Height of the observer above the ground at the point of view (POV), metres,
 *            finite, 0 or at least 2^-60 in magnitude. Targets are at ground level.
 * n_sectors  Number of sector axes over 180 degrees, 1 <= n <= 32768. Axis k points at
 *            a_k = k*pi/n from +column toward +row; each axis carries a forward and a
 *            backward line of sight (a_k and a_k + 180 deg), each the axis of a
 *            half-sector of opening pi/n (Section 3.1, Alg. 1; Section 4.1 step 1). The
 *            paper's "ns sectors" is 2n.
 * max_dist   Largest distance (metres) of a target from the POV: > 0, may be +INFINITY
 *            (the paper's own unbounded setting). A line of sight of sector s' stops at
 *            index distance m < rho = max_dist cos(s') / spacing and its last ring is
 *            clipped at rho.
 * rows, cols 1 .. 32767 each; larger grids return TVS_ERANGE. A skewed row is held in the
 *            LDS of one workgroup when it fits (float rows always; double rows up to about 19,000
 *            samples); longer rows are swept in pieces of POVs, each piece's reach (K samples
 *            either side) held in LDS, or, for lines of sight too long for that, streamed through
 *            LDS windows; with the same exact block skip and early exit. The lane-per-target sweep
 *            (TVS_FLAG_SWEEP_SCAN) and batches hold whole rows and return TVS_ERANGE beyond.
 * Results    Areas in square metres, double.
 *
 * Errors: every call returns TVS_OK (0) or a negative status; on error the outputs are
 * left untouched, except the _async variants after device work was enqueued (then the
 * status is TVS_EDEVICE). tvs_last_error() describes the last failure on the calling
 * thread. No exception crosses the ABI. Every entry point is reentrant.
 *
 * Ownership: the caller owns every buffer. Host-pointer variants are synchronous and
 * keep no pointer after return. _async variants take device pointers on the current
 * HIP device and a hipStream_t (passed as void*, NULL = the null stream); they enqueue
 * work on that stream and return; inputs must stay valid and outputs untouched until
 * the stream reaches that point. Device scratch is allocated stream-ordered per call.
 */
#ifndef LIBTVS_H
#define LIBTVS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TVS_ABI_VERSION 8

enum tvs_status {
    TVS_OK = 0,
    TVS_EINVAL = -1,  /* bad argument: null pointer, size, non-finite value, POV outside the grid */
    TVS_ENOMEM = -2,  /* host or device allocation failed */
    TVS_EDEVICE = -3, /* a HIP call or kernel launch failed (see tvs_last_error) */
    TVS_ERANGE = -4,  /* grid side above 32767, or a row the LDS cannot hold where whole rows are needed */
    TVS_ETIMEDOUT = -5 /* tvs_server_wait: the request did not finish within the timeout */
};

/* Variant flags. The default, 0, keeps the interpolated elevations in double and decides
 * visibility in double, the slope formed as the elevation difference times the double reciprocal
 * of the index distance (within one double ulp of the quotient). It steps one lane per POV in the
 * sweep, and it ends a group of 64 lines of sight early once no remaining target can rise above any
 * of their horizons. The results are those of the full walk, because the bound uses only monotone
 * roundings. Each cell is accumulated in double.
 * The paper's kernels declare their slopes float (Alg. 7/8); TVS_FLAG_SLOPE_F32 takes that
 * precision. It flips the decision of about 4e-4 of the POV-sector pairs of a 2000 x 2000 grid
 * with 1000-sample lines of sight, against about 1e-9 for the default. */
#define TVS_FLAG_SLOPE_F64 0x1u   /* double decision, slope as the correctly rounded double quotient */
#define TVS_FLAG_SWEEP_SCAN 0x2u  /* sweep with one lane per target and wavefront prefix-max */
#define TVS_FLAG_ACC_KAHAN32 0x4u /* float Kahan-compensated per-cell accumulation */
#define TVS_FLAG_SLOPE_EXACT 0x8u /* slope as the correctly rounded quotient of difference and
                                     distance in the decision's precision (an IEEE division) */
#define TVS_FLAG_NO_PRUNE 0x10u   /* walk every target in range, as Alg. 8 does (same results) */
#define TVS_FLAG_COUNT_EVALS 0x20u /* total viewshed only, needs `stats`: count the line-of-sight
                                      evaluations the sweep carries out into stats->sweep_evals_done */
#define TVS_FLAG_SLOPE_F32 0x40u  /* float elevations and float decision (the paper's precision);
                                     with TVS_FLAG_SLOPE_EXACT the float quotient. Excludes
                                     TVS_FLAG_SLOPE_F64 */
#define TVS_FLAG_AUTOTUNE 0x80u   /* batches: time the candidate launch shapes of each bucket of tiles
                                     on a sample of its rows before building the batch; total viewshed:
                                     time the sweep's waves per workgroup on a few sectors first. The
                                     fastest shape is kept per size class, device and library build
                                     (in memory and in a cache file: TVS_TUNE_CACHE, else
                                     $XDG_CACHE_HOME/libtvs or ~/.cache/libtvs), and later calls
                                     without the flag use it. Results are the same with any shape. */
#define TVS_FLAG_RELOCATE 0x200u  /* total viewshed: run the relocation as its own kernel that writes every
                                     sector's skewed elevations (skwDEM) to device memory, and sweep from
                                     there (Section 4.2's first kernel); by default each sweep workgroup
                                     gathers its skewed row from the grid with the same interpolation, and no
                                     skwDEM exists. Same results bit for bit. */
#define TVS_FLAG_COMPACT 0x100u   /* total viewshed and batches: compacted skewed buffers (Section 3.1,
                                     the second compaction of Figure 4): skewed row t of a base frame
                                     with Hx rows is stored in row t mod (Hx + 1), since rows that far
                                     apart hold disjoint column ranges. A sector then takes Hx + 1
                                     rows instead of Hx + d_max + 1, so a chunk holds more sectors
                                     within the same scratch budget. Same results bit for bit. */

/* Per-call measurement filled by the _ex entry points when `stats` is non-NULL. Kernel
 * times come from HIP events recorded around each launch on the call's stream; asking for
 * them makes the call wait for its own work before returning. */
typedef struct tvs_stats {
    double reloc_ms;        /* summed duration of the relocation launches */
    double sweep_ms;        /* summed duration of the sweep launches */
    double backproj_ms;     /* summed duration of the back-projection launches */
    int32_t reloc_launches;
    int32_t sweep_launches;
    int32_t backproj_launches;
    int32_t chunks;         /* sector groups processed one after another */
    int64_t los_evals;      /* line-of-sight cell evaluations of the call (closed form) */
    int64_t pov_sector_pairs; /* skewed samples summed over sectors (one per POV and sector) */
    int64_t reloc_bytes;    /* algorithmic bytes of the relocation: 4 read + element size written per sample */
    int64_t sweep_bytes;    /* algorithmic bytes of the sweep: element size read + 4 written per sample */
    int64_t scratch_bytes;  /* device scratch used */
    int64_t sweep_evals_done; /* evaluations carried out by the sweep (TVS_FLAG_COUNT_EVALS), else 0;
                                 equals los_evals with TVS_FLAG_NO_PRUNE */
} tvs_stats;

/* ABI version of the loaded library (TVS_ABI_VERSION of the build). */
int tvs_abi_version(void);

/* Text of the last error on the calling thread; valid until the next libtvs call on it. */
const char *tvs_last_error(void);

/* Total viewshed, Alg. 4 computed with the sDEM method of Section 4.1 (steps 1a-1d) and the
 * three kernels of Section 4.2 (relocation Alg. 6, sweep Alg. 7/8, back-projection Alg. 9):
 * out[i*cols + j] = area visible from cell (i, j), m^2. `dem` and `out` are host pointers
 * (rows*cols each). Synchronous; runs on the current HIP device. */
int tvs_total_viewshed(const float *dem, int32_t rows, int32_t cols, double spacing,
                       double obs_height, int32_t n_sectors, double max_dist, double *out);

/* Singular viewshed, Alg. 1: the area (m^2) visible from grid cell (pov_row, pov_col), each
 * line of sight passing through the POV. Host pointers. `out_mask` (nullable, rows*cols u8)
 * receives the visibility of every cell (the boolean map of Section 1; Alg. 1 itself returns the
 * area only): a cell at offset (di, dj) from the POV belongs to half-sector q, the one whose
 * interval (beta_{q-1}, beta_q] of direction angles, beta_q = (2q + 1) pi / 2n measured like the
 * sector axes, holds it (cos(beta) di - sin(beta) dj > 0 above a boundary, with cos and sin
 * computed in double); its ring index along that line of sight is
 * m = floor(sqrt(di^2 + dj^2) cos(s') + 1e-9); it is visible iff m = 0, or m is a target of the
 * line of sight (m <= its last target, m < rho) and that target is visible. */
int tvs_singular_viewshed(const float *dem, int32_t rows, int32_t cols, double spacing,
                          double obs_height, int32_t n_sectors, double max_dist,
                          int32_t pov_row, int32_t pov_col, double *out_area, uint8_t *out_mask);

/* Device-resident, stream-ordered total viewshed: d_dem and d_out are device pointers
 * (rows*cols float / double). Elevations are not read on the host; they are checked on the device
 * (finite, and 0 or at least 2^-60 m in magnitude), and a grid that breaks the rule gives a map of
 * NaN in every cell: the status, returned before the work runs, cannot report it. The same holds for
 * tvs_total_viewshed_ex, tvs_total_viewshed_noalloc and tvs_total_viewshed_tiles. */
int tvs_total_viewshed_async(const float *d_dem, int32_t rows, int32_t cols, double spacing,
                             double obs_height, int32_t n_sectors, double max_dist,
                             double *d_out, void *hip_stream);

/* Device-resident singular viewshed: *d_area (device double) receives the area; d_mask
 * (nullable, device rows*cols u8) the visibility mask as in tvs_singular_viewshed. */
int tvs_singular_viewshed_async(const float *d_dem, int32_t rows, int32_t cols, double spacing,
                                double obs_height, int32_t n_sectors, double max_dist,
                                int32_t pov_row, int32_t pov_col, double *d_area, uint8_t *d_mask,
                                void *hip_stream);

/* tvs_total_viewshed_async with variant `flags` (TVS_FLAG_*) and optional measurement. */
int tvs_total_viewshed_ex(const float *d_dem, int32_t rows, int32_t cols, double spacing,
                          double obs_height, int32_t n_sectors, double max_dist, double *d_out,
                          uint32_t flags, tvs_stats *stats, void *hip_stream);

/* tvs_singular_viewshed_async with variant flags (TVS_FLAG_SLOPE_F64, TVS_FLAG_SLOPE_EXACT,
 * TVS_FLAG_SLOPE_F32) and, when
 * d_ray_V is non-NULL, the per-line-of-sight ring sums: d_ray_V[2k] forward and [2k+1]
 * backward of sector k, packed as U | (e << 30) (U whole rings in index^2 units including
 * the POV ring, e in {0,1} clipped last ring of area rho^2 - K^2, K = ceil(rho) - 1). */
int tvs_singular_viewshed_ex(const float *d_dem, int32_t rows, int32_t cols, double spacing,
                             double obs_height, int32_t n_sectors, double max_dist,
                             int32_t pov_row, int32_t pov_col, uint32_t flags, double *d_area,
                             uint32_t *d_ray_V, void *hip_stream);

/* Multiple (cumulative) viewshed: d_count[i*cols + j] (device u32) = how many of the npov
 * POVs see cell (i, j), each POV's visibility as tvs_singular_viewshed's mask; d_areas (nullable,
 * device npov doubles) receives each POV's singular area. povs is a host array of npov
 * (row, col) pairs, read before return. All lines of sight of all POVs run in one launch, then one
 * launch computes every cell. Flags: TVS_FLAG_SLOPE_F32, _F64, _EXACT. */
int tvs_multiple_viewshed(const float *d_dem, int32_t rows, int32_t cols, double spacing,
                          double obs_height, int32_t n_sectors, double max_dist, const int32_t *povs,
                          int32_t npov, uint32_t flags, uint32_t *d_count, double *d_areas,
                          void *hip_stream);

/* ---- Allocation-free total viewshed --------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. tvs_total_viewshed_async without any allocation: every
 * device buffer of the call (reciprocal tables, skewed elevation and viewshed buffers) is carved
 * from a static device array of TVS_NOALLOC_SCRATCH_BYTES that the library holds on each device it
 * runs on until the process ends (its address is looked up on a device's first call). The skewed
 * viewshed rows take the compacted layout (TVS_FLAG_COMPACT) and the sectors are processed in groups
 * that fit the array; the map is the same as tvs_total_viewshed_async's, bit for bit.
 * Limit: one sector's skewed viewshed rows, 4 * (H_x + 1) * P bytes (H_x the sector's rows in its
 * 0..45 deg frame, P = max(rows, cols) rounded up to 64), must fit the array together with the
 * transposed grid (4 * rows * cols bytes) and the reciprocal tables (24 * max(rows, cols) bytes);
 * larger grids return TVS_ERANGE before any work is enqueued (square grids up to about 5,700).
 * Calls on one device share the array: calls whose work overlaps on a device (other streams,
 * other host threads) race and must be serialised by the caller. The call itself allocates no
 * device memory, frees none and calls no allocating library routine. */
#define TVS_NOALLOC_SCRATCH_BYTES (256u << 20)
int tvs_total_viewshed_noalloc(const float *d_dem, int32_t rows, int32_t cols, double spacing,
                               double obs_height, int32_t n_sectors, double max_dist, double *d_out,
                               void *hip_stream);

/* ---- Batches of independent tiles (uneven sizes) -------------------------------------------
 * Every tile is an independent total viewshed (tvs_total_viewshed_async semantics) with its own
 * size, spacing, observer height and max distance; all tiles share n_sectors. */
typedef struct tvs_tile {
    const float *d_dem;  /* device, rows*cols float32, row-major */
    double *d_out;       /* device, rows*cols float64: the tile's total viewshed, m^2 */
    int32_t rows, cols;
    double spacing, obs_height, max_dist;
} tvs_tile;

typedef struct tvs_batch tvs_batch; /* opaque plan of a batch, owned by the caller */

typedef struct tvs_batch_info {
    int32_t tiles;
    int32_t chunks;           /* sector groups, each one sweep and one back-projection launch */
    int32_t kernel_launches;  /* kernels in the captured graph */
    int32_t waves_per_group;  /* launch shape of bucket 0's sweep (tvs_batch_get_bucket for the others) */
    int32_t groups;           /* its workgroups per launch (persistent), or 0 (one per skewed row) */
    int32_t tuned;            /* 1 if the shape came from timing candidates */
    int64_t los_evals;        /* closed-form line-of-sight evaluations of one pass */
    int64_t pov_sector_pairs;
    int64_t sweep_evals_done; /* evaluations carried out by the last completed pass
                                 (TVS_FLAG_COUNT_EVALS), else 0 */
    int64_t scratch_bytes;    /* device memory owned by the batch */
    double tune_ms;           /* time spent timing candidates at creation */
    int32_t buckets;          /* groups of tiles with their own sweep launch and shape (tvs_batch_get_bucket) */
    int32_t pad;
} tvs_batch_info;

/* A bucket of a batch: the tiles whose longest side and longest line of sight (capped at the side)
 * fall in the same power-of-two classes; per sector chunk one sweep launch over their items, with
 * its own launch shape. */
typedef struct tvs_batch_bucket {
    int32_t side_class;       /* ceil(log2(longest side)) */
    int32_t reach_class;      /* ceil(log2(longest line of sight + 1)) */
    int32_t tiles;
    int32_t longest_side;
    int32_t longest_reach;    /* target steps of the longest line of sight */
    int32_t waves_per_group;  /* wavefronts per sweep workgroup */
    int32_t groups_per_cu;    /* persistent workgroups per CU; 0: one workgroup per skewed row */
    int32_t tuned;            /* 1 if the shape came from timing (now or remembered) */
    int64_t items;            /* (tile, sector, skewed row) items over all chunks */
} tvs_batch_bucket;

/* Plans a batch: validates every tile, groups the sectors into chunks within the scratch budget and
 * the tiles into buckets, uploads the work lists and captures one pass into a HIP graph: one
 * transposition per tile, then per chunk one fused relocate + sweep launch per bucket over its
 * (tile, sector, skewed row) items (persistent workgroups or one workgroup per item, as the bucket's
 * shape says) and one back-projection launch over every tile. The DEM and output buffers are bound to the batch: they must stay
 * allocated and in place until tvs_batch_destroy. Flags: TVS_FLAG_SLOPE_F32, TVS_FLAG_SLOPE_F64,
 * TVS_FLAG_SLOPE_EXACT, TVS_FLAG_COUNT_EVALS, TVS_FLAG_AUTOTUNE. Runs on the current HIP device
 * (synchronously at creation). Section 4.1 steps 1a-1d applied to every tile; the batching,
 * fusion and graph are this library's, not the paper's. */
int tvs_batch_create(const tvs_tile *tiles, int32_t ntiles, int32_t n_sectors, uint32_t flags,
                     tvs_batch **out_batch);

/* Enqueues one pass over every tile on hip_stream (a graph launch); outputs are complete when
 * the stream reaches that point. Passes on one batch must not overlap. */
int tvs_batch_run(tvs_batch *batch, void *hip_stream);

/* Plan, launch shape and counts of a batch (sweep_evals_done needs the last pass finished). */
int tvs_batch_get_info(const tvs_batch *batch, tvs_batch_info *info);

/* Bucket i (0 <= i < info.buckets) of a batch; bucket 0 holds the largest tiles. */
int tvs_batch_get_bucket(const tvs_batch *batch, int32_t i, tvs_batch_bucket *out);

/* Releases the batch's graph and device memory (waits for its work). NULL is ignored. */
int tvs_batch_destroy(tvs_batch *batch);

/* The plain per-tile loop the batch is measured against: tvs_total_viewshed_ex on every tile in
 * turn on hip_stream (flags as there). */
int tvs_total_viewshed_tiles(const tvs_tile *tiles, int32_t ntiles, int32_t n_sectors, uint32_t flags,
                             void *hip_stream);

/* ---- Request server: resident grids, continuous batching ------------------------------------
 * Clients on any thread submit total and singular viewshed requests against grids uploaded once.
 * A scheduler thread admits total requests in arrival order while their device memory (maps plus
 * scratch, scratch capped at a quarter of the budget) fits hbm_budget_bytes. Whenever one of two
 * group slots is free, the waiting total requests of the front request's sector count and flags
 * (up to max_total_batch) leave together as one batch (tvs_batch_create's launches, enqueued without a
 * graph: per sector chunk one fused relocate + sweep launch per bucket, with one workgroup per skewed
 * row so that singular work started later interleaves, and one back-projection launch); totals that arrive while both groups run gather into the next group. Totals the
 * batched sweep does not take (TVS_FLAG_ACC_KAHAN32, TVS_FLAG_SWEEP_SCAN, TVS_FLAG_NO_PRUNE, rows
 * longer than the LDS holds) run alone on the next of `streams` streams, overlapping with the rest.
 * Waiting singular requests are launched together, up to max_singular_batch per launch (one
 * wavefront per line of sight of every query, then one area sum per query). A result does not
 * depend on what else runs (no atomics, fixed accumulation order). The server is this library's,
 * not the paper's; the computations are the paper's (Section 4.1, Alg. 1). */
typedef struct tvs_server tvs_server; /* opaque */

typedef struct tvs_server_config {
    int64_t hbm_budget_bytes;   /* 0: half the device memory free at creation */
    int32_t streams;            /* streams for total requests, 0: 4 (at most 16) */
    int32_t max_singular_batch; /* queries per singular launch, 0: 64 */
    int32_t max_total_batch;    /* total requests per batched launch group, 0: 16 */
    int32_t pad;
} tvs_server_config;

typedef struct tvs_request_result {
    int32_t status;      /* TVS_OK, or the failure of this request */
    int32_t kind;        /* 1 total, 2 singular */
    double area_m2;      /* singular: the visible area */
    double latency_ms;   /* submission to completion seen by the scheduler */
    double queue_ms;     /* submission to launch */
    int32_t rows, cols;  /* the grid's shape (total: the map's) */
} tvs_request_result;

typedef struct tvs_server_stats {
    int32_t grids, pending, running, pad;
    int64_t completed;
    int64_t singular_batches;      /* singular launches so far */
    int64_t singular_batched;      /* singular requests they carried */
    int64_t max_concurrent_totals; /* most total requests on the device at once */
    int64_t budget_bytes, bytes_in_use, peak_bytes;
    int64_t total_batches;         /* batched launch groups of total requests so far */
    int64_t total_batched;         /* total requests they carried */
} tvs_server_stats;

/* Starts a server on the current HIP device (cfg may be NULL for the defaults). */
int tvs_server_create(const tvs_server_config *cfg, tvs_server **out_server);

/* Uploads a host grid (same rules as tvs_total_viewshed's dem) and returns its id. */
int tvs_server_add_grid(tvs_server *server, const float *dem, int32_t rows, int32_t cols, double spacing,
                        int32_t *out_grid_id);

/* Queues a total viewshed of a grid (flags as tvs_total_viewshed_ex, without
 * TVS_FLAG_COUNT_EVALS); *out_ticket names the request. */
int tvs_server_submit_total(tvs_server *server, int32_t grid_id, double obs_height, int32_t n_sectors,
                            double max_dist, uint32_t flags, uint64_t *out_ticket);

/* Queues a singular viewshed (flags: TVS_FLAG_SLOPE_F32, _F64, _EXACT). */
int tvs_server_submit_singular(tvs_server *server, int32_t grid_id, double obs_height, int32_t n_sectors,
                               double max_dist, int32_t pov_row, int32_t pov_col, uint32_t flags,
                               uint64_t *out_ticket);

/* Waits for a request (timeout_ms < 0: no limit; TVS_ETIMEDOUT when it expires) and fills *res. */
int tvs_server_wait(tvs_server *server, uint64_t ticket, double timeout_ms, tvs_request_result *res);

/* Copies a finished total request's map (rows*cols double) to `out` (host or device) on
 * hip_stream, and waits for the copy. */
int tvs_server_copy_map(tvs_server *server, uint64_t ticket, double *out, void *hip_stream);

/* Forgets a finished request and frees its map. */
int tvs_server_release(tvs_server *server, uint64_t ticket);

int tvs_server_get_stats(tvs_server *server, tvs_server_stats *stats);

/* Finishes every queued request, then stops the scheduler and frees everything. */
int tvs_server_destroy(tvs_server *server);

/* Shape of the skewed grid of sector `sector` (Section 4.1, Fig. 4b: one row per line of
 * sight): rows t = t0 .. t0 + nrows - 1, columns 0 .. ncols - 1 of the 0..45 deg base frame. */
int tvs_sector_shape(int32_t rows, int32_t cols, int32_t n_sectors, int32_t sector,
                     int32_t *out_nrows, int32_t *out_ncols, int32_t *out_t0);

/* Diagnostic: the per-sector skewed viewshed of Section 4.1 step 1c (skwVS before the
 * back-projection) for one sector, computed by the same relocation and sweep kernels as
 * the total viewshed. Host pointers; out_V is nrows x ncols (tvs_sector_shape) u32, each
 * existing sample packed as U | (e << 30) (forward + backward: U whole rings including both
 * POV rings, e in {0,1,2} clipped last rings); samples outside the grid are 0xFFFFFFFF. */
int tvs_debug_sector_rays(const float *dem, int32_t rows, int32_t cols, double spacing,
                          double obs_height, int32_t n_sectors, double max_dist, int32_t sector,
                          uint32_t flags, uint32_t *out_V);

/* tvs_debug_sector_rays on device memory: d_dem (rows*cols float) and d_out_V (nrows x ncols
 * u32) are device pointers on the current HIP device; the work is enqueued on hip_stream. */
int tvs_debug_sector_rays_async(const float *d_dem, int32_t rows, int32_t cols, double spacing,
                                double obs_height, int32_t n_sectors, double max_dist, int32_t sector,
                                uint32_t flags, uint32_t *d_out_V, void *hip_stream);

/* Work of one total viewshed call, from the sector geometry alone: line-of-sight cell
 * evaluations (per skewed row of nt samples, 2 * sum_{q<nt} min(q, K)) and POV-sector pairs. */
int tvs_los_evals(int32_t rows, int32_t cols, double spacing, int32_t n_sectors, double max_dist,
                  int64_t *out_evals, int64_t *out_pairs);

#ifdef __cplusplus
}
#endif

#endif /* LIBTVS_H */
