// tvs_internal.h -- launch-level types of libtvs (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tvs_geom.h"

// Sectors processed by one group of launches; their parameters travel as kernel arguments
// (72 x 56 B), so the library needs no host-to-device copy besides the caller's data.
#define TVS_CHUNK 72
// Sentinel columns on each side of a skewed row held in LDS by the sweep: a wavefront's 64
// lines of sight all stop at the same step, so lanes whose row ends earlier (at most 63 steps
// earlier) read these.
#define TVS_SWEEP_PAD 64

namespace tvs {

struct SecDev {
    double T;       // tan s'
    double scale;   // m^2 per index^2 unit of a half-sector ring: (pi / 2n) dx^2 / cos^2 s'
    double clip;    // area of the clipped last ring, index^2 units: rho^2 - K^2 (0 if unbounded)
    int64_t off;    // element offset of the sector's skewed buffers
    int32_t kase;   // base-frame case 0..3
    int32_t K;      // last target index in range, TVS_K_UNBOUNDED if max_dist never binds
    int32_t t0;     // first skewed row
    int32_t nrows;  // skewed rows t0 .. t0 + nrows - 1 (the last is Hx - 1)
    int32_t wrap;   // 0: row t is stored at row t - t0 of the sector's block; else (compacted
                    // layout, wrap = Hx + 1) at row t mod wrap
    float winv;     // 1 / wrap rounded to float (a first guess of the quotient)
};

struct ChunkArgs {
    SecDev s[TVS_CHUNK];
    int32_t nsec;   // sectors in this chunk
    int32_t H, W;   // grid dims
    int32_t pitch;  // row pitch (elements) of the skewed buffers
    double h0;      // observer height
    float h0f;      // observer height rounded to float
    int32_t k_base; // global index of s[0]
    int32_t pov_i, pov_j;  // singular POV (grid cell)
    int32_t rmq;    // sweep: 1 when the early exit's range-maximum table is in LDS (set by launch_sweep)
    int32_t pieces; // sweep: > 1 when each row is swept in pieces of piece_povs POVs (set by launch_sweep)
    int32_t piece_povs;
    int32_t pad1;
};
static_assert(sizeof(SecDev) == 56, "sector parameters: 56 bytes");
static_assert(sizeof(ChunkArgs) <= 4096, "chunk parameters must fit the kernel argument space");

// One (tile, sector) of a batch chunk: the sector's geometry (off = element offset of its skewed
// viewshed rows in the chunk buffer) and the tile it belongs to.
struct BatchEnt {
    SecDev s;
    const float *dem;  // the tile's DEM (device)
    const float *demT; // its transpose (W x H), or null: the 45..135 deg axes read the DEM by columns
    int32_t H, W;      // tile dims
    int32_t pitch;     // row pitch of this tile's skewed rows
    float h0f;         // observer height rounded to float
    double h0;         // observer height
};

// A tile of a batch, as the batched back-projection sees it.
struct BatchTile {
    double *out;       // the tile's total-viewshed map (device)
    int32_t H, W;
    int32_t ent0;      // first BatchEnt of this tile in the chunk (its sectors follow)
    int32_t bx;        // 64 x 64 cell blocks per block row
    int32_t blk0;      // first flat block of this tile
    int32_t pad;
};

// Singular queries launched together: one entry per (query, sector), and the queries.
struct SingSec {
    SecDev s;
    int32_t query;     // index into the query table
    int32_t pad;
};
struct SingQuery {
    const float *dem;  // the query's grid (device)
    int32_t H, W;
    int32_t pov_i, pov_j;
    int32_t sec0, nsec;  // its sectors in the SingSec table, in order
    double h0;
    float h0f;
    int32_t pad;
};

// Launchers (tvs_kernels.hip). All enqueue on `st` and return the launch status.
hipError_t launch_divtab(float2 *tab32, double2 *tab64, int n, hipStream_t st);
hipError_t launch_relocate(const ChunkArgs &a, int maxWx, int maxRows, const float *dem, void *skw,
                           bool f64, hipStream_t st);
// The sweep of a chunk. With skw null every workgroup gathers its skewed row from the grid (demT, the
// transposed grid, serves the 45..135 deg axes; null reads the grid down its columns); otherwise it
// reads the row from the skwDEM buffer the relocation wrote.
// nw: waves per workgroup of the lane-per-POV sweep (4, 8 or 16; otherwise chosen from the LDS the
// row takes); the sectors whose rows are longer than the LDS holds take the sweep in pieces or the
// streamed sweep, in launches of their own, whatever nw says. maxWx bounds every row's length (the
// frames' widths).
hipError_t launch_sweep(const ChunkArgs &a, int maxWx, const float *dem, const float *demT,
                        const void *skw, uint32_t *V, const float2 *tab32, const double2 *tab64, bool f64, bool scan,
                        bool rcp, bool prune, unsigned long long *work, hipStream_t st, int nw = 0);
// Does a skewed row of maxWx samples (with its sentinels) fit one workgroup's LDS? Longer rows are
// swept in pieces that stream their targets through LDS windows (any flags but the lane-per-target
// sweep, which needs whole rows).
bool sweep_row_fits(int maxWx, bool f64);
// demT[j][i] = dem[i][j] for an H x W grid.
hipError_t launch_transpose(const float *dem, float *demT, int H, int W, hipStream_t st);
hipError_t launch_backproj(const ChunkArgs &a, const uint32_t *V, double *out, float *kahan_sum,
                           float *kahan_c, int first, int last, hipStream_t st);
hipError_t launch_singular(const ChunkArgs &a, const float *dem, uint32_t *rayV, bool f64, bool rcp,
                           hipStream_t st);
hipError_t launch_singular_sum(const ChunkArgs &a, const uint32_t *rayV, double *area, int first,
                               hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
// *bad |= 1 when an elevation breaks the host entry points' rule (non-finite, or nonzero below 2^-60 m);
// launch_poison then fills the n map cells with NaN if *bad is set.
hipError_t launch_check_dem(const float *dem, int64_t n, uint32_t *bad, hipStream_t st);
hipError_t launch_poison(double *out, int64_t n, const uint32_t *bad, hipStream_t st);
// Batched path: a fused relocate + sweep over a chunk's (tile, sector, row) items (persistent with a
// counter, else one workgroup per item), then one back-projection launch over every tile of the
// chunk. launch_sweep_batch with grid == 0 only prepares the kernel's LDS limit.
hipError_t launch_sweep_batch(const BatchEnt *ent, const uint32_t *items, int nitems, unsigned int *counter,
                              uint32_t *V, const float2 *tab32, const double2 *tab64, bool f64, bool rcp,
                              int waves, int grid, int maxWx, int maxK, unsigned long long *work,
                              hipStream_t st);
hipError_t launch_backproj_batch(const BatchTile *tiles, int ntiles, int nblocks, const BatchEnt *ent, int nsec,
                                 const uint32_t *V, int first, hipStream_t st);
// Every query's 2 * nsec lines of sight, then each query's area (in sector order). With `bits`
// non-null also each ray's per-target visibility (`words` u32 per ray) and last target index.
hipError_t launch_singular_multi(const SingSec *secs, int nsecs, const SingQuery *qs, int nq, uint32_t *rayV,
                                 double *areas, bool f64, bool rcp, hipStream_t st, uint32_t *bits = nullptr,
                                 int words = 0, int32_t *mlast = nullptr);
// Mask / multiple viewshed over one grid from the rays of npov singular queries.
struct MaskArgs {
    int32_t H, W, n, npov;
    const int32_t *pov;     // 2 * npov (row, col)
    const double *cb, *sb;  // cos / sin of the 2n half-sector boundary angles (2q + 1) pi / 2n
    const double *ck;       // cos s' of the n sectors
    const double *rho;      // max_dist cos s' / spacing of the n sectors (inf if unbounded)
    const uint32_t *bits;   // per ray, `words` u32 of target visibility
    const int32_t *mlast;   // per ray, last target index
    int32_t words;
    int32_t pad;
    uint8_t *mask;          // nullable: 0/1 per cell
    uint32_t *count;        // nullable: POVs that see the cell
};
hipError_t launch_mask_multi(const MaskArgs &a, hipStream_t st);
// LDS of a sweep workgroup for rows of up to maxWx samples, without the early exit's
// range-maximum table (the launches add it when it fits).
size_t sweep_lds_bytes(int maxWx, bool f64);
constexpr int BATCH_BLOCK = 64;  // cells per side of a back-projection block

}  // namespace tvs
