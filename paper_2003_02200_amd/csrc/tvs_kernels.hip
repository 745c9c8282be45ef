// tvs_kernels.hip -- gfx950 kernels of libtvs, the sDEM total viewshed.
//
// Per group of sectors (Section 4.1 steps 1a-1d, Section 4.2):
//   k_relocate  DEM -> skwDEM (Alg. 6). Written as a gather: each skewed sample is produced
//               by exactly one thread as (1-r_j) X[u][j] + r_j X[u+1][j], from a tile of the
//               base frame staged in LDS by coalesced row reads of the DEM (transposed on the
//               way in for the 45..135 deg axes). Alg. 6's scatter with two "+=" per DEM
//               cell has adjacent threads updating the same skwDEM element; a gather has one
//               writer per output.
//   k_sweep     skwDEM -> skwVS (Alg. 7 / Alg. 8). One workgroup holds one skewed row (one
//               line of sight of every POV on it) in LDS. A wavefront owns 64 consecutive
//               POVs, one per lane, and steps all 64 lines of sight together: step m reads
//               z[q+m] (forward) or z[q-m] (backward), forms the slope (z - h)/m, compares it
//               with the lane's running maximum and adds the ring weight 2m+1 when visible.
//               The ring sums are integers (Alg. 8's dd^2 - open_dd^2 telescopes to a sum of
//               2m+1 over visible samples), so they are kept exactly in u32. Exact bounds from
//               elevation maxima (per block, and sliding over 40 samples where the LDS allows)
//               skip 32-step blocks no lane can see into and stop a wavefront when nothing
//               further can be visible (same results as the full walk).
//   k_backproj  skwVS -> VS (Alg. 9): each DEM cell blends the two skewed samples around it,
//               scales by the half-sector ring area (Alg. 1's pi/ns, Alg. 7's 1/cos^2) and
//               accumulates over sectors in double.
// and the singular viewshed (Alg. 1-3) as a ray scan: one wavefront per line of sight, lanes =
// 64 consecutive targets, the horizon carried by a wavefront prefix-max.
//
// Floating point: the default path keeps the interpolated elevation in double, forms h = z + h0
// and d = z - h in double and the slope as d times the double reciprocal of m, and compares in
// double. The float path rounds the interpolated elevation to float and does the same steps in
// float. Either precision can instead form the correctly rounded quotient d / m (exact mode:
// reciprocal, one product and one FMA correction, exact for every integer m in range).
// Explicit _rn intrinsics keep the compiler from contracting any step into an FMA.
#include <hip/hip_runtime.h>

#include <atomic>
#include <climits>
#include <mutex>
#include <unordered_map>
#include <math.h>
#include <stdint.h>

#include "tvs_geom.h"
#include "tvs_internal.h"

namespace tvs {

// ----------------------------------------------------------------------------- numerics

__device__ __forceinline__ float slope_div(float d, float2 t) {  // t = {m, RN(1/m)}
    float q = __fmul_rn(d, t.y);
    float r = __fmaf_rn(-q, t.x, d);
    return __fmaf_rn(r, t.y, q);
}
__device__ __forceinline__ double slope_div(double d, double2 t) {
    double q = __dmul_rn(d, t.y);
    double r = __fma_rn(-q, t.x, d);
    return __fma_rn(r, t.y, q);
}
// Default float slope: the float difference times the float reciprocal of m (one product;
// within one ulp of the correctly rounded quotient).
__device__ __forceinline__ float slope_rcp(float d, float2 t) { return __fmul_rn(d, t.y); }
template <bool RCP> __device__ __forceinline__ float slope(float d, float2 t) {
    return RCP ? slope_rcp(d, t) : slope_div(d, t);
}
// Default double slope: the double difference times the double reciprocal of m.
template <bool RCP> __device__ __forceinline__ double slope(double d, double2 t) {
    return RCP ? __dmul_rn(d, t.y) : slope_div(d, t);
}
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float sub_rn(float a, float b) { return __fsub_rn(a, b); }
__device__ __forceinline__ double sub_rn(double a, double b) { return __dsub_rn(a, b); }

// One visibility step: vis = th > mx (strict), bits = 2 bits + vis, mx = max(mx, th). The
// compare writes VCC and the add-with-carry takes it as carry-in (two VALU instructions; the
// compiler does not form this pair from C++). max equals "vis ? th : mx" here: slopes are
// never NaN except on sentinel lanes, where both keep mx.
// The maximum is taken in the same block: slopes are never NaN, so no canonicalising of the
// running maximum is needed between blocks.
__device__ __forceinline__ void vis_step(float th, float &mx, uint32_t &bits) {
    asm("v_cmp_gt_f32 vcc, %2, %1\n\t"
        "v_addc_co_u32 %0, vcc, %0, %0, vcc\n\t"
        "v_max_f32 %1, %1, %2"
        : "+v"(bits), "+v"(mx)
        : "v"(th)
        : "vcc");
}
__device__ __forceinline__ void vis_step(double th, double &mx, uint32_t &bits) {
    asm("v_cmp_gt_f64 vcc, %2, %1\n\t"
        "v_addc_co_u32 %0, vcc, %0, %0, vcc\n\t"
        "v_max_f64 %1, %1, %2"
        : "+v"(bits), "+v"(mx)
        : "v"(th)
        : "vcc");
}

template <typename Tz> struct Tab;
template <> struct Tab<float> { using type = float2; };
template <> struct Tab<double> { using type = double2; };

template <typename Tz> __device__ __forceinline__ Tz neg_inf();
template <> __device__ __forceinline__ float neg_inf<float>() { return -__builtin_inff(); }
template <> __device__ __forceinline__ double neg_inf<double>() { return -__builtin_inf(); }

// Interpolated elevation (double) of the base-frame sample at row u + r of column q, rows
// clamped to [0, Hx-1]; `row(v)` returns X[v][q] as float.
template <typename RowFn>
__device__ __forceinline__ double interp(int u, double r, int Hx, RowFn row) {
    const int ua = min(max(u, 0), Hx - 1);
    const int ub = min(max(u + 1, 0), Hx - 1);
    const float a = row(ua);
    if (r == 0.0 || ua == ub) return (double)a;
    const float b = row(ub);
    const double w = __dsub_rn(1.0, r);
    return __dadd_rn(__dmul_rn(w, (double)a), __dmul_rn(r, (double)b));
}

// ------------------------------------------------------------------- wavefront primitives
// DPP lane moves of the GFX9 family (row_shr, row_bcast, wave_shr). Lanes without a source
// keep `old`.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_mov(float old, float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL,
                                                      ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_mov(double old, double x) {
    const int2 o = *reinterpret_cast<const int2 *>(&old);
    const int2 v = *reinterpret_cast<const int2 *>(&x);
    int2 res;
    res.x = __builtin_amdgcn_update_dpp(o.x, v.x, CTRL, ROW_MASK, 0xf, false);
    res.y = __builtin_amdgcn_update_dpp(o.y, v.y, CTRL, ROW_MASK, 0xf, false);
    return *reinterpret_cast<const double *>(&res);
}
template <typename T> __device__ __forceinline__ T vmax(T a, T b) { return a > b ? a : b; }
// max of two values known not to be NaN, as one instruction (the compare-and-select form above
// takes three for doubles)
__device__ __forceinline__ double vmax_plain(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float vmax_plain(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Inclusive prefix maximum over the 64 lanes (lane l gets max of lanes 0..l).
template <typename T>
__device__ __forceinline__ T wave_prefix_max(T x) {
    const T lo = neg_inf<T>();
    x = vmax(x, dpp_mov<0x111>(lo, x));        // row_shr:1
    x = vmax(x, dpp_mov<0x112>(lo, x));        // row_shr:2
    x = vmax(x, dpp_mov<0x114>(lo, x));        // row_shr:4
    x = vmax(x, dpp_mov<0x118>(lo, x));        // row_shr:8
    x = vmax(x, dpp_mov<0x142, 0xa>(lo, x));   // row_bcast:15 into rows 1 and 3
    x = vmax(x, dpp_mov<0x143, 0xc>(lo, x));   // row_bcast:31 into rows 2 and 3
    return x;
}
// Lane l gets lane l-1's value; lane 0 gets `old` (wave_shr:1).
template <typename T>
__device__ __forceinline__ T wave_shift_up(T old, T x) { return dpp_mov<0x138>(old, x); }

template <typename T>
__device__ __forceinline__ T lane63(T x) {
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
    } else {
        int2 v = *reinterpret_cast<const int2 *>(&x);
        v.x = __builtin_amdgcn_readlane(v.x, 63);
        v.y = __builtin_amdgcn_readlane(v.y, 63);
        return *reinterpret_cast<const double *>(&v);
    }
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Stored row of skewed row t of sector s: t - t0, or in the compacted layout t mod wrap (the
// float quotient is off by at most one, corrected by one step).
__device__ __forceinline__ int skw_prow(const SecDev &s, int t) {
    if (!s.wrap) return t - s.t0;
    int p = t - s.wrap * (int)floorf((float)t * s.winv);
    if (p < 0) p += s.wrap;
    else if (p >= s.wrap) p -= s.wrap;
    return p;
}

// Element offset of skewed row t of sector s in its skewed buffers.
__device__ __forceinline__ int64_t skw_row(const SecDev &s, int t, int pitch) {
    return s.off + (int64_t)skw_prow(s, t) * pitch;
}

// ------------------------------------------------------------------------ small kernels

// Entry i holds {m, RN(1/m)} for m = i + 1, so that the 32-step blocks of the sweep, which
// start at m = 1, 33, 65, ..., begin on 256-byte boundaries of the table.
__global__ void k_divtab(float2 *tab32, double2 *tab64, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float mf = (float)(i + 1);
    const double md = (double)(i + 1);
    tab32[i] = make_float2(mf, __fdiv_rn(1.0f, mf));
    tab64[i] = make_double2(md, __ddiv_rn(1.0, md));
}

// *bad |= 1 when some elevation is not finite, or is nonzero but below 2^-60 m in magnitude (the rule
// the host entry points check on the host: biased exponent 255, or below 127 - 60 with a nonzero value).
__global__ __launch_bounds__(256) void k_check_dem(const float *__restrict__ dem, int64_t n, uint32_t *bad) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool b = false;
    for (int64_t x = i0; x < n; x += stride) {
        const uint32_t u = __float_as_uint(dem[x]);
        const uint32_t e = (u >> 23) & 0xFFu;
        b |= e == 0xFFu || (e < 67u && (u & 0x7FFFFFFFu) != 0u);
    }
    if (__builtin_amdgcn_ballot_w64(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

// Every cell of the map becomes NaN when *bad is set: the asynchronous entry points cannot return a
// status for what they find on the device.
__global__ __launch_bounds__(256) void k_poison(double *__restrict__ out, int64_t n, const uint32_t *bad) {
    if (*bad == 0u) return;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = i0; x < n; x += stride) out[x] = __builtin_nan("");
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = i; x < n; x += stride) p[x] = v;
}

// A sector's base frame X (Hx x Wx) as strides into the DEM: X[p][q] = base[p * rs + q * cs]. With
// the transposed grid `demT` (W x H, row-major) the frames of the 45..135 deg axes (cases 1 and 2)
// read along rows of demT, so consecutive columns q of X are consecutive addresses in every case.
struct FrameRef {
    const float *base;
    int64_t rs;
    int64_t cs;
};
__device__ __forceinline__ FrameRef frame_ref(int kase, int H, int W, const float *dem, const float *demT) {
    switch (kase) {
    case 0: return FrameRef{dem, W, 1};
    case 1: return demT ? FrameRef{demT, H, 1} : FrameRef{dem, 1, W};
    case 2: return demT ? FrameRef{demT + (int64_t)(W - 1) * H, -(int64_t)H, 1} : FrameRef{dem + (W - 1), -1, W};
    default: return FrameRef{dem + (W - 1), W, -1};
    }
}

// demT[j][i] = dem[i][j] for an H x W grid: 64 x 64 tiles through LDS (pitch 65), both sides coalesced.
__global__ __launch_bounds__(256) void k_transpose(const float *__restrict__ dem, float *__restrict__ demT, int H,
                                                   int W) {
    __shared__ float t[64 * 65];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int r = wv; r < 64; r += 4) {
        const int i = i0 + r, j = j0 + lane;
        if (i < H && j < W) t[r * 65 + lane] = dem[(int64_t)i * W + j];
    }
    __syncthreads();
    for (int r = wv; r < 64; r += 4) {
        const int j = j0 + r, i = i0 + lane;
        if (i < H && j < W) demT[(int64_t)j * H + i] = t[lane * 65 + r];
    }
}

// --------------------------------------------------------------------------- relocation
// A workgroup owns a strip of 64 base-frame columns of one sector and walks down RL_SEG of its
// skewed rows in batches of 32. Skewed row t of column j blends base rows t + d_j and t + d_j + 1,
// and over 64 columns d_j spans at most 64, so a batch needs at most 32 + 65 consecutive base
// rows. They sit in an LDS ring of 128 rows (slot u mod 128, row pitch 65 words so that the
// transposed stores of cases 1/2 spread over the banks); every base row is read from the DEM
// once per workgroup, clamped to the frame. While a batch is interpolated, the 32 base rows the
// next batch adds are already in flight into registers; they replace rows no later batch needs.
// Each thread interpolates one column and stores along the skewed row (64 consecutive columns
// per wavefront).
constexpr int RL_TW = 64;     // columns per strip
constexpr int RL_TB = 32;     // skewed rows per batch (= base rows added per batch)
constexpr int RL_RING = 128;  // ring rows: >= RL_TB + 65 rows in use + RL_TB rows arriving
constexpr int RL_LP = RL_TW + 1;
constexpr int RL_SEG = 512;   // skewed rows per workgroup

struct RelocFrame {
    const float *dem;
    int64_t xb;   // X[u][q] = dem[xb + u * xsu + q * xsq]
    int xsu, xsq;
    int Hx, j0, ncol;
};

// Base rows u0 .. u0 + 31 (clamped to the frame) of the strip: 8 values per thread.
__device__ __forceinline__ void reloc_load(const RelocFrame &f, int u0, int wv, int lane, float (&v)[8]) {
    if (f.xsq == 1 || f.xsq == -1) {
        // base rows are grid rows: wavefront wv takes rows u0 + wv + 4i, lanes along the row
        const int64_t col = (int64_t)(f.j0 + min(lane, f.ncol - 1)) * f.xsq;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int u = min(max(u0 + wv + 4 * i, 0), f.Hx - 1);
            v[i] = f.dem[f.xb + (int64_t)u * f.xsu + col];
        }
    } else {
        // base rows are grid columns: a half-wavefront reads 32 consecutive base rows of one base
        // column (one grid row), base column c = (lane >> 5) + 2 (wv + 4i)
        const int u = min(max(u0 + (lane & 31), 0), f.Hx - 1);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int c = (lane >> 5) + 2 * (wv + 4 * i);
            v[i] = f.dem[f.xb + (int64_t)u * f.xsu + (int64_t)(f.j0 + min(c, f.ncol - 1)) * f.xsq];
        }
    }
}

__device__ __forceinline__ void reloc_store(const RelocFrame &f, int u0, int wv, int lane, const float (&v)[8],
                                            float *ring) {
    if (f.xsq == 1 || f.xsq == -1) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (lane < f.ncol) ring[((u0 + wv + 4 * i) & (RL_RING - 1)) * RL_LP + lane] = v[i];
    } else {
        const int slot = (u0 + (lane & 31)) & (RL_RING - 1);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int c = (lane >> 5) + 2 * (wv + 4 * i);
            if (c < f.ncol) ring[slot * RL_LP + c] = v[i];
        }
    }
}

template <typename Tz>
__global__ __launch_bounds__(256) void k_relocate(const ChunkArgs a, const float *__restrict__ dem,
                                                  Tz *__restrict__ skw) {
    __shared__ float ring[RL_RING * RL_LP];
    const SecDev &s = a.s[blockIdx.z];
    RelocFrame f;
    int Wx;
    frame_dims(s.kase, a.H, a.W, f.Hx, Wx);
    f.j0 = blockIdx.x * RL_TW;
    if (f.j0 >= Wx) return;
    const int jl = min(f.j0 + RL_TW - 1, Wx - 1);
    f.ncol = jl - f.j0 + 1;
    f.dem = dem;
    switch (s.kase) {
    case 0: f.xb = 0; f.xsu = a.W; f.xsq = 1; break;
    case 1: f.xb = 0; f.xsu = 1; f.xsq = a.W; break;
    case 2: f.xb = a.W - 1; f.xsu = -1; f.xsq = a.W; break;
    default: f.xb = a.W - 1; f.xsu = a.W; f.xsq = -1; break;
    }
    int dlo, dhi;
    double rlo, rhi;
    col_offset(s.T, f.j0, dlo, rlo);
    col_offset(s.T, jl, dhi, rhi);
    // skewed rows with a sample in the strip: t + d_j in [-1, Hx - 1] for some column j
    const int tS = max(s.t0 + (int)blockIdx.y * RL_SEG, max(s.t0, -1 - dhi));
    const int tE = min(s.t0 + (int)blockIdx.y * RL_SEG + RL_SEG - 1, min(s.t0 + s.nrows - 1, f.Hx - 1 - dlo));
    if (tS > tE) return;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int uA = tS + dlo;  // first base row any batch reads
    {
        float v0[8], v1[8], v2[8], v3[8];
        reloc_load(f, uA, wv, lane, v0);
        reloc_load(f, uA + 32, wv, lane, v1);
        reloc_load(f, uA + 64, wv, lane, v2);
        reloc_load(f, uA + 96, wv, lane, v3);
        reloc_store(f, uA, wv, lane, v0, ring);
        reloc_store(f, uA + 32, wv, lane, v1, ring);
        reloc_store(f, uA + 64, wv, lane, v2, ring);
        reloc_store(f, uA + 96, wv, lane, v3, ring);
    }
    __syncthreads();
    const int q = f.j0 + min(lane, f.ncol - 1);
    int d;
    double r;
    col_offset(s.T, q, d, r);
    // existing rows of this column: u = t + d in [-1 (only if r > 0), Hx - 1]
    const int tfirst = (r != 0.0 ? -1 : 0) - d;
    const int tlast = f.Hx - 1 - d;
    const double w = __dsub_rn(1.0, r);
    const bool mine = lane < f.ncol;
    const int nb = (tE - tS) / RL_TB + 1;
    for (int b = 0; b < nb; ++b) {
        const int tb = tS + b * RL_TB;
        float v[8];
        const bool more = b + 1 < nb;
        if (more) reloc_load(f, uA + RL_RING + b * RL_TB, wv, lane, v);
        // stored row of this thread's first skewed row of the batch; the others follow 4 apart
        const int pf = skw_prow(s, tb + wv);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int t = tb + wv + 4 * i;
            int p = pf + 4 * i;
            if (s.wrap) {
                if (s.wrap > 28) p -= p >= s.wrap ? s.wrap : 0;
                else p = skw_prow(s, t);
            }
            if (mine && t <= tE && t >= tfirst && t <= tlast) {
                const int u = t + d;
                const float av = ring[(u & (RL_RING - 1)) * RL_LP + lane];
                double z = (double)av;
                if (r != 0.0 && u >= 0 && u < f.Hx - 1) {
                    const float bv = ring[((u + 1) & (RL_RING - 1)) * RL_LP + lane];
                    z = __dadd_rn(__dmul_rn(w, (double)av), __dmul_rn(r, (double)bv));
                }
                // + 0 turns a -0 elevation into +0 (no other value changes): the sweep's sign
                // tests rely on slopes never being -0
                skw[s.off + (int64_t)p * a.pitch + q] = add_rn((Tz)z, (Tz)0);
            }
        }
        if (more) {
            __syncthreads();
            reloc_store(f, uA + RL_RING + b * RL_TB, wv, lane, v, ring);
            __syncthreads();
        }
    }
}

// -------------------------------------------------------------------------------- sweep

// Levels of the early exit's range-maximum table: windows of 1, 2, .., 32 blocks of 32 samples,
// answering the maximum over any 1..64 consecutive blocks with two reads.
constexpr int RMQ_LEVELS = 6;
// Entries of the sliding maxima beyond each end of the row (copies of the end entries).
constexpr int SLIDE_PAD = 8;

// Ring sums of 32 visibility bits: step m0+s lands in bit 31-s, so the ring weight 2m+1 of set
// bit b is (2 m0 + 63) - 2b, and sum_b b = sum_k 2^k popc(bits & M_k).
struct RingAcc {
    uint32_t base = 0;                                // sum over blocks of (2 m0 + 63) popc(bits)
    uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0;  // sum over blocks of popc(bits & M_k)
    __device__ __forceinline__ void add(uint32_t bits, int m0) {
        base += __umul24((uint32_t)(2 * m0 + 63), (uint32_t)__popc(bits));
        q0 += __popc(bits & 0xAAAAAAAAu);
        q1 += __popc(bits & 0xCCCCCCCCu);
        q2 += __popc(bits & 0xF0F0F0F0u);
        q3 += __popc(bits & 0xFF00FF00u);
        q4 += __popc(bits & 0xFFFF0000u);
    }
    __device__ __forceinline__ uint32_t total() const {
        return base - 2u * (q0 + 2u * q1 + 4u * q2 + 8u * q3 + 16u * q4);
    }
};

// One direction of the lines of sight of a wavefront's 64 POVs. `zp` points at each lane's POV in
// the LDS row; `mb` is the last step any lane of the wavefront needs (lanes whose row ends earlier
// read -inf sentinels, which are never visible). Steps m < K add the whole ring 2m+1 to U; the
// step m = K (the ring clipped at rho) is returned as 0/1. Steps run in blocks of 32 whose table
// entries {m, 1/m} are wave-uniform (scalar loads); each step is subtract, slope, compare +
// add-with-carry into the bit mask, max. Returns in `done` the number of steps taken and, with
// COUNT, in `skipped` the lane's steps inside skipped blocks.
//
// Early exit (PRUNE): before each block the wavefront stops when no target from step m on can
// be visible on any live lane. zs bounds every elevation a lane still reads: the maximum over the
// 32-sample blocks from the nearest one at step m to block `bfar`, the farthest any lane of the
// wavefront reaches within K, read from the range-maximum table `rmq` (two reads, values rounded
// up to float); for ranges longer than the table covers, or without it, `bnd` holds the maxima
// accumulated away from the POVs to the row end (suffix maxima forward, prefix maxima
// backward). Rounding is monotone:
// for m' >= m, RN(z - h) <= RN(zs - h) and the slope of RN(zs - h) >= 0 does not grow with m', so
// every remaining slope is at most max(slope(RN(zs - h), m), 0) (a negative difference gives a
// negative slope). When that bound is <= the lane's horizon, no later target passes the strict
// test, the clipped last ring included, and the ring sums are those of the full walk.
// With SLIDE (the number of table levels, 0 without) the skip test reads the sliding maxima `slide`
// instead of the table's level 1, and the launch keeps every exit range within the table (there is
// no `bnd`).
template <typename Tz, int DIR, bool RCP, bool PRUNE, int SLIDE, bool COUNT>
__device__ __forceinline__ uint32_t sweep_dir(const Tz *zp, Tz h, int mb, int K,
                                              const typename Tab<Tz>::type *__restrict__ tab, uint32_t &U,
                                              const Tz *bnd, const float *rmq, int nb, int bfar, int pbase,
                                              int q, bool live, int own, int &done, int &skipped,
                                              const float *slide) {
    // a lane past the row end starts with a +inf horizon: it never sees a target and never
    // holds back the early exit (its sums are discarded)
    Tz mx = (PRUNE && !live) ? -neg_inf<Tz>() : neg_inf<Tz>();
    const int mfull = (mb == K) ? K - 1 : mb;
    constexpr int NLEV = SLIDE ? SLIDE : RMQ_LEVELS;
    // maximum over blocks lo..hi (1 <= hi - lo + 1 <= 2^NLEV) from the range table
    auto range_max = [&](int lo, int hi) -> Tz {
        const int l = min(31 - __builtin_clz(hi - lo + 1), NLEV - 1);
        const float *T = rmq + l * nb;
        float zf;  // the table holds no NaN: a plain max, without canonicalising its inputs
        asm("v_max_f32 %0, %1, %2" : "=v"(zf) : "v"(T[lo]), "v"(T[hi - (1 << l) + 1]));
        return (Tz)zf;
    };
    // Every slope of steps m' in [m1, m2] whose elevation is at most zs is at most
    // max(slope(d, m1), slope(d, m2)) with d = RN(zs - h): for d >= 0 the nearest step bounds
    // it, for d < 0 the farthest (rounding is monotone in both operands).
    auto bounded_by = [&](Tz zs, int m1, int m2) -> bool {
        const Tz d = sub_rn(zs, h);
        const Tz b = vmax_plain(slope<RCP>(d, tab[m1 - 1]), slope<RCP>(d, tab[m2 - 1]));
        // every lane of the (fully active) wavefront agrees; a wave-uniform answer keeps the
        // step counter, and with it the table loads, scalar
        return __builtin_amdgcn_ballot_w64(b <= mx) == ~0ull;
    };
    // the wavefront stops: no target from step mm to the last one (mb) can be visible
    auto hidden_from = [&](int mm) -> bool {
        // blocks a lane may still read: from the nearest at step mm to bfar, the farthest any
        // lane of the wavefront reaches within K (the range table), else to the row end
        const int bnear = (pbase + DIR * mm) >> 5;
        const int lo = DIR > 0 ? bnear : bfar, hi = DIR > 0 ? bfar : bnear;
        const int len = hi - lo + 1;
        // (with SLIDE a range past the table bounds nothing: +inf, and the wavefront walks on)
        const Tz zs = (rmq && len >= 1 && len <= 1 << NLEV) ? range_max(lo, hi)
                      : SLIDE                                ? -neg_inf<Tz>()
                                                             : bnd[bnear];
        return bounded_by(zs, mm, mb);
    };
    // the wavefront skips steps mm .. mm + 31: none of their targets can be visible on any lane.
    // A lane's 32 targets lie in two consecutive blocks, whose maximum is level 1 of the table;
    // with SLIDE, in the 40 samples from the 8-aligned position at or before the first, whose
    // maximum is slide[first >> 3]. Steps mm = 1 + 32 k put that entry 4 k after (DIR > 0) or
    // before (DIR < 0) the lane's entry for mm = 1, so the lane keeps a pointer to that one and a
    // test adds a uniform offset. Entries beyond the row's hold its end entries: the indices stay
    // within 8 of the row's (a lane's reads lie inside its sentinels), an end entry still covers
    // every target inside it, beyond it lie -inf sentinels, and a lane past the row end has a +inf
    // horizon.
    const float *sl = SLIDE != 0 ? slide + ((DIR > 0 ? q + 1 : q - 32) >> 3) : nullptr;
    auto block_hidden = [&](int mm) -> bool {
        float zf;
        if constexpr (SLIDE != 0) {
            zf = sl[DIR * ((mm - 1) >> 3)];
        } else {
            const int first = DIR > 0 ? q + mm : q - mm - 31;  // the lane's lowest target position
            const int b = min(max(first >> 5, 0), nb - 1);
            zf = rmq[nb + b];
        }
        return bounded_by((Tz)zf, mm, mm + 31);
    };
    RingAcc ra;
    uint32_t bits = 0;
    int m = 1;
    bool stop = false;
    int busy = 0;  // lanes that saw a target in the last block: from 32 on, the next is not tested
    skipped = 0;
    for (; m + 31 <= mfull; m += 32) {
        if (PRUNE) m = __builtin_amdgcn_readfirstlane(m);  // keeps the table loads on the scalar path
        // The exit test passing implies the skip test passing (its blocks lie inside the exit's
        // range and its steps inside the remaining ones), so the exit is tested only for blocks
        // that can be skipped; a block that must be evaluated costs one test.
        if (PRUNE && m > 1 && (!rmq || (busy < 32 && block_hidden(m)))) {
            if (hidden_from(m)) {
                stop = true;
                break;
            }
            if (rmq) {
                // no horizon moves and no bit is set: the block changes nothing
                if (COUNT) skipped += max(0, min(own, m + 31) - m + 1);
                continue;
            }
        }
        const auto *t = static_cast<const typename Tab<Tz>::type *>(__builtin_assume_aligned(tab + (m - 1), 256));
#pragma unroll
        for (int s = 0; s < 32; ++s) vis_step(slope<RCP>(sub_rn(zp[DIR * (m + s)], h), t[s]), mx, bits);
        // 32 steps have shifted every earlier bit out: `bits` is this block's. Far from the POVs
        // most blocks see nothing on any lane, and skip the ring sums.
        const unsigned long long seen = __builtin_amdgcn_ballot_w64(bits != 0u);
        if (seen) ra.add(bits, m);
        // skipping a test only evaluates a block it might have skipped
        busy = __builtin_amdgcn_readfirstlane((int)__popcll(seen));
    }
    if (PRUNE && !stop && m > 1 && m <= mb) stop = hidden_from(m);
    uint32_t acc = ra.total();
    uint32_t e = 0;
    if (!stop) {
        for (; m <= mfull; ++m) {
            const Tz th = slope<RCP>(sub_rn(zp[DIR * m], h), tab[m - 1]);
            acc += th > mx ? (uint32_t)(2 * m + 1) : 0u;
            mx = vmax_plain(mx, th);
        }
        if (mb == K && K >= 1) e = slope<RCP>(sub_rn(zp[DIR * K], h), tab[K - 1]) > mx ? 1u : 0u;
    }
    U += acc;
    done = stop ? m - 1 : mb;
    return e;
}

// x rounded up to float: an upper bound of x that the table can hold in half the bytes.
__device__ __forceinline__ float ru_float(double x) {
    float f = (float)x;
    if ((double)f < x) f = __int_as_float(__float_as_int(f) + (f >= 0.0f ? 1 : -1));
    return f;
}
__device__ __forceinline__ float ru_float(float x) { return x; }

// Maxima of the row's samples 8k .. 8k + 39 (sentinels past the row end), rounded up to float, at
// slide[k] for k < 4 nb. A wavefront reads 64 consecutive samples; three row shifts leave the
// maximum of each group of 8 lanes in its last lane. With `blk` the block maxima (rounded up) come
// from these groups, four per block. Then each entry takes the maximum of itself and the next
// four, in tiles of one workgroup: a tile reads before any of its entries is written, and later
// tiles read only entries at or beyond their own.
template <typename Tz>
__device__ void sliding_max40(const Tz *z, int nb, float *slide, float *blk) {
    const int lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    const int n8 = nb << 2;
    const Tz lo = neg_inf<Tz>();
    // c + 63 <= 32 nb + 31 <= nt + 62: inside the sentinels
    for (int c = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) << 6; c < n8 << 3; c += nw << 6) {
        Tz x = z[c + lane];
        x = vmax(x, dpp_mov<0x111>(lo, x));  // row_shr:1
        x = vmax(x, dpp_mov<0x112>(lo, x));  // row_shr:2
        x = vmax(x, dpp_mov<0x114>(lo, x));  // row_shr:4
        const int k = (c + lane) >> 3;
        if ((lane & 7) == 7 && k < n8) slide[k] = ru_float(x);
    }
    __syncthreads();
    if (blk) {
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
            blk[b] = fmaxf(fmaxf(slide[4 * b], slide[4 * b + 1]), fmaxf(slide[4 * b + 2], slide[4 * b + 3]));
        __syncthreads();
    }
    for (int t0 = 0; t0 < n8; t0 += blockDim.x) {
        const int k = t0 + threadIdx.x;
        float v = neg_inf<float>();
        if (k < n8) {
            v = slide[k];
#pragma unroll
            for (int i = 1; i <= 4; ++i)
                if (k + i < n8) v = fmaxf(v, slide[k + i]);
        }
        __syncthreads();
        if (k < n8) slide[k] = v;
        __syncthreads();
    }
}

// Per-block elevation maxima of a row of nt samples (followed by -inf sentinels): pre[b] is the
// maximum over blocks 0..b, suf[b] over blocks b..nb-1, each scanned by one wavefront with the
// wavefront prefix-max. With `rmq`, level l of the table holds at rmq[l nb + b] the maximum over
// blocks b .. min(b + 2^l, nb) - 1, rounded up to float. With SLIDE the table (SLIDE levels) and
// the sliding maxima of 40 samples are built instead (no suf and pre).
template <typename Tz, int SLIDE>
__device__ void block_bounds(const Tz *z, int nb, Tz *suf, Tz *pre, float *rmq, float *slide) {
    constexpr int NLEV = SLIDE ? SLIDE : RMQ_LEVELS;
    if constexpr (SLIDE != 0) {
        sliding_max40(z, nb, slide, rmq);  // the table's first level from its groups of 8
        // SLIDE_PAD copies of each end entry on either side (sliding_max40 ends with a barrier)
        if (threadIdx.x < 2 * SLIDE_PAD) {
            const int x = threadIdx.x, n8 = nb << 2;
            const float v = x < SLIDE_PAD ? slide[0] : slide[n8 - 1];
            slide[x < SLIDE_PAD ? x - SLIDE_PAD : n8 + x - SLIDE_PAD] = v;
        }
    } else {
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            Tz m = z[32 * b];
#pragma unroll
            for (int i = 1; i < 32; ++i) m = vmax(m, z[32 * b + i]);
            suf[b] = m;
            pre[b] = m;
            if (rmq) rmq[b] = ru_float(m);
        }
    }
    __syncthreads();
    if (rmq) {
        for (int l = 1; l < NLEV; ++l) {
            const float *src = rmq + (l - 1) * nb;
            float *dst = rmq + l * nb;
            const int half = 1 << (l - 1);
            for (int b = threadIdx.x; b < nb; b += blockDim.x) dst[b] = fmaxf(src[b], src[min(b + half, nb - 1)]);
            __syncthreads();
        }
    }
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (!SLIDE && wv < 2) {
        Tz *arr = wv == 0 ? pre : suf;
        Tz carry = neg_inf<Tz>();
        for (int c = 0; c < nb; c += 64) {
            const int i = c + lane;
            const int b = wv == 0 ? i : nb - 1 - i;  // wavefront 1 scans from the right
            Tz x = i < nb ? arr[b] : neg_inf<Tz>();
            x = vmax(wave_prefix_max(x), carry);
            if (i < nb) arr[b] = x;
            carry = lane63(x);
        }
    }
    __syncthreads();
}

template <typename Tz> __device__ __forceinline__ Tz h0_of(const ChunkArgs &a);
template <> __device__ __forceinline__ float h0_of<float>(const ChunkArgs &a) { return a.h0f; }
template <> __device__ __forceinline__ double h0_of<double>(const ChunkArgs &a) { return a.h0; }

// Skewed row index for workgroup b of a sector with N rows: middle-out, so the long rows of
// the parallelogram start first and the short corner rows fill the tail.
__device__ __forceinline__ int row_of_block(int b, int N) {
    const int c = (N - 1) >> 1;
    return (b & 1) ? c + ((b + 1) >> 1) : c - (b >> 1);
}

// Samples w0 .. w0 + n - 1 of skewed row t (first column jlo) gathered straight from the base frame
// into row[TVS_SWEEP_PAD ..] (Alg. 6's interpolation: the double blend (1 - r_j) X[u][j] + r_j X[u + 1][j],
// rows clamped, -0 made +0), with TVS_SWEEP_PAD -inf sentinels on both sides, so that no skwDEM buffer
// exists in HBM. Consecutive samples read consecutive columns of X: coalesced when the frame's columns
// are contiguous (the DEM for the 0..45 and 135..180 deg axes, its transpose for the others);
// neighbouring skewed rows reuse the same cache lines.
template <typename Tz>
__device__ __forceinline__ void gather_span(const FrameRef &F, int Hx, const SecDev &s, int t, int jlo, int w0, int n,
                                            Tz *row) {
    for (int x = threadIdx.x; x < n + 2 * TVS_SWEEP_PAD; x += blockDim.x) {
        const int q = x - TVS_SWEEP_PAD;
        Tz v = neg_inf<Tz>();
        if (q >= 0 && q < n) {
            const int j = jlo + w0 + q;
            int d;
            double r;
            col_offset(s.T, j, d, r);
            const int u = t + d;
            const float *col = F.base + (int64_t)j * F.cs;
            const float av = col[(int64_t)min(max(u, 0), Hx - 1) * F.rs];
            double z = (double)av;
            if (r != 0.0 && u >= 0 && u < Hx - 1) {
                const float bv = col[(int64_t)(u + 1) * F.rs];
                z = __dadd_rn(__dmul_rn(__dsub_rn(1.0, r), (double)av), __dmul_rn(r, (double)bv));
            }
            v = add_rn((Tz)z, (Tz)0);
        }
        row[x] = v;
    }
    __syncthreads();
}

// Skewed row ri of sector s, all of it. Returns nt (0 for an empty row).
template <typename Tz>
__device__ __forceinline__ int gather_row(const FrameRef &F, int Hx, int Wx, const SecDev &s, int ri, Tz *row,
                                          int &jlo) {
    const int t = s.t0 + ri;
    jlo = row_first(s.T, t, Hx, Wx);
    const int jhi = row_last(s.T, t, Hx, Wx);
    const int nt = jhi - jlo + 1;
    if (nt <= 0) return 0;
    gather_span<Tz>(F, Hx, s, t, jlo, 0, nt, row);
    return nt;
}

// Where a single-grid sweep takes its rows: gathered from the grid (and its transpose), or read
// from the skwDEM buffer the relocation kernel wrote.
struct RowSrc {
    const float *dem;
    const float *demT;  // null: cases 1 and 2 read the DEM down its columns
    int gather;         // 1: gather from the grid; 0: read skwDEM
    int pad;
};

// Skewed row `ri` (existing samples jlo .. jlo + nt - 1) into LDS with TVS_SWEEP_PAD -inf sentinels on
// both sides, from the grid or from skwDEM: all of it (pieces <= 1), or the reach of piece `piece` of
// `povs` POVs: its POVs P0 .. p1 - 1 and min(K, nt) samples either side, within the row. Every target of
// those POVs is loaded, and a POV's steps to the loaded span's ends are those to the row's ends, or more
// than K. Returns the samples loaded (0 for an empty row or piece): samples w0 .. w0 + n - 1, of which
// p_lo .. p_hi - 1 (counted from w0) are the POVs to sweep.
template <typename Tz>
__device__ __forceinline__ int load_piece(const ChunkArgs &a, const RowSrc &src, const SecDev &s, int ri, int piece,
                                          int pieces, int povs, const Tz *skw, Tz *row, int &jlo, int &w0, int &p_lo,
                                          int &p_hi) {
    int Hx, Wx;
    frame_dims(s.kase, a.H, a.W, Hx, Wx);
    const int t = s.t0 + ri;
    jlo = row_first(s.T, t, Hx, Wx);
    const int nt = row_last(s.T, t, Hx, Wx) - jlo + 1;
    if (nt <= 0) return 0;
    int n = nt;
    w0 = 0;
    p_lo = 0;
    p_hi = nt;
    if (pieces > 1) {
        const int P0 = piece * povs;
        if (P0 >= nt) return 0;
        const int Kc = min(s.K, nt), p1 = min(nt, P0 + povs);
        w0 = max(0, P0 - Kc);
        n = min(nt - 1, p1 - 1 + Kc) - w0 + 1;
        p_lo = P0 - w0;
        p_hi = p1 - w0;
    }
    if (src.gather) {
        gather_span<Tz>(frame_ref(s.kase, a.H, a.W, src.dem, src.demT), Hx, s, t, jlo, w0, n, row);
        return n;
    }
    const Tz *src_row = skw + skw_row(s, t, a.pitch) + jlo + w0;
    for (int x = threadIdx.x; x < n + 2 * TVS_SWEEP_PAD; x += blockDim.x) {
        const int q = x - TVS_SWEEP_PAD;
        row[x] = (q >= 0 && q < n) ? src_row[q] : neg_inf<Tz>();
    }
    __syncthreads();
    return n;
}

// The whole of skewed row `ri`. Returns nt (0 for an empty row).
template <typename Tz>
__device__ __forceinline__ int load_row(const ChunkArgs &a, const RowSrc &src, const SecDev &s, int ri,
                                        const Tz *skw, Tz *row, int &jlo) {
    int w0, p_lo, p_hi;
    return load_piece<Tz>(a, src, s, ri, 0, 1, 0, skw, row, jlo, w0, p_lo, p_hi);
}

// Sweeps a skewed row of nt samples held in LDS (row[TVS_SWEEP_PAD + q], -inf sentinels on both
// sides, room for the early exit's block maxima after them) and stores U | e << 30 of POV q at
// dst[q], for the POVs p_lo <= q < p_hi (every sample is a target). Returns the evaluations this
// lane carried out when COUNT is set. After the row lie
// the suffix and prefix block maxima, then (use_rmq) the range-maximum table; with SLIDE the
// table of SLIDE levels, then the sliding maxima of 40 samples at every 8th position.
template <typename Tz, int NW, bool RCP, bool PRUNE, int SLIDE, bool COUNT>
__device__ __forceinline__ uint32_t sweep_row(Tz *row, int nt, int K, Tz h0,
                                              const typename Tab<Tz>::type *__restrict__ tab,
                                              uint32_t *__restrict__ dst, bool use_rmq, int p_lo, int p_hi) {
    const int nb = (nt + 31) >> 5;
    Tz *suf = nullptr, *pre = nullptr;
    float *rmq, *slide = nullptr;
    if constexpr (SLIDE != 0) {
        // launches with SLIDE set use_rmq; a pointer the compiler cannot prove non-null keeps the
        // block loop's ring sums in place (proven, its loop copies them on every block)
        rmq = use_rmq ? reinterpret_cast<float *>(row + nt + 2 * TVS_SWEEP_PAD) : nullptr;
        slide = reinterpret_cast<float *>(row + nt + 2 * TVS_SWEEP_PAD) + SLIDE * nb + SLIDE_PAD;
    } else {
        suf = row + nt + 2 * TVS_SWEEP_PAD;
        pre = suf + nb;
        rmq = use_rmq ? reinterpret_cast<float *>(pre + nb) : nullptr;
    }
    // Segments of 64 POVs go to the wavefronts as they free up, middle of the row first (its POVs have
    // lines of sight both ways): their costs differ widely, and the workgroup holds its LDS until its
    // last wavefront ends. The k-th segment handed out is c, c + 1, c - 1, c + 2, ... (a permutation of
    // 0 .. nseg - 1).
    __shared__ int seg_next;
    if (threadIdx.x == 0) seg_next = NW;
    // rows of at most 32 samples never reach a bound test (a test needs a finished 32-step block)
    if (PRUNE && nt > 32) block_bounds<Tz, SLIDE>(row + TVS_SWEEP_PAD, nb, suf, pre, rmq, slide);  // ends with a barrier
    else __syncthreads();
    const int Kc = min(K, nt);  // K may be unbounded
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nseg = (p_hi - p_lo + 63) >> 6;
    uint32_t evals = 0;
    for (int k = wv; k < nseg;) {
        const int c = (nseg - 1) >> 1, sg = (k & 1) ? c + ((k + 1) >> 1) : c - (k >> 1);  // middle-out
        const int q0 = p_lo + (sg << 6);
        const int q = q0 + lane;
        const bool live = q < p_hi;
        const Tz *zp = row + TVS_SWEEP_PAD + q;
        const Tz h = add_rn(zp[0], h0);
        uint32_t U = (K >= 1) ? 2u : 0u;  // the POV's own ring, once per direction
        uint32_t e = (K >= 1) ? 0u : 2u;
        const int top = min(p_hi - 1, q0 + 63);
        const int fwd = min(K, nt - 1 - q0);
        const int bwd = min(K, top);
        int df, db;
        const int bfar_f = min(nb - 1, (q0 + 63 + Kc) >> 5), bfar_b = max(0, q0 - Kc) >> 5;
        const int own_f = min(K, nt - 1 - q), own_b = min(K, q);  // this lane's last step each way
        int sf, sb;
        e += sweep_dir<Tz, +1, RCP, PRUNE, SLIDE, COUNT>(zp, h, fwd, K, tab, U, suf, rmq, nb, bfar_f, q0, q, live,
                                                         own_f, df, sf, slide);
        e += sweep_dir<Tz, -1, RCP, PRUNE, SLIDE, COUNT>(zp, h, bwd, K, tab, U, pre, rmq, nb, bfar_b, top, q, live,
                                                         own_b, db, sb, slide);
        if (live) dst[q] = U | (e << 30);
        if (COUNT && live) evals += (uint32_t)(min(df, own_f) - sf + min(db, own_b) - sb);
        int nx = 0;
        if (lane == 0) nx = atomicAdd(&seg_next, 1);
        k = __builtin_amdgcn_readfirstlane(nx);
    }
    return evals;
}

// Adds a workgroup's evaluation count to one of 64 counters: one atomic per workgroup.
__device__ __forceinline__ void add_work(unsigned long long *work, unsigned long long &wg_work,
                                         unsigned long long evals, int slot) {
    for (int o = 32; o > 0; o >>= 1) evals += __shfl_xor(evals, o, 64);
    const unsigned long long wsum = evals;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) atomicAdd(&wg_work, wsum);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&work[slot & 63], wg_work);
}

// One skewed row per workgroup (a.pieces <= 1), or one piece of a row too long for the LDS: the reach
// of a.piece_povs consecutive POVs, swept as a row of its own.
template <typename Tz, int NW, bool RCP, bool PRUNE, int SLIDE = 0>
__global__ __launch_bounds__(64 * NW) void k_sweep(const ChunkArgs a, const RowSrc src, const Tz *__restrict__ skw,
                                                   uint32_t *__restrict__ V,
                                                   const typename Tab<Tz>::type *__restrict__ tab,
                                                   unsigned long long *__restrict__ work) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Tz *row = reinterpret_cast<Tz *>(lds_raw);
    __shared__ unsigned long long wg_work;
    const SecDev &s = a.s[blockIdx.y];
    // with pieces, workgroup x sweeps piece x mod pieces of row x / pieces
    const int pieces = a.pieces;
    const int rb = pieces > 1 ? (int)blockIdx.x / pieces : (int)blockIdx.x;
    if (rb >= s.nrows) return;
    const int ri = row_of_block(rb, s.nrows);
    int jlo, w0, p_lo, p_hi;
    const int n = load_piece<Tz>(a, src, s, ri, (int)blockIdx.x - rb * pieces, pieces, a.piece_povs, skw, row, jlo,
                                 w0, p_lo, p_hi);
    if (n == 0) return;
    uint32_t *dst = V + skw_row(s, s.t0 + ri, a.pitch) + jlo + w0;
    if (!work) {
        sweep_row<Tz, NW, RCP, PRUNE, SLIDE, false>(row, n, s.K, h0_of<Tz>(a), tab, dst, a.rmq != 0, p_lo, p_hi);
        return;
    }
    if (threadIdx.x == 0) wg_work = 0;
    const uint32_t evals =
        sweep_row<Tz, NW, RCP, PRUNE, SLIDE, true>(row, n, s.K, h0_of<Tz>(a), tab, dst, a.rmq != 0, p_lo, p_hi);
    add_work(work, wg_work, evals, blockIdx.x + 7 * blockIdx.y);
}

// ---------------------------------------------------------- rows longer than the LDS holds
// A skewed row too long for one workgroup's LDS (double rows beyond about 19,000 samples) whose lines of
// sight are too long for k_sweep's pieces (a piece's reach, its POVs and K samples either side, must fit
// the LDS with the range table) is swept here, also in pieces: workgroup (row, piece) owns the piece's
// 64 NW consecutive POVs, one 64-POV segment per
// wavefront, and streams the targets of both directions through an LDS window. Window c holds the
// samples of steps 1 + cM .. (c + 1) M of every POV of the piece (M + 64 NW - 1 samples, a multiple-of-32
// M, -inf outside the row); every lane carries its horizon, bit mask and ring sums from one window to
// the next, so each line of sight is walked in order over the whole row, as in the single-window sweep
// (a 32-step block never straddles two windows; the clipped step K may open the next one). Samples come
// from the grid (gathered with the relocation's interpolation) or from skwDEM.
//
// With PRUNE the walk has the single-window sweep's block skip and early exit. Before its windows the
// workgroup takes, over every position its lanes can reach (K either side of the piece), the maximum of
// each 32-sample block, rounded up to float, and from them the prefix and suffix maxima and the maxima of
// adjacent pairs. A sample's bound comes from the grid values it blends: their maximum plus 2^-40 of their
// magnitudes, above the double blend's rounding (a few double ulps of those magnitudes), so no sample
// exceeds its block's entry. A lane's 32 targets of a block lie in two consecutive blocks (the skip
// test's bound, one pair entry), and every target of the wavefront from step m on lies between the
// nearest one and the end of the reach (the exit test's). As in the single-window sweep, a block after
// one in which at least 32 lanes saw a target is not tested. A wavefront whose direction is decided
// skips its later windows' work, and the workgroup stops loading windows once every wavefront has.

// Entries of the long-row sweep's pair maxima beyond each end of a piece's reach: a lane's pair entry
// lies at most 4 blocks past the reach (its last steps' targets beyond the row end) or 3 before it.
constexpr int LONG_PAD = 8;

template <int D> struct DirTag {
    static constexpr int value = D;
};

template <typename Tz, int NW, bool RCP, bool PRUNE>
__global__ __launch_bounds__(64 * NW) void k_sweep_long(const ChunkArgs a, const RowSrc src,
                                                        const Tz *__restrict__ skw, uint32_t *__restrict__ V,
                                                        const typename Tab<Tz>::type *__restrict__ tab, int M,
                                                        int pieces, int nbs_cap, unsigned long long *__restrict__ work) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Tz *win = reinterpret_cast<Tz *>(lds_raw);
    const int L = M + 64 * NW - 1;
    // PRUNE: the block maxima's prefix and suffix maxima, then the maxima of adjacent pairs (with
    // LONG_PAD entries either side)
    float *pre = reinterpret_cast<float *>(win + L), *suf = pre + nbs_cap, *pm = suf + nbs_cap + LONG_PAD;
    __shared__ unsigned long long wg_work;
    __shared__ int ndone;  // wavefronts that have finished the current direction
    const SecDev &s = a.s[blockIdx.y];
    const int ri = (int)blockIdx.x / pieces, piece = (int)blockIdx.x % pieces;
    if (ri >= s.nrows) return;
    int Hx, Wx;
    frame_dims(s.kase, a.H, a.W, Hx, Wx);
    const int t = s.t0 + ri;
    const int jlo = row_first(s.T, t, Hx, Wx);
    const int nt = row_last(s.T, t, Hx, Wx) - jlo + 1;
    const int P0 = piece * 64 * NW;
    if (nt <= 0 || P0 >= nt) return;  // uniform over the workgroup
    const FrameRef F = frame_ref(s.kase, a.H, a.W, src.dem, src.demT);
    const Tz *srow = src.gather ? nullptr : skw + skw_row(s, t, a.pitch) + jlo;
    // elevation of sample p (0 <= p < nt) of the row
    auto sample = [&](int p) -> Tz {
        if (!src.gather) return srow[p];
        const int j = jlo + p;
        int d;
        double r;
        col_offset(s.T, j, d, r);
        const int u = t + d;
        const float *col = F.base + (int64_t)j * F.cs;
        const float av = col[(int64_t)min(max(u, 0), Hx - 1) * F.rs];
        double z = (double)av;
        if (r != 0.0 && u >= 0 && u < Hx - 1) {
            const float bv = col[(int64_t)(u + 1) * F.rs];
            z = __dadd_rn(__dmul_rn(__dsub_rn(1.0, r), (double)av), __dmul_rn(r, (double)bv));
        }
        return add_rn((Tz)z, (Tz)0);
    };
    // an upper bound of sample p, as a float
    auto sample_bound = [&](int p) -> float {
        if (!src.gather) return ru_float(srow[p]);
        const int j = jlo + p;
        int d;
        double r;
        col_offset(s.T, j, d, r);
        const int u = t + d;
        const float *col = F.base + (int64_t)j * F.cs;
        const float av = col[(int64_t)min(max(u, 0), Hx - 1) * F.rs];
        if (r != 0.0 && u >= 0 && u < Hx - 1) {
            const double bv = (double)col[(int64_t)(u + 1) * F.rs];
            return ru_float(fmax((double)av, bv) + (fabs((double)av) + fabs(bv)) * 0x1p-40);
        }
        return av;
    };
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q0 = P0 + 64 * wv, q = q0 + lane;
    const bool live = q < nt;
    const int K = s.K;
    const int last = min(nt - 1, P0 + 64 * NW - 1);  // the piece's last POV
    const int Kc = min(K, nt);
    // positions the piece's lanes can reach, and their 32-sample blocks b0 .. b0 + nbs - 1 (nbs <= nbs_cap)
    const int reach_lo = max(0, P0 - Kc), reach_hi = min(nt - 1, last + Kc);
    const int b0 = reach_lo >> 5, nbs = (reach_hi >> 5) - b0 + 1;
    if (PRUNE) {
        // one block per half wavefront, reduced across its 32 lanes
        for (int i = (int)threadIdx.x >> 5; i < nbs; i += (int)blockDim.x >> 5) {
            const int p = ((b0 + i) << 5) + (int)(threadIdx.x & 31);
            float v = (p >= reach_lo && p <= reach_hi) ? sample_bound(p) : neg_inf<float>();
            for (int o = 16; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 32));
            if ((threadIdx.x & 31) == 0) pre[i] = suf[i] = v;
        }
        __syncthreads();
        // entry i covers blocks b0 + i and b0 + i + 1; blocks outside the reach hold no target a lane
        // evaluates (positions past the row or beyond K of every lane): -inf
        for (int i = (int)threadIdx.x - LONG_PAD; i < nbs + LONG_PAD; i += (int)blockDim.x) {
            const float x = (i >= 0 && i < nbs) ? pre[i] : neg_inf<float>();
            const float y = (i + 1 >= 0 && i + 1 < nbs) ? pre[i + 1] : neg_inf<float>();
            pm[i] = fmaxf(x, y);
        }
        __syncthreads();
        if (wv < 2) {  // prefix maxima by wavefront 0, suffix maxima by wavefront 1, in place
            float *arr = wv == 0 ? pre : suf;
            float carry = neg_inf<float>();
            for (int c0 = 0; c0 < nbs; c0 += 64) {
                const int i = c0 + lane;
                const int b = wv == 0 ? i : nbs - 1 - i;
                float x = i < nbs ? arr[b] : neg_inf<float>();
                x = vmax(wave_prefix_max(x), carry);
                if (i < nbs) arr[b] = x;
                carry = lane63(x);
            }
        }
        __syncthreads();
    }
    auto entry = [&](const float *arr, int blk) -> float { return arr[min(max(blk - b0, 0), nbs - 1)]; };
    const Tz h = live ? add_rn(sample(q), h0_of<Tz>(a)) : neg_inf<Tz>();
    uint32_t U = (K >= 1) ? 2u : 0u;  // the POV's own ring, once per direction
    uint32_t e = (K >= 1) ? 0u : 2u;
    unsigned long long evals = 0;
    // one direction; a compile-time DIR folds each step's window offset into the LDS reads
    auto walk = [&](auto dir) {
        constexpr int DIR = decltype(dir)::value;
        // steps of this wavefront (its farthest-reaching lane) and of the whole piece (window count)
        const int top = min(nt - 1, q0 + 63);
        const int mb = q0 >= nt ? 0 : DIR > 0 ? min(K, nt - 1 - q0) : min(K, top);
        const int mbW = DIR > 0 ? min(K, nt - 1 - P0) : min(K, last);
        const int mfull = (mb == K) ? K - 1 : mb;
        const int nwin = mbW >= 1 ? (mbW + M - 1) / M : 0;
        const int own = DIR > 0 ? min(K, nt - 1 - q) : min(K, q);  // this lane's last step
        // a lane past the row end has a +inf horizon: it never sees a target, never holds back a test
        Tz mx = live ? neg_inf<Tz>() : -neg_inf<Tz>();
        // every target of steps m1..m2 of the wavefront with elevation at most zs is hidden
        auto bounded_by = [&](Tz zs, int m1, int m2) -> bool {
            const Tz d = sub_rn(zs, h);
            const Tz b = vmax_plain(slope<RCP>(d, tab[m1 - 1]), slope<RCP>(d, tab[m2 - 1]));
            return __builtin_amdgcn_ballot_w64(b <= mx) == ~0ull;
        };
        auto hidden_from = [&](int mm) -> bool {  // no target of the wavefront from step mm to mb
            const int bnear = (DIR > 0 ? q0 + mm : top - mm) >> 5;
            return bounded_by((Tz)entry(DIR > 0 ? suf : pre, bnear), mm, mb);
        };
        // no target of steps mm .. mm + 31 on any lane: the lane's targets from position `first` on lie
        // in blocks first >> 5 and the next; for mm = 1 + 32 k that pair's entry is k after (DIR > 0) or
        // before (DIR < 0) the one for mm = 1, and stays within LONG_PAD of the reach's entries
        const float *pl = pm + (((DIR > 0 ? q + 1 : q - 32) >> 5) - b0);
        auto block_hidden = [&](int mm) -> bool {
            return bounded_by((Tz)pl[DIR * ((mm - 1) >> 5)], mm, mm + 31);
        };
        RingAcc ra;
        uint32_t bits = 0, acc = 0;
        int m = 1, skipped = 0;
        int busy = 0;  // lanes that saw a target in the last block: from 32 on, the next is not tested
        bool stop = false, counted = false;
        if (PRUNE) {
            __syncthreads();  // the previous direction's count is read by every wavefront
            if (threadIdx.x == 0) ndone = 0;
        }
        for (int c = 0; c < nwin; ++c) {
            __syncthreads();  // the previous window is no longer read
            if (PRUNE && ndone == NW) break;  // every wavefront has finished this direction
            const int origin = DIR > 0 ? P0 + 1 + c * M : P0 - (c + 1) * M;
            for (int x = threadIdx.x; x < L; x += blockDim.x) {
                const int p = origin + x;
                win[x] = (p >= 0 && p < nt) ? sample(p) : neg_inf<Tz>();
            }
            __syncthreads();
            const int wend = (c + 1) * M;  // last step held by this window
            // position q + DIR m sits at zb[DIR m]
            const Tz *zb = win + (q - P0) + (DIR > 0 ? -1 - c * M : (c + 1) * M);
            if (!stop) {
                for (; m + 31 <= min(mfull, wend); m += 32) {
                    if (PRUNE) m = __builtin_amdgcn_readfirstlane(m);  // keeps the table loads scalar
                    if (PRUNE && m > 1 && busy < 32 && block_hidden(m)) {
                        if (hidden_from(m)) {
                            stop = true;
                            break;
                        }
                        skipped += max(0, min(own, m + 31) - m + 1);
                        continue;
                    }
                    const auto *tt = tab + (m - 1);
#pragma unroll
                    for (int k = 0; k < 32; ++k) vis_step(slope<RCP>(sub_rn(zb[DIR * (m + k)], h), tt[k]), mx, bits);
                    const unsigned long long seen = __builtin_amdgcn_ballot_w64(bits != 0u);
                    if (seen) ra.add(bits, m);
                    if (PRUNE) busy = __builtin_amdgcn_readfirstlane((int)__popcll(seen));
                }
            }
            if (!stop && m <= mfull && mfull <= wend) {  // the last steps of the wavefront, all in this window
                if (PRUNE && m > 1) stop = hidden_from(m);
                if (!stop) {
                    for (; m <= mfull; ++m) {
                        const Tz th = slope<RCP>(sub_rn(zb[DIR * m], h), tab[m - 1]);
                        acc += th > mx ? (uint32_t)(2 * m + 1) : 0u;
                        mx = vmax_plain(mx, th);
                    }
                }
            }
            // the clipped last ring, when this window holds step K
            if (!stop && mb == K && K >= 1 && m == K && K <= wend) {
                e += slope<RCP>(sub_rn(zb[DIR * K], h), tab[K - 1]) > mx ? 1u : 0u;
                m = K + 1;
            }
            if (PRUNE && !counted && (stop || (m > mfull && (mb != K || K < 1 || m > K)))) {
                counted = true;
                if (lane == 0) atomicAdd(&ndone, 1);
            }
        }
        U += ra.total() + acc;
        const int done = stop ? m - 1 : mb;
        if (live) evals += (unsigned long long)max(0, min(done, own) - skipped);
    };
    walk(DirTag<1>());
    walk(DirTag<-1>());
    if (live) V[skw_row(s, t, a.pitch) + jlo + q] = U | (e << 30);
    if (work) {
        if (threadIdx.x == 0) wg_work = 0;
        __syncthreads();
        add_work(work, wg_work, evals, blockIdx.x + 7 * blockIdx.y);
    }
}

// ------------------------------------------------------------------- batched, fused sweep
template <typename Tz> __device__ __forceinline__ Tz h0_of(const BatchEnt &e);
template <> __device__ __forceinline__ float h0_of<float>(const BatchEnt &e) { return e.h0f; }
template <> __device__ __forceinline__ double h0_of<double>(const BatchEnt &e) { return e.h0; }

// Sweep over every (tile, sector, skewed row) item of a batch chunk. Persistent (counter non-null):
// each workgroup takes the next item from a device counter until the list is exhausted (every
// workgroup reaches the end, the counter only grows). Otherwise workgroup b takes item b (one launch
// of nitems workgroups, which other kernels' workgroups interleave with). Each row is gathered from
// its tile's DEM (or the tile's transposed copy for the 45..135 deg axes) and swept.
template <typename Tz, int NW, bool RCP, int SLIDE = 0>
__global__ __launch_bounds__(64 * NW) void k_sweep_batch(const BatchEnt *__restrict__ ent,
                                                         const uint32_t *__restrict__ items, int nitems,
                                                         unsigned int *__restrict__ counter, uint32_t *__restrict__ V,
                                                         const typename Tab<Tz>::type *__restrict__ tab,
                                                         unsigned long long *__restrict__ work, int rmq) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Tz *row = reinterpret_cast<Tz *>(lds_raw);
    __shared__ int next;
    __shared__ unsigned long long wg_work;
    if (work && threadIdx.x == 0) wg_work = 0;
    unsigned long long evals = 0;
    for (int pass = 0;; ++pass) {
        int it;
        if (counter) {
            if (threadIdx.x == 0) next = (int)atomicAdd(counter, 1u);
            __syncthreads();
            it = __builtin_amdgcn_readfirstlane(next);
            __syncthreads();  // every thread has read `next` before thread 0 writes it again
        } else {
            if (pass) break;
            it = (int)blockIdx.x;
        }
        if (it >= nitems) break;
        const uint32_t item = items[it];
        const BatchEnt &E = ent[item >> 16];
        const int ri = (int)(item & 0xffffu);
        int jlo;
        int Hx, Wx;
        frame_dims(E.s.kase, E.H, E.W, Hx, Wx);
        const int nt = gather_row<Tz>(frame_ref(E.s.kase, E.H, E.W, E.dem, E.demT), Hx, Wx, E.s, ri, row, jlo);
        uint32_t *dst = V + skw_row(E.s, E.s.t0 + ri, E.pitch) + jlo;
        if (nt > 0 && !work) sweep_row<Tz, NW, RCP, true, SLIDE, false>(row, nt, E.s.K, h0_of<Tz>(E), tab, dst, rmq != 0, 0, nt);
        if (nt > 0 && work) evals += sweep_row<Tz, NW, RCP, true, SLIDE, true>(row, nt, E.s.K, h0_of<Tz>(E), tab, dst, rmq != 0, 0,
                                                                          nt);
        __syncthreads();  // the row is read by every wavefront before the next gather
    }
    if (work) add_work(work, wg_work, evals, blockIdx.x);
}

// Comparison variant: one wavefront per POV and direction, lanes = 64 consecutive targets,
// the running horizon is the exclusive wavefront prefix-max carried across 64-target chunks.
template <typename Tz, int NW, bool RCP>
__global__ __launch_bounds__(64 * NW) void k_sweep_scan(const ChunkArgs a, const RowSrc src,
                                                        const Tz *__restrict__ skw, uint32_t *__restrict__ V,
                                                        const typename Tab<Tz>::type *__restrict__ tab,
                                                        unsigned long long *__restrict__ work) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Tz *row = reinterpret_cast<Tz *>(lds_raw);
    const SecDev &s = a.s[blockIdx.y];
    if ((int)blockIdx.x >= s.nrows) return;
    const int ri = row_of_block(blockIdx.x, s.nrows);
    int jlo;
    const int nt = load_row<Tz>(a, src, s, ri, skw, row, jlo);
    if (nt == 0) return;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int K = s.K;
    const Tz h0 = h0_of<Tz>(a);
    uint32_t *dst = V + skw_row(s, s.t0 + ri, a.pitch) + jlo;
    unsigned long long evals = 0;
    for (int q = wv; q < nt; q += NW) {
        const Tz *zp = row + TVS_SWEEP_PAD + q;
        const Tz h = add_rn(zp[0], h0);
        uint32_t U = 0, e = 0;
        for (int dir = 1; dir >= -1; dir -= 2) {
            const int M = min(K, dir > 0 ? nt - 1 - q : q);  // targets in range
            Tz carry = neg_inf<Tz>();
            for (int m0 = 0; m0 < M; m0 += 64) {
                const int m = m0 + lane + 1;
                const bool ok = m <= M;
                const Tz th = ok ? slope<RCP>(sub_rn(zp[dir * m], h), tab[m - 1]) : neg_inf<Tz>();
                const Tz incl = wave_prefix_max(th);
                const Tz excl = vmax(carry, wave_shift_up(neg_inf<Tz>(), incl));
                if (ok && th > excl) {
                    if (m < K) U += (uint32_t)(2 * m + 1);
                    else e += 1;
                }
                carry = vmax(carry, lane63(incl));
            }
        }
        U = wave_sum_u32(U);
        e = wave_sum_u32(e);
        if (lane == 0) {
            if (K >= 1) U += 2u; else e += 2u;
            dst[q] = U | (e << 30);
        }
        evals += min(K, nt - 1 - q) + min(K, q);  // every target in range is evaluated
    }
    if (work && lane == 0) atomicAdd(&work[(blockIdx.x + 7 * blockIdx.y) & 63], evals);
}

// ----------------------------------------------------------------------- back-projection

__device__ __forceinline__ double ring_sum(uint32_t v, double clip) {
    return (double)(v & 0x3fffffffu) + (double)(v >> 30) * clip;
}

// A workgroup owns a 64 x 64 block of grid cells and walks the chunk's sectors in order. Per
// sector the block maps to a 64 x 64 block of the sector's base frame; the skwVS rows its cells
// blend, p - d_q - 1 .. p - d_q over the block, span at most 64 + 66 rows and are staged in LDS
// by coalesced reads along skewed rows (pitch 65 words: the transposed cases read LDS down a
// column). Each thread then forms VX = (1-r) V(p-d) + r V(p-d-1) for its 16 cells, times the
// sector's ring area, and accumulates in double -- or in float with Kahan compensation, the
// running sum and compensation kept in HBM between chunks. `first` starts from zero, `last`
// writes the double result.
constexpr int BP_T = 64;
constexpr int BP_LP = BP_T + 1;
constexpr int BP_MAXR = 2 * BP_T + 3;
constexpr int BP_CELLS = BP_T * BP_T / 256;

// The 64 x 64 cell block at (i0, j0) of an H x W grid over sectors sec(0) .. sec(nsec - 1),
// whose skewed viewshed rows have the given pitch.
template <bool KAHAN, typename SecFn>
__device__ __forceinline__ void backproj_block(SecFn sec, int nsec, int H, int W, int pitch,
                                               const uint32_t *__restrict__ V, double *__restrict__ out,
                                               float *__restrict__ ksum, float *__restrict__ kc, int first,
                                               int last, int i0, int j0) {
    __shared__ uint32_t tile[BP_MAXR * BP_LP];
    __shared__ int col_d[BP_T];
    __shared__ double col_r[BP_T];
    __shared__ int row_p[BP_MAXR];  // compacted layout: stored row of each staged skewed row
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int j = j0 + lane;
    double acc[BP_CELLS];
    float fs[BP_CELLS], fc[BP_CELLS];
#pragma unroll
    for (int c = 0; c < BP_CELLS; ++c) {
        const int i = i0 + wv + 4 * c;
        const bool in = i < H && j < W;
        const int64_t cell = (int64_t)i * W + j;
        if (KAHAN) {
            fs[c] = (first || !in) ? 0.0f : ksum[cell];
            fc[c] = (first || !in) ? 0.0f : kc[cell];
        } else {
            acc[c] = (first || !in) ? 0.0 : out[cell];
        }
    }
    const int ilast = min(i0 + BP_T, H) - 1, jlast = min(j0 + BP_T, W) - 1;
    for (int k = 0; k < nsec; ++k) {
        // the sector's parameters, once per sector in scalar registers
        SecDev s;
        {
            const SecDev &g = sec(k);
            s.T = g.T;
            s.scale = g.scale;
            s.clip = g.clip;
            s.off = g.off;
            s.kase = __builtin_amdgcn_readfirstlane(g.kase);
            s.K = g.K;
            s.t0 = __builtin_amdgcn_readfirstlane(g.t0);
            s.nrows = g.nrows;
            s.wrap = __builtin_amdgcn_readfirstlane(g.wrap);
            s.winv = g.winv;
        }
        // the block's base-frame rectangle [plo, phi] x [qlo, qhi]
        int plo, phi, qlo, qhi;
        switch (s.kase) {
        case 0: plo = i0; phi = ilast; qlo = j0; qhi = jlast; break;
        case 1: plo = j0; phi = jlast; qlo = i0; qhi = ilast; break;
        case 2: plo = W - 1 - jlast; phi = W - 1 - j0; qlo = i0; qhi = ilast; break;
        default: plo = i0; phi = ilast; qlo = W - 1 - jlast; qhi = W - 1 - j0; break;
        }
        int dlo, dhi;
        double rtmp;
        col_offset(s.T, qlo, dlo, rtmp);
        col_offset(s.T, qhi, dhi, rtmp);
        const int rbase = plo - dhi - s.t0 - 1;        // first skewed row needed
        const int nr = (phi - dlo - s.t0) - rbase + 1;  // rows needed
        const int nq = qhi - qlo + 1;
        __syncthreads();  // the previous sector's tile is no longer read
        if (threadIdx.x < nq) {
            int d;
            double r;
            col_offset(s.T, qlo + threadIdx.x, d, r);
            col_d[threadIdx.x] = d;
            col_r[threadIdx.x] = r;
        }
        if (s.wrap) {
            for (int x = threadIdx.x; x < nr; x += blockDim.x) row_p[x] = skw_prow(s, s.t0 + rbase + x);
            __syncthreads();
        }
        {
            // rows are staged in rounds of 12 per wavefront, each round's loads all in flight
            // before its LDS stores
            constexpr int RND = 12;
            const uint32_t *src = V + s.off + qlo + min(lane, nq - 1);
            for (int r0 = wv; r0 < nr; r0 += 4 * RND) {
                uint32_t v[RND];
#pragma unroll
                for (int x = 0; x < RND; ++x) {
                    const int rr = r0 + 4 * x;
                    const int p = s.wrap ? row_p[min(rr, nr - 1)] : rbase + rr;
                    if (rr < nr) v[x] = src[(int64_t)p * pitch];
                }
#pragma unroll
                for (int x = 0; x < RND; ++x) {
                    const int rr = r0 + 4 * x;
                    if (rr < nr && lane < nq) tile[rr * BP_LP + lane] = v[x];
                }
            }
        }
        __syncthreads();
        const float scf = (float)s.scale;
#pragma unroll
        for (int c = 0; c < BP_CELLS; ++c) {
            const int i = i0 + wv + 4 * c;
            if (i >= H || j >= W) continue;
            int p, q;
            to_frame(s.kase, W, i, j, p, q);
            const int cq = q - qlo;
            const int d = col_d[cq];
            const double r = col_r[cq];
            const int row = p - d - s.t0 - rbase;
            const double A = ring_sum(tile[row * BP_LP + cq], s.clip);
            if (KAHAN) {
                float vx = (float)A;
                if (r != 0.0) {
                    const float B = (float)ring_sum(tile[(row - 1) * BP_LP + cq], s.clip);
                    const float rf = (float)r;
                    vx = __fadd_rn(__fmul_rn(1.0f - rf, vx), __fmul_rn(rf, B));
                }
                const float term = __fmul_rn(scf, vx);
                const float y = __fsub_rn(term, fc[c]);
                const float t = __fadd_rn(fs[c], y);
                fc[c] = __fsub_rn(__fsub_rn(t, fs[c]), y);
                fs[c] = t;
            } else {
                double vx = A;
                if (r != 0.0) {
                    const double B = ring_sum(tile[(row - 1) * BP_LP + cq], s.clip);
                    vx = (1.0 - r) * A + r * B;
                }
                acc[c] += s.scale * vx;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < BP_CELLS; ++c) {
        const int i = i0 + wv + 4 * c;
        if (i >= H || j >= W) continue;
        const int64_t cell = (int64_t)i * W + j;
        if (KAHAN) {
            if (last) out[cell] = (double)fs[c] - (double)fc[c];
            else { ksum[cell] = fs[c]; kc[cell] = fc[c]; }
        } else {
            out[cell] = acc[c];
        }
    }
}

template <bool KAHAN>
__global__ __launch_bounds__(256) void k_backproj(const ChunkArgs a, const uint32_t *__restrict__ V,
                                                  double *__restrict__ out, float *__restrict__ ksum,
                                                  float *__restrict__ kc, int first, int last) {
    backproj_block<KAHAN>([&](int k) -> const SecDev & { return a.s[k]; }, a.nsec, a.H, a.W, a.pitch, V, out, ksum,
                          kc, first, last, blockIdx.y * BP_T, blockIdx.x * BP_T);
}

// Every tile of a batch chunk: flat block b belongs to the last tile whose first block is <= b.
__global__ __launch_bounds__(256) void k_backproj_batch(const BatchTile *__restrict__ tiles, int ntiles,
                                                        const BatchEnt *__restrict__ ent, int nsec,
                                                        const uint32_t *__restrict__ V, int first) {
    int lo = 0, hi = ntiles - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tiles[mid].blk0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const BatchTile &T = tiles[lo];
    const int b = (int)blockIdx.x - T.blk0;
    const BatchEnt *e = ent + T.ent0;
    backproj_block<false>([&](int k) -> const SecDev & { return e[k].s; }, nsec, T.H, T.W, e[0].pitch, V, T.out,
                          nullptr, nullptr, first, 1, (b / T.bx) * BP_T, (b % T.bx) * BP_T);
}

// ------------------------------------------------------------------------------ singular
// One wavefront per line of sight (2 per sector), lanes = 64 consecutive targets. Targets
// lie on the straight line through the POV: offset d_j - d_q0 rows plus fraction r_j - r_q0
// (renormalised into [0,1) and snapped like Alg. 6's weights). A target is visible iff its
// slope beats the maximum over all earlier targets: the exclusive wavefront prefix-max of the
// chunk, combined with the maximum carried from earlier chunks.
// One line of sight of a singular viewshed, walked by a whole wavefront: sector s of an H x W
// grid, POV (pov_i, pov_j), direction dir. Returns the packed ring sums (U | e << 30, the POV's
// own ring included).
// With `bits` non-null it also records the visibility of every target (bit m - 1 of the ray's
// u32 words) and, in *mlast, the last target index of the line of sight.
template <typename Tz, bool RCP>
__device__ __forceinline__ uint32_t singular_ray(const SecDev &s, int H, int W, const float *__restrict__ dem,
                                                 Tz h0, int pov_i, int pov_j, int dir,
                                                 uint32_t *__restrict__ bits = nullptr,
                                                 int32_t *__restrict__ mlast = nullptr) {
    const int lane = threadIdx.x & 63;
    int Hx, Wx;
    frame_dims(s.kase, H, W, Hx, Wx);
    int p0, q0;
    to_frame(s.kase, W, pov_i, pov_j, p0, q0);
    int d0;
    double r0;
    col_offset(s.T, q0, d0, r0);
    const float zpov = dem[frame_index(s.kase, W, p0, q0)];
    const Tz h = add_rn((Tz)zpov, h0);
    const int K = s.K;
    Tz carry = neg_inf<Tz>();
    uint32_t U = 0, e = 0;
    for (int m0 = 0;; m0 += 64) {
        const int m = m0 + lane + 1;
        const int j = q0 + dir * m;
        bool ok = j >= 0 && j < Wx && m <= K;
        Tz th = neg_inf<Tz>();
        if (ok) {
            int dj;
            double rj;
            col_offset(s.T, j, dj, rj);
            int dd = dj - d0;
            double dr = rj - r0;
            if (dr < 0.0) {
                dd -= 1;
                dr = __dadd_rn(dr, 1.0);
            }
            if (dr < 1e-9) {
                dr = 0.0;
            } else if (dr > 1.0 - 1e-9) {
                dd += 1;
                dr = 0.0;
            }
            const int u = p0 + dd;
            ok = sample_exists(u, dr, Hx);
            if (ok) {
                const double z64 = interp(u, dr, Hx, [&](int v) { return dem[frame_index(s.kase, W, v, j)]; });
                const Tz z = (Tz)z64;
                const Tz dz = sub_rn(z, h);
                if constexpr (sizeof(Tz) == 4) th = RCP ? __fmul_rn(dz, __fdiv_rn(1.0f, (float)m)) : __fdiv_rn(dz, (float)m);
                else th = RCP ? __dmul_rn(dz, __ddiv_rn(1.0, (double)m)) : __ddiv_rn(dz, (double)m);
            }
        }
        // existence is monotone along the line of sight, so the valid lanes form a prefix
        const Tz incl = wave_prefix_max(th);
        const Tz excl = vmax(carry, wave_shift_up(neg_inf<Tz>(), incl));
        const bool vis = ok && th > excl;
        if (vis) {
            if (m < K) U += (uint32_t)(2 * m + 1);
            else e += 1;
        }
        carry = vmax(carry, lane63(incl));
        const unsigned long long okm = __ballot(ok);
        if (bits) {
            const unsigned long long vm = __ballot(vis);
            if (lane == 0) {
                bits[2 * (m0 >> 6)] = (uint32_t)vm;
                bits[2 * (m0 >> 6) + 1] = (uint32_t)(vm >> 32);
                *mlast = m0 + __popcll(okm);
            }
        }
        if (okm != ~0ull) break;
    }
    U = wave_sum_u32(U);
    e = wave_sum_u32(e);
    if (K >= 1) U += 1u; else e += 1u;  // the POV's own ring
    return U | (e << 30);
}

// One wavefront per line of sight (2 per sector), lanes = 64 consecutive targets. Targets
// lie on the straight line through the POV: offset d_j - d_q0 rows plus fraction r_j - r_q0
// (renormalised into [0,1) and snapped like Alg. 6's weights). A target is visible iff its
// slope beats the maximum over all earlier targets: the exclusive wavefront prefix-max of the
// chunk, combined with the maximum carried from earlier chunks.
template <typename Tz, bool RCP>
__global__ __launch_bounds__(256) void k_singular(const ChunkArgs a, const float *__restrict__ dem,
                                                  uint32_t *__restrict__ rayV) {
    const int ray = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ray >= 2 * a.nsec) return;
    const uint32_t v = singular_ray<Tz, RCP>(a.s[ray >> 1], a.H, a.W, dem, h0_of<Tz>(a), a.pov_i, a.pov_j,
                                             (ray & 1) ? -1 : 1);
    if ((threadIdx.x & 63) == 0) rayV[2 * a.k_base + ray] = v;
}

// Many singular viewsheds in one launch (possibly on different grids): ray r walks sector
// r / 2 of the table, in direction +1 (r even) or -1 (r odd), for that sector's query.
template <typename Tz, bool RCP>
__global__ __launch_bounds__(256) void k_singular_multi(const SingSec *__restrict__ secs, int nsecs,
                                                        const SingQuery *__restrict__ qs,
                                                        uint32_t *__restrict__ rayV, uint32_t *__restrict__ bits,
                                                        int words, int32_t *__restrict__ mlast) {
    const int ray = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ray >= 2 * nsecs) return;
    const SingSec &S = secs[ray >> 1];
    const SingQuery &Q = qs[S.query];
    const Tz h0 = sizeof(Tz) == 4 ? (Tz)Q.h0f : (Tz)Q.h0;
    const uint32_t v = singular_ray<Tz, RCP>(S.s, Q.H, Q.W, Q.dem, h0, Q.pov_i, Q.pov_j, (ray & 1) ? -1 : 1,
                                             bits ? bits + (int64_t)ray * words : nullptr,
                                             bits ? mlast + ray : nullptr);
    if ((threadIdx.x & 63) == 0) rayV[ray] = v;
}

// Visibility mask / multiple viewshed from the singular lines of sight of npov POVs on one grid
// (query p's sectors are p * n .. p * n + n - 1 of the multi launch). Cell offset (di, dj) from
// a POV falls in half-sector q, the one whose interval (beta_{q-1}, beta_q] of direction angles
// holds it (beta_q = (2q + 1) pi / 2n; cos(beta) di - sin(beta) dj is > 0 above a boundary): a
// first guess from atan2, then settled by those boundary tests alone. Its ring index is
// m = floor(sqrt(di^2 + dj^2) cos s' + 1e-9) on that half-sector's line of sight; it is visible
// iff m = 0, or m is a target (m <= the last one, m < rho) and that target is visible.
__global__ __launch_bounds__(256) void k_mask_multi(MaskArgs a) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= a.H || j >= a.W) return;
    const int n2 = 2 * a.n;
    uint32_t cnt = 0;
    for (int p = 0; p < a.npov; ++p) {
        const int di = i - a.pov[2 * p], dj = j - a.pov[2 * p + 1];
        if (di == 0 && dj == 0) {
            ++cnt;
            continue;
        }
        const double fdi = (double)di, fdj = (double)dj;
        double phi = atan2(fdi, fdj);
        if (phi < 0.0) phi += 2.0 * M_PI;
        int q = (int)floor(phi * (double)a.n / M_PI + 0.5);
        q = ((q % n2) + n2) % n2;
        for (int it = 0; it < 4; ++it) {
            const double up = __dsub_rn(__dmul_rn(a.cb[q], fdi), __dmul_rn(a.sb[q], fdj));
            if (up > 0.0) {
                q = q + 1 == n2 ? 0 : q + 1;
                continue;
            }
            const int ql = q == 0 ? n2 - 1 : q - 1;
            const double lo = __dsub_rn(__dmul_rn(a.cb[ql], fdi), __dmul_rn(a.sb[ql], fdj));
            if (!(lo > 0.0)) {
                q = ql;
                continue;
            }
            break;
        }
        const int k = q % a.n;
        const int ray = 2 * (p * a.n + k) + (q >= a.n ? 1 : 0);
        const double t = __dmul_rn(__dsqrt_rn(__dadd_rn(__dmul_rn(fdi, fdi), __dmul_rn(fdj, fdj))), a.ck[k]);
        const int64_t m = (int64_t)floor(__dadd_rn(t, 1e-9));
        if (m == 0) {
            ++cnt;
            continue;
        }
        if (m > a.mlast[ray] || !((double)m < a.rho[k])) continue;
        const uint32_t w = a.bits[(int64_t)ray * a.words + ((m - 1) >> 5)];
        cnt += (w >> ((m - 1) & 31)) & 1u;
    }
    const int64_t cell = (int64_t)i * a.W + j;
    if (a.count) a.count[cell] = cnt;
    if (a.mask) a.mask[cell] = (uint8_t)(cnt != 0);
}

// Area of each query of a multi launch: its sectors summed in order, as k_singular_sum does.
__global__ void k_singular_multi_sum(const SingSec *__restrict__ secs, const SingQuery *__restrict__ qs, int nq,
                                     const uint32_t *__restrict__ rayV, double *__restrict__ areas) {
    const int qi = blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    const SingQuery &Q = qs[qi];
    double acc = 0.0;
    for (int k = 0; k < Q.nsec; ++k) {
        const SecDev &s = secs[Q.sec0 + k].s;
        const double cv = ring_sum(rayV[2 * (Q.sec0 + k)], s.clip) + ring_sum(rayV[2 * (Q.sec0 + k) + 1], s.clip);
        acc += s.scale * cv;
    }
    areas[qi] = acc;
}

__global__ void k_singular_sum(const ChunkArgs a, const uint32_t *__restrict__ rayV, double *area, int first) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = first ? 0.0 : *area;
    for (int k = 0; k < a.nsec; ++k) {
        const SecDev &s = a.s[k];
        const uint32_t f = rayV[2 * (a.k_base + k)];
        const uint32_t b = rayV[2 * (a.k_base + k) + 1];
        const double cv = ring_sum(f, s.clip) + ring_sum(b, s.clip);
        acc += s.scale * cv;
    }
    *area = acc;
}

// ------------------------------------------------------------------------------ launchers


size_t sweep_lds_bytes(int maxWx, bool f64) {
    // row with sentinels, then the per-block suffix and prefix maxima of the early exit
    return (size_t)(maxWx + 2 * TVS_SWEEP_PAD + 2 * ((maxWx + 31) / 32)) * (f64 ? sizeof(double) : sizeof(float));
}

// Largest step counts (K capped at the row length) for which every early-exit range of a
// wavefront, from the block of its nearest remaining target to the farthest block its lanes
// reach, spans at most the 64 (with one more level, 128) blocks the range-maximum table covers:
// fewer than (K + 62) / 32 + 2 blocks. Launches within them may use the sliding maxima, which need
// no suffix or prefix maxima.
constexpr int SLIDE_MAX_K = 1900, SLIDE_MAX_K_LONG = 3900;

// The sweep's LDS with the early exit's range-maximum table when it fits the workgroup limit
// (rmq = 1), else without it (rmq = 0). `slide` is the sweep's SLIDE for rows whose step counts (at
// most maxK) allow it: RMQ_LEVELS, or RMQ_LEVELS + 1 for longer lines of sight, when the row with
// those tables still fits as many workgroups per CU (up to the 8 four-wave workgroups a CU holds);
// else 0. For double rows the 6-level tables take the bytes of the suffix and prefix maxima.
// The current device's largest workgroup LDS, queried once per device (the first launch on it is not
// captured): the same limit the host checks use, the opt-in maximum, else the default one.
static int lds_cap() {
    static std::atomic<int> caps[64];
    int dev = 0, cap = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
        cap = caps[dev].load();
        if (cap == 0) {
            if (hipDeviceGetAttribute(&cap, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || cap <= 0)
                if (hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
                    cap = 0;
            if (cap > 0) caps[dev].store(cap);
        }
    }
    return cap;
}

static size_t sweep_lds_launch(int maxWx, bool f64, int maxK, int &rmq, int &slide) {
    const size_t nbx = (maxWx + 31) / 32;
    const size_t base = sweep_lds_bytes(maxWx, f64);
    const size_t full = base + (size_t)RMQ_LEVELS * nbx * sizeof(float);
    const int cap = lds_cap();
    rmq = full + 64 <= (size_t)cap ? 1 : 0;  // + the kernels' static LDS
    slide = 0;
    if (rmq && maxK <= SLIDE_MAX_K_LONG) {
        const int lev = maxK <= SLIDE_MAX_K ? RMQ_LEVELS : RMQ_LEVELS + 1;
        const size_t bytes = (size_t)(maxWx + 2 * TVS_SWEEP_PAD) * (f64 ? sizeof(double) : sizeof(float)) +
                             ((size_t)(lev + 4) * nbx + 2 * SLIDE_PAD) * sizeof(float);
        auto resident = [](size_t b) { return std::min<size_t>((160 * 1024) / (b + 64), 8); };
        if (bytes + 64 <= (size_t)cap && resident(bytes) >= resident(full)) {
            slide = lev;
            return bytes;
        }
    }
    return rmq ? full : base;
}

hipError_t launch_divtab(float2 *tab32, double2 *tab64, int n, hipStream_t st) {
    k_divtab<<<(n + 255) / 256, 256, 0, st>>>(tab32, tab64, n);
    return hipGetLastError();
}

hipError_t launch_transpose(const float *dem, float *demT, int H, int W, hipStream_t st) {
    k_transpose<<<dim3((W + 63) / 64, (H + 63) / 64), 256, 0, st>>>(dem, demT, H, W);
    return hipGetLastError();
}

hipError_t launch_check_dem(const float *dem, int64_t n, uint32_t *bad, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    k_check_dem<<<(unsigned)std::max<int64_t>(blocks, 1), 256, 0, st>>>(dem, n, bad);
    return hipGetLastError();
}

hipError_t launch_poison(double *out, int64_t n, const uint32_t *bad, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    k_poison<<<(unsigned)std::max<int64_t>(blocks, 1), 256, 0, st>>>(out, n, bad);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
    const int64_t blocks = (n + 255) / 256;
    k_fill_u32<<<(unsigned)(blocks < 65536 ? (blocks > 0 ? blocks : 1) : 65536), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_relocate(const ChunkArgs &a, int maxWx, int maxRows, const float *dem, void *skw, bool f64,
                           hipStream_t st) {
    dim3 grid((maxWx + RL_TW - 1) / RL_TW, (maxRows + RL_SEG - 1) / RL_SEG, a.nsec);
    if (f64) k_relocate<double><<<grid, 256, 0, st>>>(a, dem, (double *)skw);
    else k_relocate<float><<<grid, 256, 0, st>>>(a, dem, (float *)skw);
    return hipGetLastError();
}

// A kernel's dynamic LDS limit only ever rises (under a lock): a launch from another host thread
// with a smaller row never lowers it under a launch that needs more.
static std::mutex g_lds_mu;
static std::unordered_map<const void *, size_t> g_lds_set;

template <typename F>
static hipError_t set_lds(F f, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    const void *key = reinterpret_cast<const void *>(f);
    std::lock_guard<std::mutex> g(g_lds_mu);
    size_t &cur = g_lds_set[key];
    if (cur >= bytes) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) cur = bytes;
    return e;
}

template <typename Tz>
static hipError_t sweep_go(void (*f)(ChunkArgs, RowSrc, const Tz *, uint32_t *, const typename Tab<Tz>::type *,
                                     unsigned long long *),
                           int nw, dim3 grid, size_t lds, hipStream_t st, const ChunkArgs &a, const RowSrc &src,
                           const void *skw, uint32_t *V, const typename Tab<Tz>::type *tab,
                           unsigned long long *work) {
    hipError_t e = set_lds(f, lds);
    if (e != hipSuccess) return e;
    f<<<grid, 64 * nw, lds, st>>>(a, src, (const Tz *)skw, V, tab, work);
    return hipGetLastError();
}

template <int NW>
static hipError_t sweep_nw(const ChunkArgs &a, const RowSrc &src, dim3 grid, size_t lds, const void *skw, uint32_t *V,
                           const float2 *tab32, const double2 *tab64, bool f64, bool scan, bool rcp, bool prune,
                           int slide, unsigned long long *work, hipStream_t st) {
    constexpr int S6 = RMQ_LEVELS, S7 = RMQ_LEVELS + 1;
    if (prune && !scan && (slide == S6 || slide == S7)) {
        if (f64) {
            auto f = slide == S6 ? (rcp ? k_sweep<double, NW, true, true, S6> : k_sweep<double, NW, false, true, S6>)
                                 : (rcp ? k_sweep<double, NW, true, true, S7> : k_sweep<double, NW, false, true, S7>);
            return sweep_go<double>(f, NW, grid, lds, st, a, src, skw, V, tab64, work);
        }
        auto f = slide == S6 ? (rcp ? k_sweep<float, NW, true, true, S6> : k_sweep<float, NW, false, true, S6>)
                             : (rcp ? k_sweep<float, NW, true, true, S7> : k_sweep<float, NW, false, true, S7>);
        return sweep_go<float>(f, NW, grid, lds, st, a, src, skw, V, tab32, work);
    }
    if (f64) {
        auto f = scan ? (rcp ? k_sweep_scan<double, NW, true> : k_sweep_scan<double, NW, false>)
                 : rcp ? (prune ? k_sweep<double, NW, true, true> : k_sweep<double, NW, true, false>)
                       : (prune ? k_sweep<double, NW, false, true> : k_sweep<double, NW, false, false>);
        return sweep_go<double>(f, NW, grid, lds, st, a, src, skw, V, tab64, work);
    }
    auto f = scan ? (rcp ? k_sweep_scan<float, NW, true> : k_sweep_scan<float, NW, false>)
                  : rcp ? (prune ? k_sweep<float, NW, true, true> : k_sweep<float, NW, true, false>)
                        : (prune ? k_sweep<float, NW, false, true> : k_sweep<float, NW, false, false>);
    return sweep_go<float>(f, NW, grid, lds, st, a, src, skw, V, tab32, work);
}

// Waves per sweep workgroup: a workgroup holds one row in LDS, so long rows leave room for few
// workgroups per CU; more waves per workgroup keep about 32 waves per CU busy (4 for rows up to
// ~2600 double samples, 8 and 16 beyond).
int sweep_waves(size_t lds) {
    const size_t per_cu = 160 * 1024;
    const size_t groups = std::max<size_t>(1, per_cu / std::max<size_t>(lds + 64, 1));
    if (groups >= 8) return 4;
    if (groups >= 4) return 8;
    return 16;
}

bool sweep_row_fits(int maxWx, bool f64) { return sweep_lds_bytes(maxWx, f64) + 64 <= (size_t)lds_cap(); }

// Rows that do not fit the LDS, with lines of sight too long for k_sweep's pieces: pieces of 512 POVs
// (8 waves), windows of M steps in about 40 KB of LDS with the block tables (M a multiple of 32, no
// larger than the longest line of sight of the chunk needs).
static hipError_t launch_sweep_long(const ChunkArgs &a, const RowSrc &src, int maxWx, int maxRows, int maxK,
                                    const void *skw, uint32_t *V, const float2 *tab32, const double2 *tab64,
                                    bool f64, bool rcp, bool prune, unsigned long long *work, hipStream_t st) {
    constexpr int NW = 8;
    const size_t elem = f64 ? sizeof(double) : sizeof(float);
    const int steps = std::max(1, std::min(maxK, maxWx));
    // the blocks a piece's lanes reach: its 64 NW POVs and K either side, within the row
    const int nbs_cap = prune ? (std::min(maxWx, 2 * steps + 64 * NW) + 31) / 32 + 2 : 0;
    // prefix, suffix and padded pair maxima of the blocks
    const size_t tables = prune ? ((size_t)3 * nbs_cap + 2 * LONG_PAD) * sizeof(float) : 0;
    // four workgroups per CU (32 waves): 40 KB each, less the static LDS and the block tables (at most
    // 12.4 KB, at 32,767 samples); twice that, two per CU, ran 20 % slower
    const size_t budget = (size_t)(40 * 1024) - 64 - tables;
    const int mcap = (int)(((long long)(budget / elem) - (64 * NW - 1)) / 32) * 32;
    const int M = std::min(mcap, (steps + 31) / 32 * 32);
    if (M < 32) return hipErrorInvalidValue;  // unreachable for sides up to 32,767
    const size_t lds = (size_t)(M + 64 * NW - 1) * elem + tables;
    const int pieces = (maxWx + 64 * NW - 1) / (64 * NW);
    const dim3 grid((unsigned)maxRows * (unsigned)pieces, a.nsec);
#define TVS_LONG_GO(TZ, RC, PR, TAB)                                                                     \
    do {                                                                                                 \
        auto f = k_sweep_long<TZ, NW, RC, PR>;                                                           \
        hipError_t e = set_lds(f, lds);                                                                  \
        if (e != hipSuccess) return e;                                                                   \
        f<<<grid, 64 * NW, lds, st>>>(a, src, (const TZ *)skw, V, TAB, M, pieces, nbs_cap, work);       \
    } while (0)
    if (f64) {
        if (prune) {
            if (rcp) TVS_LONG_GO(double, true, true, tab64);
            else TVS_LONG_GO(double, false, true, tab64);
        } else {
            if (rcp) TVS_LONG_GO(double, true, false, tab64);
            else TVS_LONG_GO(double, false, false, tab64);
        }
    } else {
        if (prune) {
            if (rcp) TVS_LONG_GO(float, true, true, tab32);
            else TVS_LONG_GO(float, false, true, tab32);
        } else {
            if (rcp) TVS_LONG_GO(float, true, false, tab32);
            else TVS_LONG_GO(float, false, false, tab32);
        }
    }
#undef TVS_LONG_GO
    return hipGetLastError();
}

// Longest skewed row of a sector: row t holds the columns whose position lies in (-1, Hx), and the
// positions of successive columns differ by T (to within the offsets' rounding and snapping, far below
// a column), so at most (Hx + 1) / T + 1 columns share a row; every column of the frame when T = 0.
static int sector_row_bound(const SecDev &s, int H, int W) {
    int Hx, Wx;
    frame_dims(s.kase, H, W, Hx, Wx);
    if (!(s.T > 0.0)) return Wx;
    const double b = floor((double)(Hx + 1) / s.T) + 2.0;
    return b < (double)Wx ? (int)b : Wx;
}

// Does a row of len samples fit one workgroup's LDS with the early exit's range table?
static bool row_table_fits(int len, bool f64) {
    const size_t nbx = ((size_t)len + 31) / 32;
    return sweep_lds_bytes(len, f64) + (size_t)RMQ_LEVELS * nbx * sizeof(float) + 64 <= (size_t)lds_cap();
}

// POVs per piece for rows swept in pieces with lines of sight of at most kc steps: a multiple of 64, at
// least 2048 and 2 kc (a piece loads (P + 2 kc) / P samples per POV), as long as the reach fits the LDS
// with the range table; 0 when fewer than 512 would.
static int piece_povs(int kc, bool f64) {
    int P = (std::max(2048, 2 * kc) + 63) / 64 * 64;
    while (P >= 512 && !row_table_fits(P + 2 * kc, f64)) P -= 64;
    return P >= 512 ? P : 0;
}

hipError_t launch_sweep(const ChunkArgs &a, int maxWx, const float *dem, const float *demT,
                        const void *skw, uint32_t *V, const float2 *tab32, const double2 *tab64, bool f64, bool scan,
                        bool rcp, bool prune, unsigned long long *work, hipStream_t st, int nw) {
    RowSrc src{dem, demT, skw == nullptr ? 1 : 0, 0};
    // Sectors whose rows fit one workgroup's LDS with the early exit's range table take the
    // single-window sweep whole; with the bounds on, longer rows whose lines of sight are short enough
    // take it in pieces, each piece's reach in LDS with its own tables, and the rest stream through
    // windows (with their block tables: faster than a whole row without the range table); without the
    // bounds (or in the lane-per-target variant) rows that fit the LDS take it whole. Each group is a
    // launch of its own (a skinny grid's steep sectors have short rows even when its long side does
    // not fit).
    ChunkArgs b = a, pc = a, lng = a;
    b.nsec = pc.nsec = lng.nsec = 0;
    int fitWx = 0, fitRows = 0, pcWx = 0, pcRows = 0, pcK = 0, lngWx = 0, lngRows = 0;
    for (int k = 0; k < a.nsec; ++k) {
        const int len = std::min(maxWx, sector_row_bound(a.s[k], a.H, a.W));
        const int kc = std::min(a.s[k].K, len);
        if (!scan && prune && !row_table_fits(len, f64) && piece_povs(kc, f64) > 0) {
            pc.s[pc.nsec++] = a.s[k];
            pcWx = std::max(pcWx, len);
            pcRows = std::max(pcRows, a.s[k].nrows);
            pcK = std::max(pcK, kc);
        } else if (sweep_row_fits(len, f64) && (scan || !prune || row_table_fits(len, f64))) {
            b.s[b.nsec++] = a.s[k];
            fitWx = std::max(fitWx, len);
            fitRows = std::max(fitRows, a.s[k].nrows);
        } else {
            lng.s[lng.nsec++] = a.s[k];
            lngWx = std::max(lngWx, len);
            lngRows = std::max(lngRows, a.s[k].nrows);
        }
    }
    if (lng.nsec > 0) {
        int maxK = 0;
        for (int k = 0; k < lng.nsec; ++k) maxK = std::max(maxK, std::min(lng.s[k].K, lngWx));
        const hipError_t e =
            launch_sweep_long(lng, src, lngWx, lngRows, maxK, skw, V, tab32, tab64, f64, rcp, prune, work, st);
        if (e != hipSuccess) return e;
    }
    if (pc.nsec > 0) {
        // every piece's reach is at most P + 2 pcK samples
        const int P = piece_povs(pcK, f64);
        pc.pieces = (pcWx + P - 1) / P;
        pc.piece_povs = P;
        int slide = 0;
        const size_t lds = sweep_lds_launch(std::min(pcWx, P + 2 * pcK), f64, pcK, pc.rmq, slide);
        const dim3 grid((unsigned)pcRows * (unsigned)pc.pieces, pc.nsec);
        hipError_t e;
        switch (sweep_waves(lds)) {
        case 4: e = sweep_nw<4>(pc, src, grid, lds, skw, V, tab32, tab64, f64, false, rcp, true, slide, work, st); break;
        case 8: e = sweep_nw<8>(pc, src, grid, lds, skw, V, tab32, tab64, f64, false, rcp, true, slide, work, st); break;
        default: e = sweep_nw<16>(pc, src, grid, lds, skw, V, tab32, tab64, f64, false, rcp, true, slide, work, st);
        }
        if (e != hipSuccess) return e;
    }
    if (b.nsec == 0) return hipSuccess;
    maxWx = fitWx;
    const dim3 grid(fitRows, b.nsec);
    int maxK = 0, slide = 0;
    for (int k = 0; k < b.nsec; ++k) maxK = std::max(maxK, std::min(b.s[k].K, maxWx));
    // without the early exit or in the lane-per-target variant no sliding maxima
    const size_t lds = sweep_lds_launch(maxWx, f64, prune && !scan ? maxK : INT_MAX, b.rmq, slide);
    switch (nw == 4 || nw == 8 || nw == 16 ? nw : sweep_waves(lds)) {
    case 4: return sweep_nw<4>(b, src, grid, lds, skw, V, tab32, tab64, f64, scan, rcp, prune, slide, work, st);
    case 8: return sweep_nw<8>(b, src, grid, lds, skw, V, tab32, tab64, f64, scan, rcp, prune, slide, work, st);
    default: return sweep_nw<16>(b, src, grid, lds, skw, V, tab32, tab64, f64, scan, rcp, prune, slide, work, st);
    }
}

hipError_t launch_backproj(const ChunkArgs &a, const uint32_t *V, double *out, float *kahan_sum, float *kahan_c,
                           int first, int last, hipStream_t st) {
    dim3 grid((a.W + BP_T - 1) / BP_T, (a.H + BP_T - 1) / BP_T);
    if (kahan_sum) k_backproj<true><<<grid, 256, 0, st>>>(a, V, out, kahan_sum, kahan_c, first, last);
    else k_backproj<false><<<grid, 256, 0, st>>>(a, V, out, kahan_sum, kahan_c, first, last);
    return hipGetLastError();
}

hipError_t launch_singular(const ChunkArgs &a, const float *dem, uint32_t *rayV, bool f64, bool rcp,
                           hipStream_t st) {
    const int blocks = (2 * a.nsec + 3) / 4;
    if (f64 && rcp) k_singular<double, true><<<blocks, 256, 0, st>>>(a, dem, rayV);
    else if (f64) k_singular<double, false><<<blocks, 256, 0, st>>>(a, dem, rayV);
    else if (rcp) k_singular<float, true><<<blocks, 256, 0, st>>>(a, dem, rayV);
    else k_singular<float, false><<<blocks, 256, 0, st>>>(a, dem, rayV);
    return hipGetLastError();
}

// With grid == 0 only the kernel's LDS limit is raised (outside any graph capture). Without a
// counter the launch has one workgroup per item (grid is ignored).
hipError_t launch_sweep_batch(const BatchEnt *ent, const uint32_t *items, int nitems, unsigned int *counter,
                              uint32_t *V, const float2 *tab32, const double2 *tab64, bool f64, bool rcp,
                              int waves, int grid, int maxWx, int maxK, unsigned long long *work,
                              hipStream_t st) {
    // The rule is launch_sweep's, applied to the bucket's longest row and line of sight rather than to
    // one grid's chunk, so a tile's rows may prune with another table here than in the single-grid path
    // (and count other evaluations); both prunings are exact, so the maps are the same.
    int rmq = 0, slide = 0;
    const size_t lds = sweep_lds_launch(maxWx, f64, maxK, rmq, slide);
#define TVS_BATCH_GO(TZ, NW, RCP, SL, TAB)                                                              \
    do {                                                                                                \
        auto f = k_sweep_batch<TZ, NW, RCP, SL>;                                                        \
        if (grid == 0) return set_lds(f, lds);                                                          \
        f<<<counter ? grid : nitems, 64 * NW, lds, st>>>(ent, items, nitems, counter, V, TAB, work, rmq); \
    } while (0)
#define TVS_BATCH_NW(NW)                                                                                \
    do {                                                                                                \
        if (f64 && slide == RMQ_LEVELS) {                                                               \
            if (rcp) TVS_BATCH_GO(double, NW, true, RMQ_LEVELS, tab64);                                 \
            else TVS_BATCH_GO(double, NW, false, RMQ_LEVELS, tab64);                                    \
        } else if (f64 && slide == RMQ_LEVELS + 1) {                                                    \
            if (rcp) TVS_BATCH_GO(double, NW, true, RMQ_LEVELS + 1, tab64);                             \
            else TVS_BATCH_GO(double, NW, false, RMQ_LEVELS + 1, tab64);                                \
        } else if (f64) {                                                                               \
            if (rcp) TVS_BATCH_GO(double, NW, true, 0, tab64);                                          \
            else TVS_BATCH_GO(double, NW, false, 0, tab64);                                             \
        } else if (slide == RMQ_LEVELS) {                                                               \
            if (rcp) TVS_BATCH_GO(float, NW, true, RMQ_LEVELS, tab32);                                  \
            else TVS_BATCH_GO(float, NW, false, RMQ_LEVELS, tab32);                                     \
        } else if (slide == RMQ_LEVELS + 1) {                                                           \
            if (rcp) TVS_BATCH_GO(float, NW, true, RMQ_LEVELS + 1, tab32);                              \
            else TVS_BATCH_GO(float, NW, false, RMQ_LEVELS + 1, tab32);                                 \
        } else {                                                                                        \
            if (rcp) TVS_BATCH_GO(float, NW, true, 0, tab32);                                           \
            else TVS_BATCH_GO(float, NW, false, 0, tab32);                                              \
        }                                                                                               \
    } while (0)
    switch (waves) {
    case 2: TVS_BATCH_NW(2); break;
    case 8: TVS_BATCH_NW(8); break;
    default: TVS_BATCH_NW(4); break;
    }
#undef TVS_BATCH_NW
#undef TVS_BATCH_GO
    return hipGetLastError();
}

hipError_t launch_backproj_batch(const BatchTile *tiles, int ntiles, int nblocks, const BatchEnt *ent, int nsec,
                                 const uint32_t *V, int first, hipStream_t st) {
    k_backproj_batch<<<nblocks, 256, 0, st>>>(tiles, ntiles, ent, nsec, V, first);
    return hipGetLastError();
}

hipError_t launch_singular_multi(const SingSec *secs, int nsecs, const SingQuery *qs, int nq, uint32_t *rayV,
                                 double *areas, bool f64, bool rcp, hipStream_t st, uint32_t *bits, int words,
                                 int32_t *mlast) {
    const int blocks = (2 * nsecs + 3) / 4;
    if (f64 && rcp) k_singular_multi<double, true><<<blocks, 256, 0, st>>>(secs, nsecs, qs, rayV, bits, words, mlast);
    else if (f64) k_singular_multi<double, false><<<blocks, 256, 0, st>>>(secs, nsecs, qs, rayV, bits, words, mlast);
    else if (rcp) k_singular_multi<float, true><<<blocks, 256, 0, st>>>(secs, nsecs, qs, rayV, bits, words, mlast);
    else k_singular_multi<float, false><<<blocks, 256, 0, st>>>(secs, nsecs, qs, rayV, bits, words, mlast);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_singular_multi_sum<<<(nq + 63) / 64, 64, 0, st>>>(secs, qs, nq, rayV, areas);
    return hipGetLastError();
}

hipError_t launch_mask_multi(const MaskArgs &a, hipStream_t st) {
    const dim3 grid((a.W + 63) / 64, (a.H + 3) / 4);
    k_mask_multi<<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_singular_sum(const ChunkArgs &a, const uint32_t *rayV, double *area, int first, hipStream_t st) {
    k_singular_sum<<<1, 64, 0, st>>>(a, rayV, area, first);
    return hipGetLastError();
}

}  // namespace tvs
