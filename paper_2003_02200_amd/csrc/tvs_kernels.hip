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
//               2m+1 over visible samples), so they are kept exactly in u32.
//   k_backproj  skwVS -> VS (Alg. 9): each DEM cell blends the two skewed samples around it,
//               scales by the half-sector ring area (Alg. 1's pi/ns, Alg. 7's 1/cos^2) and
//               accumulates over sectors in double.
// and the singular viewshed (Alg. 1-3) as a ray scan: one wavefront per line of sight, lanes =
// 64 consecutive targets, the horizon carried by a wavefront prefix-max.
//
// Floating point: the float path rounds the interpolated elevation to float, forms h = z + h0
// and d = z - h, and the slope as d times the float reciprocal of m (default) or as the
// correctly rounded quotient d / m (exact mode: reciprocal, one product and one FMA
// correction, exact for every integer m in range); visibility is compared in float. The
// double path forms the correctly rounded double quotient. Explicit _rn intrinsics keep the
// compiler from contracting any step into an FMA.
#include <hip/hip_runtime.h>
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
template <bool RCP> __device__ __forceinline__ double slope(double d, double2 t) { return slope_div(d, t); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float sub_rn(float a, float b) { return __fsub_rn(a, b); }
__device__ __forceinline__ double sub_rn(double a, double b) { return __dsub_rn(a, b); }

// One visibility step: vis = th > mx (strict), bits = 2 bits + vis, mx = max(mx, th). The
// compare writes VCC and the add-with-carry takes it as carry-in (two VALU instructions; the
// compiler does not form this pair from C++). max equals "vis ? th : mx" here: slopes are
// never NaN except on sentinel lanes, where both keep mx.
__device__ __forceinline__ void vis_step(float th, float &mx, uint32_t &bits) {
    asm("v_cmp_gt_f32 vcc, %1, %2\n\t"
        "v_addc_co_u32 %0, vcc, %0, %0, vcc"
        : "+v"(bits)
        : "v"(th), "v"(mx)
        : "vcc");
    mx = __builtin_fmaxf(mx, th);
}
__device__ __forceinline__ void vis_step(double th, double &mx, uint32_t &bits) {
    asm("v_cmp_gt_f64 vcc, %1, %2\n\t"
        "v_addc_co_u32 %0, vcc, %0, %0, vcc"
        : "+v"(bits)
        : "v"(th), "v"(mx)
        : "vcc");
    mx = __builtin_fmax(mx, th);
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

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = i; x < n; x += stride) p[x] = v;
}

// --------------------------------------------------------------------------- relocation
// Output tile: 64 skewed rows x 64 columns of one sector per 256-thread workgroup. The base
// frame rows it needs, [t + d_j, t + d_j + 1] over the tile, span at most 64 + 66 rows; they
// are staged in LDS (row pitch 65 words so the transposed stores of cases 1/2 spread over
// all banks), then every thread interpolates its column for 16 rows and stores them along
// the skewed row (64 consecutive columns per wavefront).
constexpr int RL_TW = 64;
constexpr int RL_TH = 64;
constexpr int RL_LP = RL_TW + 1;
constexpr int RL_MAXR = RL_TH + RL_TW + 3;

template <typename Tz>
__global__ __launch_bounds__(256) void k_relocate(const ChunkArgs a, const float *__restrict__ dem,
                                                  Tz *__restrict__ skw) {
    __shared__ float tile[RL_MAXR * RL_LP];
    const SecDev &s = a.s[blockIdx.z];
    int Hx, Wx;
    frame_dims(s.kase, a.H, a.W, Hx, Wx);
    const int j0 = blockIdx.x * RL_TW;
    const int r0 = blockIdx.y * RL_TH;
    if (j0 >= Wx || r0 >= s.nrows) return;
    const int tb = s.t0 + r0;
    const int te = min(tb + RL_TH - 1, Hx - 1);
    const int jl = min(j0 + RL_TW - 1, Wx - 1);
    int dlo, dhi;
    double rlo, rhi;
    col_offset(s.T, j0, dlo, rlo);
    col_offset(s.T, jl, dhi, rhi);
    // no sample of the tile exists: every column's rows lie below -1 or above Hx-1
    if (te + dhi < -1 || tb + dlo > Hx - 1) return;
    const int ua = min(max(tb + dlo, 0), Hx - 1);
    const int ub = min(max(te + dhi + 1, 0), Hx - 1);
    const int nr = ub - ua + 1;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ncol = jl - j0 + 1;
    // base-frame cell X[u][q] = dem[xb + u * xsu + q * xsq]
    int64_t xb;
    int xsu, xsq;
    switch (s.kase) {
    case 0: xb = 0; xsu = a.W; xsq = 1; break;
    case 1: xb = 0; xsu = 1; xsq = a.W; break;
    case 2: xb = a.W - 1; xsu = -1; xsq = a.W; break;
    default: xb = a.W - 1; xsu = a.W; xsq = -1; break;
    }
    // Staging: every thread issues all of its loads before its first LDS store, so a wavefront
    // has up to 33 (48) reads in flight instead of one. Which rows and columns a wavefront
    // stages depends only on wv, so the guards below are uniform branches.
    const int lc = min(lane, ncol - 1);  // lanes past the tile's last column re-read it
    if (xsq == 1 || xsq == -1) {
        // base-frame rows are grid rows (reversed for case 3): coalesced along the row
        constexpr int RPW = (RL_MAXR + 3) / 4;
        const float *src = dem + xb + (int64_t)ua * xsu + (int64_t)(j0 + lc) * xsq;
        float v[RPW];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int rr = wv + 4 * i;
            if (rr < nr) v[i] = src[(int64_t)rr * xsu];
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int rr = wv + 4 * i;
            if (rr < nr && lane < ncol) tile[rr * RL_LP + lane] = v[i];
        }
    } else {
        // base-frame columns are grid rows: read along them (lanes = base-frame rows) and
        // transpose into LDS; each wavefront takes 16 columns in two halves of 8
        constexpr int RCH = (RL_MAXR + 63) / 64;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            float v[8][RCH];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = wv + 4 * (8 * half + i);
                const float *src = dem + xb + (int64_t)ua * xsu + (int64_t)(j0 + min(c, ncol - 1)) * xsq;
#pragma unroll
                for (int k = 0; k < RCH; ++k) {
                    const int rr = lane + 64 * k;
                    if (64 * k < nr) v[i][k] = src[min(rr, nr - 1) * xsu];
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = wv + 4 * (8 * half + i);
#pragma unroll
                for (int k = 0; k < RCH; ++k) {
                    const int rr = lane + 64 * k;
                    if (c < ncol && rr < nr) tile[rr * RL_LP + c] = v[i][k];
                }
            }
        }
    }
    __syncthreads();
    if (lane >= ncol) return;
    const int q = j0 + lane;
    int d;
    double r;
    col_offset(s.T, q, d, r);
    // existing rows of this column: u = t + d in [-1 (only if r > 0), Hx - 1]
    const int tfirst = max(tb, (r != 0.0 ? -1 : 0) - d);
    const int tlast = min(te, Hx - 1 - d);
    int rr = wv + (((tfirst - tb - wv) + 3) >> 2 << 2);  // first rr >= tfirst - tb with rr = wv mod 4
    if (rr < tfirst - tb) rr += 4;
    const double w = __dsub_rn(1.0, r);
    Tz *out = skw + s.off + (int64_t)(r0 + rr) * a.pitch + q;
    const int64_t step = (int64_t)4 * a.pitch;
#pragma unroll 4
    for (; rr <= tlast - tb; rr += 4, out += step) {
        const int u = tb + rr + d;
        const int uc = min(max(u, 0), Hx - 1);
        const float av = tile[(uc - ua) * RL_LP + lane];
        double z = (double)av;
        if (r != 0.0 && u >= 0 && u < Hx - 1) {
            const float bv = tile[(u + 1 - ua) * RL_LP + lane];
            z = __dadd_rn(__dmul_rn(w, (double)av), __dmul_rn(r, (double)bv));
        }
        // + 0 turns a -0 elevation into +0 (no other value changes): the sweep's sign tests
        // rely on slopes never being -0
        *out = add_rn((Tz)z, (Tz)0);
    }
}

// -------------------------------------------------------------------------------- sweep

// Ring sums of 32 visibility bits: step m0+s lands in bit 31-s, so the ring weight 2m+1 of set
// bit b is (2 m0 + 63) - 2b, and sum_b b = sum_k 2^k popc(bits & M_k).
struct RingAcc {
    uint32_t base = 0;                                // sum over blocks of (2 m0 + 63) popc(bits)
    uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0;  // sum over blocks of popc(bits & M_k)
    __device__ __forceinline__ void add(uint32_t bits, int m0) {
        base += (uint32_t)(2 * m0 + 63) * (uint32_t)__popc(bits);
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
// step m = K (the ring clipped at rho) is returned as 0/1. Steps run in blocks of 32 sharing one
// scalar load of the {m, 1/m} table; each step is subtract, slope, compare + add-with-carry into
// the bit mask, max. Returns in `done` the number of steps taken.
//
// Early exit (PRUNE): before each block the wavefront stops when no target from step m on can
// be visible on any live lane. `bnd` holds maxima of the row's elevations per 32-sample block,
// accumulated away from the POVs (suffix maxima forward, prefix maxima backward), so
// zs = bnd[(pbase + DIR m) / 32] bounds every elevation a lane still reads. Rounding is monotone:
// for m' >= m, RN(z - h) <= RN(zs - h) and the slope of RN(zs - h) >= 0 does not grow with m', so
// every remaining slope is at most max(slope(RN(zs - h), m), 0) (a negative difference gives a
// negative slope). When that bound is <= the lane's horizon, no later target passes the strict
// test, the clipped last ring included, and the ring sums are those of the full walk.
template <typename Tz, int DIR, bool RCP, bool PRUNE>
__device__ __forceinline__ uint32_t sweep_dir(const Tz *zp, Tz h, int mb, int K,
                                              const typename Tab<Tz>::type *__restrict__ tab, uint32_t &U,
                                              const Tz *bnd, int pbase, bool live, int &done) {
    // a lane past the row end starts with a +inf horizon: it never sees a target and never
    // holds back the early exit (its sums are discarded)
    Tz mx = (PRUNE && !live) ? -neg_inf<Tz>() : neg_inf<Tz>();
    const int mfull = (mb == K) ? K - 1 : mb;
    auto hidden_from = [&](int mm) -> bool {
        const Tz zs = bnd[(pbase + DIR * mm) >> 5];
        const Tz b = vmax(slope<RCP>(sub_rn(zs, h), tab[mm - 1]), (Tz)0);
        // every lane of the (fully active) wavefront agrees; a wave-uniform answer keeps the
        // step counter, and with it the table loads, scalar
        return __builtin_amdgcn_ballot_w64(b <= mx) == ~0ull;
    };
    RingAcc ra;
    int m = 1;
    bool stop = false;
    for (; m + 31 <= mfull; m += 32) {
        if (PRUNE) m = __builtin_amdgcn_readfirstlane(m);  // keeps the table loads on the scalar path
        if (PRUNE && m > 1 && hidden_from(m)) {
            stop = true;
            break;
        }
        const auto *t = static_cast<const typename Tab<Tz>::type *>(__builtin_assume_aligned(tab + (m - 1), 256));
        uint32_t bits = 0;
#pragma unroll
        for (int s = 0; s < 32; ++s) vis_step(slope<RCP>(sub_rn(zp[DIR * (m + s)], h), t[s]), mx, bits);
        ra.add(bits, m);
    }
    if (PRUNE && !stop && m > 1 && m <= mb) stop = hidden_from(m);
    uint32_t acc = ra.total();
    uint32_t e = 0;
    if (!stop) {
        for (; m <= mfull; ++m) {
            const Tz th = slope<RCP>(sub_rn(zp[DIR * m], h), tab[m - 1]);
            acc += th > mx ? (uint32_t)(2 * m + 1) : 0u;
            mx = vmax(mx, th);
        }
        if (mb == K && K >= 1) e = slope<RCP>(sub_rn(zp[DIR * K], h), tab[K - 1]) > mx ? 1u : 0u;
    }
    U += acc;
    done = stop ? m - 1 : mb;
    return e;
}

// Per-block elevation maxima of a row of nt samples (followed by -inf sentinels): pre[b] is the
// maximum over blocks 0..b, suf[b] over blocks b..nb-1, each scanned by one wavefront with the
// wavefront prefix-max.
template <typename Tz>
__device__ void block_bounds(const Tz *z, int nb, Tz *suf, Tz *pre) {
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        Tz m = z[32 * b];
#pragma unroll
        for (int i = 1; i < 32; ++i) m = vmax(m, z[32 * b + i]);
        suf[b] = m;
        pre[b] = m;
    }
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wv < 2) {
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

// Load skewed row `ri` (existing samples jlo..jlo+nt-1) into LDS with TVS_SWEEP_PAD -inf
// sentinels on both sides. Returns nt (0 for an empty row).
template <typename Tz>
__device__ __forceinline__ int load_row(const ChunkArgs &a, const SecDev &s, int ri, const Tz *skw, Tz *row,
                                        int &jlo) {
    int Hx, Wx;
    frame_dims(s.kase, a.H, a.W, Hx, Wx);
    const int t = s.t0 + ri;
    jlo = row_first(s.T, t, Hx, Wx);
    const int jhi = row_last(s.T, t, Hx, Wx);
    const int nt = jhi - jlo + 1;
    if (nt <= 0) return 0;
    const Tz *src = skw + s.off + (int64_t)ri * a.pitch + jlo;
    for (int x = threadIdx.x; x < nt + 2 * TVS_SWEEP_PAD; x += blockDim.x) {
        const int q = x - TVS_SWEEP_PAD;
        row[x] = (q >= 0 && q < nt) ? src[q] : neg_inf<Tz>();
    }
    __syncthreads();
    return nt;
}

template <typename Tz, int NW, bool RCP, bool PRUNE>
__global__ __launch_bounds__(64 * NW) void k_sweep(const ChunkArgs a, const Tz *__restrict__ skw,
                                                   uint32_t *__restrict__ V,
                                                   const typename Tab<Tz>::type *__restrict__ tab,
                                                   unsigned long long *__restrict__ work) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Tz *row = reinterpret_cast<Tz *>(lds_raw);
    __shared__ unsigned long long wg_work;
    const SecDev &s = a.s[blockIdx.y];
    if ((int)blockIdx.x >= s.nrows) return;
    const int ri = row_of_block(blockIdx.x, s.nrows);
    int jlo;
    const int nt = load_row<Tz>(a, s, ri, skw, row, jlo);
    if (nt == 0) return;
    const int nb = (nt + 31) >> 5;
    Tz *suf = row + nt + 2 * TVS_SWEEP_PAD;
    Tz *pre = suf + nb;
    if (PRUNE) block_bounds(row + TVS_SWEEP_PAD, nb, suf, pre);
    if (work && threadIdx.x == 0) wg_work = 0;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int K = s.K;
    const Tz h0 = h0_of<Tz>(a);
    const int nseg = (nt + 63) >> 6;
    uint32_t *dst = V + s.off + (int64_t)ri * a.pitch + jlo;
    uint32_t evals = 0;  // line-of-sight evaluations this lane carried out (with work counting)
    for (int sg = wv; sg < nseg; sg += NW) {
        const int q0 = sg << 6;
        const int q = q0 + lane;
        const bool live = q < nt;
        const Tz *zp = row + TVS_SWEEP_PAD + q;
        const Tz h = add_rn(zp[0], h0);
        uint32_t U = (K >= 1) ? 2u : 0u;  // the POV's own ring, once per direction
        uint32_t e = (K >= 1) ? 0u : 2u;
        const int top = min(nt - 1, q0 + 63);
        const int fwd = min(K, nt - 1 - q0);
        const int bwd = min(K, top);
        int df, db;
        e += sweep_dir<Tz, +1, RCP, PRUNE>(zp, h, fwd, K, tab, U, suf, q0, live, df);
        e += sweep_dir<Tz, -1, RCP, PRUNE>(zp, h, bwd, K, tab, U, pre, top, live, db);
        if (live) dst[q] = U | (e << 30);
        if (work && live) evals += (uint32_t)(min(df, min(K, nt - 1 - q)) + min(db, min(K, q)));
    }
    if (work) {
        // one atomic per workgroup, spread over 64 counters
        const uint32_t wsum = wave_sum_u32(evals);
        __syncthreads();
        if (lane == 0) atomicAdd(&wg_work, (unsigned long long)wsum);
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&work[(blockIdx.x + 7 * blockIdx.y) & 63], wg_work);
    }
}

// Comparison variant: one wavefront per POV and direction, lanes = 64 consecutive targets,
// the running horizon is the exclusive wavefront prefix-max carried across 64-target chunks.
template <typename Tz, int NW, bool RCP>
__global__ __launch_bounds__(64 * NW) void k_sweep_scan(const ChunkArgs a, const Tz *__restrict__ skw,
                                                        uint32_t *__restrict__ V,
                                                        const typename Tab<Tz>::type *__restrict__ tab,
                                                        unsigned long long *__restrict__ work) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Tz *row = reinterpret_cast<Tz *>(lds_raw);
    const SecDev &s = a.s[blockIdx.y];
    if ((int)blockIdx.x >= s.nrows) return;
    const int ri = row_of_block(blockIdx.x, s.nrows);
    int jlo;
    const int nt = load_row<Tz>(a, s, ri, skw, row, jlo);
    if (nt == 0) return;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int K = s.K;
    const Tz h0 = h0_of<Tz>(a);
    uint32_t *dst = V + s.off + (int64_t)ri * a.pitch + jlo;
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

template <bool KAHAN>
__global__ __launch_bounds__(256) void k_backproj(const ChunkArgs a, const uint32_t *__restrict__ V,
                                                  double *__restrict__ out, float *__restrict__ ksum,
                                                  float *__restrict__ kc, int first, int last) {
    __shared__ uint32_t tile[BP_MAXR * BP_LP];
    __shared__ int col_d[BP_T];
    __shared__ double col_r[BP_T];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int i0 = blockIdx.y * BP_T, j0 = blockIdx.x * BP_T;
    const int j = j0 + lane;
    double acc[BP_CELLS];
    float fs[BP_CELLS], fc[BP_CELLS];
#pragma unroll
    for (int c = 0; c < BP_CELLS; ++c) {
        const int i = i0 + wv + 4 * c;
        const bool in = i < a.H && j < a.W;
        const int64_t cell = (int64_t)i * a.W + j;
        if (KAHAN) {
            fs[c] = (first || !in) ? 0.0f : ksum[cell];
            fc[c] = (first || !in) ? 0.0f : kc[cell];
        } else {
            acc[c] = (first || !in) ? 0.0 : out[cell];
        }
    }
    const int ilast = min(i0 + BP_T, a.H) - 1, jlast = min(j0 + BP_T, a.W) - 1;
    for (int k = 0; k < a.nsec; ++k) {
        const SecDev &s = a.s[k];
        // the block's base-frame rectangle [plo, phi] x [qlo, qhi]
        int plo, phi, qlo, qhi;
        switch (s.kase) {
        case 0: plo = i0; phi = ilast; qlo = j0; qhi = jlast; break;
        case 1: plo = j0; phi = jlast; qlo = i0; qhi = ilast; break;
        case 2: plo = a.W - 1 - jlast; phi = a.W - 1 - j0; qlo = i0; qhi = ilast; break;
        default: plo = i0; phi = ilast; qlo = a.W - 1 - jlast; qhi = a.W - 1 - j0; break;
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
        if (lane < nq) {
            const uint32_t *src = V + s.off + (int64_t)rbase * a.pitch + qlo + lane;
            for (int rr = wv; rr < nr; rr += 4) tile[rr * BP_LP + lane] = src[(int64_t)rr * a.pitch];
        }
        __syncthreads();
        const float scf = (float)s.scale;
#pragma unroll
        for (int c = 0; c < BP_CELLS; ++c) {
            const int i = i0 + wv + 4 * c;
            if (i >= a.H || j >= a.W) continue;
            int p, q;
            to_frame(s.kase, a.W, i, j, p, q);
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
        if (i >= a.H || j >= a.W) continue;
        const int64_t cell = (int64_t)i * a.W + j;
        if (KAHAN) {
            if (last) out[cell] = (double)fs[c] - (double)fc[c];
            else { ksum[cell] = fs[c]; kc[cell] = fc[c]; }
        } else {
            out[cell] = acc[c];
        }
    }
}

// ------------------------------------------------------------------------------ singular
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
    const int lane = threadIdx.x & 63;
    const SecDev &s = a.s[ray >> 1];
    const int dir = (ray & 1) ? -1 : 1;
    int Hx, Wx;
    frame_dims(s.kase, a.H, a.W, Hx, Wx);
    int p0, q0;
    to_frame(s.kase, a.W, a.pov_i, a.pov_j, p0, q0);
    int d0;
    double r0;
    col_offset(s.T, q0, d0, r0);
    const float zpov = dem[frame_index(s.kase, a.W, p0, q0)];
    const Tz h = add_rn((Tz)zpov, h0_of<Tz>(a));
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
                const double z64 =
                    interp(u, dr, Hx, [&](int v) { return dem[frame_index(s.kase, a.W, v, j)]; });
                const Tz z = (Tz)z64;
                const Tz dz = sub_rn(z, h);
                if constexpr (sizeof(Tz) == 4) th = RCP ? __fmul_rn(dz, __fdiv_rn(1.0f, (float)m)) : __fdiv_rn(dz, (float)m);
                else th = __ddiv_rn(dz, (double)m);
            }
        }
        // existence is monotone along the line of sight, so the valid lanes form a prefix
        const Tz incl = wave_prefix_max(th);
        const Tz excl = vmax(carry, wave_shift_up(neg_inf<Tz>(), incl));
        if (ok && th > excl) {
            if (m < K) U += (uint32_t)(2 * m + 1);
            else e += 1;
        }
        carry = vmax(carry, lane63(incl));
        if (!__all(ok)) break;
    }
    U = wave_sum_u32(U);
    e = wave_sum_u32(e);
    if (lane == 0) {
        if (K >= 1) U += 1u; else e += 1u;  // the POV's own ring
        rayV[2 * a.k_base + ray] = U | (e << 30);
    }
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

constexpr int SWEEP_WAVES = 4;

size_t sweep_lds_bytes(int maxWx, bool f64) {
    // row with sentinels, then the per-block suffix and prefix maxima of the early exit
    return (size_t)(maxWx + 2 * TVS_SWEEP_PAD + 2 * ((maxWx + 31) / 32)) * (f64 ? sizeof(double) : sizeof(float));
}

hipError_t launch_divtab(float2 *tab32, double2 *tab64, int n, hipStream_t st) {
    k_divtab<<<(n + 255) / 256, 256, 0, st>>>(tab32, tab64, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
    const int64_t blocks = (n + 255) / 256;
    k_fill_u32<<<(unsigned)(blocks < 65536 ? (blocks > 0 ? blocks : 1) : 65536), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_relocate(const ChunkArgs &a, int maxWx, int maxRows, const float *dem, void *skw, bool f64,
                           hipStream_t st) {
    dim3 grid((maxWx + RL_TW - 1) / RL_TW, (maxRows + RL_TH - 1) / RL_TH, a.nsec);
    if (f64) k_relocate<double><<<grid, 256, 0, st>>>(a, dem, (double *)skw);
    else k_relocate<float><<<grid, 256, 0, st>>>(a, dem, (float *)skw);
    return hipGetLastError();
}

template <typename F>
static hipError_t set_lds(F f, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <typename Tz>
static hipError_t sweep_go(void (*f)(ChunkArgs, const Tz *, uint32_t *, const typename Tab<Tz>::type *,
                                     unsigned long long *),
                           dim3 grid, size_t lds, hipStream_t st, const ChunkArgs &a, const void *skw, uint32_t *V,
                           const typename Tab<Tz>::type *tab, unsigned long long *work) {
    hipError_t e = set_lds(f, lds);
    if (e != hipSuccess) return e;
    f<<<grid, 64 * SWEEP_WAVES, lds, st>>>(a, (const Tz *)skw, V, tab, work);
    return hipGetLastError();
}

hipError_t launch_sweep(const ChunkArgs &a, int maxWx, int maxRows, const void *skw, uint32_t *V,
                        const float2 *tab32, const double2 *tab64, bool f64, bool scan, bool rcp, bool prune,
                        unsigned long long *work, hipStream_t st) {
    const dim3 grid(maxRows, a.nsec);
    const size_t lds = sweep_lds_bytes(maxWx, f64);
    constexpr int NW = SWEEP_WAVES;
    if (f64) {
        auto f = scan ? k_sweep_scan<double, NW, false>
                      : (prune ? k_sweep<double, NW, false, true> : k_sweep<double, NW, false, false>);
        return sweep_go<double>(f, grid, lds, st, a, skw, V, tab64, work);
    }
    auto f = scan ? (rcp ? k_sweep_scan<float, NW, true> : k_sweep_scan<float, NW, false>)
                  : rcp ? (prune ? k_sweep<float, NW, true, true> : k_sweep<float, NW, true, false>)
                        : (prune ? k_sweep<float, NW, false, true> : k_sweep<float, NW, false, false>);
    return sweep_go<float>(f, grid, lds, st, a, skw, V, tab32, work);
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
    if (f64) k_singular<double, false><<<blocks, 256, 0, st>>>(a, dem, rayV);
    else if (rcp) k_singular<float, true><<<blocks, 256, 0, st>>>(a, dem, rayV);
    else k_singular<float, false><<<blocks, 256, 0, st>>>(a, dem, rayV);
    return hipGetLastError();
}

hipError_t launch_singular_sum(const ChunkArgs &a, const uint32_t *rayV, double *area, int first, hipStream_t st) {
    k_singular_sum<<<1, 64, 0, st>>>(a, rayV, area, first);
    return hipGetLastError();
}

}  // namespace tvs
