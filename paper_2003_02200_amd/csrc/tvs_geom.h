// tvs_geom.h -- sector geometry of the sDEM method, shared by the host planner and the
// gfx950 kernels of libtvs.
//
// Sector axes (Section 3.1, Alg. 1; Section 4.1 step 1): axis k of n points at k*pi/n from
// +column toward +row and carries a forward and a backward line of sight. The relocation
// and back-projection kernels of Section 4.2 (Alg. 6, Alg. 9) are stated for axes between
// 0 and 45 degrees; every other axis is brought into that range by a transpose and/or flip
// of the grid, the "base frame" X (Hx x Wx) of the sector:
//   case 0: 4k <= n        X = D              s' = pi*k/n
//   case 1: n < 4k <= 2n   X = D^T            s' = pi*(n-2k)/(2n)
//   case 2: 2n < 4k < 3n   X = flipud(D^T)    s' = pi*(2k-n)/(2n)
//   case 3: 4k >= 3n       X = fliplr(D)      s' = pi*(n-k)/n
// Skew (Alg. 6): column j of X is shifted by y_j = j*tan(s'), split into the integer row
// offset d_j = floor(y_j) and the interpolation weight r_j = y_j - d_j, with r_j snapped to
// 0 within 1e-9 of an integer. Skewed sample (t, j) lies at fractional row t + d_j + r_j;
// it exists iff that position is strictly inside (-1, Hx).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define TVS_HD __host__ __device__ __forceinline__
#else
#define TVS_HD static inline
#endif

#define TVS_MAX_SIDE 32767
#define TVS_MAX_SECTORS 32768
// Sentinel for "no distance bound": larger than any line of sight (sides <= 32767).
#define TVS_K_UNBOUNDED (1 << 30)

namespace tvs {

// Skew offset of base-frame column j for slope T (Alg. 6: y = tan(s) j, dest = int(y),
// r = y - dest), computed with one IEEE multiply so host and device agree bit for bit.
TVS_HD void col_offset(double T, int j, int &d, double &r) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __dmul_rn((double)j, T);
    double fl = floor(y);
    double rr = __dsub_rn(y, fl);
#else
    double y = (double)j * T;
    double fl = __builtin_floor(y);
    double rr = y - fl;
#endif
    int dd = (int)fl;
    if (rr < 1e-9) {
        rr = 0.0;
    } else if (rr > 1.0 - 1e-9) {
        dd += 1;
        rr = 0.0;
    }
    d = dd;
    r = rr;
}

// Does the sample at row u (+ fraction r) of a base frame with Hx rows exist, i.e. is
// -1 < u + r < Hx?
TVS_HD bool sample_exists(int u, double r, int Hx) {
    return u >= -1 && u <= Hx - 1 && !(u == -1 && r == 0.0);
}

// Base-frame dims of a case.
TVS_HD void frame_dims(int kase, int H, int W, int &Hx, int &Wx) {
    if (kase == 0 || kase == 3) {
        Hx = H;
        Wx = W;
    } else {
        Hx = W;
        Wx = H;
    }
}

// Linear index into D of base-frame cell X[p][q].
TVS_HD int64_t frame_index(int kase, int W, int p, int q) {
    switch (kase) {
    case 0: return (int64_t)p * W + q;
    case 1: return (int64_t)q * W + p;
    case 2: return (int64_t)q * W + (W - 1 - p);
    default: return (int64_t)p * W + (W - 1 - q);
    }
}

// Grid cell (i, j) -> base-frame cell (p, q).
TVS_HD void to_frame(int kase, int W, int i, int j, int &p, int &q) {
    switch (kase) {
    case 0: p = i; q = j; break;
    case 1: p = j; q = i; break;
    case 2: p = W - 1 - j; q = i; break;
    default: p = i; q = W - 1 - j; break;
    }
}

// First column of skewed row t whose sample exists (Wx if none): the existence test is
// monotone along a row because y_j is non-decreasing.
TVS_HD int row_first(double T, int t, int Hx, int Wx) {
    int lo = 0, hi = Wx;  // answer in [lo, hi]
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int d;
        double r;
        col_offset(T, mid, d, r);
        int u = t + d;
        bool above_top = u > -1 || (u == -1 && r != 0.0);  // position > -1
        if (above_top) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Last column of skewed row t whose position is < Hx (-1 if none).
TVS_HD int row_last(double T, int t, int Hx, int Wx) {
    int lo = -1, hi = Wx - 1;  // answer in [lo, hi]
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int d;
        double r;
        col_offset(T, mid, d, r);
        if (t + d <= Hx - 1) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace tvs
