/*
 * tvs_oracle.c -- plain, slow CPU oracle for the sDEM total viewshed.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or load this
 * file. Only the tests, the smoke check and the bench's CPU-baseline leg use it. It
 * shares no code, header or table with the GPU library.
 *
 * What it computes (Sanchez-Fernandez, Romero, Bandera, Tabik, "A data relocation
 * approach for terrain surface analysis on multi-GPU systems: a case study on the
 * total viewshed problem"):
 *
 *   total viewshed, Alg. 4: every grid cell is a point of view (POV); its value is
 *   the visible area around it. It follows the sDEM method of Section 4.1 (steps 1a-1d)
 *   but walks each line of sight separately per POV (the Alg. 4 -> Alg. 1 shape)
 *   instead of building skewed buffers:
 *
 *   1. Sectors (Section 3.1, Alg. 1; Section 4.1 step 1): n axis directions
 *      a_k = k*pi/n, k = 0..n-1, measured from +column toward +row. Each axis
 *      carries a forward and a backward line of sight (sectors s and s+180 deg,
 *      step 1c-i), each the axis of a half-sector of opening pi/n.
 *   2. Base frame: the kernels of Section 4.2 (Alg. 6 and Alg. 9) are stated for
 *      0 <= s <= 45 deg only. Other axes are brought into that range by a
 *      transpose / flip of the grid (reading R9 in the design notes):
 *        case 0: 4k <= n        X = D              s' = pi*k/n
 *        case 1: n < 4k <= 2n   X = D^T            s' = pi*(n-2k)/(2n)
 *        case 2: 2n < 4k < 3n   X = flipud(D^T)    s' = pi*(2k-n)/(2n)
 *        case 3: 4k >= 3n       X = fliplr(D)      s' = pi*(n-k)/n
 *   3. Skew (Alg. 6, "simplified Bresenham"): column j is shifted by y_j = j*tan(s');
 *      d_j = floor(y_j), r_j = y_j - d_j, with r_j snapped to 0 within 1e-9 of an
 *      integer. Skewed sample (t, j) sits at fractional row f = t + d_j + r_j and
 *      its elevation is the linear interpolation (1-r_j) X[u][j] + r_j X[u+1][j],
 *      u = t + d_j, rows clamped to the grid. It exists iff -1 < f < Hx.
 *      Every skewed row t is one line of sight (Section 4.1: each skwDEM row is the
 *      band of sight of every point in it).
 *   4. Visibility (Alg. 3, Alg. 8): along a line of sight from POV height
 *      h = z_POV + h0, target m (index distance m) has slope theta_m = (z_m - h)/m;
 *      it is visible iff theta_m exceeds every earlier slope (strictly).
 *   5. Ring sectors (Section 3.1 area equation, Alg. 8's dd^2 - open_dd^2 update):
 *      sample m owns the ring [m, m+1) in index units; a visible sample adds
 *      min(m+1, rho)^2 - m^2 where rho = R cos(s')/dx bounds the line of sight;
 *      the POV's own ring [0, min(1, rho)) always counts. Targets stop at m < rho.
 *   6. Back-projection (Alg. 9): base-frame cell (p, q) takes
 *      (1-r_q) V(p-d_q, q) + r_q V(p-d_q-1, q), V = forward + backward ring sums.
 *   7. Scale (Alg. 1's pi/ns "Pappus" factor, Alg. 7's (1/cos s)^2 deformation
 *      correction): one index^2 unit of a half-sector ring is
 *      (pi/(2n)) * dx^2 / cos^2(s') square metres. TVS = sum over sectors.
 *
 * Precision: prec = 64 takes every step in double. prec = 32 takes the visibility
 * decision the way the paper's single-precision kernels do (Alg. 7/8 declare float):
 * the interpolated elevation rounded to float, h = z + h0 in float, the slope as a
 * float division, compared in float. Ring sums and areas stay in double. prec = 33 is the
 * same float decision with the slope formed as the float difference times the float
 * reciprocal of m -- not the paper's arithmetic but that of the GPU's reciprocal-product
 * variant, kept here so that variant can be checked bit for bit. prec = 65 is the double
 * decision with the slope formed as the double difference times the double reciprocal of m
 * (within one ulp of the double quotient), the arithmetic of the GPU's default path.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no -ffast-math).
 */
#include <limits.h>
#include <omp.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

typedef struct {
    int kase;          /* 0..3, base-frame case */
    int H, W;          /* grid dims */
    int Hx, Wx;        /* base-frame dims */
    double sp;         /* s' in radians */
    double T;          /* tan s' */
    double rho;        /* R cos s' / dx (may be +inf) */
    long long K;       /* ceil(rho) - 1; LLONG_MAX when rho is infinite */
    double scale;      /* m^2 per index^2 unit of one half-sector ring */
    long long t0;      /* first skewed row */
    long long nrows;   /* number of skewed rows, t in [t0, Hx-1] */
    int *d;            /* d_j, j in [0, Wx) */
    double *r;         /* r_j */
} sector_t;

/* ---------------------------------------------------------------- sectors -- */

static int sector_init(sector_t *S, int k, int n, int H, int W, double dx, double R)
{
    long long num, den;
    int kase;
    if (4LL * k <= n) {
        kase = 0; num = k; den = n;
    } else if (4LL * k <= 2LL * n) {
        kase = 1; num = n - 2LL * k; den = 2LL * n;
    } else if (4LL * k < 3LL * n) {
        kase = 2; num = 2LL * k - n; den = 2LL * n;
    } else {
        kase = 3; num = n - k; den = n;
    }
    S->kase = kase;
    S->H = H;
    S->W = W;
    if (kase == 0 || kase == 3) { S->Hx = H; S->Wx = W; }
    else { S->Hx = W; S->Wx = H; }
    S->sp = (M_PI * (double)num) / (double)den;
    if (num == 0) S->T = 0.0;
    else if (4 * num == den) S->T = 1.0;
    else S->T = tan(S->sp);
    double c = cos(S->sp);
    S->scale = (M_PI / (2.0 * (double)n)) * (dx * dx) / (c * c);
    if (isinf(R)) {
        S->rho = INFINITY;
        S->K = LLONG_MAX;
    } else {
        S->rho = (R * c) / dx;
        S->K = (long long)ceil(S->rho) - 1;
    }
    S->d = (int *)malloc(sizeof(int) * (size_t)S->Wx);
    S->r = (double *)malloc(sizeof(double) * (size_t)S->Wx);
    if (!S->d || !S->r) return ORC_ENOMEM;
    for (int j = 0; j < S->Wx; j++) {
        double y = (double)j * S->T;
        double fl = floor(y);
        double rr = y - fl;
        int dd = (int)fl;
        if (rr < 1e-9) rr = 0.0;
        else if (rr > 1.0 - 1e-9) { dd += 1; rr = 0.0; }
        S->d[j] = dd;
        S->r[j] = rr;
    }
    S->t0 = -(long long)S->d[S->Wx - 1] - 1;
    S->nrows = (long long)S->Hx - S->t0;
    return ORC_OK;
}

static void sector_free(sector_t *S)
{
    free(S->d);
    free(S->r);
    S->d = NULL;
    S->r = NULL;
}

/* base-frame cell X[p][q] of grid D */
static double X_at(const float *D, const sector_t *S, long long p, long long q)
{
    int W = S->W;
    switch (S->kase) {
    case 0: return (double)D[p * W + q];                 /* X = D */
    case 1: return (double)D[q * W + p];                 /* X[p][q] = D[q][p] */
    case 2: return (double)D[q * W + (W - 1 - p)];       /* X[p][q] = D^T[W-1-p][q] */
    default: return (double)D[p * W + (W - 1 - q)];      /* X[p][q] = D[p][W-1-q] */
    }
}

/* grid cell (i, j) -> base-frame cell (p, q) */
static void to_base(const sector_t *S, int i, int j, long long *p, long long *q)
{
    switch (S->kase) {
    case 0: *p = i; *q = j; break;
    case 1: *p = j; *q = i; break;
    case 2: *p = S->W - 1 - j; *q = i; break;
    default: *p = i; *q = S->W - 1 - j; break;
    }
}

/* A sample at integer row u plus fraction fr (0 <= fr < 1) of base-frame column j.
 * It exists iff -1 < u + fr < Hx. */
static int sample_exists(const sector_t *S, long long u, double fr)
{
    if (u < -1 || u > (long long)S->Hx - 1) return 0;
    if (u == -1 && fr == 0.0) return 0;
    return 1;
}

static long long clamp_row(const sector_t *S, long long u)
{
    if (u < 0) return 0;
    if (u > S->Hx - 1) return S->Hx - 1;
    return u;
}

/* interpolated elevation (double) of the sample at row u + fr of column j */
static double sample_z(const float *D, const sector_t *S, long long u, double fr, long long j)
{
    long long ua = clamp_row(S, u), ub = clamp_row(S, u + 1);
    double a = X_at(D, S, ua, j);
    if (fr == 0.0 || ua == ub) return a;
    double b = X_at(D, S, ub, j);
    double w = 1.0 - fr;
    double pa = w * a;
    double pb = fr * b;
    return pa + pb;
}

/* ------------------------------------------------------------- visibility -- */

/* One line of sight. For m = 1, 2, ... the target is column j0 + delta*m at row
 * rowoff(m) + frac(m) as produced by the callback-free helper below. Returns the ring
 * sum cv (double), and its split into the integer part U (rings wholly inside rho,
 * including the POV ring when rho >= 1) and e (1 if the clipped last ring m = K is
 * visible, or the POV ring itself is clipped). Optionally records per-target
 * visibility and slope for tests. */
typedef struct {
    double cv;
    unsigned long long U;
    int e;
    long long M;       /* number of targets walked */
} ray_t;

/* geometry of the m-th target of a line of sight:
 *   mode 0 (total viewshed): skewed row t, target column j: u = t + d_j, fr = r_j
 *   mode 1 (singular): POV at base cell (p0, q0): u = p0 + (d_j - d_q0) [-1], fr = r_j - r_q0 [+1], snapped */
static void target_pos(const sector_t *S, int mode, long long t_or_p0, long long q0, long long j,
                       long long *u, double *fr)
{
    if (mode == 0) {
        *u = t_or_p0 + S->d[j];
        *fr = S->r[j];
        return;
    }
    long long dd = (long long)S->d[j] - S->d[q0];
    double dr = S->r[j] - S->r[q0];
    if (dr < 0.0) { dd -= 1; dr += 1.0; }
    if (dr < 1e-9) dr = 0.0;
    else if (dr > 1.0 - 1e-9) { dd += 1; dr = 0.0; }
    *u = t_or_p0 + dd;
    *fr = dr;
}

static ray_t walk(const float *D, const sector_t *S, int mode, long long t_or_p0, long long q0, int delta,
                  double h64, float h32, int prec, unsigned char *vis_out, double *theta_out,
                  double *z_out, long long cap)
{
    ray_t R;
    double rho = S->rho;
    long long K = S->K;
    /* the POV's own ring [0, min(1, rho)) */
    double w0 = rho < 1.0 ? rho * rho : 1.0;
    R.cv = w0;
    if (K == 0) { R.U = 0; R.e = 1; }
    else { R.U = 1; R.e = 0; }
    R.M = 0;
    double mx64 = -INFINITY;
    float mx32 = -INFINITY;
    for (long long m = 1;; m++) {
        long long j = q0 + (long long)delta * m;
        if (j < 0 || j >= S->Wx) break;
        long long u;
        double fr;
        target_pos(S, mode, t_or_p0, q0, j, &u, &fr);
        if (!sample_exists(S, u, fr)) break;
        if (!((double)m < rho)) break;
        double z = sample_z(D, S, u, fr, j);
        int visible;
        double th_rec;
        if (prec == 64 || prec == 65) {
            double dz = z - h64;
            double th = prec == 64 ? dz / (double)m : dz * (1.0 / (double)m);
            visible = th > mx64;
            if (visible) mx64 = th;
            th_rec = th;
        } else {
            float z32 = (float)z;
            float dz = z32 - h32;
            float th;
            if (prec == 32) th = dz / (float)m;
            else th = dz * (1.0f / (float)m);  /* prec 33: the reciprocal-product variant */
            visible = th > mx32;
            if (visible) mx32 = th;
            th_rec = (double)th;
        }
        if (m - 1 < cap) {
            if (vis_out) vis_out[m - 1] = (unsigned char)visible;
            if (theta_out) theta_out[m - 1] = th_rec;
            if (z_out) z_out[m - 1] = z;
        }
        if (visible) {
            double hi = (double)(m + 1) < rho ? (double)(m + 1) : rho;
            R.cv += hi * hi - (double)m * (double)m;
            if (m < K) R.U += (unsigned long long)(2 * m + 1);
            else R.e += 1;
        }
        R.M = m;
    }
    return R;
}

/* POV heights in both precisions */
static void pov_height(double zpov, double h0, double *h64, float *h32)
{
    *h64 = zpov + h0;
    *h32 = (float)zpov + (float)h0;
}

/* V at skewed sample (t, q): forward + backward ring sums (Section 4.1 step 1c). */
static ray_t pair_at(const float *D, const sector_t *S, long long t, long long q, double h0, int prec)
{
    double zp = sample_z(D, S, t + S->d[q], S->r[q], q);
    double h64;
    float h32;
    pov_height(zp, h0, &h64, &h32);
    ray_t a = walk(D, S, 0, t, q, +1, h64, h32, prec, NULL, NULL, NULL, 0);
    ray_t b = walk(D, S, 0, t, q, -1, h64, h32, prec, NULL, NULL, NULL, 0);
    ray_t v;
    v.cv = a.cv + b.cv;
    v.U = a.U + b.U;
    v.e = a.e + b.e;
    v.M = a.M + b.M;
    return v;
}

/* ------------------------------------------------------------- validation -- */

static int check_args(const float *dem, int rows, int cols, double dx, double h0, int n, double R)
{
    if (!dem) return ORC_EINVAL;
    if (rows < 1 || cols < 1 || rows > 32767 || cols > 32767) return ORC_EINVAL;
    if (!(dx > 0.0) || !isfinite(dx)) return ORC_EINVAL;
    if (!isfinite(h0)) return ORC_EINVAL;
    if (n < 1 || n > 32768) return ORC_EINVAL;
    if (isnan(R) || !(R > 0.0)) return ORC_EINVAL;
    for (long long x = 0; x < (long long)rows * cols; x++)
        if (!isfinite(dem[x])) return ORC_EINVAL;
    return ORC_OK;
}

static sector_t *make_sectors(int rows, int cols, double dx, int n, double R)
{
    sector_t *S = (sector_t *)calloc((size_t)n, sizeof(sector_t));
    if (!S) return NULL;
    for (int k = 0; k < n; k++) {
        if (sector_init(&S[k], k, n, rows, cols, dx, R) != ORC_OK) {
            for (int q = 0; q <= k; q++) sector_free(&S[q]);
            free(S);
            return NULL;
        }
    }
    return S;
}

static void free_sectors(sector_t *S, int n)
{
    for (int k = 0; k < n; k++) sector_free(&S[k]);
    free(S);
}

/* ------------------------------------------------------------ public API -- */

int oracle_abi_version(void) { return 1; }

/* Per-sector parameters (for tests). */
int oracle_sector_info(int rows, int cols, double dx, int n, double R, int k,
                       int *out_case, int *out_Hx, int *out_Wx, long long *out_t0, long long *out_nrows,
                       double *out_T, double *out_rho, long long *out_K, double *out_scale,
                       int *out_d, double *out_r)
{
    if (k < 0 || k >= n || rows < 1 || cols < 1) return ORC_EINVAL;
    sector_t S;
    memset(&S, 0, sizeof(S));
    if (sector_init(&S, k, n, rows, cols, dx, R) != ORC_OK) { sector_free(&S); return ORC_ENOMEM; }
    if (out_case) *out_case = S.kase;
    if (out_Hx) *out_Hx = S.Hx;
    if (out_Wx) *out_Wx = S.Wx;
    if (out_t0) *out_t0 = S.t0;
    if (out_nrows) *out_nrows = S.nrows;
    if (out_T) *out_T = S.T;
    if (out_rho) *out_rho = S.rho;
    if (out_K) *out_K = S.K;
    if (out_scale) *out_scale = S.scale;
    if (out_d) memcpy(out_d, S.d, sizeof(int) * (size_t)S.Wx);
    if (out_r) memcpy(out_r, S.r, sizeof(double) * (size_t)S.Wx);
    sector_free(&S);
    return ORC_OK;
}

/* Per-sector skewed viewshed V for every skewed sample (Section 4.1 steps 1a-1c):
 * arrays of nrows x Wx (row t - t0, column j). U and e as in walk(); valid = 1 where
 * the sample exists. cv (optional) holds the double ring sum. */
int oracle_sector_V(const float *dem, int rows, int cols, double dx, double h0, int n, double R, int k, int prec,
                    uint32_t *out_U, uint8_t *out_e, uint8_t *out_valid, double *out_cv)
{
    int rc = check_args(dem, rows, cols, dx, h0, n, R);
    if (rc) return rc;
    if (k < 0 || k >= n || (prec != 32 && prec != 33 && prec != 64 && prec != 65)) return ORC_EINVAL;
    sector_t S;
    memset(&S, 0, sizeof(S));
    if (sector_init(&S, k, n, rows, cols, dx, R) != ORC_OK) { sector_free(&S); return ORC_ENOMEM; }
    long long nr = S.nrows;
    int Wx = S.Wx;
#pragma omp parallel for schedule(dynamic, 4)
    for (long long ti = 0; ti < nr; ti++) {
        long long t = S.t0 + ti;
        for (int j = 0; j < Wx; j++) {
            size_t o = (size_t)ti * (size_t)Wx + (size_t)j;
            if (!sample_exists(&S, t + S.d[j], S.r[j])) {
                if (out_U) out_U[o] = 0;
                if (out_e) out_e[o] = 0;
                if (out_valid) out_valid[o] = 0;
                if (out_cv) out_cv[o] = 0.0;
                continue;
            }
            ray_t v = pair_at(dem, &S, t, j, h0, prec);
            if (out_U) out_U[o] = (uint32_t)v.U;
            if (out_e) out_e[o] = (uint8_t)v.e;
            if (out_valid) out_valid[o] = 1;
            if (out_cv) out_cv[o] = v.cv;
        }
    }
    sector_free(&S);
    return ORC_OK;
}

/* Total viewshed (m^2) for the window of cells rows [r0, r0+nr), cols [c0, c0+nc)
 * (Alg. 4 with Alg. 9's back-projection and the per-sector scale). out is nr x nc. */
int oracle_total(const float *dem, int rows, int cols, double dx, double h0, int n, double R, int prec,
                 int r0, int c0, int nr, int nc, double *out, long long *out_evals)
{
    long long evals = 0;
    int rc = check_args(dem, rows, cols, dx, h0, n, R);
    if (rc) return rc;
    if (!out || (prec != 32 && prec != 33 && prec != 64 && prec != 65)) return ORC_EINVAL;
    if (r0 < 0 || c0 < 0 || nr < 0 || nc < 0 || r0 + nr > rows || c0 + nc > cols) return ORC_EINVAL;
    sector_t *S = make_sectors(rows, cols, dx, n, R);
    if (!S) return ORC_ENOMEM;
#pragma omp parallel for schedule(dynamic, 1) collapse(2) reduction(+ : evals)
    for (int a = 0; a < nr; a++) {
        for (int b = 0; b < nc; b++) {
            int i = r0 + a, j = c0 + b;
            double acc = 0.0;
            for (int k = 0; k < n; k++) {
                const sector_t *s = &S[k];
                long long p, q;
                to_base(s, i, j, &p, &q);
                long long ta = p - s->d[q];
                double rq = s->r[q];
                ray_t va = pair_at(dem, s, ta, q, h0, prec);
                double vx;
                evals += va.M;
                if (rq == 0.0) {
                    vx = va.cv;
                } else {
                    ray_t vb = pair_at(dem, s, ta - 1, q, h0, prec);
                    vx = (1.0 - rq) * va.cv + rq * vb.cv;
                    evals += vb.M;
                }
                acc += s->scale * vx;
            }
            out[(size_t)a * nc + b] = acc;
        }
    }
    free_sectors(S, n);
    if (out_evals) *out_evals = evals;
    return ORC_OK;
}

/* Threads the oracle's parallel loops use. */
int oracle_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}

/* Singular viewshed (Alg. 1): the area visible from grid cell (i0, j0), in m^2. The line
 * of sight of each sector passes through the POV itself (reading R18/O-11 in the design
 * notes). ray_U/ray_e/ray_cv (optional, 2n entries: [2k] forward, [2k+1] backward). */
int oracle_singular(const float *dem, int rows, int cols, double dx, double h0, int n, double R, int prec,
                    int i0, int j0, double *out_area, uint32_t *ray_U, uint8_t *ray_e, double *ray_cv)
{
    int rc = check_args(dem, rows, cols, dx, h0, n, R);
    if (rc) return rc;
    if (!out_area || (prec != 32 && prec != 33 && prec != 64 && prec != 65)) return ORC_EINVAL;
    if (i0 < 0 || i0 >= rows || j0 < 0 || j0 >= cols) return ORC_EINVAL;
    sector_t *S = make_sectors(rows, cols, dx, n, R);
    if (!S) return ORC_ENOMEM;
    double area = 0.0;
    for (int k = 0; k < n; k++) {
        const sector_t *s = &S[k];
        long long p0, q0;
        to_base(s, i0, j0, &p0, &q0);
        double zp = X_at(dem, s, p0, q0);
        double h64;
        float h32;
        pov_height(zp, h0, &h64, &h32);
        ray_t a = walk(dem, s, 1, p0, q0, +1, h64, h32, prec, NULL, NULL, NULL, 0);
        ray_t b = walk(dem, s, 1, p0, q0, -1, h64, h32, prec, NULL, NULL, NULL, 0);
        if (ray_U) { ray_U[2 * k] = (uint32_t)a.U; ray_U[2 * k + 1] = (uint32_t)b.U; }
        if (ray_e) { ray_e[2 * k] = (uint8_t)a.e; ray_e[2 * k + 1] = (uint8_t)b.e; }
        if (ray_cv) { ray_cv[2 * k] = a.cv; ray_cv[2 * k + 1] = b.cv; }
        area += s->scale * (a.cv + b.cv);
    }
    *out_area = area;
    free_sectors(S, n);
    return ORC_OK;
}

/* Singular visibility mask (reading R18 in the design notes; Alg. 1 returns only the area, the
 * problem statement of Section 1 speaks of a boolean map). A grid cell at offset (di, dj) from
 * the POV belongs to half-sector q (axis angle q*pi/n, q < n forward of sector q, q >= n backward
 * of sector q - n) whose angular interval (beta_{q-1}, beta_q] holds its direction, where
 * beta_q = (2q + 1) pi / (2n): the cross product cos(beta) di - sin(beta) dj is > 0 above a
 * boundary and <= 0 on or below it. Its ring index along that line of sight is
 * m = floor(sqrt(di^2 + dj^2) cos(s') + 1e-9) (index units, snapped like the skew offsets). It is
 * visible iff m = 0, or m is a target of that line of sight (m <= the last target) and that
 * target is visible. The search below simply tries every half-sector. */
static int mask_half_sector(int di, int dj, int n, const double *cb, const double *sb)
{
    for (int q = 0; q < 2 * n; q++) {
        int ql = (q + 2 * n - 1) % (2 * n);
        double up = cb[q] * (double)di - sb[q] * (double)dj;
        double lo = cb[ql] * (double)di - sb[ql] * (double)dj;
        if (up <= 0.0 && lo > 0.0) return q;
    }
    return -1;
}

/* Ring visibility of the 2n singular lines of sight from (i0, j0): vis[r * cap + m - 1] for target
 * m of ray r = 2k (forward) or 2k + 1 (backward), and each ray's last target in M[r]. */
static int singular_rays(const float *dem, const sector_t *S, int n, int i0, int j0, double h0, int prec,
                         unsigned char *vis, long long cap, long long *M)
{
    for (int k = 0; k < n; k++) {
        const sector_t *s = &S[k];
        long long p0, q0;
        to_base(s, i0, j0, &p0, &q0);
        double zp = X_at(dem, s, p0, q0);
        double h64;
        float h32;
        pov_height(zp, h0, &h64, &h32);
        ray_t a = walk(dem, s, 1, p0, q0, +1, h64, h32, prec, vis + (size_t)(2 * k) * cap, NULL, NULL, cap);
        ray_t b = walk(dem, s, 1, p0, q0, -1, h64, h32, prec, vis + (size_t)(2 * k + 1) * cap, NULL, NULL, cap);
        M[2 * k] = a.M;
        M[2 * k + 1] = b.M;
    }
    return ORC_OK;
}

static int cell_visible(int di, int dj, int n, const sector_t *S, const double *cb, const double *sb,
                        const unsigned char *vis, long long cap, const long long *M)
{
    if (di == 0 && dj == 0) return 1;
    int q = mask_half_sector(di, dj, n, cb, sb);
    if (q < 0) return 0;
    int k = q % n;
    int ray = 2 * k + (q >= n ? 1 : 0);
    double c = cos(S[k].sp);
    double t = sqrt((double)di * (double)di + (double)dj * (double)dj) * c;
    long long m = (long long)floor(t + 1e-9);
    if (m == 0) return 1;
    if (m > M[ray] || !((double)m < S[k].rho)) return 0;
    return vis[(size_t)ray * cap + (size_t)(m - 1)] ? 1 : 0;
}

/* Multiple (cumulative) viewshed: count[i][j] = number of the npov POVs (pov[2p], pov[2p+1])
 * whose singular mask holds cell (i, j); with npov = 1 it is the mask itself. */
int oracle_multiple(const float *dem, int rows, int cols, double dx, double h0, int n, double R, int prec,
                    const int *pov, int npov, uint32_t *count)
{
    int rc = check_args(dem, rows, cols, dx, h0, n, R);
    if (rc) return rc;
    if (!count || !pov || npov < 1 || (prec != 32 && prec != 33 && prec != 64 && prec != 65)) return ORC_EINVAL;
    for (int p = 0; p < npov; p++)
        if (pov[2 * p] < 0 || pov[2 * p] >= rows || pov[2 * p + 1] < 0 || pov[2 * p + 1] >= cols) return ORC_EINVAL;
    sector_t *S = make_sectors(rows, cols, dx, n, R);
    if (!S) return ORC_ENOMEM;
    long long cap = (rows > cols ? rows : cols) + 1;
    double *cb = malloc(sizeof(double) * 2 * (size_t)n);
    double *sb = malloc(sizeof(double) * 2 * (size_t)n);
    unsigned char *vis = malloc((size_t)2 * n * (size_t)cap);
    long long *M = malloc(sizeof(long long) * 2 * (size_t)n);
    if (!cb || !sb || !vis || !M) {
        free(cb); free(sb); free(vis); free(M); free_sectors(S, n);
        return ORC_ENOMEM;
    }
    for (int q = 0; q < 2 * n; q++) {
        double beta = (M_PI * (double)(2 * q + 1)) / (double)(2 * n);
        cb[q] = cos(beta);
        sb[q] = sin(beta);
    }
    memset(count, 0, sizeof(uint32_t) * (size_t)rows * cols);
    for (int p = 0; p < npov; p++) {
        int i0 = pov[2 * p], j0 = pov[2 * p + 1];
        memset(vis, 0, (size_t)2 * n * (size_t)cap);
        singular_rays(dem, S, n, i0, j0, h0, prec, vis, cap, M);
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < rows; i++)
            for (int j = 0; j < cols; j++)
                count[(size_t)i * cols + j] += (uint32_t)cell_visible(i - i0, j - j0, n, S, cb, sb, vis, cap, M);
    }
    free(cb); free(sb); free(vis); free(M);
    free_sectors(S, n);
    return ORC_OK;
}

/* The half-sector of offset (di, dj) (-1 for the POV itself), for tests of the assignment. */
int oracle_half_sector(int n, int di, int dj)
{
    if (n < 1 || (di == 0 && dj == 0)) return -1;
    double *cb = malloc(sizeof(double) * 2 * (size_t)n);
    double *sb = malloc(sizeof(double) * 2 * (size_t)n);
    if (!cb || !sb) { free(cb); free(sb); return -2; }
    for (int q = 0; q < 2 * n; q++) {
        double beta = (M_PI * (double)(2 * q + 1)) / (double)(2 * n);
        cb[q] = cos(beta);
        sb[q] = sin(beta);
    }
    int q = mask_half_sector(di, dj, n, cb, sb);
    free(cb); free(sb);
    return q;
}

/* One line of sight in detail, for tests: mode 0 = skewed row t through column q0;
 * mode 1 = singular through base cell (t_or_p0, q0). Fills up to cap entries of
 * per-target visibility, slope and interpolated elevation; returns the number of
 * targets in *out_M and the ring sum in *out_cv. */
int oracle_ray(const float *dem, int rows, int cols, double dx, double h0, int n, double R, int prec,
               int k, int mode, long long t_or_p0, long long q0, int delta,
               uint8_t *vis, double *theta, double *zs, long long cap,
               long long *out_M, double *out_cv, uint32_t *out_U, int *out_e, double *out_h)
{
    int rc = check_args(dem, rows, cols, dx, h0, n, R);
    if (rc) return rc;
    if (k < 0 || k >= n || (delta != 1 && delta != -1) || (mode != 0 && mode != 1)) return ORC_EINVAL;
    sector_t S;
    memset(&S, 0, sizeof(S));
    if (sector_init(&S, k, n, rows, cols, dx, R) != ORC_OK) { sector_free(&S); return ORC_ENOMEM; }
    if (q0 < 0 || q0 >= S.Wx) { sector_free(&S); return ORC_EINVAL; }
    double zp;
    if (mode == 0) {
        if (!sample_exists(&S, t_or_p0 + S.d[q0], S.r[q0])) { sector_free(&S); return ORC_EINVAL; }
        zp = sample_z(dem, &S, t_or_p0 + S.d[q0], S.r[q0], q0);
    } else {
        if (t_or_p0 < 0 || t_or_p0 >= S.Hx) { sector_free(&S); return ORC_EINVAL; }
        zp = X_at(dem, &S, t_or_p0, q0);
    }
    double h64;
    float h32;
    pov_height(zp, h0, &h64, &h32);
    ray_t a = walk(dem, &S, mode, t_or_p0, q0, delta, h64, h32, prec, vis, theta, zs, cap);
    if (out_M) *out_M = a.M;
    if (out_cv) *out_cv = a.cv;
    if (out_U) *out_U = (uint32_t)a.U;
    if (out_e) *out_e = a.e;
    if (out_h) *out_h = prec >= 64 ? h64 : (double)h32;
    sector_free(&S);
    return ORC_OK;
}

/* Number of LoS cell-evaluations of the whole method: per skewed row with nt samples,
 * 2 * sum_{q<nt} min(q, K). Counted here by walking the sample existence test. */
int oracle_los_evals(int rows, int cols, double dx, int n, double R, long long *out_evals, long long *out_pairs)
{
    if (rows < 1 || cols < 1 || n < 1 || !(dx > 0.0) || isnan(R) || !(R > 0.0)) return ORC_EINVAL;
    long long ev = 0, pairs = 0;
    for (int k = 0; k < n; k++) {
        sector_t S;
        memset(&S, 0, sizeof(S));
        if (sector_init(&S, k, n, rows, cols, dx, R) != ORC_OK) { sector_free(&S); return ORC_ENOMEM; }
        for (long long ti = 0; ti < S.nrows; ti++) {
            long long t = S.t0 + ti;
            long long nt = 0;
            for (int j = 0; j < S.Wx; j++) nt += sample_exists(&S, t + S.d[j], S.r[j]);
            pairs += nt;
            for (long long q = 0; q < nt; q++) ev += 2 * (q < S.K ? q : S.K);
        }
        sector_free(&S);
    }
    *out_evals = ev;
    *out_pairs = pairs;
    return ORC_OK;
}
