/*
 * fbs_oracle.c - plain FP64 CPU oracle for fast bilateral stereo (FBS).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The GPU library never
 * links it; the two share no source, header, table or helper.
 *
 * Everything is evaluated in double precision, directly from the definitions
 * of "Real-Time Subpixel Fast Bilateral Stereo" (Fan et al.), with the left
 * image as the reference view:
 *
 *   cost       Section II-A.  Either the truncated absolute difference (TAD)
 *              min(mean_ch |L(x,y) - R(x-d,y)|, tau), or the normalised
 *              cross-correlation of Eqs. (1)-(3) turned into a cost 1 - c.
 *   weights    Section II-B, Eqs. (7) and (8): w = omega_d * omega_r with
 *              omega_d = exp(-(dx^2+dy^2)/gamma_d^2) and
 *              omega_r = exp(-(i(q)-i(p))^2/gamma_r^2).
 *   aggregate  Section II-B, Eq. (6): A(p,d) = sum_t w c / sum_t w.
 *   WTA        Section II-C: the disparity of the lowest aggregated cost.
 *   subpixel   Section II-D, Eq. (10): parabola through d*-1, d*, d*+1.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - right column x-d outside the image: TAD cost = tau, NCC cost = 2;
 *   - NCC block pixels outside the image: clamp-to-edge coordinates;
 *   - NCC block with zero variance: c = 0 (cost 1);
 *   - RGB: TAD averages |diff| over channels before the cap; the range weight
 *     uses the mean over channels of the squared differences;
 *   - window taps outside the image are left out of both sums of Eq. (6);
 *   - gamma values are used as printed (no factor 2); gamma = +inf gives 1;
 *   - WTA ties go to the lowest d; Eq. (10) is applied to the aggregated
 *     costs, and returns d* at d_min, d_max or when its denominator is <= 0.
 *
 * Right reference (Section II-A, the right cost volume; Section II-C, WTA on
 * both volumes; Section II-D, Eq. 9):
 *   cost       the right volume holds, at (u,v,d), the cost of matching right
 *              pixel (u,v) with left pixel (u+d,v), i.e. the left volume's
 *              value at (u+d,v,d) - the two volumes store each cost once
 *              each.  Where u+d is outside the image: TAD tau, NCC 2.
 *   weights    Eqs. (7)-(8) with i(x,y) taken from the right image.
 *   LRC        Eq. (9): a left pixel keeps its disparity d only if u-d is in
 *              the image and the right map at (u-d,v) holds d (within an
 *              optional tolerance, 0 = Eq. 9 as printed).
 *   final map  Eq. (10) on the left aggregated costs where the check passes,
 *              -1 where it fails (the match is removed).
 *
 * Weighted median filter (Section II-D names weighted median filtering among
 * the refinement steps, without using it): each pixel's output is the
 * weighted median of the disparities in its (2r+1)^2 window, with the
 * weights of Eqs. (7)-(8) from the reference image; values outside
 * [d_min, d_max] are holes that take no part; a window without any valid
 * value gives -1.  The weighted median is the smallest window value m whose
 * cumulative weight (the weights of values <= m) reaches half of the
 * window's total weight.
 *
 * Guided search range (Section V, future work): reliable pixels suggest the
 * search range of their neighbourhood, and only that range is searched.
 * Reading: the image is cut into tiles of tile_w x tile_h pixels; a tile's
 * range is [min - margin, max + margin] (clipped to [d_min, d_max]) of the
 * disparities of the reliable seeds in the tile grown by `halo` pixels on
 * every side, or the whole range where there is none; each pixel then takes
 * WTA (Section II-C) and Eq. (10) over its tile's range only, on the same
 * aggregated costs as the full search - Eq. (10) falls back to d* at the ends
 * of the tile's range.
 *
 * Volumes are [D][H][W] with index d - d_min; weights are [H][W][(2r+1)^2]
 * in row-major tap order (dy outer, dx inner).  Images are HWC uint8 with a
 * row stride in bytes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t width, height, channels, row_stride;
    int32_t d_min, d_max, radius, ncc_radius;
    int32_t cost_type; /* 0 = TAD, 1 = NCC */
    int32_t reserved;
    double gamma_d, gamma_r, tau;
} orc_params;

enum { ORC_TAD = 0, ORC_NCC = 1 };

static int orc_check(const orc_params* p)
{
    if (!p) return -1;
    if (p->width <= 0 || p->height <= 0) return -1;
    if (p->channels != 1 && p->channels != 3) return -1;
    if (p->row_stride < p->width * p->channels) return -1;
    if (p->d_min < 0 || p->d_max < p->d_min || p->d_max >= p->width) return -1;
    if (p->radius < 0) return -1;
    if (!(p->gamma_d > 0.0) || !(p->gamma_r > 0.0)) return -1;
    if (p->cost_type == ORC_TAD) {
        if (!(p->tau > 0.0)) return -1;
    } else if (p->cost_type == ORC_NCC) {
        if (p->channels != 1 || p->ncc_radius < 0) return -1;
    } else {
        return -1;
    }
    return 0;
}

/* Checks for the map filters, where the disparity range only labels holes. */
static int orc_check_filter(const orc_params* p)
{
    if (!p) return -1;
    if (p->width <= 0 || p->height <= 0) return -1;
    if (p->channels != 1 && p->channels != 3) return -1;
    if (p->row_stride < p->width * p->channels) return -1;
    if (p->d_min < 0 || p->d_max < p->d_min || p->radius < 0) return -1;
    if (!(p->gamma_d > 0.0) || !(p->gamma_r > 0.0)) return -1;
    return 0;
}

static inline double pix(const uint8_t* img, const orc_params* p, int x, int y, int ch)
{
    return (double)img[(size_t)y * (size_t)p->row_stride + (size_t)x * (size_t)p->channels + ch];
}

static inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Truncated absolute difference between L(x,y) and R(x-d,y). */
static double cost_tad(const orc_params* p, const uint8_t* L, const uint8_t* R,
                       int x, int y, int d)
{
    if (x - d < 0 || x - d >= p->width) return p->tau;
    double s = 0.0;
    for (int ch = 0; ch < p->channels; ++ch)
        s += fabs(pix(L, p, x, y, ch) - pix(R, p, x - d, y, ch));
    double m = s / (double)p->channels;
    return m < p->tau ? m : p->tau;
}

/* Eqs. (1)-(3): correlation of the (2*varrho+1)^2 blocks centred on (u,v) in
 * the left image and (u-d,v) in the right image, returned as the cost 1 - c. */
static double cost_ncc(const orc_params* p, const uint8_t* L, const uint8_t* R,
                       int u, int v, int d)
{
    if (u - d < 0 || u - d >= p->width) return 2.0;
    const int rr = p->ncc_radius;
    const double n = (double)((2 * rr + 1) * (2 * rr + 1));
    double sl = 0, sr = 0, sll = 0, srr = 0, slr = 0;
    for (int y = v - rr; y <= v + rr; ++y) {
        for (int x = u - rr; x <= u + rr; ++x) {
            int yc = clampi(y, 0, p->height - 1);
            int xl = clampi(x, 0, p->width - 1);
            int xr = clampi(x - d, 0, p->width - 1);
            double il = pix(L, p, xl, yc, 0);
            double ir = pix(R, p, xr, yc, 0);
            sl += il; sr += ir; sll += il * il; srr += ir * ir; slr += il * ir;
        }
    }
    double mu_l = sl / n, mu_r = sr / n;
    double var_l = sll / n - mu_l * mu_l;   /* sigma_l^2, Eq. (2) */
    double var_r = srr / n - mu_r * mu_r;   /* sigma_r^2, Eq. (3) */
    double c = 0.0;
    if (var_l > 0.0 && var_r > 0.0)
        c = (slr - n * mu_l * mu_r) / (n * sqrt(var_l) * sqrt(var_r));
    return 1.0 - c;
}

static double cost_at(const orc_params* p, const uint8_t* L, const uint8_t* R,
                      int x, int y, int d)
{
    return p->cost_type == ORC_NCC ? cost_ncc(p, L, R, x, y, d) : cost_tad(p, L, R, x, y, d);
}

/* Right-reference cost at right pixel (u,v) and disparity d: the match of
 * right pixel u is left pixel u + d, so this is the left-reference cost at
 * (u + d, v, d); where u + d leaves the image, the off-image value. */
static double cost_right_at(const orc_params* p, const uint8_t* L, const uint8_t* R,
                            int u, int v, int d)
{
    if (u + d >= p->width) return p->cost_type == ORC_NCC ? 2.0 : p->tau;
    return cost_at(p, L, R, u + d, v, d);
}

/* Eqs. (7)-(8): weight of tap q = p + (dx,dy) for centre p; 0 off-image. */
static double weight_at(const orc_params* p, const uint8_t* L, int u, int v, int dx, int dy)
{
    int x = u + dx, y = v + dy;
    if (x < 0 || x >= p->width || y < 0 || y >= p->height) return 0.0;
    double dist2 = (double)(dx * dx + dy * dy);
    double wd = exp(-dist2 / (p->gamma_d * p->gamma_d));
    double diff2 = 0.0;
    for (int ch = 0; ch < p->channels; ++ch) {
        double t = pix(L, p, x, y, ch) - pix(L, p, u, v, ch);
        diff2 += t * t;
    }
    diff2 /= (double)p->channels;
    double wr = exp(-diff2 / (p->gamma_r * p->gamma_r));
    return wd * wr;
}

int orc_cost(const orc_params* p, const uint8_t* L, const uint8_t* R, double* cost)
{
    if (orc_check(p)) return -1;
    const int W = p->width, H = p->height, D = p->d_max - p->d_min + 1;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int k = 0; k < D; ++k)
            for (int x = 0; x < W; ++x)
                cost[((size_t)k * H + y) * W + x] = cost_at(p, L, R, x, y, p->d_min + k);
    return 0;
}

/* The right cost volume [D][H][W]: C_R(u,v,d) = C_L(u+d,v,d). */
int orc_cost_right(const orc_params* p, const uint8_t* L, const uint8_t* R, double* cost)
{
    if (orc_check(p)) return -1;
    const int W = p->width, H = p->height, D = p->d_max - p->d_min + 1;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int k = 0; k < D; ++k)
            for (int u = 0; u < W; ++u)
                cost[((size_t)k * H + y) * W + u] = cost_right_at(p, L, R, u, y, p->d_min + k);
    return 0;
}

int orc_weights(const orc_params* p, const uint8_t* L, double* w)
{
    if (orc_check(p)) return -1;
    const int W = p->width, H = p->height, r = p->radius, T = (2 * r + 1) * (2 * r + 1);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double* wp = w + ((size_t)y * W + x) * T;
            int t = 0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx)
                    wp[t++] = weight_at(p, L, x, y, dx, dy);
        }
    return 0;
}

/* Eq. (6) over a materialised cost volume and weight field. */
int orc_aggregate(const orc_params* p, const double* cost, const double* w, double* agg)
{
    if (orc_check(p)) return -1;
    const int W = p->width, H = p->height, r = p->radius, T = (2 * r + 1) * (2 * r + 1);
    const int D = p->d_max - p->d_min + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const double* wp = w + ((size_t)y * W + x) * T;
            double den = 0.0;
            for (int t = 0; t < T; ++t) den += wp[t];
            for (int k = 0; k < D; ++k) {
                const double* plane = cost + (size_t)k * H * W;
                double num = 0.0;
                int t = 0;
                for (int dy = -r; dy <= r; ++dy)
                    for (int dx = -r; dx <= r; ++dx, ++t) {
                        int qx = x + dx, qy = y + dy;
                        if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                        num += wp[t] * plane[(size_t)qy * W + qx];
                    }
                agg[((size_t)k * H + y) * W + x] = num / den;
            }
        }
    return 0;
}

/* WTA (Section II-C) and the parabola of Eq. (10) for one pixel; a[k] is the
 * aggregated cost at d = d_min + k, the stride between consecutive d is sd. */
static void wta_subpixel_one(const orc_params* p, const double* a, size_t sd,
                             int32_t* disp, double* disp_sub)
{
    const int D = p->d_max - p->d_min + 1;
    int best = 0;
    for (int k = 1; k < D; ++k)
        if (a[(size_t)k * sd] < a[(size_t)best * sd]) best = k;
    double ds = (double)(p->d_min + best);
    if (best > 0 && best < D - 1) {
        double cm = a[(size_t)(best - 1) * sd];
        double c0 = a[(size_t)best * sd];
        double cp = a[(size_t)(best + 1) * sd];
        double den = 2.0 * cm + 2.0 * cp - 4.0 * c0;
        if (den > 0.0) ds += (cm - cp) / den;
    }
    *disp = p->d_min + best;
    *disp_sub = ds;
}

int orc_wta_subpixel(const orc_params* p, const double* agg, int32_t* disp, double* disp_sub)
{
    if (orc_check(p)) return -1;
    const int W = p->width, H = p->height;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            wta_subpixel_one(p, agg + i, (size_t)W * H, disp + i, disp_sub + i);
        }
    return 0;
}

/* The whole left-reference pipeline: cost, weights, Eq. (6), WTA, Eq. (10).
 * agg_out may be NULL. Returns -2 when the volumes cannot be allocated. */
int orc_fbs(const orc_params* p, const uint8_t* L, const uint8_t* R,
            int32_t* disp, double* disp_sub, double* agg_out)
{
    if (orc_check(p)) return -1;
    const size_t N = (size_t)p->width * p->height;
    const size_t D = (size_t)(p->d_max - p->d_min + 1);
    const size_t T = (size_t)(2 * p->radius + 1) * (2 * p->radius + 1);
    double* cost = (double*)malloc(N * D * sizeof(double));
    double* w = (double*)malloc(N * T * sizeof(double));
    double* agg = agg_out ? agg_out : (double*)malloc(N * D * sizeof(double));
    int rc = 0;
    if (!cost || !w || !agg) {
        rc = -2;
    } else {
        orc_cost(p, L, R, cost);
        orc_weights(p, L, w);
        orc_aggregate(p, cost, w, agg);
        orc_wta_subpixel(p, agg, disp, disp_sub);
    }
    free(cost);
    free(w);
    if (!agg_out) free(agg);
    return rc;
}

/* The right-reference pipeline: right cost volume, weights from the right
 * image, Eq. (6), WTA and Eq. (10).  agg_out may be NULL. */
int orc_fbs_right(const orc_params* p, const uint8_t* L, const uint8_t* R,
                  int32_t* disp, double* disp_sub, double* agg_out)
{
    if (orc_check(p)) return -1;
    const size_t N = (size_t)p->width * p->height;
    const size_t D = (size_t)(p->d_max - p->d_min + 1);
    const size_t T = (size_t)(2 * p->radius + 1) * (2 * p->radius + 1);
    double* cost = (double*)malloc(N * D * sizeof(double));
    double* w = (double*)malloc(N * T * sizeof(double));
    double* agg = agg_out ? agg_out : (double*)malloc(N * D * sizeof(double));
    int rc = 0;
    if (!cost || !w || !agg) {
        rc = -2;
    } else {
        orc_cost_right(p, L, R, cost);
        orc_weights(p, R, w);
        orc_aggregate(p, cost, w, agg);
        orc_wta_subpixel(p, agg, disp, disp_sub);
    }
    free(cost);
    free(w);
    if (!agg_out) free(agg);
    return rc;
}

/* Eq. (9): valid[v][u] = 1 when u - dl(u,v) >= 0 and
 * |dr(u - dl(u,v), v) - dl(u,v)| <= max_diff, else 0. */
int orc_lrc(const orc_params* p, const int32_t* dl, const int32_t* dr, int32_t max_diff,
            uint8_t* valid)
{
    if (orc_check(p) || max_diff < 0) return -1;
    const int W = p->width, H = p->height;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int d = dl[(size_t)y * W + x];
            const int u = x - d;
            int ok = 0;
            if (u >= 0 && u < W) {
                const int diff = dr[(size_t)y * W + u] - d;
                ok = (diff <= max_diff && -diff <= max_diff);
            }
            valid[(size_t)y * W + x] = (uint8_t)ok;
        }
    return 0;
}

/* The paper's full path: both disparity maps, the LRC check of Eq. (9) and
 * Eq. (10) on the left map; disp_sub is -1 where the check removes the match. */
int orc_fbs_lrc(const orc_params* p, const uint8_t* L, const uint8_t* R, int32_t max_diff,
                int32_t* disp_l, int32_t* disp_r, uint8_t* valid, double* disp_sub)
{
    if (orc_check(p) || max_diff < 0) return -1;
    const size_t N = (size_t)p->width * p->height;
    double* sub_r = (double*)malloc(N * sizeof(double));
    int rc = sub_r ? 0 : -2;
    if (!rc) rc = orc_fbs(p, L, R, disp_l, disp_sub, NULL);
    if (!rc) rc = orc_fbs_right(p, L, R, disp_r, sub_r, NULL);
    if (!rc) rc = orc_lrc(p, disp_l, disp_r, max_diff, valid);
    if (!rc)
        for (size_t i = 0; i < N; ++i)
            if (!valid[i]) disp_sub[i] = -1.0;
    free(sub_r);
    return rc;
}

/* The same pipeline evaluated at n chosen pixels only (xs[i], ys[i]), for
 * images too large for full volumes.  agg is [n][D]. */
int orc_fbs_pixels(const orc_params* p, const uint8_t* L, const uint8_t* R, int32_t n,
                   const int32_t* xs, const int32_t* ys, double* agg, int32_t* disp,
                   double* disp_sub)
{
    if (orc_check(p)) return -1;
    const int r = p->radius, D = p->d_max - p->d_min + 1;
    for (int i = 0; i < n; ++i)
        if (xs[i] < 0 || xs[i] >= p->width || ys[i] < 0 || ys[i] >= p->height) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i) {
        const int x = xs[i], y = ys[i];
        double* a = agg + (size_t)i * D;
        double den = 0.0;
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) den += weight_at(p, L, x, y, dx, dy);
        for (int k = 0; k < D; ++k) {
            double num = 0.0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    int qx = x + dx, qy = y + dy;
                    if (qx < 0 || qx >= p->width || qy < 0 || qy >= p->height) continue;
                    num += weight_at(p, L, x, y, dx, dy) * cost_at(p, L, R, qx, qy, p->d_min + k);
                }
            a[k] = num / den;
        }
        wta_subpixel_one(p, a, 1, disp + i, disp_sub + i);
    }
    return 0;
}

/* The right-reference pipeline at n chosen right-image pixels (weights from
 * the right image, costs of the right volume).  agg is [n][D]. */
int orc_fbs_right_pixels(const orc_params* p, const uint8_t* L, const uint8_t* R, int32_t n,
                         const int32_t* xs, const int32_t* ys, double* agg, int32_t* disp,
                         double* disp_sub)
{
    if (orc_check(p)) return -1;
    const int r = p->radius, D = p->d_max - p->d_min + 1;
    for (int i = 0; i < n; ++i)
        if (xs[i] < 0 || xs[i] >= p->width || ys[i] < 0 || ys[i] >= p->height) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i) {
        const int x = xs[i], y = ys[i];
        double* a = agg + (size_t)i * D;
        double den = 0.0;
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) den += weight_at(p, R, x, y, dx, dy);
        for (int k = 0; k < D; ++k) {
            double num = 0.0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    int qx = x + dx, qy = y + dy;
                    if (qx < 0 || qx >= p->width || qy < 0 || qy >= p->height) continue;
                    num += weight_at(p, R, x, y, dx, dy) *
                           cost_right_at(p, L, R, qx, qy, p->d_min + k);
                }
            a[k] = num / den;
        }
        wta_subpixel_one(p, a, 1, disp + i, disp_sub + i);
    }
    return 0;
}

/* Number of OpenMP threads the oracle runs on. */
/* Per-tile search ranges from reliable seeds (see the header): ranges is
 * [tiles_y][tiles_x][2] int32 (lo, hi); a seed is a pixel with valid != 0 and
 * disp within [d_min, d_max]. */
int orc_guided_ranges(const orc_params* p, const int32_t* disp, const uint8_t* valid,
                      int32_t tile_w, int32_t tile_h, int32_t halo, int32_t margin,
                      int32_t* ranges)
{
    if (orc_check_filter(p) || tile_w < 1 || tile_h < 1 || halo < 0 || margin < 0) return -1;
    const int W = p->width, H = p->height;
    const int tx_n = (W + tile_w - 1) / tile_w, ty_n = (H + tile_h - 1) / tile_h;
    for (int ty = 0; ty < ty_n; ++ty)
        for (int tx = 0; tx < tx_n; ++tx) {
            int lo = p->d_max + 1, hi = p->d_min - 1;
            for (int y = ty * tile_h - halo; y < (ty + 1) * tile_h + halo; ++y)
                for (int x = tx * tile_w - halo; x < (tx + 1) * tile_w + halo; ++x) {
                    if (x < 0 || x >= W || y < 0 || y >= H) continue;
                    const size_t o = (size_t)y * W + x;
                    const int d = disp[o];
                    if (!valid[o] || d < p->d_min || d > p->d_max) continue;
                    if (d < lo) lo = d;
                    if (d > hi) hi = d;
                }
            int32_t* r = ranges + 2 * ((size_t)ty * tx_n + tx);
            if (lo > hi) {
                r[0] = p->d_min;
                r[1] = p->d_max;
            } else {
                r[0] = lo - margin < p->d_min ? p->d_min : lo - margin;
                r[1] = hi + margin > p->d_max ? p->d_max : hi + margin;
            }
        }
    return 0;
}

/* The four steps with each pixel's WTA and Eq. (10) restricted to its tile's
 * range (ranges as for orc_guided_ranges); aggregated costs as orc_fbs. */
int orc_fbs_ranged(const orc_params* p, const uint8_t* L, const uint8_t* R, int32_t tile_w,
                   int32_t tile_h, const int32_t* ranges, int32_t* disp, double* disp_sub)
{
    if (orc_check(p) || tile_w < 1 || tile_h < 1) return -1;
    const int W = p->width, H = p->height;
    const size_t N = (size_t)W * H;
    const int D = p->d_max - p->d_min + 1;
    const int tx_n = (W + tile_w - 1) / tile_w;
    double* agg = (double*)malloc(N * D * sizeof(double));
    int32_t* tmp = (int32_t*)malloc(N * sizeof(int32_t));
    double* tsub = (double*)malloc(N * sizeof(double));
    int rc = (agg && tmp && tsub) ? 0 : -2;
    if (!rc) rc = orc_fbs(p, L, R, tmp, tsub, agg);
    for (int y = 0; y < H && !rc; ++y)
        for (int x = 0; x < W; ++x) {
            const int32_t* r = ranges + 2 * ((size_t)(y / tile_h) * tx_n + x / tile_w);
            if (r[0] < p->d_min || r[1] > p->d_max || r[0] > r[1]) {
                rc = -1;
                break;
            }
            orc_params q = *p;
            q.d_min = r[0];
            q.d_max = r[1];
            const size_t o = (size_t)y * W + x;
            wta_subpixel_one(&q, agg + (size_t)(r[0] - p->d_min) * N + o, N, disp + o, disp_sub + o);
        }
    free(agg);
    free(tmp);
    free(tsub);
    return rc;
}

typedef struct {
    int32_t value;
    double weight;
} wmf_item;

static int wmf_cmp(const void* a, const void* b)
{
    const int32_t va = ((const wmf_item*)a)->value, vb = ((const wmf_item*)b)->value;
    return (va > vb) - (va < vb);
}

/* Weighted median filter of an integer disparity map (see the header). */
int orc_wmf(const orc_params* p, const uint8_t* img, const int32_t* din, int32_t* dout)
{
    if (orc_check_filter(p)) return -1;
    const int W = p->width, H = p->height, r = p->radius;
    const size_t T = (size_t)(2 * r + 1) * (2 * r + 1);
    int rc = 0;
#pragma omp parallel
    {
        wmf_item* it = (wmf_item*)malloc(T * sizeof(wmf_item));
        if (!it) {
#pragma omp atomic write
            rc = -2;
        }
#pragma omp for schedule(static)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                if (!it) continue;
                size_t n = 0;
                double total = 0.0;
                for (int dy = -r; dy <= r; ++dy)
                    for (int dx = -r; dx <= r; ++dx) {
                        const int qx = x + dx, qy = y + dy;
                        if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                        const int32_t v = din[(size_t)qy * W + qx];
                        if (v < p->d_min || v > p->d_max) continue;
                        it[n].value = v;
                        it[n].weight = weight_at(p, img, x, y, dx, dy);
                        total += it[n].weight;
                        ++n;
                    }
                int32_t out = -1;
                if (n > 0) {
                    qsort(it, n, sizeof(wmf_item), wmf_cmp);
                    double cum = 0.0;
                    for (size_t i = 0; i < n; ++i) {
                        cum += it[i].weight;
                        /* the last item of a run of equal values decides */
                        if (i + 1 < n && it[i + 1].value == it[i].value) continue;
                        if (cum >= 0.5 * total) {
                            out = it[i].value;
                            break;
                        }
                    }
                }
                dout[(size_t)y * W + x] = out;
            }
        free(it);
    }
    return rc;
}

/* For a candidate map m (one value per pixel): the window weights of valid
 * values below m, of valid values up to m, and the total (Eqs. 7-8 weights
 * from the reference image, as for orc_wmf).  m is a weighted median of the
 * pixel's window exactly when below < total / 2 <= upto. */
int orc_wmf_cumulative(const orc_params* p, const uint8_t* img, const int32_t* din,
                       const int32_t* m, double* below, double* upto, double* total)
{
    if (orc_check_filter(p)) return -1;
    const int W = p->width, H = p->height, r = p->radius;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const size_t o = (size_t)y * W + x;
            double b = 0.0, u = 0.0, t = 0.0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    const int qx = x + dx, qy = y + dy;
                    if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                    const int32_t v = din[(size_t)qy * W + qx];
                    if (v < p->d_min || v > p->d_max) continue;
                    const double w = weight_at(p, img, x, y, dx, dy);
                    t += w;
                    if (v < m[o]) b += w;
                    if (v <= m[o]) u += w;
                }
            below[o] = b;
            upto[o] = u;
            total[o] = t;
        }
    return 0;
}

int orc_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
