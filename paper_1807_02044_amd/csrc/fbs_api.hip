// fbs_api.hip - the extern "C" entry points of include/fbs.h.
//
// Host side only: parameter validation (before anything is enqueued), the
// weight tables of Eqs. 7-8 in double precision rounded once to float, the
// choice of kernel, and error reporting.  No entry point allocates memory or
// synchronises the stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "fbs_internal.h"

namespace {

thread_local std::string g_last_error;

fbs_status fail(fbs_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

fbs_status fail(fbs_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

fbs_status hip_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return FBS_OK;
    return fail(FBS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool sigma_ok(float s) { return !isnan(s) && s > 0.0f; }

// Full check of the parameters of the cost / aggregation / fused paths.
fbs_status check_params(const fbs_params* p)
{
    if (!p) return fail(FBS_E_INVALID, "params is NULL");
    if (p->width < 1 || p->height < 1) return fail(FBS_E_INVALID, "width/height must be >= 1");
    if (p->width > 65535 || p->height > 65535)
        return fail(FBS_E_UNSUPPORTED, "width/height above 65535");
    if (p->channels != 1 && p->channels != 3) return fail(FBS_E_INVALID, "channels must be 1 or 3");
    if ((long long)p->row_stride < (long long)p->width * p->channels)
        return fail(FBS_E_INVALID, "row_stride %d < width*channels", p->row_stride);
    if (p->d_min < 0 || p->d_max < p->d_min || p->d_max >= p->width)
        return fail(FBS_E_INVALID, "need 0 <= d_min <= d_max < width (got %d..%d, width %d)",
                    p->d_min, p->d_max, p->width);
    if (p->d_max - p->d_min + 1 > FBS_MAX_DISP)
        return fail(FBS_E_UNSUPPORTED, "more than %d disparities", FBS_MAX_DISP);
    if (p->radius < 0) return fail(FBS_E_INVALID, "radius must be >= 0");
    if (p->radius > FBS_MAX_RADIUS)
        return fail(FBS_E_UNSUPPORTED, "radius %d above %d", p->radius, FBS_MAX_RADIUS);
    if (!sigma_ok(p->sigma_s) || !sigma_ok(p->sigma_r))
        return fail(FBS_E_INVALID, "sigma_s and sigma_r must be > 0");
    if (p->cost_type == FBS_COST_TAD) {
        if (!isfinite(p->cost_cap) || !(p->cost_cap > 0.0f))
            return fail(FBS_E_INVALID, "cost_cap must be finite and > 0");
    } else if (p->cost_type == FBS_COST_NCC) {
        if (p->channels != 1) return fail(FBS_E_UNSUPPORTED, "NCC cost needs channels == 1");
        if (p->ncc_radius < 0 || p->ncc_radius > FBS_MAX_NCC_RADIUS)
            return fail(FBS_E_UNSUPPORTED, "ncc_radius must be in 0..%d", FBS_MAX_NCC_RADIUS);
    } else {
        return fail(FBS_E_INVALID, "unknown cost_type %d", p->cost_type);
    }
    if (p->flags & ~FBS_F_FORCE_VALU) return fail(FBS_E_INVALID, "unknown flags 0x%x", p->flags);
    return FBS_OK;
}

fbs::Geom make_geom(const fbs_params* p)
{
    fbs::Geom g;
    g.W = p->width;
    g.H = p->height;
    g.C = p->channels;
    g.stride = p->row_stride;
    g.dmin = p->d_min;
    g.D = p->d_max - p->d_min + 1;
    g.r = p->radius;
    g.tau = p->cost_cap;
    g.ncc_r = p->ncc_radius;
    g.gd = p->sigma_s;
    g.gr = p->sigma_r;
    return g;
}

// Eqs. 7-8 factor tables, in double precision, rounded once to float.
fbs::Tables make_tables(const fbs_params* p)
{
    fbs::Tables t;
    const double gd = (double)p->sigma_s, gr = (double)p->sigma_r;
    for (int k = 0; k <= FBS_MAX_RADIUS; ++k) t.gs[k] = (float)exp(-(double)(k * k) / (gd * gd));
    const double scale = (p->channels == 3) ? 3.0 : 1.0;
    for (int i = 0; i < 256; ++i) t.gr[i] = (float)exp(-(double)(i * i) / (scale * gr * gr));
    return t;
}

fbs::Tables64 make_tables64(const fbs_params* p)
{
    fbs::Tables64 t;
    const double gd = (double)p->sigma_s, gr = (double)p->sigma_r;
    for (int k = 0; k <= FBS_MAX_RADIUS; ++k) t.gs[k] = exp(-(double)(k * k) / (gd * gd));
    const double scale = (p->channels == 3) ? 3.0 : 1.0;
    for (int i = 0; i < 256; ++i) t.gr[i] = exp(-(double)(i * i) / (scale * gr * gr));
    return t;
}

size_t ncc_ws_bytes(const fbs_params* p)
{
    const size_t b = (size_t)16 * p->width * p->height;
    return (b + 255) & ~(size_t)255;
}

bool aligned4(const void* q) { return ((uintptr_t)q & 3u) == 0; }

// Checks of the parameters that a map-only call reads (size and range).
fbs_status check_map_params(const fbs_params* p)
{
    if (!p) return fail(FBS_E_INVALID, "params is NULL");
    if (p->width < 1 || p->height < 1) return fail(FBS_E_INVALID, "width/height must be >= 1");
    if (p->width > 65535 || p->height > 65535)
        return fail(FBS_E_UNSUPPORTED, "width/height above 65535");
    if (p->d_min < 0 || p->d_max < p->d_min)
        return fail(FBS_E_INVALID, "need 0 <= d_min <= d_max");
    if (p->d_max - p->d_min + 1 > FBS_MAX_DISP)
        return fail(FBS_E_UNSUPPORTED, "more than %d disparities", FBS_MAX_DISP);
    return FBS_OK;
}

// The fused path on validated parameters: NCC on the matrix cores where they
// apply (gray, block radius <= 1), else block sums then the vector-ALU kernel;
// TAD on the matrix cores where they apply, else the vector ALUs.
fbs_status run_fused(const fbs_params* p, const fbs::Geom& g, const uint8_t* left,
                     const uint8_t* right, int32_t* disp, float* disp_sub, float* agg_out,
                     int2* stats, hipStream_t s, const char* what)
{
    const fbs::Tables t = make_tables(p);
    if (p->cost_type == FBS_COST_NCC) {
        if (!(p->flags & FBS_F_FORCE_VALU) && fbs::mfma_ncc_supported(g))
            return hip_status(fbs::launch_mfma_ncc(g, t, left, right, disp, disp_sub, agg_out, s), what);
        fbs_status st = hip_status(fbs::launch_ncc_stats(g, left, right, stats, s), what);
        if (st != FBS_OK) return st;
        return hip_status(fbs::launch_valu(g, t, fbs::SRC_NCC, left, right, nullptr, stats, agg_out,
                                           disp, disp_sub, s),
                          what);
    }
    if (!(p->flags & FBS_F_FORCE_VALU) && fbs::mfma_supported(g))
        return hip_status(fbs::launch_mfma(g, t, left, right, disp, disp_sub, agg_out, s), what);
    return hip_status(fbs::launch_valu(g, t, fbs::SRC_TAD, left, right, nullptr, nullptr, agg_out,
                                       disp, disp_sub, s),
                      what);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace of the fused left-right path: NCC block sums (NCC only), the two
// mirrored images, the mirrored right map and the left map.
struct LrLayout {
    size_t off_stats, off_lm, off_rm, off_drm, off_dl, total;
};

LrLayout lr_layout(const fbs_params* p)
{
    const size_t n = (size_t)p->width * p->height;
    const size_t img = align256(n * p->channels);
    LrLayout l;
    l.off_stats = 0;
    l.off_lm = p->cost_type == FBS_COST_NCC ? ncc_ws_bytes(p) : 0;
    l.off_rm = l.off_lm + img;
    l.off_drm = l.off_rm + img;
    l.off_dl = l.off_drm + align256(n * 4);
    l.total = l.off_dl + align256(n * 4);
    return l;
}

// Section II-C on both volumes and Eq. 9, fused: the right-reference run is
// the left-reference run on the mirrored pair (its map comes out mirrored),
// then the left run, then the check, which also unmirrors the right map.
fbs_status run_lr(const fbs_params* p, const uint8_t* left, const uint8_t* right, int max_diff,
                  int32_t* disp_left, int32_t* disp_right, uint8_t* valid, float* disp_sub,
                  unsigned char* ws, const LrLayout& lay, hipStream_t s, const char* what)
{
    const fbs::Geom g = make_geom(p);
    int2* stats = (int2*)(ws + lay.off_stats);
    uint8_t* lm = ws + lay.off_lm;
    uint8_t* rm = ws + lay.off_rm;
    int32_t* drm = (int32_t*)(ws + lay.off_drm);
    int32_t* dl = disp_left ? disp_left : (int32_t*)(ws + lay.off_dl);
    fbs_status st = hip_status(fbs::launch_mirror(g, left, right, lm, rm, s), what);
    if (st != FBS_OK) return st;
    fbs_params pm = *p;
    pm.row_stride = p->width * p->channels;
    fbs::Geom gm = make_geom(&pm);
    st = run_fused(&pm, gm, rm, lm, drm, nullptr, nullptr, stats, s, what);
    if (st != FBS_OK) return st;
    st = run_fused(p, g, left, right, dl, disp_sub, nullptr, stats, s, what);
    if (st != FBS_OK) return st;
    return hip_status(fbs::launch_lrc(g, dl, drm, true, max_diff, valid, disp_sub, disp_right, s),
                      what);
}


}  // namespace

namespace fbs {
// Shared with the no-allocation entry point (fbs_noalloc.hip).
size_t api_lr_workspace_bytes(const fbs_params* p) { return lr_layout(p).total; }
fbs_status api_run_lr(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                      int max_diff, int32_t* disp_left, int32_t* disp_right, uint8_t* valid,
                      float* disp_sub, unsigned char* ws, hipStream_t s, const char* what)
{
    return run_lr(p, left, right, max_diff, disp_left, disp_right, valid, disp_sub, ws,
                  lr_layout(p), s, what);
}
fbs_status api_hip_status(hipError_t e, const char* what) { return hip_status(e, what); }
bool api_aligned4(const void* q) { return aligned4(q); }
// Shared with the plan layer (fbs_plan.hip).
fbs_status api_check_params(const fbs_params* p) { return check_params(p); }
Geom api_geom(const fbs_params* p) { return make_geom(p); }
Tables api_tables(const fbs_params* p) { return make_tables(p); }
fbs_status api_fail(fbs_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}
}  // namespace fbs

extern "C" {

fbs_status fbs_validate(const fbs_params* p) { return check_params(p); }

fbs_status fbs_workspace_bytes(const fbs_params* p, size_t* bytes)
{
    fbs_status st = check_params(p);
    if (st != FBS_OK) return st;
    if (!bytes) return fail(FBS_E_INVALID, "bytes is NULL");
    *bytes = p->cost_type == FBS_COST_NCC ? ncc_ws_bytes(p) : 0;
    return FBS_OK;
}

fbs_status fbs_cost(const fbs_params* p, const uint8_t* left, const uint8_t* right, float* cost,
                    void* workspace, void* stream)
{
    fbs_status st = check_params(p);
    if (st != FBS_OK) return st;
    if (!left || !right || !cost) return fail(FBS_E_INVALID, "left, right and cost are required");
    if (!aligned4(cost)) return fail(FBS_E_INVALID, "cost must be 4-byte aligned");
    if (p->cost_type == FBS_COST_NCC && !workspace)
        return fail(FBS_E_WORKSPACE, "NCC cost needs %zu bytes of workspace", ncc_ws_bytes(p));
    if (workspace && ((uintptr_t)workspace & 15u))
        return fail(FBS_E_INVALID, "workspace must be 16-byte aligned");
    const fbs::Geom g = make_geom(p);
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    if (p->cost_type == FBS_COST_TAD)
        return hip_status(fbs::launch_cost_tad(g, left, right, cost, nullptr, s), "fbs_cost");
    int2* stats = (int2*)workspace;
    st = hip_status(fbs::launch_ncc_stats(g, left, right, stats, s), "fbs_cost(stats)");
    if (st != FBS_OK) return st;
    return hip_status(fbs::launch_cost_ncc(g, left, right, stats, cost, nullptr, s), "fbs_cost(ncc)");
}

fbs_status fbs_aggregate(const fbs_params* p, const uint8_t* left, const float* cost, float* agg,
                         void* stream)
{
    fbs_status st = check_params(p);
    if (st != FBS_OK) return st;
    if (!left || !cost || !agg) return fail(FBS_E_INVALID, "left, cost and agg are required");
    if (!aligned4(cost) || !aligned4(agg)) return fail(FBS_E_INVALID, "volumes must be 4-byte aligned");
    const fbs::Geom g = make_geom(p);
    const size_t vol = (size_t)g.W * g.H * g.D * sizeof(float);
    if ((const char*)cost < (const char*)agg + vol && (const char*)agg < (const char*)cost + vol)
        return fail(FBS_E_INVALID, "cost and agg overlap");
    const fbs::Tables t = make_tables(p);
    (void)hipGetLastError();
    return hip_status(fbs::launch_valu(g, t, fbs::SRC_VOLUME, left, nullptr, cost, nullptr, agg,
                                       nullptr, nullptr, (hipStream_t)stream),
                      "fbs_aggregate");
}

fbs_status fbs_wta_subpixel(const fbs_params* p, const float* agg, int32_t* disp, float* disp_sub,
                            void* stream)
{
    if (!p) return fail(FBS_E_INVALID, "params is NULL");
    if (p->width < 1 || p->height < 1) return fail(FBS_E_INVALID, "width/height must be >= 1");
    if (p->width > 65535 || p->height > 65535)
        return fail(FBS_E_UNSUPPORTED, "width/height above 65535");
    if (p->d_min < 0 || p->d_max < p->d_min)
        return fail(FBS_E_INVALID, "need 0 <= d_min <= d_max");
    if (p->d_max - p->d_min + 1 > FBS_MAX_DISP)
        return fail(FBS_E_UNSUPPORTED, "more than %d disparities", FBS_MAX_DISP);
    if (!agg) return fail(FBS_E_INVALID, "agg is required");
    if (!aligned4(agg) || !aligned4(disp) || !aligned4(disp_sub))
        return fail(FBS_E_INVALID, "pointers must be 4-byte aligned");
    if (!disp && !disp_sub) return FBS_OK;
    fbs::Geom g = make_geom(p);
    (void)hipGetLastError();
    return hip_status(fbs::launch_wta_subpixel(g, agg, disp, disp_sub, (hipStream_t)stream),
                      "fbs_wta_subpixel");
}

int fbs_run_variant(const fbs_params* p)
{
    fbs_status st = check_params(p);
    if (st != FBS_OK) return st;
    if (p->flags & FBS_F_FORCE_VALU) return 0;
    const fbs::Geom g = make_geom(p);
    if (p->cost_type == FBS_COST_NCC) return fbs::mfma_ncc_supported(g) ? 1 : 0;
    return fbs::mfma_supported(g) ? 1 : 0;
}

fbs_status fbs_run(const fbs_params* p, const uint8_t* left, const uint8_t* right, int32_t* disp,
                   float* disp_sub, float* agg_out, void* workspace, void* stream)
{
    fbs_status st = check_params(p);
    if (st != FBS_OK) return st;
    if (!left || !right) return fail(FBS_E_INVALID, "left and right are required");
    if (!aligned4(disp) || !aligned4(disp_sub) || !aligned4(agg_out))
        return fail(FBS_E_INVALID, "outputs must be 4-byte aligned");
    if (p->cost_type == FBS_COST_NCC && !workspace)
        return fail(FBS_E_WORKSPACE, "NCC cost needs %zu bytes of workspace", ncc_ws_bytes(p));
    if (workspace && ((uintptr_t)workspace & 15u))
        return fail(FBS_E_INVALID, "workspace must be 16-byte aligned");
    if (!disp && !disp_sub && !agg_out) return FBS_OK;
    (void)hipGetLastError();
    return run_fused(p, make_geom(p), left, right, disp, disp_sub, agg_out, (int2*)workspace,
                     (hipStream_t)stream, "fbs_run");
}

fbs_status fbs_cost_lr(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                       float* cost_left, float* cost_right, void* workspace, void* stream)
{
    fbs_status st = check_params(p);
    if (st != FBS_OK) return st;
    if (!left || !right || !cost_left || !cost_right)
        return fail(FBS_E_INVALID, "left, right, cost_left and cost_right are required");
    if (!aligned4(cost_left) || !aligned4(cost_right))
        return fail(FBS_E_INVALID, "volumes must be 4-byte aligned");
    const fbs::Geom g = make_geom(p);
    const size_t vol = (size_t)g.W * g.H * g.D * sizeof(float);
    if ((const char*)cost_left < (const char*)cost_right + vol &&
        (const char*)cost_right < (const char*)cost_left + vol)
        return fail(FBS_E_INVALID, "cost_left and cost_right overlap");
    if (p->cost_type == FBS_COST_NCC && !workspace)
        return fail(FBS_E_WORKSPACE, "NCC cost needs %zu bytes of workspace", ncc_ws_bytes(p));
    if (workspace && ((uintptr_t)workspace & 15u))
        return fail(FBS_E_INVALID, "workspace must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    if (p->cost_type == FBS_COST_TAD)
        return hip_status(fbs::launch_cost_tad(g, left, right, cost_left, cost_right, s),
                          "fbs_cost_lr");
    int2* stats = (int2*)workspace;
    st = hip_status(fbs::launch_ncc_stats(g, left, right, stats, s), "fbs_cost_lr(stats)");
    if (st != FBS_OK) return st;
    return hip_status(fbs::launch_cost_ncc(g, left, right, stats, cost_left, cost_right, s),
                      "fbs_cost_lr(ncc)");
}

fbs_status fbs_lrc(const fbs_params* p, const int32_t* disp_left, const int32_t* disp_right,
                   int32_t max_diff, uint8_t* valid, float* disp_sub, void* stream)
{
    fbs_status st = check_map_params(p);
    if (st != FBS_OK) return st;
    if (!disp_left || !disp_right) return fail(FBS_E_INVALID, "disp_left and disp_right are required");
    if (max_diff < 0) return fail(FBS_E_INVALID, "max_diff must be >= 0");
    if (!aligned4(disp_left) || !aligned4(disp_right) || !aligned4(disp_sub))
        return fail(FBS_E_INVALID, "maps must be 4-byte aligned");
    if (!valid && !disp_sub) return FBS_OK;
    (void)hipGetLastError();
    return hip_status(fbs::launch_lrc(make_geom(p), disp_left, disp_right, false, max_diff, valid,
                                      disp_sub, nullptr, (hipStream_t)stream),
                      "fbs_lrc");
}

fbs_status fbs_lr_workspace_bytes(const fbs_params* p, size_t* bytes)
{
    fbs_status st = check_params(p);
    if (st != FBS_OK) return st;
    if (!bytes) return fail(FBS_E_INVALID, "bytes is NULL");
    *bytes = lr_layout(p).total;
    return FBS_OK;
}

fbs_status fbs_run_lr(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                      int32_t max_diff, int32_t* disp_left, int32_t* disp_right, uint8_t* valid,
                      float* disp_sub, void* workspace, void* stream)
{
    fbs_status st = check_params(p);
    if (st != FBS_OK) return st;
    if (!left || !right) return fail(FBS_E_INVALID, "left and right are required");
    if (max_diff < 0) return fail(FBS_E_INVALID, "max_diff must be >= 0");
    if (!aligned4(disp_left) || !aligned4(disp_right) || !aligned4(disp_sub))
        return fail(FBS_E_INVALID, "outputs must be 4-byte aligned");
    const LrLayout lay = lr_layout(p);
    if (!workspace) return fail(FBS_E_WORKSPACE, "fbs_run_lr needs %zu bytes of workspace", lay.total);
    if ((uintptr_t)workspace & 255u) return fail(FBS_E_INVALID, "workspace must be 256-byte aligned");
    if (!disp_left && !disp_right && !valid && !disp_sub) return FBS_OK;
    (void)hipGetLastError();
    return run_lr(p, left, right, max_diff, disp_left, disp_right, valid, disp_sub,
                  (unsigned char*)workspace, lay, (hipStream_t)stream, "fbs_run_lr");
}

fbs_status fbs_wmf(const fbs_params* p, const uint8_t* reference, const int32_t* disp_in,
                   int32_t* disp_out, void* stream)
{
    if (!p) return fail(FBS_E_INVALID, "params is NULL");
    if (p->width < 1 || p->height < 1) return fail(FBS_E_INVALID, "width/height must be >= 1");
    if (p->width > 65535 || p->height > 65535)
        return fail(FBS_E_UNSUPPORTED, "width/height above 65535");
    if (p->channels != 1 && p->channels != 3) return fail(FBS_E_INVALID, "channels must be 1 or 3");
    if ((long long)p->row_stride < (long long)p->width * p->channels)
        return fail(FBS_E_INVALID, "row_stride %d < width*channels", p->row_stride);
    if (p->d_min < 0 || p->d_max < p->d_min)
        return fail(FBS_E_INVALID, "need 0 <= d_min <= d_max");
    if (p->d_max - p->d_min + 1 > FBS_MAX_DISP)
        return fail(FBS_E_UNSUPPORTED, "more than %d disparities", FBS_MAX_DISP);
    if (p->radius < 0) return fail(FBS_E_INVALID, "radius must be >= 0");
    if (p->radius > FBS_MAX_RADIUS)
        return fail(FBS_E_UNSUPPORTED, "radius %d above %d", p->radius, FBS_MAX_RADIUS);
    if (!sigma_ok(p->sigma_s) || !sigma_ok(p->sigma_r))
        return fail(FBS_E_INVALID, "sigma_s and sigma_r must be > 0");
    if (!reference || !disp_in || !disp_out)
        return fail(FBS_E_INVALID, "reference, disp_in and disp_out are required");
    if (!aligned4(disp_in) || !aligned4(disp_out))
        return fail(FBS_E_INVALID, "maps must be 4-byte aligned");
    const size_t map = (size_t)p->width * p->height * 4;
    if ((const char*)disp_in < (const char*)disp_out + map &&
        (const char*)disp_out < (const char*)disp_in + map)
        return fail(FBS_E_INVALID, "disp_in and disp_out overlap");
    (void)hipGetLastError();
    return hip_status(fbs::launch_wmf(make_geom(p), make_tables64(p), reference, disp_in, disp_out,
                                      (hipStream_t)stream),
                      "fbs_wmf");
}

fbs_status fbs_range_tile(const fbs_params* p, int32_t* tile_w, int32_t* tile_h)
{
    fbs_status st = check_params(p);
    if (st != FBS_OK) return st;
    const fbs::Geom g = make_geom(p);
    if (p->cost_type != FBS_COST_TAD || (p->flags & FBS_F_FORCE_VALU) || !fbs::mfma_supported(g))
        return fail(FBS_E_UNSUPPORTED, "search ranges need the matrix-core TAD kernel");
    if (tile_w) *tile_w = 2 * fbs::mfma_default_cfg(g).nw;
    if (tile_h) *tile_h = fbs::mfma_tile_rows();
    return FBS_OK;
}

fbs_status fbs_guided_ranges(const fbs_params* p, const int32_t* disp_seed, const uint8_t* valid,
                             int32_t halo, int32_t margin, int32_t* ranges, void* stream)
{
    int32_t tw = 0, th = 0;
    fbs_status st = fbs_range_tile(p, &tw, &th);
    if (st != FBS_OK) return st;
    if (!disp_seed || !valid || !ranges)
        return fail(FBS_E_INVALID, "disp_seed, valid and ranges are required");
    if (halo < 0 || margin < 0) return fail(FBS_E_INVALID, "halo and margin must be >= 0");
    if (halo > 64) return fail(FBS_E_UNSUPPORTED, "halo above 64");
    if (!aligned4(disp_seed) || ((uintptr_t)ranges & 7u))
        return fail(FBS_E_INVALID, "disp_seed must be 4-byte and ranges 8-byte aligned");
    (void)hipGetLastError();
    return hip_status(fbs::launch_guided_ranges(make_geom(p), disp_seed, valid, tw, th, halo, margin,
                                                (int2*)ranges, (hipStream_t)stream),
                      "fbs_guided_ranges");
}

fbs_status fbs_run_ranged(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                          const int32_t* ranges, int32_t* disp, float* disp_sub, void* stream)
{
    fbs_status st = fbs_range_tile(p, nullptr, nullptr);
    if (st != FBS_OK) return st;
    if (!left || !right || !ranges) return fail(FBS_E_INVALID, "left, right and ranges are required");
    if ((uintptr_t)ranges & 7u) return fail(FBS_E_INVALID, "ranges must be 8-byte aligned");
    if (!aligned4(disp) || !aligned4(disp_sub))
        return fail(FBS_E_INVALID, "outputs must be 4-byte aligned");
    if (!disp && !disp_sub) return FBS_OK;
    (void)hipGetLastError();
    return hip_status(fbs::launch_mfma_ranged(make_geom(p), make_tables(p), left, right,
                                              (const int2*)ranges, disp, disp_sub, (hipStream_t)stream),
                      "fbs_run_ranged");
}

const char* fbs_status_str(int status)
{
    switch (status) {
    case FBS_OK: return "ok";
    case FBS_E_INVALID: return "invalid argument";
    case FBS_E_UNSUPPORTED: return "unsupported";
    case FBS_E_HIP: return "HIP error";
    case FBS_E_WORKSPACE: return "workspace missing";
    default: return "unknown status";
    }
}

const char* fbs_last_error(void) { return g_last_error.c_str(); }

const char* fbs_version(void) { return "0.1.0"; }

}  // extern "C"
