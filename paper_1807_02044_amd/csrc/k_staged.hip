// k_staged.hip - the materialising kernels of the staged path:
//   cost volume (TAD, or the paper's NCC with pre-computed block sums) and
//   WTA + subpixel over an aggregated volume; the small per-pixel kernels
//   of the left-right path (image mirroring, the consistency check of
//   Eq. 9); and the per-tile search ranges from reliable seeds.
//
// The cost kernels optionally also write the right volume by dual storage
// (Section II-A).  All of them are bound by HBM traffic: each writes or reads
// 4*W*H*D bytes of float volume once, with lanes along x so every access is a
// coalesced row segment of the [D][H][W] layout.
#include <climits>

#include "fbs_device.h"
#include "fbs_internal.h"

namespace fbs {

namespace {

constexpr int kRowThreads = 256;  // lanes along x per workgroup
constexpr int kSlab = 16;         // disparities per thread in the cost kernels

// Dual storage of the right volume (Section II-A): the cost computed at left
// pixel x and disparity d is also the right volume's value at (x - d, d), so
// a thread that computes it writes it to both volumes.  Right-volume entries
// whose match x = u + d lies past the right edge have no such thread; the
// thread at x = u (u >= W - d) writes them with the off-image value.
__device__ __forceinline__ void store_right(const Geom& g, float* __restrict__ cost_r, size_t plane_k,
                                            int x, int y, int d, bool computed, float c, float off)
{
    float* row = cost_r + plane_k + (size_t)y * g.W;
    if (computed) row[x - d] = c;
    if (x >= g.W - d) row[x] = off;
}

// TAD cost (Section II-A cost step with the truncated absolute difference):
// C(x,y,d) = min(mean_ch |L - R(x-d)|, tau); tau where x-d is off-image.
// cost_r (may be null): the right volume, by dual storage.
template <int CH>
__global__ __launch_bounds__(kRowThreads) void k_cost_tad(Geom g, const uint8_t* __restrict__ L,
                                                          const uint8_t* __restrict__ R,
                                                          float* __restrict__ cost,
                                                          float* __restrict__ cost_r)
{
    const int x = blockIdx.x * kRowThreads + threadIdx.x;
    const int y = blockIdx.y;
    const int k0 = blockIdx.z * kSlab;
    if (x >= g.W) return;
    const uint8_t* lrow = L + (size_t)y * g.stride;
    const uint8_t* rrow = R + (size_t)y * g.stride;
    int lv[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) lv[c] = lrow[x * CH + c];
    const size_t plane = (size_t)g.W * g.H;
    float* out = cost + (size_t)y * g.W + x;
    const int kend = min(k0 + kSlab, g.D);
    for (int k = k0; k < kend; ++k) {
        const int xr = x - (g.dmin + k);
        float c = g.tau;
        if (xr >= 0) {
            int s = 0;
#pragma unroll
            for (int ch = 0; ch < CH; ++ch) s += abs(lv[ch] - (int)rrow[xr * CH + ch]);
            const float m = (CH == 1) ? (float)s : (float)s / 3.0f;
            c = fminf(m, g.tau);
        }
        out[(size_t)k * plane] = c;
        if (cost_r) store_right(g, cost_r, (size_t)k * plane, x, y, g.dmin + k, xr >= 0, c, g.tau);
    }
}

// Per-pixel block sums S = sum i and S2 = sum i^2 over the clamp-to-edge
// (2*varrho+1)^2 block: the mean / deviation pre-computation of Section III.
// stats[0] holds the left image, stats[1] the right image, as [H][W] int2.
__global__ __launch_bounds__(kRowThreads) void k_ncc_stats(Geom g, const uint8_t* __restrict__ L,
                                                           const uint8_t* __restrict__ R,
                                                           int2* __restrict__ stats)
{
    const int x = blockIdx.x * kRowThreads + threadIdx.x;
    const int y = blockIdx.y;
    const int which = blockIdx.z;
    if (x >= g.W) return;
    const uint8_t* img = which ? R : L;
    int s = 0, s2 = 0;
    for (int j = -g.ncc_r; j <= g.ncc_r; ++j) {
        const int yy = min(max(y + j, 0), g.H - 1);
        const uint8_t* row = img + (size_t)yy * g.stride;
        for (int i = -g.ncc_r; i <= g.ncc_r; ++i) {
            const int v = row[min(max(x + i, 0), g.W - 1)];
            s += v;
            s2 += v * v;
        }
    }
    stats[(size_t)which * g.W * g.H + (size_t)y * g.W + x] = make_int2(s, s2);
}

// NCC cost 1 - c (Eq. 1): only the cross term sum i_l * i_r is formed here;
// the block sums come from k_ncc_stats.  cost_r as for k_cost_tad.
__global__ __launch_bounds__(kRowThreads) void k_cost_ncc(Geom g, const uint8_t* __restrict__ L,
                                                          const uint8_t* __restrict__ R,
                                                          const int2* __restrict__ stats,
                                                          float* __restrict__ cost,
                                                          float* __restrict__ cost_r)
{
    const int x = blockIdx.x * kRowThreads + threadIdx.x;
    const int y = blockIdx.y;
    const int k0 = blockIdx.z * kSlab;
    if (x >= g.W) return;
    const size_t plane = (size_t)g.W * g.H;
    const int n = (2 * g.ncc_r + 1) * (2 * g.ncc_r + 1);
    const int2 sl = stats[(size_t)y * g.W + x];
    float* out = cost + (size_t)y * g.W + x;
    const int kend = min(k0 + kSlab, g.D);
    for (int k = k0; k < kend; ++k) {
        const int d = g.dmin + k;
        float c = 2.0f;
        if (x - d >= 0) {
            int slr = 0;
            for (int j = -g.ncc_r; j <= g.ncc_r; ++j) {
                const int yy = min(max(y + j, 0), g.H - 1);
                const uint8_t* lrow = L + (size_t)yy * g.stride;
                const uint8_t* rrow = R + (size_t)yy * g.stride;
                for (int i = -g.ncc_r; i <= g.ncc_r; ++i) {
                    const int xl = min(max(x + i, 0), g.W - 1);
                    const int xr = min(max(x + i - d, 0), g.W - 1);
                    slr += (int)lrow[xl] * (int)rrow[xr];
                }
            }
            const int2 sr = stats[plane + (size_t)y * g.W + (x - d)];
            c = ncc_cost(n, sl.x, sl.y, sr.x, sr.y, slr);
        }
        out[(size_t)k * plane] = c;
        if (cost_r) store_right(g, cost_r, (size_t)k * plane, x, y, d, x - d >= 0, c, 2.0f);
    }
}

// WTA (Section II-C) and Eq. 10 over a materialised aggregated volume; one
// lane per pixel, reading the D planes in order.
__global__ __launch_bounds__(kRowThreads) void k_wta_subpixel(Geom g,
                                                              const float* __restrict__ agg,
                                                              int32_t* __restrict__ disp,
                                                              float* __restrict__ sub)
{
    const int x = blockIdx.x * kRowThreads + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.W) return;
    const size_t plane = (size_t)g.W * g.H;
    const float* a = agg + (size_t)y * g.W + x;
    Wta w;
    w.init();
    for (int k = 0; k < g.D; ++k) w.push(a[(size_t)k * plane], k);
    int32_t d;
    float ds;
    w.finish(g.dmin, g.D, &d, &ds);
    if (disp) disp[(size_t)y * g.W + x] = d;
    if (sub) sub[(size_t)y * g.W + x] = ds;
}

// Left-right mirror of both images into packed copies: column x of the copy
// is column W-1-x of the image, channels kept in order.  Mirroring turns the
// right-reference problem (match of right pixel u is left pixel u + d,
// weights from the right image) into the left-reference one on the mirrored
// pair (reference = mirrored right image, target = mirrored left image).
template <int CH>
__global__ __launch_bounds__(kRowThreads) void k_mirror(Geom g, const uint8_t* __restrict__ L,
                                                        const uint8_t* __restrict__ R,
                                                        uint8_t* __restrict__ Lm,
                                                        uint8_t* __restrict__ Rm)
{
    const int x = blockIdx.x * kRowThreads + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.W) return;
    const uint8_t* src = (blockIdx.z ? R : L) + (size_t)y * g.stride + (size_t)(g.W - 1 - x) * CH;
    uint8_t* dst = (blockIdx.z ? Rm : Lm) + ((size_t)y * g.W + x) * CH;
#pragma unroll
    for (int c = 0; c < CH; ++c) dst[c] = src[c];
}

// Left-right consistency, Eq. 9: left pixel (x, y) with disparity d keeps it
// when x - d is in the image and the right map holds d there (within
// max_diff).  Where the check fails the refined map gets -1 (match removed).
// MIRRORED: the right map is stored mirrored (column W-1-u holds u); it is
// also written out unmirrored to right_out when that is given.
template <bool MIRRORED>
__global__ __launch_bounds__(kRowThreads) void k_lrc(Geom g, const int32_t* __restrict__ dl,
                                                     const int32_t* __restrict__ dr, int max_diff,
                                                     uint8_t* __restrict__ valid,
                                                     float* __restrict__ sub,
                                                     int32_t* __restrict__ right_out)
{
    const int x = blockIdx.x * kRowThreads + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.W) return;
    const size_t row = (size_t)y * g.W;
    const int d = dl[row + x];
    const int u = x - d;
    bool ok = false;
    if (u >= 0 && u < g.W) {
        const int diff = dr[row + (MIRRORED ? g.W - 1 - u : u)] - d;
        ok = diff <= max_diff && -diff <= max_diff;
    }
    if (valid) valid[row + x] = ok ? 1 : 0;
    if (sub && !ok) sub[row + x] = -1.0f;
    if (right_out) right_out[row + x] = dr[row + (MIRRORED ? g.W - 1 - x : x)];
}

// Per-tile search ranges from reliable seeds (Section V, future work): tile
// (tx, ty) of tile_w x tile_h pixels gets [min - margin, max + margin] of the
// seed disparities (valid != 0, inside [d_min, d_max]) in the tile grown by
// `halo` pixels, clipped to [d_min, d_max]; the whole range without seeds.
// One workgroup per tile; lanes stride over the grown tile, then a wave and a
// workgroup min/max reduction.
__global__ __launch_bounds__(kRowThreads) void k_guided_ranges(Geom g, const int32_t* __restrict__ disp,
                                                               const uint8_t* __restrict__ valid,
                                                               int tile_w, int tile_h, int halo,
                                                               int margin, int2* __restrict__ ranges)
{
    __shared__ int s_lo[kRowThreads / 64], s_hi[kRowThreads / 64];
    const int tx = blockIdx.x, ty = blockIdx.y;
    const int dmax = g.dmin + g.D - 1;
    const int gw = tile_w + 2 * halo, gh = tile_h + 2 * halo;
    const int x0 = tx * tile_w - halo, y0 = ty * tile_h - halo;
    int lo = INT_MAX, hi = INT_MIN;
    for (int i = threadIdx.x; i < gw * gh; i += kRowThreads) {
        const int y = y0 + i / gw, x = x0 + i % gw;
        if (x < 0 || x >= g.W || y < 0 || y >= g.H) continue;
        const size_t o = (size_t)y * g.W + x;
        const int d = disp[o];
        if (!valid[o] || d < g.dmin || d > dmax) continue;
        lo = min(lo, d);
        hi = max(hi, d);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off));
        hi = max(hi, __shfl_xor(hi, off));
    }
    if ((threadIdx.x & 63) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kRowThreads / 64; ++w) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
        int2 r = make_int2(g.dmin, dmax);
        if (lo <= hi) r = make_int2(max(lo - margin, g.dmin), min(hi + margin, dmax));
        ranges[(size_t)ty * gridDim.x + tx] = r;
    }
}

}  // namespace

hipError_t launch_cost_tad(const Geom& g, const uint8_t* L, const uint8_t* R, float* cost,
                           float* cost_r, hipStream_t s)
{
    dim3 grid((g.W + kRowThreads - 1) / kRowThreads, g.H, (g.D + kSlab - 1) / kSlab);
    if (g.C == 3)
        hipLaunchKernelGGL(k_cost_tad<3>, grid, dim3(kRowThreads), 0, s, g, L, R, cost, cost_r);
    else
        hipLaunchKernelGGL(k_cost_tad<1>, grid, dim3(kRowThreads), 0, s, g, L, R, cost, cost_r);
    return hipGetLastError();
}

hipError_t launch_ncc_stats(const Geom& g, const uint8_t* L, const uint8_t* R, int2* stats,
                            hipStream_t s)
{
    dim3 grid((g.W + kRowThreads - 1) / kRowThreads, g.H, 2);
    hipLaunchKernelGGL(k_ncc_stats, grid, dim3(kRowThreads), 0, s, g, L, R, stats);
    return hipGetLastError();
}

hipError_t launch_cost_ncc(const Geom& g, const uint8_t* L, const uint8_t* R,
                           const int2* stats, float* cost, float* cost_r, hipStream_t s)
{
    dim3 grid((g.W + kRowThreads - 1) / kRowThreads, g.H, (g.D + kSlab - 1) / kSlab);
    hipLaunchKernelGGL(k_cost_ncc, grid, dim3(kRowThreads), 0, s, g, L, R, stats, cost, cost_r);
    return hipGetLastError();
}

hipError_t launch_wta_subpixel(const Geom& g, const float* agg, int32_t* disp, float* sub,
                               hipStream_t s)
{
    dim3 grid((g.W + kRowThreads - 1) / kRowThreads, g.H);
    hipLaunchKernelGGL(k_wta_subpixel, grid, dim3(kRowThreads), 0, s, g, agg, disp, sub);
    return hipGetLastError();
}

hipError_t launch_mirror(const Geom& g, const uint8_t* L, const uint8_t* R, uint8_t* Lm,
                         uint8_t* Rm, hipStream_t s)
{
    dim3 grid((g.W + kRowThreads - 1) / kRowThreads, g.H, 2);
    if (g.C == 3)
        hipLaunchKernelGGL(k_mirror<3>, grid, dim3(kRowThreads), 0, s, g, L, R, Lm, Rm);
    else
        hipLaunchKernelGGL(k_mirror<1>, grid, dim3(kRowThreads), 0, s, g, L, R, Lm, Rm);
    return hipGetLastError();
}

hipError_t launch_lrc(const Geom& g, const int32_t* dl, const int32_t* dr, bool right_mirrored,
                      int max_diff, uint8_t* valid, float* sub, int32_t* right_out, hipStream_t s)
{
    dim3 grid((g.W + kRowThreads - 1) / kRowThreads, g.H);
    if (right_mirrored)
        hipLaunchKernelGGL(k_lrc<true>, grid, dim3(kRowThreads), 0, s, g, dl, dr, max_diff, valid,
                           sub, right_out);
    else
        hipLaunchKernelGGL(k_lrc<false>, grid, dim3(kRowThreads), 0, s, g, dl, dr, max_diff, valid,
                           sub, right_out);
    return hipGetLastError();
}

hipError_t launch_guided_ranges(const Geom& g, const int32_t* disp, const uint8_t* valid, int tile_w,
                                int tile_h, int halo, int margin, int2* ranges, hipStream_t s)
{
    dim3 grid((g.W + tile_w - 1) / tile_w, (g.H + tile_h - 1) / tile_h);
    hipLaunchKernelGGL(k_guided_ranges, grid, dim3(kRowThreads), 0, s, g, disp, valid, tile_w, tile_h,
                       halo, margin, ranges);
    return hipGetLastError();
}

}  // namespace fbs
