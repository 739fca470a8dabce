// k_wmf.hip - weighted median filter of an integer disparity map (the
// refinement step Section II-D names beside the left-right check), with the
// support weights of Eqs. 7-8 from the reference image, in double precision
// (weights and sums: a window whose valid values all sit far from the centre
// in intensity keeps weights far below float's range, and only relative
// weights within a window decide its median).
//
// Output per pixel: the smallest window value m whose cumulative weight (the
// weights of window values <= m) reaches half the window's total; values
// outside [d_min, d_max] are holes; -1 where a window holds none.
//
// One lane per pixel, 16x16 pixels per workgroup.  The image and the map of
// the tile plus an r halo are staged in LDS once.  The median is found by a
// radix descent over the disparity range: each level spreads the window's
// weights over 16 bins of the current range (per-lane histograms in LDS,
// lane-major so the 64 lanes of a wave hit 64 distinct banks), walks the
// cumulative sum to the bin that crosses half the total, and narrows the
// range to that bin; ceil(log16 D) levels reach single values (2 for D <= 256).
// Each level recomputes the window's weights (no per-tap storage).  The
// weight tables come from the host in double precision.
#include "fbs_internal.h"

namespace fbs {

namespace {

constexpr int kWmfTile = 16;
constexpr int kWmfThreads = kWmfTile * kWmfTile;
constexpr int kBins = 16;

struct WmfLayout {
    int side;          // tile side with halo
    int off_hist, off_img, off_disp, bytes;
};

__host__ __device__ inline WmfLayout wmf_layout(int r, int ch)
{
    WmfLayout l;
    l.side = kWmfTile + 2 * r;
    l.off_hist = (256 + 32) * 8;                              // range LUT, spatial factors
    l.off_disp = l.off_hist + kBins * kWmfThreads * 8;
    l.off_img = l.off_disp + l.side * l.side * 4;
    l.bytes = l.off_img + ((l.side * l.side * ch + 15) & ~15);
    return l;
}

template <int CH>
__global__ __launch_bounds__(kWmfThreads) void k_wmf(Geom g, Tables64 tb, const uint8_t* __restrict__ img,
                                                     const int32_t* __restrict__ din,
                                                     int32_t* __restrict__ dout)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int r = g.r;
    const WmfLayout lay = wmf_layout(r, CH);
    double* s_gr = reinterpret_cast<double*>(smem);
    double* s_gs = s_gr + 256;
    double* s_hist = reinterpret_cast<double*>(smem + lay.off_hist);
    int32_t* s_d = reinterpret_cast<int32_t*>(smem + lay.off_disp);
    uint8_t* s_img = smem + lay.off_img;
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * kWmfTile - r, y0 = blockIdx.y * kWmfTile - r;
    const int side = lay.side;
    const int dmax = g.dmin + g.D - 1;

    for (int i = tid; i < 256; i += kWmfThreads) s_gr[i] = tb.gr[i];
    if (tid < 32) s_gs[tid] = tid <= FBS_MAX_RADIUS ? tb.gs[tid] : 0.0;
    // halo positions off the image are holes; their image bytes are never read
    for (int i = tid; i < side * side; i += kWmfThreads) {
        const int ty = i / side, tx = i - ty * side;
        const int x = x0 + tx, y = y0 + ty;
        const bool in = x >= 0 && x < g.W && y >= 0 && y < g.H;
        int32_t v = -1;
        if (in) {
            v = din[(size_t)y * g.W + x];
            if (v < g.dmin || v > dmax) v = -1;
#pragma unroll
            for (int c = 0; c < CH; ++c) s_img[i * CH + c] = img[(size_t)y * g.stride + (size_t)x * CH + c];
        }
        s_d[i] = v;
    }
    __syncthreads();

    const int lx = tid % kWmfTile, ly = tid / kWmfTile;
    const int px = blockIdx.x * kWmfTile + lx, py = blockIdx.y * kWmfTile + ly;
    if (px >= g.W || py >= g.H) return;  // no barrier follows
    const int cpos = (ly + r) * side + (lx + r);
    int ip[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) ip[c] = s_img[cpos * CH + c];

    int lo = g.dmin, span = g.D;
    double below = 0.0, total = 0.0, half = 0.0;
    bool first = true;
    int32_t out = -1;
    for (;;) {
        const int bw = (span + kBins - 1) / kBins;
#pragma unroll
        for (int b = 0; b < kBins; ++b) s_hist[b * kWmfThreads + tid] = 0.0;
        for (int dy = -r; dy <= r; ++dy) {
            const double wy = s_gs[dy < 0 ? -dy : dy];
            const int row = (ly + r + dy) * side + lx + r;
            for (int dx = -r; dx <= r; ++dx) {
                const int q = row + dx;
                const int v = s_d[q];
                if (v < 0) continue;
                double w = wy * s_gs[dx < 0 ? -dx : dx];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int di = (int)s_img[q * CH + c] - ip[c];
                    w *= s_gr[di < 0 ? -di : di];
                }
                if (first) total += w;
                const int k = v - lo;
                if (k >= 0 && k < span) s_hist[(k / bw) * kWmfThreads + tid] += w;
            }
        }
        if (first) {
            if (!(total > 0.0)) break;  // no valid value (or all weights below double's range)
            half = 0.5 * total;
            first = false;
        }
        // the first bin whose cumulative weight reaches half; if rounding
        // leaves every bin short, the last bin that holds weight
        int pick = -1, last = -1;
        double cum = below, before_last = below;
        for (int b = 0; b < kBins && pick < 0; ++b) {
            const double h = s_hist[b * kWmfThreads + tid];
            if (h > 0.0) {
                last = b;
                before_last = cum;
            }
            if (cum + h >= half) pick = b;
            else cum += h;
        }
        if (pick < 0) {
            pick = last;
            cum = before_last;
        }
        below = cum;
        lo += pick * bw;
        span = min(bw, span - pick * bw);
        if (bw == 1) {
            out = lo;
            break;
        }
    }
    dout[(size_t)py * g.W + px] = out;
}

}  // namespace

int wmf_lds_bytes(int r, int ch) { return wmf_layout(r, ch).bytes; }

hipError_t launch_wmf(const Geom& g, const Tables64& t, const uint8_t* img, const int32_t* din,
                      int32_t* dout, hipStream_t s)
{
    dim3 grid((g.W + kWmfTile - 1) / kWmfTile, (g.H + kWmfTile - 1) / kWmfTile);
    const int lds = wmf_layout(g.r, g.C).bytes;
    if (g.C == 3)
        hipLaunchKernelGGL(k_wmf<3>, grid, dim3(kWmfThreads), lds, s, g, t, img, din, dout);
    else
        hipLaunchKernelGGL(k_wmf<1>, grid, dim3(kWmfThreads), lds, s, g, t, img, din, dout);
    return hipGetLastError();
}

}  // namespace fbs
