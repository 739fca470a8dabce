// k_valu.hip - bilateral cost aggregation (Eq. 6) on the vector ALUs.
//
// One workgroup = a 16x16 pixel tile, one lane per pixel.  The left image
// tile (with the window halo, plus the NCC block halo) is staged once in LDS.
// The disparity axis is walked in slabs of DS: per slab the workgroup fills
// an LDS cost slab [UH][UW][DS] for every position of the tile's window union
// (read from a volume, or computed from the LDS image tiles), then each lane
// walks its (2r+1)^2 taps, forms the weight of Eqs. 7-8 once per tap from the
// LDS lookup tables and applies it to the DS costs of that tap with DS fused
// multiply-adds into per-lane accumulators.  After each slab the lane divides
// by the weight sum and feeds the running WTA / Eq. 10 state, so the fused
// path never writes a volume unless agg is requested.
//
// Tap order (dy outer, dx inner) and arithmetic are identical for every cost
// source, so the fused result equals cost -> aggregate -> WTA bit for bit.
#include "fbs_device.h"
#include "fbs_internal.h"

namespace fbs {

namespace {

constexpr int TW = 16, TH = 16, NT = TW * TH;

struct Layout {
    int UW, UH;   // window union of the tile
    int hal;      // NCC block halo
    int LW, LH;   // left tile
    int RW;       // right tile width per slab
    size_t bytes;
};

__host__ __device__ inline Layout make_layout(int r, int ncc_r, int src, int ds)
{
    Layout l;
    l.UW = TW + 2 * r;
    l.UH = TH + 2 * r;
    l.hal = (src == SRC_NCC) ? ncc_r : 0;
    l.LW = l.UW + 2 * l.hal;
    l.LH = l.UH + 2 * l.hal;
    l.RW = l.LW + ds - 1;
    l.bytes = (size_t)(256 + 32) * 4 + (size_t)l.UH * l.UW * ds * 4 + (size_t)l.LH * l.LW * 4 +
              (src != SRC_VOLUME ? (size_t)l.LH * l.RW * 4 : 0);
    return l;
}

__device__ __forceinline__ uint32_t load_px(const uint8_t* img, int stride, int C, int x, int y)
{
    const uint8_t* p = img + (size_t)y * stride + (size_t)x * C;
    if (C == 1) return p[0];
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
}

template <int CH>
__device__ __forceinline__ float range_weight(const float* gr, uint32_t a, uint32_t b)
{
    if (CH == 1) return gr[abs((int)a - (int)b)];
    const float w0 = gr[abs((int)(a & 0xff) - (int)(b & 0xff))];
    const float w1 = gr[abs((int)((a >> 8) & 0xff) - (int)((b >> 8) & 0xff))];
    const float w2 = gr[abs((int)((a >> 16) & 0xff) - (int)((b >> 16) & 0xff))];
    return (w0 * w1) * w2;
}

template <int CH>
__device__ __forceinline__ float tad_cost(uint32_t a, uint32_t b, float tau)
{
    if (CH == 1) return fminf((float)abs((int)a - (int)b), tau);
    const int s = abs((int)(a & 0xff) - (int)(b & 0xff)) +
                  abs((int)((a >> 8) & 0xff) - (int)((b >> 8) & 0xff)) +
                  abs((int)((a >> 16) & 0xff) - (int)((b >> 16) & 0xff));
    return fminf((float)s / 3.0f, tau);
}

template <int SRC, int CH, int DS>
__global__ __launch_bounds__(NT) void k_valu(Geom g, Tables tb, const uint8_t* __restrict__ L,
                                             const uint8_t* __restrict__ R,
                                             const float* __restrict__ cost,
                                             const int2* __restrict__ stats,
                                             float* __restrict__ agg, int32_t* __restrict__ disp,
                                             float* __restrict__ sub)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int r = g.r;
    const Layout lay = make_layout(r, g.ncc_r, SRC, DS);
    const int UW = lay.UW, UH = lay.UH, hal = lay.hal, LW = lay.LW, LH = lay.LH, RW = lay.RW;
    float* s_gr = reinterpret_cast<float*>(smem);
    float* s_gs = s_gr + 256;
    float* s_cost = s_gs + 32;
    uint32_t* s_L = reinterpret_cast<uint32_t*>(s_cost + (size_t)UH * UW * DS);
    uint32_t* s_R = s_L + (size_t)LH * LW;

    const int tid = threadIdx.x;
    const int tx = tid % TW, ty = tid / TW;
    const int X0 = blockIdx.x * TW, Y0 = blockIdx.y * TH;
    const int x = X0 + tx, y = Y0 + ty;
    const bool inside = x < g.W && y < g.H;

    // lookup tables and the clamp-to-edge left tile
    for (int i = tid; i < 256; i += NT) s_gr[i] = tb.gr[i];
    if (tid <= FBS_MAX_RADIUS) s_gs[tid] = tb.gs[tid];
    const int bx = X0 - r - hal, by = Y0 - r - hal;
    for (int i = tid; i < LW * LH; i += NT) {
        const int u = i % LW, v = i / LW;
        const int xx = min(max(bx + u, 0), g.W - 1);
        const int yy = min(max(by + v, 0), g.H - 1);
        s_L[i] = load_px(L, g.stride, CH, xx, yy);
    }
    __syncthreads();

    const uint32_t Lp = s_L[(ty + r + hal) * LW + tx + r + hal];
    const int n_ncc = (2 * g.ncc_r + 1) * (2 * g.ncc_r + 1);
    const size_t plane = (size_t)g.W * g.H;
    float den = 0.f;
    Wta wta;
    wta.init();
    const int nslab = (g.D + DS - 1) / DS;

    for (int s = 0; s < nslab; ++s) {
        const int k0 = s * DS;
        const int d0 = g.dmin + k0;
        const int kvalid = min(DS, g.D - k0);
        if (SRC != SRC_VOLUME) {
            // right tile: columns bx - (d0 + DS - 1) ... bx + LW - 1 - d0
            const int rbx = bx - (d0 + DS - 1);
            for (int i = tid; i < LH * RW; i += NT) {
                const int u = i % RW, v = i / RW;
                const int xx = min(max(rbx + u, 0), g.W - 1);
                const int yy = min(max(by + v, 0), g.H - 1);
                s_R[i] = load_px(R, g.stride, CH, xx, yy);
            }
            __syncthreads();
        }
        // cost slab over the window union
        if (SRC == SRC_VOLUME) {
            for (int i = tid; i < DS * UH * UW; i += NT) {
                const int k = i / (UH * UW);
                const int q = i - k * (UH * UW);
                const int ui = q % UW, uj = q / UW;
                const int X = X0 - r + ui, Y = Y0 - r + uj;
                float c = 0.f;
                if (k < kvalid && X >= 0 && X < g.W && Y >= 0 && Y < g.H)
                    c = cost[(size_t)(k0 + k) * plane + (size_t)Y * g.W + X];
                s_cost[q * DS + k] = c;
            }
        } else {
            for (int i = tid; i < DS * UH * UW; i += NT) {
                const int k = i % DS;
                const int q = i / DS;
                const int ui = q % UW, uj = q / UW;
                const int X = X0 - r + ui, Y = Y0 - r + uj;
                const int d = d0 + k;
                float c = 0.f;
                if (k < kvalid && X >= 0 && X < g.W && Y >= 0 && Y < g.H) {
                    if (SRC == SRC_TAD) {
                        c = g.tau;
                        if (X - d >= 0)
                            c = tad_cost<CH>(s_L[(uj + hal) * LW + ui + hal],
                                             s_R[(uj + hal) * RW + ui + hal + DS - 1 - k], g.tau);
                    } else {
                        c = 2.0f;
                        if (X - d >= 0) {
                            int slr = 0;
                            for (int b = -g.ncc_r; b <= g.ncc_r; ++b) {
                                const uint32_t* lr = s_L + (uj + hal + b) * LW + ui + hal;
                                const uint32_t* rr = s_R + (uj + hal + b) * RW + ui + hal + DS - 1 - k;
                                for (int a = -g.ncc_r; a <= g.ncc_r; ++a)
                                    slr += (int)lr[a] * (int)rr[a];
                            }
                            const int2 sl = stats[(size_t)Y * g.W + X];
                            const int2 sr = stats[plane + (size_t)Y * g.W + (X - d)];
                            c = ncc_cost(n_ncc, sl.x, sl.y, sr.x, sr.y, slr);
                        }
                    }
                }
                s_cost[q * DS + k] = c;
            }
        }
        __syncthreads();

        if (inside) {
            float acc[DS];
#pragma unroll
            for (int k = 0; k < DS; ++k) acc[k] = 0.f;
            for (int dy = -r; dy <= r; ++dy) {
                const int Y = y + dy;
                const bool rowok = Y >= 0 && Y < g.H;
                const float wdy = s_gs[dy < 0 ? -dy : dy];
                const uint32_t* lrow = s_L + (ty + r + dy + hal) * LW + tx + r + hal;
                const float* crow = s_cost + ((ty + r + dy) * UW + tx + r) * DS;
                for (int dx = -r; dx <= r; ++dx) {
                    const int X = x + dx;
                    float w = 0.f;
                    if (rowok && X >= 0 && X < g.W)
                        w = (wdy * s_gs[dx < 0 ? -dx : dx]) * range_weight<CH>(s_gr, lrow[dx], Lp);
                    if (s == 0) den += w;
                    const float4* cp = reinterpret_cast<const float4*>(crow + dx * DS);
#pragma unroll
                    for (int k4 = 0; k4 < DS / 4; ++k4) {
                        const float4 c = cp[k4];
                        acc[4 * k4 + 0] = fmaf(w, c.x, acc[4 * k4 + 0]);
                        acc[4 * k4 + 1] = fmaf(w, c.y, acc[4 * k4 + 1]);
                        acc[4 * k4 + 2] = fmaf(w, c.z, acc[4 * k4 + 2]);
                        acc[4 * k4 + 3] = fmaf(w, c.w, acc[4 * k4 + 3]);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < DS; ++k) {
                if (k < kvalid) {
                    const float a = acc[k] / den;
                    wta.push(a, k0 + k);
                    if (agg) agg[(size_t)(k0 + k) * plane + (size_t)y * g.W + x] = a;
                }
            }
        }
        __syncthreads();  // the next slab overwrites s_R and s_cost
    }
    if (inside && (disp || sub)) {
        int32_t d;
        float ds;
        wta.finish(g.dmin, g.D, &d, &ds);
        if (disp) disp[(size_t)y * g.W + x] = d;
        if (sub) sub[(size_t)y * g.W + x] = ds;
    }
}

template <int SRC, int CH>
hipError_t launch_ds(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                     const float* cost, const int2* stats, float* agg, int32_t* disp, float* sub,
                     hipStream_t s, size_t lds_limit)
{
    dim3 grid((g.W + TW - 1) / TW, (g.H + TH - 1) / TH);
    Layout l16 = make_layout(g.r, g.ncc_r, SRC, 16);
    Layout l8 = make_layout(g.r, g.ncc_r, SRC, 8);
    Layout l4 = make_layout(g.r, g.ncc_r, SRC, 4);
    if (l16.bytes <= lds_limit && g.D >= 16)
        hipLaunchKernelGGL((k_valu<SRC, CH, 16>), grid, dim3(NT), l16.bytes, s, g, t, L, R, cost,
                           stats, agg, disp, sub);
    else if (l8.bytes <= lds_limit)
        hipLaunchKernelGGL((k_valu<SRC, CH, 8>), grid, dim3(NT), l8.bytes, s, g, t, L, R, cost,
                           stats, agg, disp, sub);
    else if (l4.bytes <= lds_limit)
        hipLaunchKernelGGL((k_valu<SRC, CH, 4>), grid, dim3(NT), l4.bytes, s, g, t, L, R, cost,
                           stats, agg, disp, sub);
    else
        return hipErrorInvalidConfiguration;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_valu(const Geom& g, const Tables& t, CostSrc src, const uint8_t* L,
                       const uint8_t* R, const float* cost, const int2* stats, float* agg,
                       int32_t* disp, float* sub, hipStream_t s)
{
    const size_t lds_limit = 64 * 1024;
    if (src == SRC_VOLUME) {
        return g.C == 3 ? launch_ds<SRC_VOLUME, 3>(g, t, L, R, cost, stats, agg, disp, sub, s, lds_limit)
                        : launch_ds<SRC_VOLUME, 1>(g, t, L, R, cost, stats, agg, disp, sub, s, lds_limit);
    }
    if (src == SRC_TAD) {
        return g.C == 3 ? launch_ds<SRC_TAD, 3>(g, t, L, R, cost, stats, agg, disp, sub, s, lds_limit)
                        : launch_ds<SRC_TAD, 1>(g, t, L, R, cost, stats, agg, disp, sub, s, lds_limit);
    }
    return launch_ds<SRC_NCC, 1>(g, t, L, R, cost, stats, agg, disp, sub, s, lds_limit);
}

}  // namespace fbs
