// fbs_device.h - device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fbs {

// NCC cost 1 - c from integer block sums (Eq. 1 with Eqs. 2-3 substituted
// and numerator and denominator multiplied by n):
//   c = (n*Slr - Sl*Sr) / sqrt((n*Sll - Sl^2) * (n*Srr - Sr^2)).
// All sums are exact integers; a flat block (zero variance) gives c = 0.
__device__ __forceinline__ float ncc_cost(int n, int sl, int sll, int sr, int srr, int slr)
{
    const long long vl = (long long)n * sll - (long long)sl * sl;
    const long long vr = (long long)n * srr - (long long)sr * sr;
    if (vl <= 0 || vr <= 0) return 1.0f;
    const long long num = (long long)n * slr - (long long)sl * sr;
    const double c = (double)num / sqrt((double)vl * (double)vr);
    return (float)(1.0 - c);
}

// Eq. 10: d^s = d + (c(d-1) - c(d+1)) / (2c(d-1) + 2c(d+1) - 4c(d)); d itself
// at the ends of the range or where the denominator is not positive.  Every
// operation rounds in the order written (no contraction into fused
// multiply-adds), so all kernels produce the same bits from the same costs.
__device__ __forceinline__ float eq10_subpixel(int d, bool interior, float cm, float c0, float cp)
{
#pragma clang fp contract(off)
    float ds = (float)d;
    if (interior) {
        const float den = 2.0f * cm + 2.0f * cp - 4.0f * c0;
        if (den > 0.0f) ds += (cm - cp) / den;
    }
    return ds;
}

// Running winner-take-all over ascending disparities (Section II-C, ties to
// the lowest d) that also keeps the two neighbours of the current best for
// the parabola of Eq. 10.
struct Wta {
    float best, cm, cp, prev;
    int bi;
    bool need_cp;

    __device__ __forceinline__ void init()
    {
        best = 0.f; cm = 0.f; cp = 0.f; prev = 0.f;
        bi = -1; need_cp = false;
    }
    // v is the aggregated cost at disparity index k (k = 0, 1, 2, ... in order)
    __device__ __forceinline__ void push(float v, int k)
    {
        if (bi < 0 || v < best) {
            cm = prev;
            best = v;
            bi = k;
            need_cp = true;
        } else if (need_cp) {
            cp = v;
            need_cp = false;
        }
        prev = v;
    }
    __device__ __forceinline__ void finish(int dmin, int D, int32_t* disp, float* sub) const
    {
        *disp = dmin + bi;
        *sub = eq10_subpixel(dmin + bi, bi > 0 && bi < D - 1, cm, best, cp);
    }
};

}  // namespace fbs
