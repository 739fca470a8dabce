// k_mfma_ncc.hip - per-frame matrix-core launches of fbs_run with the NCC
// cost of Eq. 1 (block radius varrho <= 1), gray images; the tile code is
// mfma_tile.h's NCC path.
#include "mfma_tile.h"

namespace fbs {

namespace {
constexpr int kNccMaxBlockR = 1;  // one dword per block row in the cost build
}

bool mfma_ncc_supported(const Geom& g)
{
    if (g.C != 1 || g.r < 1 || g.r > kMaxR || g.ncc_r < 0 || g.ncc_r > kNccMaxBlockR) return false;
    return mfma_layout(g.r, 1, g.D, 1, 4, true).bytes <= kLdsLimit;
}

// 8 waves where they are built and one slab of a block fits, else 4; the
// deepest slab that fits
MfmaCfg mfma_ncc_cfg(const Geom& g)
{
    const int nw = g.r <= kNccMaxR8 && mfma_layout(g.r, 1, g.D, 1, 8, true).bytes <= kLdsLimit ? 8 : 4;
    return MfmaCfg{nw, max_nb(g.r, 1, g.D, nw, true)};
}

hipError_t launch_mfma_ncc(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                           int32_t* disp, float* sub, float* agg, hipStream_t s)
{
    if (!mfma_ncc_supported(g)) return hipErrorInvalidValue;
    const MfmaCfg cfg = mfma_ncc_cfg(g);
    // NCC costs lie in [0, 2]; scaled by 2^10 their cap is 2048
    const TileJob job{g, 2048.0f, cfg.nb, L, R, disp, sub, agg, nullptr};
    if (cfg.nw == 8) return dispatch_r<NccLauncher, 1, 8>(g.r, job, t, s);
    return dispatch_r<NccLauncher, 1, 4>(g.r, job, t, s);
}

}  // namespace fbs
