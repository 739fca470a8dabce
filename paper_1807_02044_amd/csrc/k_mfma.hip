// k_mfma.hip - per-frame matrix-core launches of fbs_run and their default
// configuration (the tile code is in mfma_tile.h).
#include "mfma_tile.h"

namespace fbs {

bool mfma_supported(const Geom& g)
{
    float scap;
    if (g.r < 1 || g.r > kMaxR) return false;
    if (g.C != 1 && g.C != 3) return false;
    if (!scaled_cap(g, &scap)) return false;
    return mfma_layout(g.r, g.C, g.D, 1, 8).bytes <= kLdsLimit &&
           mfma_layout(g.r, g.C, g.D, 1, 4).bytes <= kLdsLimit;
}

float mfma_scaled_cap(const Geom& g)
{
    float scap = 0.0f;
    scaled_cap(g, &scap);
    return scap;
}

int mfma_max_nb(const Geom& g, int nw) { return max_nb(g.r, g.C, g.D, nw); }

int mfma_lds_bytes(const Geom& g, int nb, int nw) { return mfma_layout(g.r, g.C, g.D, nb, nw).bytes; }

hipError_t launch_mfma_cfg(const Geom& g, const Tables& t, const MfmaCfg& cfg, const uint8_t* L,
                           const uint8_t* R, int32_t* disp, float* sub, float* agg, hipStream_t s)
{
    float scap;
    if (!mfma_supported(g) || !scaled_cap(g, &scap)) return hipErrorInvalidValue;
    if (!mfma_nw_valid(g, cfg.nw) || cfg.nb < 1 || cfg.nb > max_nb(g.r, g.C, g.D, cfg.nw))
        return hipErrorInvalidValue;
    const TileJob job{g, scap, cfg.nb, L, R, disp, sub, agg, nullptr};
    return dispatch<FrameLauncher>(g.r, g.C, cfg.nw, job, t, s);
}

bool mfma_nw_valid(const Geom& g, int nw)
{
    return (nw == 4 || nw == 8 || (nw == 12 && g.r <= kMaxR12)) &&
           mfma_layout(g.r, g.C, g.D, 1, nw).bytes <= kLdsLimit;
}

// Default configuration: per candidate waves per workgroup, the chunk-outer
// path (one slab with every disparity block) where it fits, else the
// deepest slab whose LDS keeps the register-limited number of workgroups per
// CU resident; the candidate with the most resident waves per CU wins (ties:
// chunk-outer first, then 8, 12, 4 waves).  Cached per (radius, channels,
// disparity blocks) once the device has answered.

MfmaCfg mfma_default_cfg(const Geom& g)
{
    static std::atomic<int> cache[kMaxR + 1][2][FBS_MAX_DISP / 16 + 1];
    const int nblk = (g.D + 15) >> 4;
    std::atomic<int>& slot = cache[g.r][g.C == 3][nblk];
    int packed = slot.load(std::memory_order_relaxed);
    if (packed == 0) {
        static const int cands[3] = {8, 12, 4};
        MfmaCfg c{8, 1};
        if (pick_cfg<FrameOccupancy>(g, cands, 3, &c)) {
            packed = (c.nw << 8) | c.nb;
            slot.store(packed, std::memory_order_relaxed);
        } else {
            packed = (8 << 8) | max_nb(g.r, g.C, g.D, 8);
        }
    }
    return MfmaCfg{packed >> 8, packed & 255};
}

hipError_t launch_mfma(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                       int32_t* disp, float* sub, float* agg, hipStream_t s)
{
    return launch_mfma_cfg(g, t, mfma_default_cfg(g), L, R, disp, sub, agg, s);
}

int mfma_tile_rows() { return kTileH; }

hipError_t launch_mfma_ranged(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                              const int2* ranges, int32_t* disp, float* sub, hipStream_t s)
{
    float scap;
    if (!mfma_supported(g) || !scaled_cap(g, &scap)) return hipErrorInvalidValue;
    const MfmaCfg cfg = mfma_default_cfg(g);
    TileJob job{g, scap, cfg.nb, L, R, disp, sub, nullptr, nullptr};
    job.ranges = ranges;
    job.ranges_tx = (g.W + 2 * cfg.nw - 1) / (2 * cfg.nw);
    return dispatch<FrameLauncher>(g.r, g.C, cfg.nw, job, t, s);
}

}  // namespace fbs
