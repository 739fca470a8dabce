// k_mfma_feat.hip - the cheap run of the learned surrogate with its top-8
// features, on the matrix cores (tile code in mfma_tile.h).
#include "mfma_tile.h"

namespace fbs {

hipError_t launch_mfma_features(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                                float* sub, uint16_t* feat, hipStream_t s)
{
    float scap;
    if (g.C != 1 || g.D < 8 || !mfma_supported(g) || !scaled_cap(g, &scap) || !feat)
        return hipErrorInvalidValue;
    // 8 or 12 waves and the slab depth picked as for fbs_run (most resident
    // waves), cached per radius and disparity blocks
    static std::atomic<int> cache[kMaxR + 1][FBS_MAX_DISP / 16 + 1];
    const int nblk = (g.D + 15) >> 4;
    int packed = cache[g.r][nblk].load(std::memory_order_relaxed);
    if (packed == 0) {
        static const int cands[2] = {8, 12};
        MfmaCfg c{8, 1};
        packed = pick_cfg<FeatOccupancyAny>(g, cands, 2, &c) ? (c.nw << 8) | c.nb : (8 << 8) | 1;
        cache[g.r][nblk].store(packed, std::memory_order_relaxed);
    }
    const TileJob job{g, scap, packed & 255, L, R, nullptr, sub, nullptr, feat};
    if ((packed >> 8) == 12) return dispatch_r<FeatLauncher, 1, 12>(g.r, job, t, s);
    return dispatch_r<FeatLauncher, 1, 8>(g.r, job, t, s);
}

}  // namespace fbs
