// fbs_internal.h - types shared by the HIP kernels and the C-ABI layer.
//
// Everything here is device-side plumbing for the gfx950 kernels; the public
// contract is include/fbs.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fbs.h"

namespace fbs {

// Problem geometry, passed to kernels by value.
struct Geom {
    int W, H, C;      // image size and channel count (1 or 3)
    int stride;       // bytes between image rows
    int dmin, D;      // first disparity and number of disparities
    int r;            // aggregation radius rho
    float tau;        // TAD cap
    int ncc_r;        // NCC block radius varrho
    float gd, gr;     // gamma_d, gamma_r of Eqs. 7-8 (the matrix-core kernel's
                      // double-precision recheck of near ties)
};

// Support-weight factors, computed on the host in double precision and
// rounded once to float (Eqs. 7-8):
//   gs[k] = exp(-k^2 / gamma_d^2)            k = |dx| or |dy|
//   gr[i] = exp(-i^2 / gamma_r^2)            gray, i = |I(q) - I(p)|
//   gr[i] = exp(-i^2 / (3 gamma_r^2))        RGB, one factor per channel
// so that w = gs[|dx|] * gs[|dy|] * prod_ch gr[|dI_ch|].
struct Tables {
    float gs[FBS_MAX_RADIUS + 1];
    float gr[256];
};

// The same factors in double precision (the weighted median filter).
struct Tables64 {
    double gs[FBS_MAX_RADIUS + 1];
    double gr[256];
};

enum CostSrc { SRC_VOLUME = 0, SRC_TAD = 1, SRC_NCC = 2 };

// ---- launchers (each returns the launch status; no synchronisation) ----
// cost_r (may be null): the right volume as well, by dual storage
hipError_t launch_cost_tad(const Geom& g, const uint8_t* L, const uint8_t* R, float* cost,
                           float* cost_r, hipStream_t s);
hipError_t launch_ncc_stats(const Geom& g, const uint8_t* L, const uint8_t* R, int2* stats,
                            hipStream_t s);
hipError_t launch_cost_ncc(const Geom& g, const uint8_t* L, const uint8_t* R,
                           const int2* stats, float* cost, float* cost_r, hipStream_t s);
// Both images mirrored left-right into packed copies (row stride W*C).
hipError_t launch_mirror(const Geom& g, const uint8_t* L, const uint8_t* R, uint8_t* Lm,
                         uint8_t* Rm, hipStream_t s);
// Eq. 9 on a left map and a right map (right_mirrored: the right map is
// stored mirrored, column W-1-u holds u); valid, sub, right_out optional.
hipError_t launch_lrc(const Geom& g, const int32_t* dl, const int32_t* dr, bool right_mirrored,
                      int max_diff, uint8_t* valid, float* sub, int32_t* right_out, hipStream_t s);
hipError_t launch_wta_subpixel(const Geom& g, const float* agg, int32_t* disp, float* sub,
                               hipStream_t s);

// Per-tile search ranges (int2 lo, hi per tile) from seed disparities.
hipError_t launch_guided_ranges(const Geom& g, const int32_t* disp, const uint8_t* valid, int tile_w,
                                int tile_h, int halo, int margin, int2* ranges, hipStream_t s);
// fbs_run's matrix-core kernel with one search range per kernel tile
// (ranges [tiles_y][tiles_x], tiles of 8 rows x 2 * mfma_default_cfg(g).nw).
int mfma_tile_rows();  // rows of a matrix-core kernel tile
hipError_t launch_mfma_ranged(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                              const int2* ranges, int32_t* disp, float* sub, hipStream_t s);

// Weighted median filter of an int32 map (g.r = window radius; values
// outside [g.dmin, g.dmin + g.D - 1] are holes).
hipError_t launch_wmf(const Geom& g, const Tables64& t, const uint8_t* img, const int32_t* din,
                      int32_t* dout, hipStream_t s);
int wmf_lds_bytes(int r, int ch);

// Bilateral aggregation on the vector ALUs.  src selects where costs come
// from (a materialised volume, or TAD / NCC computed in the kernel); agg,
// disp and sub are each optional.
hipError_t launch_valu(const Geom& g, const Tables& t, CostSrc src, const uint8_t* L,
                       const uint8_t* R, const float* cost, const int2* stats, float* agg,
                       int32_t* disp, float* sub, hipStream_t s);

// Fused TAD path on the matrix cores.
struct MfmaCfg {
    int nw;  // waves per workgroup: 4, 8 or 12 (8x8, 8x16 or 8x24 pixel tiles)
    int nb;  // 16-disparity blocks per LDS slab
};
bool mfma_supported(const Geom& g);
// NCC frames on the matrix cores (gray, block radius <= 1)
bool mfma_ncc_supported(const Geom& g);
float mfma_scaled_cap(const Geom& g);
int mfma_max_nb(const Geom& g, int nw);
bool mfma_nw_valid(const Geom& g, int nw);   // 4, 8 or 12 waves and the layout fits
MfmaCfg mfma_default_cfg(const Geom& g);     // what fbs_run uses
// Gray TAD frame with the learned surrogate's features (D >= 8): sub map and
// feat [H][W][32] BF16, equal to fbs_run's sub and to the features of its
// agg_out.
hipError_t launch_mfma_features(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                                float* sub, uint16_t* feat, hipStream_t s);
int mfma_lds_bytes(const Geom& g, int nb, int nw);
hipError_t launch_mfma(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                       int32_t* disp, float* sub, float* agg, hipStream_t s);
hipError_t launch_mfma_ncc(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                           int32_t* disp, float* sub, float* agg, hipStream_t s);
hipError_t launch_mfma_cfg(const Geom& g, const Tables& t, const MfmaCfg& cfg, const uint8_t* L,
                           const uint8_t* R, int32_t* disp, float* sub, float* agg, hipStream_t s);

// One pair of a batch, as the persistent kernel reads it from device memory.
struct BatchPair {
    Geom g;
    float scap;
    int nb;
    int tiles_x;
    int pad;
};

// One persistent launch: every (pair, tile) item of one (radius, channels,
// waves) class; items[i] = (pair index, tile index), pointer arrays indexed
// by pair.
struct BatchClass {
    int r, ch, nw;
    int lds;  // dynamic LDS bytes: the largest layout of any pair in the class
    int grid;             // persistent workgroups
    int one_wg_per_item;  // 1: one workgroup per item instead of persistent ones
    int co;               // 1: every pair's slab holds all its disparity blocks
    Tables tb;            // weight tables, shared by every pair of the class
    const BatchPair* pairs;
    const int2* items;
    int n_items;
    const int* n_dev;     // non-null: the list length is read from here (n_items: its bound)
    int tiles_per_item;   // persistent: consecutive tiles of one pair per item (>= 1)
    int* counter;
    const uint8_t* const* L;
    const uint8_t* const* R;
    int32_t* const* disp;
    float* const* sub;
};
hipError_t launch_mfma_batch(const BatchClass& bc, hipStream_t s);
int mfma_batch_blocks_per_cu(int r, int ch, int nw, int lds_bytes, bool co);
bool mfma_use_co(int D, int nb);  // chunk-outer kernels: one slab holds every block

}  // namespace fbs
