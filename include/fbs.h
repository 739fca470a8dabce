/*
 * fbs.h - C ABI of the MI355X (gfx950) fast bilateral stereo library.
 *
 * The library computes the left-reference hot path of fast bilateral stereo
 * (Fan et al., "Real-Time Subpixel Fast Bilateral Stereo"): a per-pixel,
 * per-disparity matching-cost volume (Section II-A), bilateral aggregation of
 * that volume (Section II-B, Eqs. 6-8), winner-take-all disparity selection
 * (Section II-C) and parabola subpixel refinement (Section II-D, Eq. 10).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Images     rectified pair, HWC uint8, `row_stride` bytes between rows,
 *            `channels` 1 (gray) or 3 (RGB).  Disparity d maps left column x
 *            to right column x - d on the same row.
 * Volumes    float32 [D][H][W], plane k holds d = d_min + k, D = d_max-d_min+1,
 *            densely packed (plane stride H*W, row stride W elements).
 * Maps       int32 / float32 [H][W], densely packed, absolute disparities.
 * Pointers   image, volume, map and workspace pointers are DEVICE pointers
 *            (hipMalloc or equivalent) owned by the caller; the library never
 *            frees them, never keeps them after the call returns, and
 *            allocates nothing on these paths.  `params` is a HOST pointer,
 *            read during the call only.
 * Streams    `stream` is a hipStream_t passed as void* (NULL = the null
 *            stream).  Work is enqueued asynchronously; outputs are valid
 *            once the stream has been synchronised.
 * Errors     every call validates all parameters before it enqueues anything.
 *            On failure nothing is enqueued, the status is negative and
 *            fbs_last_error() returns a message (per calling thread).  A
 *            failed kernel launch returns FBS_E_HIP.
 *
 * Readings of the paper fixed by this ABI (left image is the reference):
 *   TAD cost      C = min(mean over channels of |L(x,y) - R(x-d,y)|, cost_cap);
 *                 C = cost_cap where x - d is outside the image.
 *   NCC cost      1 - c with c of Eq. 1 over a (2*ncc_radius+1)^2 block,
 *                 clamp-to-edge block pixels, c = 0 for a flat block, cost 2
 *                 where x - d is outside the image; gray only.
 *   weights       w = exp(-(dx^2+dy^2)/sigma_s^2) * exp(-dI^2/sigma_r^2)
 *                 (Eqs. 7-8 with gamma_d = sigma_s, gamma_r = sigma_r, no
 *                 factor 2); dI^2 is the channel mean of squared left-image
 *                 differences; sigma = +INFINITY makes that factor 1; taps
 *                 outside the image take no part in either sum of Eq. 6.
 *   WTA           lowest aggregated cost, ties to the lowest d.
 *   subpixel      Eq. 10 on the aggregated costs; d* itself at d_min, d_max,
 *                 or where the parabola's denominator is not positive.
 */
#ifndef FBS_H
#define FBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fbs_status {
    FBS_OK = 0,
    FBS_E_INVALID = -1,     /* bad parameter, null or misaligned pointer */
    FBS_E_UNSUPPORTED = -2, /* valid request outside the kernels' limits */
    FBS_E_HIP = -3,         /* HIP runtime error or failed kernel launch */
    FBS_E_WORKSPACE = -4    /* workspace required but NULL */
} fbs_status;

typedef enum fbs_cost_type {
    FBS_COST_TAD = 0, /* truncated absolute difference */
    FBS_COST_NCC = 1  /* normalised cross-correlation, Eqs. 1-3 */
} fbs_cost_type;

/* Kernel limits. */
#define FBS_MAX_RADIUS 16     /* rho: window (2*rho+1)^2 <= 33x33 */
#define FBS_MAX_NCC_RADIUS 3  /* varrho: NCC block <= 7x7 */
#define FBS_MAX_DISP 1024     /* d_max - d_min + 1 */

/* fbs_params.flags */
#define FBS_F_FORCE_VALU 0x1u /* fbs_run: use the vector-ALU kernel even where
                                 the matrix-core kernel applies */

typedef struct fbs_params {
    int32_t width;      /* W >= 1 */
    int32_t height;     /* H >= 1 */
    int32_t channels;   /* 1 or 3 */
    int32_t row_stride; /* bytes between image rows, >= width * channels */
    int32_t d_min;      /* 0 <= d_min <= d_max < width */
    int32_t d_max;
    int32_t radius;     /* rho of Eq. 6, 0 <= radius <= FBS_MAX_RADIUS */
    float sigma_s;      /* gamma_d of Eq. 7, > 0 (+INFINITY allowed) */
    float sigma_r;      /* gamma_r of Eq. 8, > 0 (+INFINITY allowed) */
    float cost_cap;     /* tau of the TAD cost, finite and > 0 (TAD only) */
    int32_t cost_type;  /* fbs_cost_type */
    int32_t ncc_radius; /* varrho of Eq. 1, 0..FBS_MAX_NCC_RADIUS (NCC only) */
    uint32_t flags;     /* FBS_F_* */
} fbs_params;

/* Host-only check of `p` (no device access, usable without a GPU).
 * Returns FBS_OK, FBS_E_INVALID or FBS_E_UNSUPPORTED. */
fbs_status fbs_validate(const fbs_params* p);

/* Bytes of device workspace fbs_cost and fbs_run need for `p` (0 for TAD;
 * 16*W*H rounded up to 256 for NCC, which holds the per-pixel block sums that
 * the paper pre-computes, Section III).  Host only. */
fbs_status fbs_workspace_bytes(const fbs_params* p, size_t* bytes);

/* Cost step, Section II-A (TAD, or NCC of Eqs. 1-3 as 1 - c).
 * left, right: images; cost: volume [D][H][W] written in full;
 * workspace: fbs_workspace_bytes(p) bytes, may be NULL when that is 0. */
fbs_status fbs_cost(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                    float* cost, void* workspace, void* stream);

/* Aggregation step, Section II-B, Eq. 6 with the weights of Eqs. 7-8 taken
 * from the reference image: the left image for the left volume, the right
 * image for the right volume of fbs_cost_lr.  cost: volume [D][H][W] (any
 * float values); agg: volume [D][H][W] written in full; cost and agg must not
 * overlap. */
fbs_status fbs_aggregate(const fbs_params* p, const uint8_t* reference, const float* cost,
                         float* agg, void* stream);

/* Optimisation and refinement, Sections II-C and II-D (Eq. 10).
 * agg: volume [D][H][W]; disp: int32 map, disp_sub: float32 map.  Either
 * output may be NULL (not written); only width, height, d_min, d_max of `p`
 * are read (radius and sigmas are not checked). */
fbs_status fbs_wta_subpixel(const fbs_params* p, const float* agg, int32_t* disp,
                            float* disp_sub, void* stream);

/* The whole left-reference path fused: cost, weights, aggregation, WTA and
 * Eq. 10 without materialising the cost volume.  disp, disp_sub: maps
 * (either may be NULL); agg_out: optional volume [D][H][W] of aggregated
 * costs (NULL = not written); workspace as for fbs_cost. */
fbs_status fbs_run(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                   int32_t* disp, float* disp_sub, float* agg_out, void* workspace,
                   void* stream);

/* Which fused kernel fbs_run picks for `p`: 1 = matrix-core (MFMA) kernel
 * (TAD; or NCC with ncc_radius <= 1), 0 = vector-ALU kernel.  Host only;
 * FBS_E_* on invalid `p`. */
int fbs_run_variant(const fbs_params* p);

/* ---- Both views: right volume, right map, left-right check ----
 *
 * Right reference (Section II-A, II-C): the right volume holds at (u, v, d)
 * the cost of right pixel (u, v) against left pixel (u + d, v), i.e. the left
 * volume's value at (u + d, v, d) (TAD cap / NCC 2 where u + d >= W); it is
 * aggregated with the weights of Eqs. 7-8 from the right image, and its WTA
 * gives the right map (ties to the lowest d).  Eq. 9 (Section II-D): a left
 * pixel (x, y) keeps its disparity d when x - d is in the image and
 * |right(x - d, y) - d| <= max_diff (0 = the equality printed in Eq. 9); where
 * it fails the match is removed.  */

/* Cost step with dual storage (Section II-A): each cost is computed once and
 * written to both volumes, cost_left[d][y][x] and cost_right[d][y][x - d];
 * right entries with x = u + d >= W get the off-image value.  Both volumes
 * [D][H][W], written in full, must not overlap; workspace as for fbs_cost. */
fbs_status fbs_cost_lr(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                       float* cost_left, float* cost_right, void* workspace, void* stream);

/* Eq. 9 on two integer maps (any source, e.g. fbs_wta_subpixel of the left
 * and the right aggregated volumes).  valid[H][W] (uint8, may be NULL)
 * receives 1 where the left match survives, else 0; disp_sub (float32, may be
 * NULL) is overwritten with -1 where the check fails and left unchanged where
 * it holds.  Only width, height, d_min, d_max of `p` are read. */
fbs_status fbs_lrc(const fbs_params* p, const int32_t* disp_left, const int32_t* disp_right,
                   int32_t max_diff, uint8_t* valid, float* disp_sub, void* stream);

/* Weighted median filter, the refinement step Section II-D names beside the
 * left-right check: disp_out[y][x] is the weighted median of the values of
 * disp_in in the (2 radius + 1)^2 window around (x, y), each weighted by
 * Eqs. 7-8 (sigma_s, sigma_r) from the reference image - the smallest
 * window value whose cumulative weight (weights of values <= it) reaches half
 * the window's total.  Values outside [d_min, d_max] are holes (e.g. the -1
 * left by a failed check, or a map masked with fbs_lrc's valid): they take no
 * part, and a window without any valid value gives -1.  From `p` only the
 * image geometry, d_min, d_max (d_max may exceed width here), radius and
 * sigma_s, sigma_r are read.  disp_in, disp_out: int32 [H][W], not
 * overlapping.  Weights and sums in double precision. */
fbs_status fbs_wmf(const fbs_params* p, const uint8_t* reference, const int32_t* disp_in,
                   int32_t* disp_out, void* stream);

/* ---- Search ranges suggested by reliable pixels (Section V) ----
 *
 * The paper's future work: reliable feature points suggest the search range
 * of their neighbourhood, and only that range is searched.  Ranges are given
 * per tile of the matrix-core kernel (fbs_range_tile), as int32 pairs
 * (lo, hi) of absolute disparities, [tiles_y][tiles_x][2] with
 * tiles_x = ceil(W / tile_w), tiles_y = ceil(H / tile_h).  TAD, radius 1..10
 * (the matrix-core kernel) only; FBS_E_UNSUPPORTED otherwise. */

/* Tile shape of the ranges for `p` (host only). */
fbs_status fbs_range_tile(const fbs_params* p, int32_t* tile_w, int32_t* tile_h);

/* Ranges from seeds: a tile's range is [min - margin, max + margin] of the
 * disparities disp_seed holds where valid != 0 (and inside [d_min, d_max])
 * in the tile grown by `halo` pixels on each side (0..64), clipped to
 * [d_min, d_max]; the whole range where the grown tile has no seed.  Seeds
 * are typically the pixels a cheap run's left-right check keeps
 * (fbs_run_lr at a small radius: disp_left and valid). */
fbs_status fbs_guided_ranges(const fbs_params* p, const int32_t* disp_seed, const uint8_t* valid,
                             int32_t halo, int32_t margin, int32_t* ranges, void* stream);

/* fbs_run restricted to the ranges: each pixel's costs are aggregated, and
 * its WTA and Eq. 10 run, only over its tile's range (Eq. 10 returns d* at
 * the range's ends).  A range is clipped to [d_min, d_max]; an empty one
 * (lo > hi after clipping) means the whole range.  disp, disp_sub as for
 * fbs_run (either may be NULL). */
fbs_status fbs_run_ranged(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                          const int32_t* ranges, int32_t* disp, float* disp_sub, void* stream);

/* Bytes of device workspace fbs_run_lr needs for `p` (mirrored image copies,
 * the right map, the left map, and NCC's block sums).  Host only. */
fbs_status fbs_lr_workspace_bytes(const fbs_params* p, size_t* bytes);

/* The paper's whole path for both views, fused (Sections II-A to II-D):
 * the right-reference run, the left-reference run, Eq. 9 and Eq. 10.
 * disp_left, disp_right: int32 [H][W] integer maps; valid: uint8 [H][W]
 * (Eq. 9); disp_sub: float32 [H][W], Eq. 10 on the left aggregated costs where
 * Eq. 9 holds and -1 where it fails.  Any output may be NULL.  workspace:
 * fbs_lr_workspace_bytes(p) bytes, 256-byte aligned, required.  The right run
 * is the left-reference kernel applied to the left-right mirrored pair
 * (mirrored right image as reference), so both views use the same kernels
 * and arithmetic as fbs_run.  Calls sharing one workspace must not overlap. */
fbs_status fbs_run_lr(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                      int32_t max_diff, int32_t* disp_left, int32_t* disp_right, uint8_t* valid,
                      float* disp_sub, void* workspace, void* stream);

/* Bytes of the static device scratch of fbs_run_lr_noalloc (per GPU). */
#define FBS_NOALLOC_SCRATCH_BYTES (32u << 20)

/* fbs_run_lr without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * outputs and arithmetic as fbs_run_lr; the workspace is a static device
 * array of FBS_NOALLOC_SCRATCH_BYTES on each GPU, which the library holds
 * until the process ends (its address is looked up on the first call on
 * each device, on the current device).  FBS_E_UNSUPPORTED when
 * fbs_lr_workspace_bytes(p) exceeds FBS_NOALLOC_SCRATCH_BYTES (e.g. above
 * about 5.5 Mpixel gray or 3.3 Mpixel RGB).  Every call on one GPU uses the
 * same scratch: calls that overlap on one GPU (different streams, threads
 * or processes' graphs replaying concurrently) race and must be ordered by
 * the caller.  Nothing in the scratch needs to start at zero. */
fbs_status fbs_run_lr_noalloc(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                              int32_t max_diff, int32_t* disp_left, int32_t* disp_right,
                              uint8_t* valid, float* disp_sub, void* stream);

/* ---- Batched plans: many pairs of uneven sizes in one graph launch ---- */

typedef struct fbs_plan fbs_plan;

/* fbs_plan_create flags */
#define FBS_PLAN_TUNE 0x1u     /* time candidates for shapes missing from the cache */
#define FBS_PLAN_PER_TILE 0x2u /* one workgroup per (pair, tile) item instead of
                                  persistent workgroups draining a queue */

/* Builds a plan for n pairs (params is a HOST array of n fbs_params; every
 * pair TAD).  Each pair gets the matrix-core kernel where fbs_run would use
 * it, with its waves-per-workgroup and disparity-slab depth taken from the
 * tuning cache at tune_cache_path (JSON, may be NULL), or - with
 * FBS_PLAN_TUNE and no cache entry for the pair's (W, H, C, D, r) - by
 * timing every candidate on synthetic data of that shape (the cache file is
 * then rewritten), else from the same heuristic as fbs_run.  Pairs of equal
 * radius, channels and waves share one launch over their (pair, tile) items:
 * persistent workgroups pulling items from a work queue, or with
 * FBS_PLAN_PER_TILE one workgroup per item; the whole launch sequence is
 * captured once into a hipGraph.  Allocates device and pinned host memory
 * and synchronises the device (tuning); not for the hot path.  *out is NULL
 * on failure.  The per-pixel arithmetic equals fbs_run's, so results are
 * bit-identical to n separate fbs_run calls. */
fbs_status fbs_plan_create(fbs_plan** out, int32_t n, const fbs_params* params,
                           const char* tune_cache_path, uint32_t flags);

/* Runs the plan: left, right, disp, disp_sub are HOST arrays of n DEVICE
 * pointers (images as described by the pair's params; dense int32 / float32
 * [H][W] maps).  Enqueues a pointer upload, one graph launch and, for pairs
 * the matrix cores cannot take, one vector-ALU launch each, on `stream`.
 * A plan holds one device pointer table and one set of work-queue counters,
 * so launches of one plan are ordered: each launch waits on the device for
 * the previous one to finish, whatever stream either was given (launches on
 * two streams therefore do not overlap; use one plan per stream for that).
 * Waits (on the host) only for the previous launch's pointer upload.  Calls
 * on one plan from several host threads must be serialised by the caller. */
fbs_status fbs_plan_launch(fbs_plan* plan, const uint8_t* const* left,
                           const uint8_t* const* right, int32_t* const* disp,
                           float* const* disp_sub, void* stream);

/* Configuration chosen for one pair: matrix_cores (1/0), waves per
 * workgroup (4, 8 or 12; 12 only up to radius 7) and disparity-slab depth in
 * blocks of 16 (0 for a vector-ALU pair).  Any output may be NULL. */
fbs_status fbs_plan_pair_config(const fbs_plan* plan, int32_t pair, int32_t* matrix_cores,
                                int32_t* waves, int32_t* slab_blocks);

/* Host-side launches per fbs_plan_launch (1 graph + vector-ALU pairs). */
int32_t fbs_plan_num_launches(const fbs_plan* plan);

/* Waits for the plan's last launch, then frees it.  NULL is a no-op. */
void fbs_plan_destroy(fbs_plan* plan);

/* ---- Learned surrogate of the full-radius run ----
 *
 * A small convolutional net predicts the subpixel disparity map of a
 * full-radius run (Section II, all steps) from a cheap small-radius run:
 *   features  17 BF16 channels per pixel, channel-last [H][W][32] (channels
 *             17..31 are written as zero): the 8 lowest aggregated costs of
 *             the cheap run in ascending order (ties to the lower d) divided
 *             by its cost_cap, their disparity indices (d - d_min)/(D - 1)
 *             in the same order, and the left intensity / 255.
 *   net       3x3 zero-padded convolutions 17 -> 32 -> 32 -> 32 -> 1, ReLU
 *             after the first three; BF16 weights and activations, float32
 *             sums; the output is added to the cheap run's subpixel map.
 *   training  mean absolute error against a label map, Adam (beta1 0.9,
 *             beta2 0.999, eps 1e-8) on float32 master weights.
 * Parameters are one float32 array of fbs_surrogate_num_params() values:
 * w0 [3][3][32][17], b0 [32], w1 [3][3][32][32], b1 [32], w2 [3][3][32][32],
 * b2 [32], w3 [3][3][1][32], b3 [1]; weight [ky][kx][out][in] multiplies the
 * input at image offset (ky - 1, kx - 1).  Feature, map and gradient
 * pointers are DEVICE pointers; feat must be 16-byte aligned. */
typedef struct fbs_surrogate fbs_surrogate;

int32_t fbs_surrogate_num_params(void);

/* Allocates weights (all zero), Adam state and buffers for frames up to
 * max_width x max_height and, for fbs_surrogate_run, cheap runs of up to
 * max_disp disparities (8..FBS_MAX_DISP).  Synchronises the device. */
fbs_status fbs_surrogate_create(fbs_surrogate** out, int32_t max_width, int32_t max_height,
                                int32_t max_disp);

/* Waits for the device, then frees the object.  NULL is a no-op. */
void fbs_surrogate_destroy(fbs_surrogate* s);

/* Copies fbs_surrogate_num_params() float32 values from / to HOST memory.
 * set_params also clears the Adam state.  Both synchronise the device. */
fbs_status fbs_surrogate_set_params(fbs_surrogate* s, const float* host_params);
fbs_status fbs_surrogate_get_params(fbs_surrogate* s, float* host_params);

/* Features of a cheap run: `cheap` describes it (gray TAD, D >= 8), agg is
 * its aggregated volume [D][H][W] (fbs_run's agg_out), feat receives
 * [H][W][32] BF16 (uint16 bit patterns). */
fbs_status fbs_surrogate_features(fbs_surrogate* s, const fbs_params* cheap, const uint8_t* left,
                                  const float* agg, uint16_t* feat, void* stream);

/* The cheap run and its features in one call: cheap_sub[H][W] receives the
 * cheap run's subpixel map (as fbs_run), feat [H][W][32] its features (as
 * fbs_surrogate_features on fbs_run's agg_out), bit for bit.  Where the
 * matrix-core kernel applies this is one launch that keeps the volume out of
 * HBM; otherwise fbs_run plus fbs_surrogate_features through the object's
 * volume buffer (D <= max_disp). */
fbs_status fbs_surrogate_cheap_run(fbs_surrogate* s, const fbs_params* cheap, const uint8_t* left,
                                   const uint8_t* right, float* cheap_sub, uint16_t* feat,
                                   void* stream);

/* Prediction: pred[H][W] = cheap_sub + net(feat). */
fbs_status fbs_surrogate_forward(fbs_surrogate* s, int32_t width, int32_t height,
                                 const uint16_t* feat, const float* cheap_sub, float* pred,
                                 void* stream);

/* Forward plus backward of the mean absolute error against label[H][W]:
 * pred receives the prediction, grads (num_params float32, device) the
 * gradient in the packed order, loss (device float, may be NULL) the loss.
 * Uses the object's buffers: calls on one object must not overlap. */
fbs_status fbs_surrogate_gradients(fbs_surrogate* s, int32_t width, int32_t height,
                                   const uint16_t* feat, const float* cheap_sub,
                                   const float* label, float* pred, float* grads, float* loss,
                                   void* stream);

/* One Adam step with learning rate lr on the master weights (device grads). */
fbs_status fbs_surrogate_adam(fbs_surrogate* s, const float* grads, float lr, void* stream);

/* Inference with fallback: runs `cheap` and its features
 * (fbs_surrogate_cheap_run) and the net into disp_sub; counts pixels where
 * the prediction and the cheap subpixel map differ by more than gate_px, and
 * when that count exceeds gate_frac * W * H reruns `full` (same pair and
 * disparity range, e.g. the full radius) into disp_sub and sets *fell_back
 * to 1 (else 0; fell_back may be NULL).  Synchronises `stream` once, for the
 * count. */
fbs_status fbs_surrogate_run(fbs_surrogate* s, const fbs_params* cheap, const fbs_params* full,
                             const uint8_t* left, const uint8_t* right, float* disp_sub,
                             float gate_px, float gate_frac, int32_t* fell_back, void* stream);

/* Inference with a fallback per tile: runs `cheap` and its features, then
 * the net into disp_sub, then reruns `full` (same pair and disparity range)
 * on every tile of the full run's matrix-core kernel (8 rows by 8, 16 or 24
 * columns, as fbs_run picks for `full`) in which more than tile_frac of the
 * pixels have |prediction - cheap subpixel map| > gate_px; those tiles of
 * disp_sub then hold exactly fbs_run(full)'s values.  tile_frac < 0 reruns
 * every tile, tile_frac >= 1 none.  No host synchronisation: the tile list
 * is built and consumed on the device.  FBS_E_UNSUPPORTED when `full` is
 * not a gray TAD run the matrix-core kernel takes (or forces the vector
 * ALUs).  Calls on one object must not overlap. */
fbs_status fbs_surrogate_run_tiled(fbs_surrogate* s, const fbs_params* cheap,
                                   const fbs_params* full, const uint8_t* left,
                                   const uint8_t* right, float* disp_sub, float gate_px,
                                   float tile_frac, void* stream);

/* Static description of a status code. */
const char* fbs_status_str(int status);

/* Message of the calling thread's last failed call ("" if none). */
const char* fbs_last_error(void);

/* Library version, e.g. "0.1.0". */
const char* fbs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FBS_H */
