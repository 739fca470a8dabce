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
 * from the left image.  cost: volume [D][H][W] (any float values);
 * agg: volume [D][H][W] written in full; cost and agg must not overlap. */
fbs_status fbs_aggregate(const fbs_params* p, const uint8_t* left, const float* cost,
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

/* Which fused kernel fbs_run picks for `p`: 1 = matrix-core (MFMA) kernel,
 * 0 = vector-ALU kernel.  Host only; FBS_E_* on invalid `p`. */
int fbs_run_variant(const fbs_params* p);

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
