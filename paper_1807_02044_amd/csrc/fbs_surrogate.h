// fbs_surrogate.h - layout constants and launchers of the learned surrogate.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fbs_internal.h"

// Packed parameter order (float32): w0 [3][3][32][17], b0 [32], w1 [3][3][32][32],
// b1 [32], w2 [3][3][32][32], b2 [32], w3 [3][3][1][32], b3 [1].
#define SUR_CH 32
#define SUR_CIN 17
#define SUR_TOPK 8
#define SUR_OFF_W0 0
#define SUR_OFF_B0 4896
#define SUR_OFF_W1 4928
#define SUR_OFF_B1 14144
#define SUR_OFF_W2 14176
#define SUR_OFF_B2 23392
#define SUR_OFF_W3 23424
#define SUR_OFF_B3 23712
#define SUR_NPARAM 23713
#define SUR_PART (9 * SUR_CH * SUR_CH + SUR_CH)  // per-tile partial gradient sums
#define SUR_FWD 0
#define SUR_BWD 1

namespace fbs {
// The full-radius job of a tile-gated surrogate run, as the fallback kernel
// reads it: one pair and its image / output pointers.
struct SurFallbackJob {
    BatchPair pair;
    const uint8_t* L;
    const uint8_t* R;
    int32_t* disp;
    float* sub;
};
hipError_t sur_features(int W, int H, int D, float tau, const float* agg, const uint8_t* L,
                        int lstride, uint16_t* F, hipStream_t s);
hipError_t sur_conv(int mode, int W, int H, const uint16_t* in, const uint16_t* A,
                    const float* bias, const uint16_t* mask_act, uint16_t* out, hipStream_t s);
hipError_t sur_last_fwd(int W, int H, const uint16_t* a3, const float* w3, const float* b3,
                        const float* cheap, float* pred, const float* label, float* g4,
                        float* loss_part, hipStream_t s);
int sur_loss_parts(int W, int H);
hipError_t sur_last_bwd(int W, int H, const float* g4, const float* w3, const uint16_t* a3,
                        uint16_t* gz, hipStream_t s);
int sur_wgrad_tiles(int W, int H);
hipError_t sur_wgrad(int W, int H, const uint16_t* g, const uint16_t* a, float* part,
                     float* reduced, hipStream_t s);
hipError_t sur_wgrad_last(int W, int H, const float* g4, const uint16_t* a3, float* part,
                          float* reduced, hipStream_t s);
hipError_t sur_unpack_grads(const float* r0, const float* r1, const float* r2, const float* r3,
                            float* grads, hipStream_t s);
hipError_t sur_adam(float* w, float* m, float* v, const float* g, float lr, float b1, float b2,
                    float bc1, float bc2, float eps, hipStream_t s);
hipError_t sur_pack(const float* master, uint16_t* fwd, uint16_t* bwd, float* w3, float* bias,
                    hipStream_t s);
hipError_t sur_gate(int n, const float* pred, const float* cheap, float gate_px, int* count,
                    hipStream_t s);
// fused inference of the whole net; zero2 (nullable): two ints set to 0
size_t sur_net_lds_bytes();
hipError_t sur_net_fwd(int W, int H, const uint16_t* feat, const uint16_t* fwd, const float* bias,
                       const float* w3, const float* b3, const float* cheap, float* pred,
                       int* zero2, hipStream_t s);
hipError_t sur_tile_gate(int W, int H, const float* pred, const float* cheap, float gate_px,
                         float tile_frac, int tw, int2* items, int* n_items,
                         const SurFallbackJob& job, SurFallbackJob* job_out, hipStream_t s);
}  // namespace fbs
