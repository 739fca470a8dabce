// k_surrogate.hip - kernels of the learned FBS surrogate (inference and training).
//
// Network: four 3x3 'same' convolutions 17 -> 32 -> 32 -> 32 -> 1, ReLU after
// the first three, output = residual added to the cheap subpixel disparity.
// Activations and gradients between layers are BF16, channel-last
// [H][W][32] (the 17 input channels padded with zeros to 32); sums are FP32.
//
//   k_sur_features     top-8 aggregated costs / disparities + intensity
//   k_sur_conv<MODE>   32 -> 32 conv on the matrix cores (BF16 MFMA):
//                        forward  out = relu(conv(in, W) + b)
//                        backward out = conv(g, flip(W)^T) * [act > 0]
//   k_sur_last_fwd     32 -> 1 conv, residual, L1 loss gradient (vector ALU)
//   k_sur_last_bwd     gradient through the 32 -> 1 conv and the ReLU mask
//   k_sur_wgrad        weight / bias gradients of a 32 -> 32 layer (vector ALU)
//   k_sur_wgrad_last   weight / bias gradients of the 32 -> 1 layer
//   k_sur_reduce       fixed-order sum of per-tile partial gradients
//   k_sur_adam         Adam on the float32 master weights
//   k_sur_pack         BF16 kernel copies of the master weights
//   k_sur_gate         count of pixels where prediction and cheap differ
#include "fbs_internal.h"
#include "fbs_surrogate.h"

namespace fbs {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (no NaN inputs here)
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int kC = SUR_CH;  // padded channels

// ---------------------------------------------------------------- features

__global__ __launch_bounds__(256) void k_sur_features(int W, int H, int D, float tau,
                                                      const float* __restrict__ agg,
                                                      const uint8_t* __restrict__ L, int lstride,
                                                      uint16_t* __restrict__ F)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const size_t plane = (size_t)W * H;
    const float* a = agg + (size_t)y * W + x;
    float bv[SUR_TOPK];
    int bk[SUR_TOPK];
#pragma unroll
    for (int i = 0; i < SUR_TOPK; ++i) {
        bv[i] = __builtin_inff();
        bk[i] = 0;
    }
    for (int k = 0; k < D; ++k) {
        const float v = a[(size_t)k * plane];
        if (v < bv[SUR_TOPK - 1]) {
            // insert after equal values: ties keep the lower disparity first
#pragma unroll
            for (int i = SUR_TOPK - 1; i >= 0; --i) {
                const bool shift = i > 0 && v < bv[i > 0 ? i - 1 : 0];
                if (shift) {
                    bv[i] = bv[i - 1];
                    bk[i] = bk[i - 1];
                } else if (v < bv[i]) {
                    bv[i] = v;
                    bk[i] = k;
                }
            }
        }
    }
    uint32_t w[16];
    const float dn = (float)(D - 1);
#pragma unroll
    for (int i = 0; i < SUR_TOPK; i += 2) {
        w[i / 2] = (uint32_t)to_bf16(bv[i] / tau) | ((uint32_t)to_bf16(bv[i + 1] / tau) << 16);
        w[4 + i / 2] = (uint32_t)to_bf16((float)bk[i] / dn) | ((uint32_t)to_bf16((float)bk[i + 1] / dn) << 16);
    }
    w[8] = to_bf16((float)L[(size_t)y * lstride + x] / 255.0f);
#pragma unroll
    for (int i = 9; i < 16; ++i) w[i] = 0u;
    uint4* dst = reinterpret_cast<uint4*>(F + ((size_t)y * W + x) * kC);
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
}

// ------------------------------------------------------- 32 -> 32 conv (MFMA)
//
// out[p][m] = sum_{tap, k} A[tap][m][k] * in[p + off(tap)][k], off(tap) =
// (tap/3 - 1, tap%3 - 1), in = 0 off the image.  One workgroup: an 8 x 32
// pixel tile, 4 waves, each wave 4 groups of 16 pixels of one row.  Per group,
// cout block cb and tap: v_mfma_f32_16x16x32_bf16 with A = weights (16 out
// channels x 32 in channels, in registers) and B = 32 in channels x 16 pixels
// read from the LDS input tile; lane l of the result holds out channels
// 16cb + 4(l/16) + j of pixel l%16.
constexpr int CT_H = 8, CT_W = 32;

template <int MODE>
__global__ __launch_bounds__(256) void k_sur_conv(int W, int H, const uint16_t* __restrict__ in,
                                                  const uint16_t* __restrict__ A,
                                                  const float* __restrict__ bias,
                                                  const uint16_t* __restrict__ mask_act,
                                                  uint16_t* __restrict__ out)
{
    __shared__ __align__(16) uint16_t s_in[(CT_H + 2) * (CT_W + 2) * kC];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int X0 = blockIdx.x * CT_W, Y0 = blockIdx.y * CT_H;
    // input tile with a one-pixel zero halo, 16-byte chunks
    constexpr int kChunks = (CT_H + 2) * (CT_W + 2) * (kC / 8);
    for (int i = tid; i < kChunks; i += 256) {
        const int px = i / (kC / 8), c8 = i - px * (kC / 8);
        const int ty = px / (CT_W + 2), tx = px - ty * (CT_W + 2);
        const int y = Y0 - 1 + ty, x = X0 - 1 + tx;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (x >= 0 && x < W && y >= 0 && y < H)
            v = reinterpret_cast<const uint4*>(in + ((size_t)y * W + x) * kC)[c8];
        reinterpret_cast<uint4*>(s_in)[i] = v;
    }
    // weights: A operands of all taps and both 16-channel output blocks
    bf8 aw[9][2];
    const int m = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
            aw[t][cb] = *reinterpret_cast<const bf8*>(A + ((size_t)(t * kC + cb * 16 + m) * kC + 8 * kq));
    __syncthreads();

#pragma unroll 1
    for (int gi = 0; gi < 4; ++gi) {
        const int grp = wave * 4 + gi;
        const int ty = grp >> 1, tx0 = (grp & 1) * 16;
        const int y = Y0 + ty;
        const int x = X0 + tx0 + m;  // this lane's pixel (B operand column / result column)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int ky = t / 3, kx = t - 3 * (t / 3);
                const bf8 b = *reinterpret_cast<const bf8*>(
                    s_in + ((ty + ky) * (CT_W + 2) + (tx0 + m + kx)) * kC + 8 * kq);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[t][cb], b, acc, 0, 0, 0);
            }
            if (x < W && y < H) {
                const int c0 = cb * 16 + 4 * kq;
                const size_t o = ((size_t)y * W + x) * kC + c0;
                uint16_t r[4];
                if (MODE == SUR_FWD) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) r[j] = to_bf16(fmaxf(acc[j] + bias[c0 + j], 0.0f));
                } else {
                    const uint2 mk = *reinterpret_cast<const uint2*>(mask_act + o);
                    const uint16_t mv[4] = {(uint16_t)(mk.x & 0xffff), (uint16_t)(mk.x >> 16),
                                            (uint16_t)(mk.y & 0xffff), (uint16_t)(mk.y >> 16)};
#pragma unroll
                    for (int j = 0; j < 4; ++j) r[j] = from_bf16(mv[j]) > 0.0f ? to_bf16(acc[j]) : 0;
                }
                *reinterpret_cast<uint2*>(out + o) =
                    make_uint2((uint32_t)r[0] | ((uint32_t)r[1] << 16), (uint32_t)r[2] | ((uint32_t)r[3] << 16));
            }
        }
    }
}

// ------------------------------------------------------------- last layer

// resid[p] = sum_{tap, c} W3[tap][c] a3[p + off][c] + b3; pred = cheap + resid;
// with a label: g4 = bf16(sign(pred - label) / N) and per-block |pred - label| sums.
__global__ __launch_bounds__(256) void k_sur_last_fwd(int W, int H, const uint16_t* __restrict__ a3,
                                                      const float* __restrict__ w3,
                                                      const float* __restrict__ b3,
                                                      const float* __restrict__ cheap,
                                                      float* __restrict__ pred,
                                                      const float* __restrict__ label,
                                                      float* __restrict__ g4,
                                                      float* __restrict__ loss_part)
{
    __shared__ float s_w[9 * kC];
    __shared__ float s_red[256];
    for (int i = threadIdx.x; i < 9 * kC; i += 256) s_w[i] = w3[i];
    __syncthreads();
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    float err = 0.0f;
    if (x < W && y < H) {
        float acc = *b3;
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
            const uint4* src = reinterpret_cast<const uint4*>(a3 + ((size_t)yy * W + xx) * kC);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 v = src[q];
                const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = 8 * q + 2 * e;
                    acc = fmaf(s_w[t * kC + c], from_bf16((uint16_t)(u[e] & 0xffff)), acc);
                    acc = fmaf(s_w[t * kC + c + 1], from_bf16((uint16_t)(u[e] >> 16)), acc);
                }
            }
        }
        const size_t o = (size_t)y * W + x;
        const float pv = cheap[o] + acc;
        pred[o] = pv;
        if (label) {
            const float d = pv - label[o];
            err = fabsf(d);
            const float s = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
            g4[o] = from_bf16(to_bf16(s / (float)((size_t)W * H)));
        }
    }
    if (label) {
        s_red[threadIdx.x] = err;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) s_red[threadIdx.x] += s_red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) loss_part[blockIdx.y * gridDim.x + blockIdx.x] = s_red[0];
    }
}

// dL/dz2[p][c] = bf16( sum_tap W3[tap][c] g4[p - off(tap)] ) if a3[p][c] > 0
__global__ __launch_bounds__(256) void k_sur_last_bwd(int W, int H, const float* __restrict__ g4,
                                                      const float* __restrict__ w3,
                                                      const uint16_t* __restrict__ a3,
                                                      uint16_t* __restrict__ gz)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    float gv[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y - (t / 3 - 1), xx = x - (t % 3 - 1);
        gv[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? g4[(size_t)yy * W + xx] : 0.0f;
    }
    const size_t o = ((size_t)y * W + x) * kC;
    for (int c = 0; c < kC; c += 2) {
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            s0 = fmaf(w3[t * kC + c], gv[t], s0);
            s1 = fmaf(w3[t * kC + c + 1], gv[t], s1);
        }
        const uint32_t av = *reinterpret_cast<const uint32_t*>(a3 + o + c);
        const uint16_t r0 = from_bf16((uint16_t)(av & 0xffff)) > 0.f ? to_bf16(s0) : 0;
        const uint16_t r1 = from_bf16((uint16_t)(av >> 16)) > 0.f ? to_bf16(s1) : 0;
        *reinterpret_cast<uint32_t*>(gz + o + c) = (uint32_t)r0 | ((uint32_t)r1 << 16);
    }
}

// ---------------------------------------------------------- weight gradients
//
// Per 16 x 16 pixel tile: part[tile][tap][co][ci] = sum_p g[p][co] a[p + off][ci]
// and part[tile][9*32*32 + co] = sum_p g[p][co]; thread (co = t/8, 4 input
// channels ci4 = 4*(t%8)) owns 36 sums.
constexpr int WG_T = 16;

__global__ __launch_bounds__(256) void k_sur_wgrad(int W, int H, const uint16_t* __restrict__ g,
                                                   const uint16_t* __restrict__ a,
                                                   float* __restrict__ part)
{
    __shared__ __align__(16) uint16_t s_a[(WG_T + 2) * (WG_T + 2) * kC];
    __shared__ __align__(16) uint16_t s_g[WG_T * WG_T * kC];
    const int tid = threadIdx.x;
    const int X0 = blockIdx.x * WG_T, Y0 = blockIdx.y * WG_T;
    for (int i = tid; i < (WG_T + 2) * (WG_T + 2) * (kC / 8); i += 256) {
        const int px = i / (kC / 8), c8 = i - px * (kC / 8);
        const int ty = px / (WG_T + 2), tx = px - ty * (WG_T + 2);
        const int y = Y0 - 1 + ty, x = X0 - 1 + tx;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (x >= 0 && x < W && y >= 0 && y < H)
            v = reinterpret_cast<const uint4*>(a + ((size_t)y * W + x) * kC)[c8];
        reinterpret_cast<uint4*>(s_a)[i] = v;
    }
    for (int i = tid; i < WG_T * WG_T * (kC / 8); i += 256) {
        const int px = i / (kC / 8), c8 = i - px * (kC / 8);
        const int ty = px / WG_T, tx = px - ty * WG_T;
        const int y = Y0 + ty, x = X0 + tx;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (x < W && y < H) v = reinterpret_cast<const uint4*>(g + ((size_t)y * W + x) * kC)[c8];
        reinterpret_cast<uint4*>(s_g)[i] = v;
    }
    __syncthreads();
    const int co = tid >> 3, ci4 = 4 * (tid & 7);
    float acc[9][4];
    float bsum = 0.0f;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[t][e] = 0.0f;
    for (int py = 0; py < WG_T; ++py) {
        for (int px = 0; px < WG_T; ++px) {
            const float gv = from_bf16(s_g[(py * WG_T + px) * kC + co]);
            bsum += gv;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const uint2 av = *reinterpret_cast<const uint2*>(
                    s_a + ((py + t / 3) * (WG_T + 2) + px + t % 3) * kC + ci4);
                acc[t][0] = fmaf(gv, from_bf16((uint16_t)(av.x & 0xffff)), acc[t][0]);
                acc[t][1] = fmaf(gv, from_bf16((uint16_t)(av.x >> 16)), acc[t][1]);
                acc[t][2] = fmaf(gv, from_bf16((uint16_t)(av.y & 0xffff)), acc[t][2]);
                acc[t][3] = fmaf(gv, from_bf16((uint16_t)(av.y >> 16)), acc[t][3]);
            }
        }
    }
    const int tile = blockIdx.y * gridDim.x + blockIdx.x;
    float* pt = part + (size_t)tile * SUR_PART;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) pt[(t * kC + co) * kC + ci4 + e] = acc[t][e];
    if ((tid & 7) == 0) pt[9 * kC * kC + co] = bsum;
}

// Last layer: part[tile][tap*32 + c] = sum_p g4[p] a3[p + off][c]; part[tile][288] = sum g4.
__global__ __launch_bounds__(256) void k_sur_wgrad_last(int W, int H, const float* __restrict__ g4,
                                                        const uint16_t* __restrict__ a3,
                                                        float* __restrict__ part)
{
    __shared__ float s_g[WG_T * WG_T];
    const int tid = threadIdx.x;
    const int X0 = blockIdx.x * WG_T, Y0 = blockIdx.y * WG_T;
    {
        const int y = Y0 + tid / WG_T, x = X0 + tid % WG_T;
        s_g[tid] = (x < W && y < H) ? g4[(size_t)y * W + x] : 0.0f;
    }
    __syncthreads();
    const int tile = blockIdx.y * gridDim.x + blockIdx.x;
    float* pt = part + (size_t)tile * SUR_PART;
    // threads 0..287: one (tap, channel) each; thread 288 would be the bias
    for (int o = tid; o < 9 * kC + 1; o += 256) {
        float s = 0.0f;
        if (o < 9 * kC) {
            const int t = o / kC, c = o % kC;
            for (int i = 0; i < WG_T * WG_T; ++i) {
                const int y = Y0 + i / WG_T + t / 3 - 1, x = X0 + i % WG_T + t % 3 - 1;
                if (x < 0 || x >= W || y < 0 || y >= H) continue;
                s = fmaf(s_g[i], from_bf16(a3[((size_t)y * W + x) * kC + c]), s);
            }
        } else {
            for (int i = 0; i < WG_T * WG_T; ++i) s += s_g[i];
        }
        pt[o] = s;
    }
}

// out[j] = sum_{tile} part[tile][j] in tile order (deterministic)
__global__ __launch_bounds__(256) void k_sur_reduce(const float* __restrict__ part, int ntiles,
                                                    int n, float* __restrict__ out)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    float s = 0.0f;
    for (int t = 0; t < ntiles; ++t) s += part[(size_t)t * SUR_PART + j];
    out[j] = s;
}

// ------------------------------------------------------------ optimiser

__global__ __launch_bounds__(256) void k_sur_adam(float* __restrict__ w, float* __restrict__ m,
                                                  float* __restrict__ v,
                                                  const float* __restrict__ g, int n, float lr,
                                                  float b1, float b2, float bc1, float bc2,
                                                  float eps)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Kernel copies of the packed master weights:
//   fwd[l][tap][co][ci]  BF16, input channels padded with zeros (l = 0, 1, 2)
//   bwd[l][tap'][ci][co] BF16 = W_l[8 - tap'][co][ci]           (l = 1, 2)
//   w3[tap][c]           BF16-rounded float32;  bias[l][co] float32
__global__ __launch_bounds__(256) void k_sur_pack(const float* __restrict__ master,
                                                  uint16_t* __restrict__ fwd,
                                                  uint16_t* __restrict__ bwd,
                                                  float* __restrict__ w3, float* __restrict__ bias)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    constexpr int LW = 9 * kC * kC;
    if (i < 3 * LW) {
        const int l = i / LW, r = i - l * LW;
        const int t = r / (kC * kC), co = (r / kC) % kC, ci = r % kC;
        const int cin = l == 0 ? SUR_CIN : kC;
        const int wofs = l == 0 ? SUR_OFF_W0 : (l == 1 ? SUR_OFF_W1 : SUR_OFF_W2);
        const float v = ci < cin ? master[wofs + (t * kC + co) * cin + ci] : 0.0f;
        const uint16_t h = to_bf16(v);
        fwd[i] = h;
        if (l > 0) bwd[(size_t)(l - 1) * LW + ((8 - t) * kC + ci) * kC + co] = h;
    } else if (i < 3 * LW + 9 * kC) {
        const int j = i - 3 * LW;
        w3[j] = from_bf16(to_bf16(master[SUR_OFF_W3 + j]));
    } else if (i < 3 * LW + 9 * kC + 3 * kC) {
        const int j = i - 3 * LW - 9 * kC, l = j / kC, c = j % kC;
        const int bofs = l == 0 ? SUR_OFF_B0 : (l == 1 ? SUR_OFF_B1 : SUR_OFF_B2);
        bias[j] = master[bofs + c];
    }
}

// Gradients from the reduced per-layer sums into the packed parameter order.
__global__ __launch_bounds__(256) void k_sur_unpack_grads(const float* __restrict__ red0,
                                                          const float* __restrict__ red1,
                                                          const float* __restrict__ red2,
                                                          const float* __restrict__ red3,
                                                          float* __restrict__ grads)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= SUR_NPARAM) return;
    float v;
    if (i < SUR_OFF_B0) {
        const int r = i - SUR_OFF_W0, t = r / (kC * SUR_CIN), co = (r / SUR_CIN) % kC, ci = r % SUR_CIN;
        v = red0[(t * kC + co) * kC + ci];
    } else if (i < SUR_OFF_W1) {
        v = red0[9 * kC * kC + (i - SUR_OFF_B0)];
    } else if (i < SUR_OFF_B1) {
        v = red1[i - SUR_OFF_W1];
    } else if (i < SUR_OFF_W2) {
        v = red1[9 * kC * kC + (i - SUR_OFF_B1)];
    } else if (i < SUR_OFF_B2) {
        v = red2[i - SUR_OFF_W2];
    } else if (i < SUR_OFF_W3) {
        v = red2[9 * kC * kC + (i - SUR_OFF_B2)];
    } else {
        v = red3[i - SUR_OFF_W3];  // 288 weights then the bias
    }
    grads[i] = v;
}

// ------------------------------------------------------------------ gate

__global__ void k_sur_zero(int* p) { *p = 0; }

__global__ __launch_bounds__(256) void k_sur_gate(int n, const float* __restrict__ pred,
                                                  const float* __restrict__ cheap, float gate_px,
                                                  int* __restrict__ count)
{
    __shared__ int s_c;
    if (threadIdx.x == 0) s_c = 0;
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n && fabsf(pred[i] - cheap[i]) > gate_px) atomicAdd(&s_c, 1);
    __syncthreads();
    if (threadIdx.x == 0 && s_c) atomicAdd(count, s_c);
}

inline dim3 pix_grid(int W, int H) { return dim3((W + 63) / 64, (H + 3) / 4); }

}  // namespace

hipError_t sur_features(int W, int H, int D, float tau, const float* agg, const uint8_t* L,
                        int lstride, uint16_t* F, hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_features, pix_grid(W, H), dim3(256), 0, s, W, H, D, tau, agg, L,
                       lstride, F);
    return hipGetLastError();
}

hipError_t sur_conv(int mode, int W, int H, const uint16_t* in, const uint16_t* A,
                    const float* bias, const uint16_t* mask_act, uint16_t* out, hipStream_t s)
{
    dim3 grid((W + CT_W - 1) / CT_W, (H + CT_H - 1) / CT_H);
    if (mode == SUR_FWD)
        hipLaunchKernelGGL(k_sur_conv<SUR_FWD>, grid, dim3(256), 0, s, W, H, in, A, bias, mask_act, out);
    else
        hipLaunchKernelGGL(k_sur_conv<SUR_BWD>, grid, dim3(256), 0, s, W, H, in, A, bias, mask_act, out);
    return hipGetLastError();
}

hipError_t sur_last_fwd(int W, int H, const uint16_t* a3, const float* w3, const float* b3,
                        const float* cheap, float* pred, const float* label, float* g4,
                        float* loss_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_last_fwd, pix_grid(W, H), dim3(256), 0, s, W, H, a3, w3, b3, cheap,
                       pred, label, g4, loss_part);
    return hipGetLastError();
}

int sur_loss_parts(int W, int H) { return ((W + 63) / 64) * ((H + 3) / 4); }

hipError_t sur_last_bwd(int W, int H, const float* g4, const float* w3, const uint16_t* a3,
                        uint16_t* gz, hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_last_bwd, pix_grid(W, H), dim3(256), 0, s, W, H, g4, w3, a3, gz);
    return hipGetLastError();
}

int sur_wgrad_tiles(int W, int H) { return ((W + WG_T - 1) / WG_T) * ((H + WG_T - 1) / WG_T); }

hipError_t sur_wgrad(int W, int H, const uint16_t* g, const uint16_t* a, float* part,
                     float* reduced, hipStream_t s)
{
    dim3 grid((W + WG_T - 1) / WG_T, (H + WG_T - 1) / WG_T);
    hipLaunchKernelGGL(k_sur_wgrad, grid, dim3(256), 0, s, W, H, g, a, part);
    const int n = 9 * kC * kC + kC;
    hipLaunchKernelGGL(k_sur_reduce, dim3((n + 255) / 256), dim3(256), 0, s, part,
                       (int)(grid.x * grid.y), n, reduced);
    return hipGetLastError();
}

hipError_t sur_wgrad_last(int W, int H, const float* g4, const uint16_t* a3, float* part,
                          float* reduced, hipStream_t s)
{
    dim3 grid((W + WG_T - 1) / WG_T, (H + WG_T - 1) / WG_T);
    hipLaunchKernelGGL(k_sur_wgrad_last, grid, dim3(256), 0, s, W, H, g4, a3, part);
    const int n = 9 * kC + 1;
    hipLaunchKernelGGL(k_sur_reduce, dim3((n + 255) / 256), dim3(256), 0, s, part,
                       (int)(grid.x * grid.y), n, reduced);
    return hipGetLastError();
}

hipError_t sur_unpack_grads(const float* r0, const float* r1, const float* r2, const float* r3,
                            float* grads, hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_unpack_grads, dim3((SUR_NPARAM + 255) / 256), dim3(256), 0, s, r0, r1,
                       r2, r3, grads);
    return hipGetLastError();
}

hipError_t sur_adam(float* w, float* m, float* v, const float* g, float lr, float b1, float b2,
                    float bc1, float bc2, float eps, hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_adam, dim3((SUR_NPARAM + 255) / 256), dim3(256), 0, s, w, m, v, g,
                       SUR_NPARAM, lr, b1, b2, bc1, bc2, eps);
    return hipGetLastError();
}

hipError_t sur_pack(const float* master, uint16_t* fwd, uint16_t* bwd, float* w3, float* bias,
                    hipStream_t s)
{
    const int n = 3 * 9 * kC * kC + 9 * kC + 3 * kC;
    hipLaunchKernelGGL(k_sur_pack, dim3((n + 255) / 256), dim3(256), 0, s, master, fwd, bwd, w3, bias);
    return hipGetLastError();
}

hipError_t sur_gate(int n, const float* pred, const float* cheap, float gate_px, int* count,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_zero, dim3(1), dim3(1), 0, s, count);
    hipLaunchKernelGGL(k_sur_gate, dim3((n + 255) / 256), dim3(256), 0, s, n, pred, cheap, gate_px,
                       count);
    return hipGetLastError();
}

}  // namespace fbs
