// k_surrogate.hip - kernels of the learned FBS surrogate (inference and training).
//
// Network: four 3x3 'same' convolutions 17 -> 32 -> 32 -> 32 -> 1, ReLU after
// the first three, output = residual added to the cheap subpixel disparity.
// Activations and gradients between layers are BF16, channel-last
// [H][W][32] (the 17 input channels padded with zeros to 32); sums are FP32.
//
//   k_sur_features     top-8 aggregated costs / disparities + intensity
//   k_sur_net_fwd      inference: all four layers and the residual in one
//                        launch, bit-identical to the per-layer kernels
//   k_sur_conv<MODE>   32 -> 32 conv on the matrix cores (BF16 MFMA):
//                        forward  out = relu(conv(in, W) + b)
//                        backward out = conv(g, flip(W)^T) * [act > 0]
//   k_sur_last_fwd     32 -> 1 conv (matrix cores), residual, L1 loss gradient
//   k_sur_last_bwd     gradient through the 32 -> 1 conv and the ReLU mask
//   k_sur_wgrad        weight / bias gradients of a 32 -> 32 layer (vector ALU)
//   k_sur_wgrad_last   weight / bias gradients of the 32 -> 1 layer
//   k_sur_reduce       fixed-order sum of per-tile partial gradients
//   k_sur_adam         Adam on the float32 master weights
//   k_sur_pack         BF16 kernel copies of the master weights
//   k_sur_gate         count of pixels where prediction and cheap differ
//   k_sur_tile_gate    list of the full-radius tiles to rerun (tile-gated run)
#include <algorithm>

#include "fbs_internal.h"
#include "fbs_surrogate.h"

namespace fbs {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int kC = SUR_CH;  // padded channels
typedef float f4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (no NaN inputs here)
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
// two floats -> packed bfloat16 (a in the low half), round to nearest even:
// one v_cvt_pk_bf16_f32, the same bits as to_bf16 on each
__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v{a, b}), bf2));
}
// A operand of the 32 -> 1 layer for one tap: output row 0 holds the weights
// of the 32 input channels (BF16-exact floats), rows 1..15 are zero
__device__ __forceinline__ bf8 last_layer_a(const float* __restrict__ w3, int tap, int m, int kq)
{
    bf8 a;
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = (__bf16)(m == 0 ? w3[tap * kC + 8 * kq + i] : 0.0f);
    return a;
}


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
    // keys: the cost's bits with the low kbits (the width of D - 1) replaced
    // by the disparity index (costs are >= 0): ascending keys order by cost at
    // that resolution, then by disparity
    const int kbits = 32 - __builtin_clz((unsigned)max(D - 1, 1));
    const uint32_t kmask = (1u << kbits) - 1u;
    uint32_t key[SUR_TOPK];
#pragma unroll
    for (int i = 0; i < SUR_TOPK; ++i) key[i] = ~0u;
    for (int k = 0; k < D; ++k) {
        const uint32_t q = (__float_as_uint(a[(size_t)k * plane]) & ~kmask) | (uint32_t)k;
        if (q < key[SUR_TOPK - 1]) {
#pragma unroll
            for (int i = SUR_TOPK - 1; i >= 0; --i) {
                const bool shift = i > 0 && q < key[i > 0 ? i - 1 : 0];
                if (shift) key[i] = key[i - 1];
                else if (q < key[i]) key[i] = q;
            }
        }
    }
    uint32_t w[16];
    const float dn = (float)(D - 1);
#pragma unroll
    for (int i = 0; i < SUR_TOPK; i += 2) {
        w[i / 2] = (uint32_t)to_bf16(__uint_as_float(key[i] & ~kmask) / tau) |
                   ((uint32_t)to_bf16(__uint_as_float(key[i + 1] & ~kmask) / tau) << 16);
        w[4 + i / 2] = (uint32_t)to_bf16((float)(int)(key[i] & kmask) / dn) |
                       ((uint32_t)to_bf16((float)(int)(key[i + 1] & kmask) / dn) << 16);
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
        f4 acc2[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int t = 0; t < 9; ++t) {  // one B operand serves both output blocks
            const int ky = t / 3, kx = t - 3 * (t / 3);
            const bf8 b = *reinterpret_cast<const bf8*>(
                s_in + ((ty + ky) * (CT_W + 2) + (tx0 + m + kx)) * kC + 8 * kq);
            acc2[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[t][0], b, acc2[0], 0, 0, 0);
            acc2[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[t][1], b, acc2[1], 0, 0, 0);
        }
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const f4& acc = acc2[cb];
            if (x < W && y < H) {
                const int c0 = cb * 16 + 4 * kq;
                const size_t o = ((size_t)y * W + x) * kC + c0;
                uint2 v;
                if (MODE == SUR_FWD) {
                    v.x = pack_bf16(fmaxf(acc[0] + bias[c0], 0.0f), fmaxf(acc[1] + bias[c0 + 1], 0.0f));
                    v.y = pack_bf16(fmaxf(acc[2] + bias[c0 + 2], 0.0f), fmaxf(acc[3] + bias[c0 + 3], 0.0f));
                } else {
                    // keep the gradient where the forward activation is > 0
                    const uint2 mk = *reinterpret_cast<const uint2*>(mask_act + o);
                    const uint32_t mw[2] = {mk.x, mk.y};
                    uint32_t r[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t keep = (from_bf16((uint16_t)(mw[h] & 0xffff)) > 0.0f ? 0xffffu : 0u) |
                                              (from_bf16((uint16_t)(mw[h] >> 16)) > 0.0f ? 0xffff0000u : 0u);
                        r[h] = pack_bf16(acc[2 * h], acc[2 * h + 1]) & keep;
                    }
                    v = make_uint2(r[0], r[1]);
                }
                *reinterpret_cast<uint2*>(out + o) = v;
            }
        }
    }
}

// ------------------------------------------------ fused inference (whole net)
//
// One workgroup (4 waves) per NT x NT tile of predictions.  The tile's
// features plus a 4-pixel halo (the receptive radius of four 3x3 layers) are
// staged in one LDS buffer, and each layer overwrites it in place: a layer's
// output square is one pixel smaller per side (34 -> 32 -> 30 -> 28 -> 26)
// and output (r, c) only reads inputs (r..r+2, c..c+2), so every wave keeps
// its results in registers until all waves have read their inputs, then
// stores them at (r, c).  Activations of positions off the image are stored
// as 0: every layer sees the zero padding of a 'same' convolution.  At 75 KB
// of LDS two workgroups share a compute unit, one staging while the other
// computes.
//
// The buffer holds activations by channel octet: plane q keeps channels
// 8q..8q+7 of every pixel in 16 bytes, so the 16 pixels of an MFMA B operand
// are 256 contiguous bytes (no bank conflicts).  A wave item is 16 columns x
// 4 rows of a layer's output; each B operand (input row, column shift) it
// loads serves the (up to) three output rows that use it.  Every output is
// summed in the same order as in k_sur_conv / k_sur_last_fwd, so the
// predictions are bit-identical to the per-layer kernels'.
constexpr int NT = 26, NS0 = NT + 8;
constexpr int kNetThreads = 256, kNetWaves = kNetThreads / 64;
constexpr int kPlane = NS0 * NS0;  // pixels per channel-octet plane, pitch NS0

// The MFMA sums of one item: output rows r0..r0+3 (those below so), columns
// 16 seg .. 16 seg + 15 of a layer whose input square has side si.
template <int NCB>
__device__ __forceinline__ void net_item(const uint16_t* __restrict__ plane, const bf8 (&aw)[9][NCB],
                                         int si, int so, int r0, int c, f4 (&acc)[4][NCB])
{
#pragma unroll
    for (int qi = 0; qi < 6; ++qi) {
        const int q = r0 + qi;  // input row
        if (q >= si) break;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            // columns past the output are computed from clamped reads and dropped
            const int col = min(c + kx, si - 1);
            const bf8 b = *reinterpret_cast<const bf8*>(plane + (size_t)(q * NS0 + col) * 8);
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
                const int r = qi - ky;  // output row r0 + r takes input row q as tap row ky
                if (r >= 0 && r < 4 && r0 + r < so) {
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
                        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[3 * ky + kx][cb], b, acc[r][cb], 0, 0, 0);
                }
            }
        }
    }
}

// One 32 -> 32 layer, input side SI, in place.
template <int SI>
__device__ __forceinline__ void net_layer(uint16_t* __restrict__ buf, const uint16_t* __restrict__ A,
                                          const float* __restrict__ bias, int W, int H, int oy,
                                          int ox, int lane, int wave)
{
    constexpr int SO = SI - 2, NSEG = (SO + 15) / 16, NSTRIP = (SO + 3) / 4;
    constexpr int NITEM = NSEG * NSTRIP, PER = (NITEM + kNetWaves - 1) / kNetWaves;
    const int m = lane & 15, kq = lane >> 4;
    bf8 aw[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
            aw[t][cb] = *reinterpret_cast<const bf8*>(A + ((size_t)(t * kC + cb * 16 + m) * kC + 8 * kq));
    float bs[2][4];  // this lane's output channels 16cb + 4kq + j
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j) bs[cb][j] = bias[cb * 16 + 4 * kq + j];
    const uint16_t* plane = buf + (size_t)kq * kPlane * 8;
    uint2 res[PER][4][2];  // packed BF16 results, stored after the barrier
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int item = wave + kNetWaves * k;
        if (item < NITEM) {
            const int seg = item % NSEG, r0 = (item / NSEG) * 4;
            const int c = seg * 16 + m;
            f4 acc[4][2];
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r][0] = acc[r][1] = f4{0.f, 0.f, 0.f, 0.f};
            net_item<2>(plane, aw, SI, SO, r0, c, acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int y = oy + r0 + r, x = ox + c;
                const uint32_t keep = (x >= 0 && x < W && y >= 0 && y < H) ? 0xffffffffu : 0u;
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const f4& a = acc[r][cb];
                    res[k][r][cb] = make_uint2(
                        pack_bf16(fmaxf(a[0] + bs[cb][0], 0.0f), fmaxf(a[1] + bs[cb][1], 0.0f)) & keep,
                        pack_bf16(fmaxf(a[2] + bs[cb][2], 0.0f), fmaxf(a[3] + bs[cb][3], 0.0f)) & keep);
                }
            }
        }
    }
    __syncthreads();  // every wave has read this layer's input
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int item = wave + kNetWaves * k;
        if (item < NITEM) {
            const int seg = item % NSEG, r0 = (item / NSEG) * 4;
            const int c = seg * 16 + m;
            if (c < SO) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r0 + r < SO) {
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb) {
                            const int c0 = cb * 16 + 4 * kq;
                            *reinterpret_cast<uint2*>(buf + ((size_t)(c0 >> 3) * kPlane + (r0 + r) * NS0 + c) * 8 +
                                                      (c0 & 7)) = res[k][r][cb];
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kNetThreads) void k_sur_net_fwd(int W, int H, const uint16_t* __restrict__ feat,
                                                             const uint16_t* __restrict__ fwd,
                                                             const float* __restrict__ bias,
                                                             const float* __restrict__ w3,
                                                             const float* __restrict__ b3,
                                                             const float* __restrict__ cheap,
                                                             float* __restrict__ pred,
                                                             int* __restrict__ zero2)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* buf = reinterpret_cast<uint16_t*>(smem);
    float* s_w3 = reinterpret_cast<float*>(buf + (size_t)kPlane * kC);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (zero2 && blockIdx.x == 0 && blockIdx.y == 0 && tid < 2) zero2[tid] = 0;
    for (int i = tid; i < 9 * kC; i += kNetThreads) s_w3[i] = w3[i];
    const int X0 = blockIdx.x * NT - 4, Y0 = blockIdx.y * NT - 4;  // image position of the buffer's origin
    for (int i = tid; i < kPlane * 4; i += kNetThreads) {
        const int px = i >> 2, q = i & 3;
        const int ty = px / NS0, tx = px - ty * NS0;
        const int y = Y0 + ty, x = X0 + tx;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (x >= 0 && x < W && y >= 0 && y < H)
            v = reinterpret_cast<const uint4*>(feat + ((size_t)y * W + x) * kC)[q];
        reinterpret_cast<uint4*>(buf)[(size_t)q * kPlane + px] = v;
    }
    __syncthreads();
    constexpr int LW = 9 * kC * kC;
    net_layer<NS0>(buf, fwd, bias, W, H, Y0 + 1, X0 + 1, lane, wave);
    net_layer<NS0 - 2>(buf, fwd + LW, bias + kC, W, H, Y0 + 2, X0 + 2, lane, wave);
    net_layer<NS0 - 4>(buf, fwd + 2 * LW, bias + 2 * kC, W, H, Y0 + 3, X0 + 3, lane, wave);
    // 32 -> 1 layer and the residual: the same MFMA scheme with only output
    // row 0 weighted, started from the bias (the sums of k_sur_last_fwd, in
    // its order)
    constexpr int SI = NS0 - 6, SO = NT, NSEG = (SO + 15) / 16, NSTRIP = (SO + 3) / 4;
    const int m = lane & 15, kq = lane >> 4;
    bf8 aw[9][1];
#pragma unroll
    for (int t = 0; t < 9; ++t) aw[t][0] = last_layer_a(s_w3, t, m, kq);
    const float bias3 = *b3;
    const uint16_t* plane = buf + (size_t)kq * kPlane * 8;
#pragma unroll 1
    for (int item = wave; item < NSEG * NSTRIP; item += kNetWaves) {
        const int seg = item % NSEG, r0 = (item / NSEG) * 4;
        const int c = seg * 16 + m;
        f4 acc[4][1];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r][0] = f4{lane < 16 ? bias3 : 0.0f, 0.f, 0.f, 0.f};
        net_item<1>(plane, aw, SI, SO, r0, c, acc);
        if (lane < 16 && c < SO) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int y = Y0 + 4 + r0 + r, x = X0 + 4 + c;
                if (r0 + r < SO && x < W && y < H) {
                    const size_t o = (size_t)y * W + x;
                    pred[o] = cheap[o] + acc[r][0][0];
                }
            }
        }
    }
}

// ------------------------------------------------------------- last layer

// resid[p] = b3 + sum_{tap, c} W3[tap][c] a3[p + off][c]; pred = cheap + resid;
// with a label: g4 = bf16(sign(pred - label) / N) and per-tile |pred - label|
// sums.  Tiles and MFMA scheme of k_sur_conv with one weighted output row,
// the accumulator started from the bias.
__global__ __launch_bounds__(256) void k_sur_last_fwd(int W, int H, const uint16_t* __restrict__ a3,
                                                      const float* __restrict__ w3,
                                                      const float* __restrict__ b3,
                                                      const float* __restrict__ cheap,
                                                      float* __restrict__ pred,
                                                      const float* __restrict__ label,
                                                      float* __restrict__ g4,
                                                      float* __restrict__ loss_part)
{
    __shared__ __align__(16) uint16_t s_in[(CT_H + 2) * (CT_W + 2) * kC];
    __shared__ float s_red[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int X0 = blockIdx.x * CT_W, Y0 = blockIdx.y * CT_H;
    constexpr int kChunks = (CT_H + 2) * (CT_W + 2) * (kC / 8);
    for (int i = tid; i < kChunks; i += 256) {
        const int px = i / (kC / 8), c8 = i - px * (kC / 8);
        const int ty = px / (CT_W + 2), tx = px - ty * (CT_W + 2);
        const int y = Y0 - 1 + ty, x = X0 - 1 + tx;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (x >= 0 && x < W && y >= 0 && y < H)
            v = reinterpret_cast<const uint4*>(a3 + ((size_t)y * W + x) * kC)[c8];
        reinterpret_cast<uint4*>(s_in)[i] = v;
    }
    const int m = lane & 15, kq = lane >> 4;
    bf8 aw[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) aw[t] = last_layer_a(w3, t, m, kq);
    const float bias3 = *b3;
    __syncthreads();
    float err = 0.0f;
#pragma unroll 1
    for (int gi = 0; gi < 4; ++gi) {
        const int grp = wave * 4 + gi;
        const int ty = grp >> 1, tx0 = (grp & 1) * 16;
        const int y = Y0 + ty, x = X0 + tx0 + m;
        f4 acc = {lane < 16 ? bias3 : 0.0f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ky = t / 3, kx = t - 3 * (t / 3);
            const bf8 b = *reinterpret_cast<const bf8*>(
                s_in + ((ty + ky) * (CT_W + 2) + (tx0 + m + kx)) * kC + 8 * kq);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[t], b, acc, 0, 0, 0);
        }
        if (lane < 16 && x < W && y < H) {
            const size_t o = (size_t)y * W + x;
            const float pv = cheap[o] + acc[0];
            pred[o] = pv;
            if (label) {
                const float d = pv - label[o];
                err += fabsf(d);
                const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
                g4[o] = from_bf16(to_bf16(sg / (float)((size_t)W * H)));
            }
        }
    }
    if (label) {
        // fixed-order sum: lanes of a wave, then the four waves
        for (int off = 32; off > 0; off >>= 1) err += __shfl_xor(err, off);
        if (lane == 0) s_red[wave] = err;
        __syncthreads();
        if (tid == 0) loss_part[blockIdx.y * gridDim.x + blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
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

// grid-stride count; one atomic per workgroup
__global__ __launch_bounds__(256) void k_sur_gate(int n, const float* __restrict__ pred,
                                                  const float* __restrict__ cheap, float gate_px,
                                                  int* __restrict__ count)
{
    __shared__ int s_c[4];
    int c = 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        c += fabsf(pred[i] - cheap[i]) > gate_px ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = s_c[0] + s_c[1] + s_c[2] + s_c[3];
        if (t) atomicAdd(count, t);
    }
}

// Sixteen lanes per fallback tile (tw x 8 pixels of the full-radius run), 16
// tiles per workgroup: a tile is listed when more than tile_frac of its
// pixels in the image have |pred - cheap| > gate_px.  One atomic per
// workgroup reserves the list slots.  Block 0 also publishes the full-radius
// job for the fallback kernel.  n_items and the fallback's queue counter
// start at 0 (cleared by k_sur_net_fwd).
__global__ __launch_bounds__(256) void k_sur_tile_gate(int W, int H, const float* __restrict__ pred,
                                                       const float* __restrict__ cheap, float gate_px,
                                                       float tile_frac, int tw, int tiles_x,
                                                       int n_tiles, int2* __restrict__ items,
                                                       int* __restrict__ n_items, SurFallbackJob job,
                                                       SurFallbackJob* __restrict__ job_out)
{
    __shared__ int s_n, s_base;
    if (blockIdx.x == 0 && threadIdx.x == 0) *job_out = job;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const int t = blockIdx.x * 16 + (threadIdx.x >> 4), sub = threadIdx.x & 15;
    int cnt = 0, npx = 0;
    if (t < n_tiles) {
        const int tx = t % tiles_x, ty = t / tiles_x;
        for (int i = sub; i < tw * 8; i += 16) {
            const int x = tx * tw + i % tw, y = ty * 8 + i / tw;
            if (x < W && y < H) {
                const size_t o = (size_t)y * W + x;
                ++npx;
                cnt += fabsf(pred[o] - cheap[o]) > gate_px ? 1 : 0;
            }
        }
    }
    for (int off = 8; off > 0; off >>= 1) {  // within the 16 lanes of the tile
        cnt += __shfl_xor(cnt, off);
        npx += __shfl_xor(npx, off);
    }
    const bool listed = t < n_tiles && sub == 0 && (float)cnt > tile_frac * (float)npx;
    const int slot = listed ? atomicAdd(&s_n, 1) : 0;
    __syncthreads();
    if (threadIdx.x == 0) s_base = s_n ? atomicAdd(n_items, s_n) : 0;
    __syncthreads();
    if (listed) items[s_base + slot] = make_int2(0, t);
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
    dim3 grid((W + CT_W - 1) / CT_W, (H + CT_H - 1) / CT_H);
    hipLaunchKernelGGL(k_sur_last_fwd, grid, dim3(256), 0, s, W, H, a3, w3, b3, cheap, pred,
                       label, g4, loss_part);
    return hipGetLastError();
}

int sur_loss_parts(int W, int H) { return ((W + CT_W - 1) / CT_W) * ((H + CT_H - 1) / CT_H); }

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
    hipLaunchKernelGGL(k_sur_gate, dim3(std::max(1, std::min((n + 255) / 256, 512))), dim3(256), 0, s,
                       n, pred, cheap, gate_px, count);
    return hipGetLastError();
}

size_t sur_net_lds_bytes() { return (size_t)kPlane * kC * sizeof(uint16_t) + 9 * kC * sizeof(float); }

hipError_t sur_net_fwd(int W, int H, const uint16_t* feat, const uint16_t* fwd, const float* bias,
                       const float* w3, const float* b3, const float* cheap, float* pred,
                       int* zero2, hipStream_t s)
{
    dim3 grid((W + NT - 1) / NT, (H + NT - 1) / NT);
    hipLaunchKernelGGL(k_sur_net_fwd, grid, dim3(kNetThreads), sur_net_lds_bytes(), s, W, H, feat,
                       fwd, bias, w3, b3, cheap, pred, zero2);
    return hipGetLastError();
}

hipError_t sur_tile_gate(int W, int H, const float* pred, const float* cheap, float gate_px,
                         float tile_frac, int tw, int2* items, int* n_items,
                         const SurFallbackJob& job, SurFallbackJob* job_out, hipStream_t s)
{
    const int tiles_x = (W + tw - 1) / tw, n_tiles = tiles_x * ((H + 7) / 8);
    hipLaunchKernelGGL(k_sur_tile_gate, dim3((n_tiles + 15) / 16), dim3(256), 0, s, W, H, pred, cheap,
                       gate_px, tile_frac, tw, tiles_x, n_tiles, items, n_items, job, job_out);
    return hipGetLastError();
}

}  // namespace fbs
