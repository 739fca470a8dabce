// fbs_surrogate.hip - C ABI of the learned surrogate (see include/fbs.h).
//
// The object owns the float32 master weights, Adam state, BF16 kernel copies
// and the activation / gradient buffers for frames up to max_width x
// max_height (and, for fbs_surrogate_run, the cheap run's aggregated volume
// up to max_disp disparities).  Everything is allocated at creation; the
// per-frame entry points allocate nothing.
#include <math.h>
#include <string.h>

#include <vector>

#include "fbs_internal.h"
#include "fbs_surrogate.h"

namespace fbs {
fbs_status api_check_params(const fbs_params* p);
Geom api_geom(const fbs_params* p);
Tables api_tables(const fbs_params* p);
fbs_status api_fail(fbs_status st, const char* fmt, ...);

namespace {
__global__ void k_sum_ordered(const float* __restrict__ parts, int n, float scale,
                              float* __restrict__ out)
{
    __shared__ float s[256];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) acc += parts[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0] * scale;
}
}  // namespace
}  // namespace fbs

struct fbs_surrogate {
    int max_w = 0, max_h = 0, max_d = 0;
    long long t = 0;  // Adam steps taken
    float *master = nullptr, *m = nullptr, *v = nullptr, *grads = nullptr;
    uint16_t *fwd = nullptr, *bwd = nullptr;
    float *w3 = nullptr, *bias = nullptr;
    uint16_t *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *g2 = nullptr, *g1 = nullptr,
             *g0 = nullptr, *feat = nullptr;
    float *g4 = nullptr, *loss_parts = nullptr, *part = nullptr;
    float *red0 = nullptr, *red1 = nullptr, *red2 = nullptr, *red3 = nullptr;
    float *vol = nullptr, *cheap = nullptr;
    int* count = nullptr;
    int* h_count = nullptr;  // pinned
    // tile-gated runs: listed fallback tiles, {list length, queue counter},
    // the full-radius job as the fallback kernel reads it
    int2* items = nullptr;
    int* qctr = nullptr;
    fbs::SurFallbackJob* job = nullptr;
    int max_tiles = 0;
    int cus = 0;
};

namespace {

using fbs::api_fail;

template <typename T>
bool dalloc(T** p, size_t n)
{
    return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (n ? n : 1)) == hipSuccess;
}

void sur_free(fbs_surrogate* s)
{
    if (!s) return;
    void* ptrs[] = {s->master, s->m, s->v, s->grads, s->fwd, s->bwd, s->w3, s->bias, s->a1,
                    s->a2, s->a3, s->g2, s->g1, s->g0, s->feat, s->g4, s->loss_parts, s->part,
                    s->red0, s->red1, s->red2, s->red3, s->vol, s->cheap, s->count,
                    s->items, s->qctr, s->job};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (s->h_count) (void)hipHostFree(s->h_count);
    delete s;
}

fbs_status check_frame(const fbs_surrogate* s, int w, int h)
{
    if (!s) return api_fail(FBS_E_INVALID, "surrogate is NULL");
    if (w < 1 || h < 1 || w > s->max_w || h > s->max_h)
        return api_fail(FBS_E_INVALID, "frame %dx%d outside 1..%dx%d", w, h, s->max_w, s->max_h);
    return FBS_OK;
}

fbs_status hipst(hipError_t e, const char* what)
{
    if (e == hipSuccess) return FBS_OK;
    return api_fail(FBS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Forward of the three 32 -> 32 layers and the last layer.  Inference
// (no label) is one fused kernel; with a label the layers run one by one,
// keeping the activations for the backward pass, and the last layer also
// forms the L1 gradient.  Both give the same bits.
fbs_status forward(fbs_surrogate* s, int W, int H, const uint16_t* feat, const float* cheap,
                   float* pred, const float* label, hipStream_t st, int* zero2 = nullptr)
{
    using namespace fbs;
    constexpr int LW = 9 * SUR_CH * SUR_CH;
    if (!label)
        return hipst(sur_net_fwd(W, H, feat, s->fwd, s->bias, s->w3, s->master + SUR_OFF_B3, cheap,
                                 pred, zero2, st),
                     "surrogate forward");
    hipError_t e = sur_conv(SUR_FWD, W, H, feat, s->fwd, s->bias, nullptr, s->a1, st);
    if (e == hipSuccess) e = sur_conv(SUR_FWD, W, H, s->a1, s->fwd + LW, s->bias + SUR_CH, nullptr, s->a2, st);
    if (e == hipSuccess) e = sur_conv(SUR_FWD, W, H, s->a2, s->fwd + 2 * LW, s->bias + 2 * SUR_CH, nullptr, s->a3, st);
    if (e == hipSuccess)
        e = sur_last_fwd(W, H, s->a3, s->w3, s->master + SUR_OFF_B3, cheap, pred, label, s->g4,
                         s->loss_parts, st);
    return hipst(e, "surrogate forward");
}

}  // namespace

extern "C" {

int32_t fbs_surrogate_num_params(void) { return SUR_NPARAM; }

fbs_status fbs_surrogate_create(fbs_surrogate** out, int32_t max_width, int32_t max_height,
                                int32_t max_disp)
{
    if (!out) return api_fail(FBS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (max_width < 1 || max_height < 1 || max_width > 65535 || max_height > 65535)
        return api_fail(FBS_E_INVALID, "bad maximum frame size");
    if (max_disp < SUR_TOPK || max_disp > FBS_MAX_DISP)
        return api_fail(FBS_E_INVALID, "max_disp must be in %d..%d", SUR_TOPK, FBS_MAX_DISP);
    fbs_surrogate* s = new fbs_surrogate();
    s->max_w = max_width;
    s->max_h = max_height;
    s->max_d = max_disp;
    const size_t N = (size_t)max_width * max_height;
    const size_t tiles = (size_t)fbs::sur_wgrad_tiles(max_width, max_height);
    const size_t parts = (size_t)fbs::sur_loss_parts(max_width, max_height);
    constexpr int LW = 9 * SUR_CH * SUR_CH;
    bool ok = dalloc(&s->master, SUR_NPARAM) && dalloc(&s->m, SUR_NPARAM) &&
              dalloc(&s->v, SUR_NPARAM) && dalloc(&s->grads, SUR_NPARAM) &&
              dalloc(&s->fwd, 3 * LW) && dalloc(&s->bwd, 2 * LW) && dalloc(&s->w3, 9 * SUR_CH) &&
              dalloc(&s->bias, 3 * SUR_CH) && dalloc(&s->a1, N * SUR_CH) &&
              dalloc(&s->a2, N * SUR_CH) && dalloc(&s->a3, N * SUR_CH) &&
              dalloc(&s->g2, N * SUR_CH) && dalloc(&s->g1, N * SUR_CH) &&
              dalloc(&s->g0, N * SUR_CH) && dalloc(&s->feat, N * SUR_CH) && dalloc(&s->g4, N) &&
              dalloc(&s->loss_parts, parts) && dalloc(&s->part, tiles * SUR_PART) &&
              dalloc(&s->red0, SUR_PART) && dalloc(&s->red1, SUR_PART) &&
              dalloc(&s->red2, SUR_PART) && dalloc(&s->red3, 9 * SUR_CH + 1) &&
              dalloc(&s->vol, N * max_disp) && dalloc(&s->cheap, N) && dalloc(&s->count, 1) &&
              hipHostMalloc(&s->h_count, sizeof(int), hipHostMallocDefault) == hipSuccess;
    // fallback tiles are at least 8 x 8 pixels
    s->max_tiles = ((max_width + 7) / 8) * ((max_height + 7) / 8);
    ok = ok && dalloc(&s->items, s->max_tiles) && dalloc(&s->qctr, 2) && dalloc(&s->job, 1);
    int dev = 0;
    if (ok && hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (s->cus <= 0) s->cus = 256;
    if (!ok) {
        sur_free(s);
        return api_fail(FBS_E_HIP, "surrogate: device allocation failed");
    }
    std::vector<float> zero(SUR_NPARAM, 0.0f);
    if (hipMemcpy(s->master, zero.data(), sizeof(float) * SUR_NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->m, zero.data(), sizeof(float) * SUR_NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->v, zero.data(), sizeof(float) * SUR_NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        fbs::sur_pack(s->master, s->fwd, s->bwd, s->w3, s->bias, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        sur_free(s);
        return api_fail(FBS_E_HIP, "surrogate: initialisation failed");
    }
    *out = s;
    return FBS_OK;
}

void fbs_surrogate_destroy(fbs_surrogate* s)
{
    if (!s) return;
    (void)hipDeviceSynchronize();
    sur_free(s);
}

fbs_status fbs_surrogate_set_params(fbs_surrogate* s, const float* host_params)
{
    if (!s || !host_params) return api_fail(FBS_E_INVALID, "surrogate and params are required");
    std::vector<float> zero(SUR_NPARAM, 0.0f);
    if (hipMemcpy(s->master, host_params, sizeof(float) * SUR_NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->m, zero.data(), sizeof(float) * SUR_NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->v, zero.data(), sizeof(float) * SUR_NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        fbs::sur_pack(s->master, s->fwd, s->bwd, s->w3, s->bias, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        return api_fail(FBS_E_HIP, "surrogate: parameter upload failed");
    s->t = 0;
    return FBS_OK;
}

fbs_status fbs_surrogate_get_params(fbs_surrogate* s, float* host_params)
{
    if (!s || !host_params) return api_fail(FBS_E_INVALID, "surrogate and params are required");
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(host_params, s->master, sizeof(float) * SUR_NPARAM, hipMemcpyDeviceToHost) != hipSuccess)
        return api_fail(FBS_E_HIP, "surrogate: parameter download failed");
    return FBS_OK;
}

fbs_status fbs_surrogate_features(fbs_surrogate* s, const fbs_params* cheap, const uint8_t* left,
                                  const float* agg, uint16_t* feat, void* stream)
{
    fbs_status st = fbs::api_check_params(cheap);
    if (st != FBS_OK) return st;
    st = check_frame(s, cheap->width, cheap->height);
    if (st != FBS_OK) return st;
    const int D = cheap->d_max - cheap->d_min + 1;
    if (cheap->channels != 1 || cheap->cost_type != FBS_COST_TAD || D < SUR_TOPK)
        return api_fail(FBS_E_UNSUPPORTED, "features need a gray TAD run with >= %d disparities", SUR_TOPK);
    if (!left || !agg || !feat) return api_fail(FBS_E_INVALID, "left, agg and feat are required");
    if (((uintptr_t)feat & 15u) || ((uintptr_t)agg & 3u))
        return api_fail(FBS_E_INVALID, "feat must be 16-byte and agg 4-byte aligned");
    (void)hipGetLastError();
    return hipst(fbs::sur_features(cheap->width, cheap->height, D, cheap->cost_cap, agg, left,
                                   cheap->row_stride, feat, (hipStream_t)stream),
                 "surrogate features");
}

fbs_status fbs_surrogate_cheap_run(fbs_surrogate* s, const fbs_params* cheap, const uint8_t* left,
                                   const uint8_t* right, float* cheap_sub, uint16_t* feat,
                                   void* stream)
{
    fbs_status st = fbs::api_check_params(cheap);
    if (st != FBS_OK) return st;
    st = check_frame(s, cheap->width, cheap->height);
    if (st != FBS_OK) return st;
    const int D = cheap->d_max - cheap->d_min + 1;
    if (cheap->channels != 1 || cheap->cost_type != FBS_COST_TAD || D < SUR_TOPK)
        return api_fail(FBS_E_UNSUPPORTED, "features need a gray TAD run with >= %d disparities", SUR_TOPK);
    if (!left || !right || !cheap_sub || !feat)
        return api_fail(FBS_E_INVALID, "left, right, cheap_sub and feat are required");
    if (((uintptr_t)feat & 15u) || ((uintptr_t)cheap_sub & 3u))
        return api_fail(FBS_E_INVALID, "feat must be 16-byte and cheap_sub 4-byte aligned");
    const fbs::Geom g = fbs::api_geom(cheap);
    if (!(cheap->flags & FBS_F_FORCE_VALU) && fbs::mfma_supported(g)) {
        (void)hipGetLastError();
        return hipst(fbs::launch_mfma_features(g, fbs::api_tables(cheap), left, right, cheap_sub,
                                               feat, (hipStream_t)stream),
                     "surrogate cheap run");
    }
    if (D > s->max_d) return api_fail(FBS_E_INVALID, "%d disparities above the maximum %d", D, s->max_d);
    st = fbs_run(cheap, left, right, nullptr, cheap_sub, s->vol, nullptr, stream);
    if (st == FBS_OK) st = fbs_surrogate_features(s, cheap, left, s->vol, feat, stream);
    return st;
}

fbs_status fbs_surrogate_forward(fbs_surrogate* s, int32_t width, int32_t height,
                                 const uint16_t* feat, const float* cheap_sub, float* pred,
                                 void* stream)
{
    fbs_status st = check_frame(s, width, height);
    if (st != FBS_OK) return st;
    if (!feat || !cheap_sub || !pred) return api_fail(FBS_E_INVALID, "feat, cheap_sub, pred required");
    if ((uintptr_t)feat & 15u) return api_fail(FBS_E_INVALID, "feat must be 16-byte aligned");
    (void)hipGetLastError();
    return forward(s, width, height, feat, cheap_sub, pred, nullptr, (hipStream_t)stream);
}

fbs_status fbs_surrogate_gradients(fbs_surrogate* s, int32_t width, int32_t height,
                                   const uint16_t* feat, const float* cheap_sub,
                                   const float* label, float* pred, float* grads, float* loss,
                                   void* stream)
{
    using namespace fbs;
    fbs_status st = check_frame(s, width, height);
    if (st != FBS_OK) return st;
    if (!feat || !cheap_sub || !label || !pred || !grads)
        return api_fail(FBS_E_INVALID, "feat, cheap_sub, label, pred and grads are required");
    if ((uintptr_t)feat & 15u) return api_fail(FBS_E_INVALID, "feat must be 16-byte aligned");
    hipStream_t q = (hipStream_t)stream;
    const int W = width, H = height;
    constexpr int LW = 9 * SUR_CH * SUR_CH;
    (void)hipGetLastError();
    st = forward(s, W, H, feat, cheap_sub, pred, label, q);
    if (st != FBS_OK) return st;
    hipError_t e = hipSuccess;
    if (loss) {
        hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, q, s->loss_parts,
                           sur_loss_parts(W, H), 1.0f / (float)((size_t)W * H), loss);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = sur_wgrad_last(W, H, s->g4, s->a3, s->part, s->red3, q);
    if (e == hipSuccess) e = sur_last_bwd(W, H, s->g4, s->w3, s->a3, s->g2, q);
    if (e == hipSuccess) e = sur_wgrad(W, H, s->g2, s->a2, s->part, s->red2, q);
    if (e == hipSuccess) e = sur_conv(SUR_BWD, W, H, s->g2, s->bwd + LW, nullptr, s->a2, s->g1, q);
    if (e == hipSuccess) e = sur_wgrad(W, H, s->g1, s->a1, s->part, s->red1, q);
    if (e == hipSuccess) e = sur_conv(SUR_BWD, W, H, s->g1, s->bwd, nullptr, s->a1, s->g0, q);
    if (e == hipSuccess) e = sur_wgrad(W, H, s->g0, feat, s->part, s->red0, q);
    if (e == hipSuccess) e = sur_unpack_grads(s->red0, s->red1, s->red2, s->red3, grads, q);
    return hipst(e, "surrogate backward");
}

fbs_status fbs_surrogate_adam(fbs_surrogate* s, const float* grads, float lr, void* stream)
{
    if (!s || !grads) return api_fail(FBS_E_INVALID, "surrogate and grads are required");
    if (!(lr > 0.0f)) return api_fail(FBS_E_INVALID, "lr must be > 0");
    const double b1 = 0.9, b2 = 0.999;
    const long long t = s->t + 1;
    const float bc1 = (float)(1.0 - pow(b1, (double)t)), bc2 = (float)(1.0 - pow(b2, (double)t));
    hipStream_t q = (hipStream_t)stream;
    (void)hipGetLastError();
    hipError_t e = fbs::sur_adam(s->master, s->m, s->v, grads, lr, (float)b1, (float)b2, bc1, bc2,
                                 1e-8f, q);
    if (e == hipSuccess) e = fbs::sur_pack(s->master, s->fwd, s->bwd, s->w3, s->bias, q);
    if (e == hipSuccess) s->t = t;
    return hipst(e, "surrogate adam");
}

}  // extern "C"

namespace {
// arguments shared by the gated runs
fbs_status check_pair(fbs_surrogate* s, const fbs_params* cheap, const fbs_params* full,
                      const uint8_t* left, const uint8_t* right, float* disp_sub)
{
    fbs_status st = fbs::api_check_params(cheap);
    if (st == FBS_OK) st = fbs::api_check_params(full);
    if (st != FBS_OK) return st;
    st = check_frame(s, cheap->width, cheap->height);
    if (st != FBS_OK) return st;
    const int W = cheap->width, H = cheap->height, D = cheap->d_max - cheap->d_min + 1;
    if (full->width != W || full->height != H || full->row_stride != cheap->row_stride ||
        full->channels != cheap->channels || full->d_min != cheap->d_min || full->d_max != cheap->d_max)
        return api_fail(FBS_E_INVALID, "cheap and full runs must describe the same pair");
    if (D > s->max_d) return api_fail(FBS_E_INVALID, "%d disparities above the maximum %d", D, s->max_d);
    if (!left || !right || !disp_sub) return api_fail(FBS_E_INVALID, "left, right, disp_sub required");
    if ((uintptr_t)disp_sub & 3u) return api_fail(FBS_E_INVALID, "disp_sub must be 4-byte aligned");
    return FBS_OK;
}
}  // namespace

extern "C" {

fbs_status fbs_surrogate_run(fbs_surrogate* s, const fbs_params* cheap, const fbs_params* full,
                             const uint8_t* left, const uint8_t* right, float* disp_sub,
                             float gate_px, float gate_frac, int32_t* fell_back, void* stream)
{
    fbs_status st = check_pair(s, cheap, full, left, right, disp_sub);
    if (st != FBS_OK) return st;
    const int W = cheap->width, H = cheap->height;
    if (!(gate_px >= 0.0f) || !(gate_frac >= 0.0f)) return api_fail(FBS_E_INVALID, "bad gate");
    hipStream_t q = (hipStream_t)stream;
    st = fbs_surrogate_cheap_run(s, cheap, left, right, s->cheap, s->feat, stream);
    if (st != FBS_OK) return st;
    (void)hipGetLastError();
    st = forward(s, W, H, s->feat, s->cheap, disp_sub, nullptr, q);
    if (st != FBS_OK) return st;
    const int n = W * H;
    hipError_t e = fbs::sur_gate(n, disp_sub, s->cheap, gate_px, s->count, q);
    if (e == hipSuccess) e = hipMemcpyAsync(s->h_count, s->count, sizeof(int), hipMemcpyDeviceToHost, q);
    if (e == hipSuccess) e = hipStreamSynchronize(q);
    if (e != hipSuccess) return hipst(e, "surrogate gate");
    const bool fb = (double)*s->h_count > (double)gate_frac * (double)n;
    if (fell_back) *fell_back = fb ? 1 : 0;
    if (fb) return fbs_run(full, left, right, nullptr, disp_sub, nullptr, nullptr, stream);
    return FBS_OK;
}

fbs_status fbs_surrogate_run_tiled(fbs_surrogate* s, const fbs_params* cheap,
                                   const fbs_params* full, const uint8_t* left,
                                   const uint8_t* right, float* disp_sub, float gate_px,
                                   float tile_frac, void* stream)
{
    using namespace fbs;
    fbs_status st = check_pair(s, cheap, full, left, right, disp_sub);
    if (st != FBS_OK) return st;
    if (!(gate_px >= 0.0f) || tile_frac != tile_frac) return api_fail(FBS_E_INVALID, "bad gate");
    const Geom gf = api_geom(full);
    if ((full->flags & FBS_F_FORCE_VALU) || full->cost_type != FBS_COST_TAD || !mfma_supported(gf))
        return api_fail(FBS_E_UNSUPPORTED, "tile-gated runs need the matrix-core kernel for the full run");
    const int W = cheap->width, H = cheap->height;
    hipStream_t q = (hipStream_t)stream;
    st = fbs_surrogate_cheap_run(s, cheap, left, right, s->cheap, s->feat, stream);
    if (st != FBS_OK) return st;
    (void)hipGetLastError();
    // the net also clears the tile list and the fallback queue
    st = forward(s, W, H, s->feat, s->cheap, disp_sub, nullptr, q, s->qctr);
    if (st != FBS_OK) return st;
    const MfmaCfg cfg = mfma_default_cfg(gf);
    const int tw = 2 * cfg.nw, tiles_x = (W + tw - 1) / tw;
    if (tiles_x * ((H + 7) / 8) > s->max_tiles) return api_fail(FBS_E_INVALID, "too many tiles");
    SurFallbackJob job{};
    job.pair.g = gf;
    job.pair.scap = mfma_scaled_cap(gf);
    job.pair.nb = cfg.nb;
    job.pair.tiles_x = tiles_x;
    job.L = left;
    job.R = right;
    job.disp = nullptr;
    job.sub = disp_sub;
    hipError_t e = sur_tile_gate(W, H, disp_sub, s->cheap, gate_px, tile_frac, tw, s->items,
                                 s->qctr, job, s->job, q);
    if (e != hipSuccess) return hipst(e, "surrogate tile gate");
    BatchClass bc{};
    bc.r = gf.r;
    bc.ch = gf.C;
    bc.nw = cfg.nw;
    bc.co = mfma_use_co(gf.D, cfg.nb) ? 1 : 0;
    bc.lds = mfma_lds_bytes(gf, cfg.nb, cfg.nw);
    bc.tb = api_tables(full);
    // one workgroup per listed tile (the grid covers every tile; those past
    // the list's end leave at once)
    bc.grid = 0;
    bc.one_wg_per_item = 1;
    bc.tiles_per_item = 1;
    bc.pairs = &s->job->pair;
    bc.items = s->items;
    bc.n_items = tiles_x * ((H + 7) / 8);
    bc.n_dev = s->qctr;
    bc.counter = s->qctr + 1;
    bc.L = &s->job->L;
    bc.R = &s->job->R;
    bc.disp = &s->job->disp;
    bc.sub = &s->job->sub;
    return hipst(launch_mfma_batch(bc, q), "surrogate tile fallback");
}

}  // extern "C"
