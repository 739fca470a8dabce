// fbs_plan.hip - many stereo pairs of uneven sizes in one graph launch.
//
// fbs_plan_create validates every pair, picks each pair's matrix-core
// configuration (waves per workgroup, disparity-slab depth) - from a JSON
// tuning cache, by timing the candidates on synthetic data of that shape, or
// by the built-in heuristic - and groups pairs into classes of equal
// (radius, channels, waves).  Each class becomes one persistent kernel whose
// workgroups pop (pair, tile) items from an atomic queue, most expensive
// items first.  The launch sequence (a counter-reset kernel, then one
// persistent kernel per class) is captured once into a hipGraph; pairs the
// matrix-core kernel cannot take run through the vector-ALU kernel after it.
//
// The per-pixel arithmetic of a batched pair is the one fbs_run uses (the
// group shape, and so the accumulation order, depends on the radius only),
// so batched outputs equal fbs_run's bit for bit.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "fbs_internal.h"

namespace fbs {
fbs_status api_check_params(const fbs_params* p);
Geom api_geom(const fbs_params* p);
Tables api_tables(const fbs_params* p);
fbs_status api_fail(fbs_status st, const char* fmt, ...);
}  // namespace fbs

struct fbs_plan {
    int n = 0;
    int device = 0;
    std::vector<fbs_params> params;
    std::vector<int> mfma;            // 1: batched on the matrix cores, 0: vector-ALU launch
    std::vector<fbs::MfmaCfg> cfg;
    std::vector<fbs::BatchClass> classes;
    fbs::BatchPair* d_pairs = nullptr;
    int2* d_items = nullptr;
    int* d_counters = nullptr;
    void** d_ptrs = nullptr;          // [4][n]: left, right, disp, disp_sub
    void** h_ptrs = nullptr;          // pinned mirror of d_ptrs
    hipEvent_t copied = nullptr;      // the last pointer upload has been consumed
    hipEvent_t done = nullptr;        // the last launch has finished
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
constexpr int kTilesPerItem = 4;

__global__ void k_zero(int* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

std::string shape_key(const fbs::Geom& g)
{
    char b[96];
    snprintf(b, sizeof b, "%d,%d,%d,%d,%d", g.W, g.H, g.C, g.D, g.r);
    return b;
}

// ---- tuning cache: {"arch": "gfx950", "entries": {"W,H,C,D,r": [nw, nb, us, "path"], ...}}
// where path names the loop order the depth implies: "chunk-outer" (one slab
// holds every disparity block) or "slab"; a reader needs only the first three
struct TuneEntry {
    int nw, nb;
    double us;
};

std::map<std::string, TuneEntry> read_cache(const char* path)
{
    std::map<std::string, TuneEntry> m;
    if (!path) return m;
    FILE* f = fopen(path, "rb");
    if (!f) return m;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
    fclose(f);
    size_t pos = s.find("\"entries\"");
    if (pos != std::string::npos) pos += 9;  // past the token, at the ':'
    while (pos != std::string::npos) {
        size_t q0 = s.find('"', pos);
        if (q0 == std::string::npos) break;
        size_t q1 = s.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
        size_t lb = s.find('[', q1);
        if (lb == std::string::npos) break;
        TuneEntry e{};
        if (sscanf(s.c_str() + lb, "[%d , %d , %lf", &e.nw, &e.nb, &e.us) == 3 ||
            sscanf(s.c_str() + lb, "[%d,%d,%lf", &e.nw, &e.nb, &e.us) == 3)
            m[key] = e;
        pos = s.find(']', lb);
    }
    return m;
}

void write_cache(const char* path, const std::map<std::string, TuneEntry>& m)
{
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return;
    fprintf(f, "{\"arch\": \"gfx950\", \"entries\": {");
    bool first = true;
    for (const auto& kv : m) {
        int D = 0;
        (void)sscanf(kv.first.c_str(), "%*d,%*d,%*d,%d", &D);
        const bool co = fbs::mfma_use_co(D, kv.second.nb);
        fprintf(f, "%s\n  \"%s\": [%d, %d, %.3f, \"%s\"]", first ? "" : ",", kv.first.c_str(),
                kv.second.nw, kv.second.nb, kv.second.us, co ? "chunk-outer" : "slab");
        first = false;
    }
    fprintf(f, "\n}}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}

// Times every (waves, slab depth) candidate of one shape on synthetic data.
fbs_status tune_shape(const fbs_params& p, TuneEntry* out)
{
    const fbs::Geom g = fbs::api_geom(&p);
    const fbs::Tables t = fbs::api_tables(&p);
    const size_t img = (size_t)(g.H - 1) * g.stride + (size_t)g.W * g.C;
    std::vector<uint8_t> host(img);
    uint32_t x = 12345u;
    for (auto& v : host) {
        x = x * 1664525u + 1013904223u;
        v = (uint8_t)(x >> 24);
    }
    uint8_t *L = nullptr, *R = nullptr;
    int32_t* disp = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    fbs_status st = FBS_OK;
    if (hipMalloc(&L, img) != hipSuccess || hipMalloc(&R, img) != hipSuccess ||
        hipMalloc(&disp, (size_t)g.W * g.H * 4) != hipSuccess || hipStreamCreate(&s) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = fbs::api_fail(FBS_E_HIP, "tuning: allocation failed");
    }
    if (st == FBS_OK) {
        (void)hipMemcpy(L, host.data(), img, hipMemcpyHostToDevice);
        (void)hipMemcpy(R, host.data(), img, hipMemcpyHostToDevice);
        out->us = 1e30;
        for (int nw : {4, 8, 12}) {
            const int nbmax = fbs::mfma_max_nb(g, nw);
            for (int nb = 1; nb <= nbmax; ++nb) {
                const fbs::MfmaCfg c{nw, nb};
                float best = 1e30f;
                bool ok = true;
                for (int rep = 0; rep < 7 && ok; ++rep) {
                    (void)hipEventRecord(e0, s);
                    ok = fbs::launch_mfma_cfg(g, t, c, L, R, disp, nullptr, nullptr, s) == hipSuccess;
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (rep >= 2) best = std::min(best, ms);   // first two are warm-up
                }
                if (ok && best * 1e3 < out->us) *out = TuneEntry{nw, nb, best * 1e3};
            }
        }
        if (out->us >= 1e29) st = fbs::api_fail(FBS_E_HIP, "tuning: no candidate ran");
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (L) (void)hipFree(L);
    if (R) (void)hipFree(R);
    if (disp) (void)hipFree(disp);
    return st;
}

void release(fbs_plan* p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->copied) (void)hipEventDestroy(p->copied);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->d_pairs) (void)hipFree(p->d_pairs);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_counters) (void)hipFree(p->d_counters);
    if (p->d_ptrs) (void)hipFree(p->d_ptrs);
    if (p->h_ptrs) (void)hipHostFree(p->h_ptrs);
    delete p;
}

}  // namespace

extern "C" {

fbs_status fbs_plan_create(fbs_plan** out, int32_t n, const fbs_params* params,
                           const char* tune_cache_path, uint32_t flags)
{
    using namespace fbs;
    if (!out) return api_fail(FBS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || !params) return api_fail(FBS_E_INVALID, "need n >= 1 pairs and their params");
    for (int i = 0; i < n; ++i) {
        fbs_status st = api_check_params(&params[i]);
        if (st != FBS_OK) return st;
        if (params[i].cost_type != FBS_COST_TAD)
            return api_fail(FBS_E_UNSUPPORTED, "pair %d: plans take the TAD cost only", i);
    }
    fbs_plan* p = new fbs_plan();
    p->n = n;
    p->params.assign(params, params + n);
    p->mfma.assign(n, 0);
    p->cfg.assign(n, MfmaCfg{8, 1});
    if (hipGetDevice(&p->device) != hipSuccess) {
        release(p);
        return api_fail(FBS_E_HIP, "no HIP device");
    }

    // per-pair configuration: cache, tuning, or the heuristic of fbs_run
    std::map<std::string, TuneEntry> cache = read_cache(tune_cache_path);
    bool cache_dirty = false;
    for (int i = 0; i < n; ++i) {
        const Geom g = api_geom(&params[i]);
        if ((params[i].flags & FBS_F_FORCE_VALU) || !mfma_supported(g)) continue;
        p->mfma[i] = 1;
        const std::string key = shape_key(g);
        auto it = cache.find(key);
        if (it != cache.end() && mfma_nw_valid(g, it->second.nw) &&
            it->second.nb >= 1 && it->second.nb <= mfma_max_nb(g, it->second.nw)) {
            p->cfg[i] = MfmaCfg{it->second.nw, it->second.nb};
        } else if (flags & FBS_PLAN_TUNE) {
            TuneEntry e{};
            fbs_status st = tune_shape(params[i], &e);
            if (st != FBS_OK) {
                release(p);
                return st;
            }
            cache[key] = e;
            cache_dirty = true;
            p->cfg[i] = MfmaCfg{e.nw, e.nb};
        } else {
            p->cfg[i] = mfma_default_cfg(g);
        }
    }
    if (cache_dirty) write_cache(tune_cache_path, cache);

    // classes and their work lists (most expensive pairs first)
    // classes: (r*1000 + ch*100 + nw/4*10 + co, sigma_s bits, sigma_r bits) - the
    // pairs of a class share one kernel and one set of weight tables
    std::map<std::tuple<int, uint32_t, uint32_t>, std::vector<int>> by_class;
    for (int i = 0; i < n; ++i)
        if (p->mfma[i]) {
            const Geom g = api_geom(&params[i]);
            const int co = mfma_use_co(g.D, p->cfg[i].nb) ? 1 : 0;
            uint32_t ss, sr;
            memcpy(&ss, &params[i].sigma_s, 4);
            memcpy(&sr, &params[i].sigma_r, 4);
            by_class[std::make_tuple(g.r * 1000 + g.C * 100 + p->cfg[i].nw / 4 * 10 + co, ss, sr)]
                .push_back(i);
        }
    std::vector<BatchPair> pairs(n);
    std::vector<int2> items;
    // persistent workgroups take kTilesPerItem consecutive tiles of a pair per
    // queue item (one descriptor chain for them); per-tile mode one tile
    const int per_item = (flags & FBS_PLAN_PER_TILE) ? 1 : kTilesPerItem;
    struct Span {
        int r, ch, nw, co, first, count, lds;
        Tables tb;
    };
    std::vector<Span> spans;
    for (auto& kv : by_class) {
        std::vector<int>& ids = kv.second;
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
            const Geom ga = api_geom(&params[a]), gb = api_geom(&params[b]);
            return ga.D > gb.D;  // cost per tile grows with D
        });
        const int key = std::get<0>(kv.first);
        Span sp{key / 1000, (key / 100) % 10, ((key / 10) % 10) * 4, key % 10, (int)items.size(), 0, 0,
                api_tables(&params[ids[0]])};
        for (int i : ids) {
            const Geom g = api_geom(&params[i]);
            const int tw = 2 * p->cfg[i].nw;
            const int tx = (g.W + tw - 1) / tw, ty = (g.H + 7) / 8;
            for (int t = 0; t < tx * ty; t += per_item) items.push_back(make_int2(i, t));
            pairs[i].g = g;
            pairs[i].scap = mfma_scaled_cap(g);
            pairs[i].nb = p->cfg[i].nb;
            pairs[i].tiles_x = tx;
            pairs[i].pad = 0;
            // each tile lays out LDS for its own pair's D and slab depth
            sp.lds = std::max(sp.lds, mfma_lds_bytes(g, p->cfg[i].nb, p->cfg[i].nw));
        }
        sp.count = (int)items.size() - sp.first;
        spans.push_back(sp);
    }

    int cus = 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
    const size_t nptr = (size_t)4 * n;
    bool ok = hipMalloc(&p->d_pairs, sizeof(BatchPair) * n) == hipSuccess &&
              hipMalloc(&p->d_items, sizeof(int2) * std::max<size_t>(1, items.size())) == hipSuccess &&
              hipMalloc(&p->d_counters, sizeof(int) * std::max<size_t>(1, spans.size())) == hipSuccess &&
              hipMalloc(&p->d_ptrs, sizeof(void*) * nptr) == hipSuccess &&
              hipHostMalloc(&p->h_ptrs, sizeof(void*) * nptr, hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&p->copied, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&p->done, hipEventDisableTiming) == hipSuccess;
    if (ok) {
        ok = hipMemcpy(p->d_pairs, pairs.data(), sizeof(BatchPair) * n, hipMemcpyHostToDevice) == hipSuccess &&
             (items.empty() || hipMemcpy(p->d_items, items.data(), sizeof(int2) * items.size(),
                                         hipMemcpyHostToDevice) == hipSuccess);
    }
    if (!ok) {
        release(p);
        return api_fail(FBS_E_HIP, "plan: device allocation or upload failed");
    }
    void** dp = p->d_ptrs;
    for (size_t c = 0; c < spans.size(); ++c) {
        const Span& sp = spans[c];
        BatchClass bc{};
        bc.r = sp.r;
        bc.ch = sp.ch;
        bc.nw = sp.nw;
        bc.lds = sp.lds;
        bc.co = sp.co;
        bc.tb = sp.tb;
        const int per_cu = mfma_batch_blocks_per_cu(sp.r, sp.ch, sp.nw, sp.lds, sp.co != 0);
        bc.grid = std::max(1, std::min(sp.count, cus * per_cu));
        bc.one_wg_per_item = (flags & FBS_PLAN_PER_TILE) ? 1 : 0;
        bc.tiles_per_item = per_item;
        bc.pairs = p->d_pairs;
        bc.items = p->d_items + sp.first;
        bc.n_items = sp.count;
        bc.counter = p->d_counters + c;
        bc.L = reinterpret_cast<const uint8_t* const*>(dp);
        bc.R = reinterpret_cast<const uint8_t* const*>(dp + n);
        bc.disp = reinterpret_cast<int32_t* const*>(dp + 2 * n);
        bc.sub = reinterpret_cast<float* const*>(dp + 3 * n);
        p->classes.push_back(bc);
    }

    // capture: reset the queue counters, then one kernel per class; the class
    // kernels are independent branches of the graph (fork after the reset,
    // join at the end), so one class's last tiles overlap the next class
    if (!p->classes.empty()) {
        const int nc = (int)p->classes.size();
        hipStream_t cs = nullptr;
        std::vector<hipStream_t> side(nc - 1, nullptr);
        std::vector<hipEvent_t> ev(nc, nullptr);
        bool cap = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
        for (int c = 0; c < nc && cap; ++c)
            cap = hipEventCreateWithFlags(&ev[c], hipEventDisableTiming) == hipSuccess &&
                  (c == 0 || hipStreamCreateWithFlags(&side[c - 1], hipStreamNonBlocking) == hipSuccess);
        cap = cap && hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) == hipSuccess;
        if (cap) {
            hipLaunchKernelGGL(k_zero, dim3((nc + 63) / 64), dim3(64), 0, cs, p->d_counters, nc);
            cap = hipEventRecord(ev[0], cs) == hipSuccess;
            for (int c = 1; c < nc && cap; ++c)
                cap = hipStreamWaitEvent(side[c - 1], ev[0], 0) == hipSuccess &&
                      launch_mfma_batch(p->classes[c], side[c - 1]) == hipSuccess &&
                      hipEventRecord(ev[c], side[c - 1]) == hipSuccess;
            cap = cap && launch_mfma_batch(p->classes[0], cs) == hipSuccess;
            for (int c = 1; c < nc && cap; ++c) cap = hipStreamWaitEvent(cs, ev[c], 0) == hipSuccess;
            hipGraph_t gr = nullptr;
            const bool ended = hipStreamEndCapture(cs, &gr) == hipSuccess;
            cap = cap && ended && gr;
            if (gr) p->graph = gr;
            if (cap) cap = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
        }
        for (hipStream_t q : side)
            if (q) (void)hipStreamDestroy(q);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (cs) (void)hipStreamDestroy(cs);
        if (!cap) {
            release(p);
            return api_fail(FBS_E_HIP, "plan: graph capture failed");
        }
    }
    *out = p;
    return FBS_OK;
}

fbs_status fbs_plan_launch(fbs_plan* p, const uint8_t* const* left, const uint8_t* const* right,
                           int32_t* const* disp, float* const* disp_sub, void* stream)
{
    using namespace fbs;
    if (!p) return api_fail(FBS_E_INVALID, "plan is NULL");
    if (!left || !right || !disp || !disp_sub)
        return api_fail(FBS_E_INVALID, "left, right, disp and disp_sub arrays are required");
    const int n = p->n;
    for (int i = 0; i < n; ++i) {
        if (!left[i] || !right[i] || !disp[i] || !disp_sub[i])
            return api_fail(FBS_E_INVALID, "pair %d: null buffer", i);
        if (((uintptr_t)disp[i] & 3u) || ((uintptr_t)disp_sub[i] & 3u))
            return api_fail(FBS_E_INVALID, "pair %d: maps must be 4-byte aligned", i);
    }
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    // the previous launch's pointer upload must have left the pinned mirror
    if (hipEventSynchronize(p->copied) != hipSuccess)
        return api_fail(FBS_E_HIP, "plan: event wait failed");
    // One pointer table and one set of queue counters per plan: this launch
    // starts on the device only after the previous launch (on any stream)
    // has finished with them.
    if (hipStreamWaitEvent(s, p->done, 0) != hipSuccess)
        return api_fail(FBS_E_HIP, "plan: ordering after the previous launch failed");
    for (int i = 0; i < n; ++i) {
        p->h_ptrs[i] = (void*)left[i];
        p->h_ptrs[n + i] = (void*)right[i];
        p->h_ptrs[2 * n + i] = (void*)disp[i];
        p->h_ptrs[3 * n + i] = (void*)disp_sub[i];
    }
    if (hipMemcpyAsync(p->d_ptrs, p->h_ptrs, sizeof(void*) * 4 * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(p->copied, s) != hipSuccess)
        return api_fail(FBS_E_HIP, "plan: pointer upload failed");
    if (p->exec && hipGraphLaunch(p->exec, s) != hipSuccess)
        return api_fail(FBS_E_HIP, "plan: graph launch failed");
    for (int i = 0; i < n; ++i) {
        if (p->mfma[i]) continue;
        const Geom g = api_geom(&p->params[i]);
        const Tables t = api_tables(&p->params[i]);
        if (launch_valu(g, t, SRC_TAD, left[i], right[i], nullptr, nullptr, nullptr, disp[i],
                        disp_sub[i], s) != hipSuccess)
            return api_fail(FBS_E_HIP, "plan: pair %d launch failed", i);
    }
    if (hipEventRecord(p->done, s) != hipSuccess) return api_fail(FBS_E_HIP, "plan: event record failed");
    return FBS_OK;
}

fbs_status fbs_plan_pair_config(const fbs_plan* p, int32_t pair, int32_t* matrix_cores,
                                int32_t* waves, int32_t* slab_blocks)
{
    if (!p || pair < 0 || pair >= p->n) return fbs::api_fail(FBS_E_INVALID, "bad plan or pair");
    if (matrix_cores) *matrix_cores = p->mfma[pair];
    if (waves) *waves = p->mfma[pair] ? p->cfg[pair].nw : 0;
    if (slab_blocks) *slab_blocks = p->mfma[pair] ? p->cfg[pair].nb : 0;
    return FBS_OK;
}

int32_t fbs_plan_num_launches(const fbs_plan* p)
{
    if (!p) return -1;
    int v = 0;
    for (int i = 0; i < p->n; ++i) v += p->mfma[i] ? 0 : 1;
    return (p->classes.empty() ? 0 : 1) + v;
}

void fbs_plan_destroy(fbs_plan* p)
{
    if (!p) return;
    (void)hipEventSynchronize(p->done);  // the plan's buffers outlive its last launch
    release(p);
}

}  // extern "C"
