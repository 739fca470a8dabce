// k_mfma.hip - fused TAD path with Eq. 6 on the matrix cores (gfx950).
//
// For a group of 16 pixels (a 2x8 or 4x4 block) let Q be the union of their
// (2r+1)^2 windows.  Eq. 6's numerator for the group is a dense contraction
//     num(d, p) = sum_{q in Q} C(q, d) * W(p, q),   W(p, q) = 0 outside p's window,
// so each 16-disparity x 16-pixel block is a chain of v_mfma_f32_16x16x32_f16
// over K = |Q| padded to a multiple of 32:
//   * A operand (16 x 32): costs.  TAD costs are small integers (gray
//     min(|dI|, tau); RGB 3*min(mean |dI|, tau) = min(sum |dI|, 3 tau)), exact
//     in fp16 whenever the cap is (checked on the host).
//   * B operand (32 x 16): support weights of Eqs. 7-8, computed once per
//     (pixel, window position), scaled by 2^14 and split into fp16 hi + lo
//     (|w - hi - lo| <= 2^-22 w); both halves stay in registers for the whole
//     disparity range, so each weight is formed once and used for every d.
//   * C/D (16 x 16): fp32 accumulators, one chain for hi and one for lo.
// The denominator of Eq. 6 does not depend on d, so the WTA and Eq. 10 run on
// the numerators directly (Eq. 10 is invariant under positive scaling); it is
// only formed when the aggregated volume is requested.
//
// Workgroup: 8 waves, one 16-pixel group per wave, covering an 8x16 pixel
// tile.  The left tile and the right strip it can match are staged in LDS as
// bytes once.  The disparity axis is walked in slabs of nb 16-disparity
// blocks: per slab all waves build the fp16 cost planes of the tile's window
// union in LDS (each cost computed once per workgroup), then every wave runs
// its MFMA chains.  Lane group g (lanes 16g..16g+15) of the 16x16 result holds
// disparities g*Q + 4b + j (Q = padded D / 4) of pixel lane%16, so each lane
// sees one contiguous quarter of the disparity range in ascending order and
// keeps a running first-minimum WTA with the Eq. 10 neighbours; the four
// quarters are merged with lane shuffles at the end.
#include "fbs_device.h"
#include "fbs_internal.h"

namespace fbs {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;
constexpr int kThreads = kWaves * 64;
constexpr int kTileH = 8, kTileW = 16;
constexpr float kWScale = 16384.0f;  // 2^14: keeps small weights in fp16's normal range
constexpr int kMaxR = 10;

constexpr int n_chunks(int gh, int gw, int r) { return (((gh + 2 * r) * ((gw + 2 * r + 7) / 8)) + 3) / 4; }

// Geometry of one radius: group shape (the one with fewer K chunks), octets,
// chunks, and the LDS tile of the 8x16 workgroup tile.
struct Cfg {
    int GH, GW;  // group shape
    int OPR;     // 8-wide octets per union row
    int NOCT;    // octets of the group's union
    int NCH;     // K chunks of 32
    int GX, GY;  // groups across / down the tile
    int LH, LW;  // rows / padded columns of the tile's union
    // cost plane stride in halves: PS/2 = 4 (mod 64) dwords, so the 16 lanes
    // reading 16 planes at one offset hit 16 distinct 4-bank groups
    int PS;
};

__host__ __device__ constexpr Cfg cfg_of(int r)
{
    const bool wide = n_chunks(2, 8, r) <= n_chunks(4, 4, r);
    Cfg c{};
    c.GH = wide ? 2 : 4;
    c.GW = wide ? 8 : 4;
    c.OPR = (c.GW + 2 * r + 7) / 8;
    c.NOCT = (c.GH + 2 * r) * c.OPR;
    c.NCH = (c.NOCT + 3) / 4;
    c.GX = kTileW / c.GW;
    c.GY = kTileH / c.GH;
    c.LH = kTileH + 2 * r;
    c.LW = ((c.GX - 1) * c.GW + 8 * c.OPR + 7) / 8 * 8;
    c.PS = ((c.LH * c.LW + 127) / 128) * 128 + 8;
    return c;
}

__host__ __device__ constexpr int align16(int b) { return (b + 15) & ~15; }

struct MfmaLayout {
    int rw;           // bytes per right-strip row
    int off_L, off_R, off_cost;
    int bytes;
};

__host__ __device__ constexpr MfmaLayout mfma_layout(int r, int ch, int D, int nb)
{
    const Cfg c = cfg_of(r);
    MfmaLayout m{};
    m.rw = (c.LW + D - 1 + 4 + 3) & ~3;  // +4: the last unaligned 8-byte read
    m.off_L = (256 + 32) * 4;
    m.off_R = m.off_L + align16(ch * c.LH * c.LW);
    m.off_cost = m.off_R + align16(ch * c.LH * m.rw);
    m.bytes = m.off_cost + 16 * nb * c.PS * 2;
    return m;
}

template <bool kAligned16>
__device__ __forceinline__ h8 lds_h8(const _Float16* p)
{
    if (kAligned16) return *reinterpret_cast<const h8*>(p);
    const h4 a = *reinterpret_cast<const h4*>(p);
    const h4 b = *reinterpret_cast<const h4*>(p + 4);
    return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// Bytes b0,b1 of v as the fp16 pair (1024 + b0, 1024 + b1): the byte fills the
// mantissa under the exponent of 1024 (0x6400), so differences are exact.
__device__ __forceinline__ h2 bytes01_f16(uint32_t v)
{
    return __builtin_bit_cast(h2, (v & 0xffu) | ((v & 0xff00u) << 8) | 0x64006400u);
}
__device__ __forceinline__ h2 bytes23_f16(uint32_t v)
{
    return __builtin_bit_cast(h2, ((v >> 16) & 0xffu) | ((v >> 8) & 0xff0000u) | 0x64006400u);
}

// 8 right-image bytes starting at an arbitrary byte offset (3 aligned dword
// reads; the row padding of the strip keeps the third read in bounds).
__device__ __forceinline__ void load8_unaligned(const uint8_t* p, uint32_t& lo, uint32_t& hi)
{
    const uintptr_t a = (uintptr_t)p;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(a & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(a & 3);
    const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
    lo = __builtin_amdgcn_alignbyte(w1, w0, sh);
    hi = __builtin_amdgcn_alignbyte(w2, w1, sh);
}

// TAD cost (times the channel count) of 8 interior positions in packed fp16:
// min(sum_ch |L - R|, scap), exact because every term is an integer <= 765.
template <int CH>
__device__ __forceinline__ h8 octet_cost(const uint8_t* l, const uint8_t* r, int lplane,
                                         int rplane, float scap)
{
    h2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const uint2 lv = *reinterpret_cast<const uint2*>(l + ch * lplane);
        uint32_t r0, r1;
        load8_unaligned(r + ch * rplane, r0, r1);
        const h2 lp[4] = {bytes01_f16(lv.x), bytes23_f16(lv.x), bytes01_f16(lv.y), bytes23_f16(lv.y)};
        const h2 rp[4] = {bytes01_f16(r0), bytes23_f16(r0), bytes01_f16(r1), bytes23_f16(r1)};
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += __builtin_elementwise_abs(lp[i] - rp[i]);
    }
    const _Float16 ch = (_Float16)scap;
    const h2 cap = {ch, ch};
    h8 out;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const h2 c = __builtin_elementwise_min(acc[i], cap);
        out[2 * i] = c[0];
        out[2 * i + 1] = c[1];
    }
    return out;
}

template <int R, int CH>
__global__ __launch_bounds__(kThreads) void k_fbs_mfma(Geom g, Tables tb, int nb, float scap,
                                                       const uint8_t* __restrict__ Lg,
                                                       const uint8_t* __restrict__ Rg,
                                                       int32_t* __restrict__ disp,
                                                       float* __restrict__ sub,
                                                       float* __restrict__ agg)
{
    constexpr Cfg C = cfg_of(R);
    constexpr int GH = C.GH, GW = C.GW, OPR = C.OPR, NOCT = C.NOCT, NCH = C.NCH;
    constexpr int LH = C.LH, LW = C.LW, PS = C.PS;
    static_assert(C.GX * C.GY == kWaves, "one group per wave");
    extern __shared__ __align__(16) unsigned char smem[];

    const int D = g.D;
    const int nblk = (D + 15) >> 4;   // 16-disparity blocks
    const int Q = nblk * 4;           // disparities per lane group
    const MfmaLayout lay = mfma_layout(R, CH, D, nb);
    const int RW = lay.rw;
    float* s_gr = reinterpret_cast<float*>(smem);
    float* s_gs = s_gr + 256;
    uint8_t* s_L = smem + lay.off_L;
    uint8_t* s_R = smem + lay.off_R;
    _Float16* s_cost = reinterpret_cast<_Float16*>(smem + lay.off_cost);

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int X0 = blockIdx.x * kTileW, Y0 = blockIdx.y * kTileH;
    const int ox = X0 - R, oy = Y0 - R;           // image position of LDS tile (0,0)
    const int dmax = g.dmin + D - 1;
    const int rox = ox - dmax;                    // image x of right-strip column 0

    // ---- stage lookup tables, left tile and right strip (0 off-image) ----
    for (int i = tid; i < 256; i += kThreads) s_gr[i] = tb.gr[i];
    if (tid < 32) s_gs[tid] = (tid <= R) ? tb.gs[tid] : 0.0f;
    for (int i = tid; i < CH * LH * LW; i += kThreads) {
        const int ch = i / (LH * LW), rem = i - ch * (LH * LW);
        const int row = rem / LW, col = rem - row * LW;
        const int x = ox + col, y = oy + row;
        uint8_t v = 0;
        if (x >= 0 && x < g.W && y >= 0 && y < g.H) v = Lg[(size_t)y * g.stride + (size_t)x * CH + ch];
        s_L[i] = v;
    }
    for (int i = tid; i < CH * LH * RW; i += kThreads) {
        const int ch = i / (LH * RW), rem = i - ch * (LH * RW);
        const int row = rem / RW, col = rem - row * RW;
        const int x = rox + col, y = oy + row;
        uint8_t v = 0;
        if (x >= 0 && x < g.W && y >= 0 && y < g.H) v = Rg[(size_t)y * g.stride + (size_t)x * CH + ch];
        s_R[i] = v;
    }
    __syncthreads();

    // ---- this wave's group and this lane's pixel / octet group ----
    const int gcol0 = (wave % C.GX) * GW, grow0 = (wave / C.GX) * GH;  // in the tile
    const int n = lane & 15, gq = lane >> 4;
    const int prow = grow0 + n / GW, pcol = gcol0 + n % GW;               // pixel in the tile
    const int px = X0 + pcol, py = Y0 + prow;
    const bool pin = px < g.W && py < g.H;

    // ---- support weights (Eqs. 7-8) for this lane's pixel, hi/lo fp16 ----
    uint32_t lp[CH];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) lp[ch] = s_L[(ch * LH + prow + R) * LW + pcol + R];
    h8 whi[NCH], wlo[NCH];
    float den = 0.0f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int o = 4 * c + gq;
        const bool real = o < NOCT;
        const int urow = real ? o / OPR : 0;
        const int ucol0 = real ? (o % OPR) * 8 : 0;
        const int dy = urow - R - n / GW;
        const float wdy = s_gs[min(abs(dy), 31)];
        const int qy = oy + grow0 + urow;
        const bool rowok = real && qy >= 0 && qy < g.H;
        const uint8_t* lrow = s_L + (grow0 + urow) * LW + gcol0 + ucol0;
        uint32_t hb[4], lb[4];
#pragma unroll
        for (int j2 = 0; j2 < 4; ++j2) {
            uint32_t hh = 0, ll = 0;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int j = 2 * j2 + e;
                const int ucol = ucol0 + j;
                const int dx = ucol - R - n % GW;
                const int qx = ox + gcol0 + ucol;
                float w = 0.0f;
                if (rowok && ucol < GW + 2 * R && qx >= 0 && qx < g.W) {
                    float wr = s_gr[abs((int)lrow[j] - (int)lp[0])];
                    if (CH == 3) {
                        wr *= s_gr[abs((int)lrow[LH * LW + j] - (int)lp[1])];
                        wr *= s_gr[abs((int)lrow[2 * LH * LW + j] - (int)lp[2])];
                    }
                    w = ((wdy * s_gs[min(abs(dx), 31)]) * wr) * kWScale;
                }
                const _Float16 hi = (_Float16)w;
                const _Float16 lo = (_Float16)(w - (float)hi);
                hh |= (uint32_t)__builtin_bit_cast(uint16_t, hi) << (16 * e);
                ll |= (uint32_t)__builtin_bit_cast(uint16_t, lo) << (16 * e);
            }
            hb[j2] = hh;
            lb[j2] = ll;
        }
        whi[c] = __builtin_bit_cast(h8, make_uint4(hb[0], hb[1], hb[2], hb[3]));
        wlo[c] = __builtin_bit_cast(h8, make_uint4(lb[0], lb[1], lb[2], lb[3]));
        __builtin_amdgcn_sched_barrier(0);  // keep one chunk's temporaries live at a time
    }
    if (agg) {
        // Eq. 6's denominator: an all-ones A operand sums each weight column,
        // giving sum_q (hi + lo)(p, q) for pixel p in every lane of that pixel
        h8 ones;
#pragma unroll
        for (int j = 0; j < 8; ++j) ones[j] = (_Float16)1.0f;
        f4 dh = {0.f, 0.f, 0.f, 0.f}, dl = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            dh = __builtin_amdgcn_mfma_f32_16x16x32_f16(ones, whi[c], dh, 0, 0, 0);
            dl = __builtin_amdgcn_mfma_f32_16x16x32_f16(ones, wlo[c], dl, 0, 0, 0);
        }
        den = dh[0] + dl[0];
    }
    const float inv_scale = 1.0f / (CH == 3 ? 3.0f : 1.0f);

    // ---- running WTA over this lane's quarter of the disparity range ----
    const float kInf = __builtin_inff();
    float best = kInf, cm = kInf, cp = kInf, prev = kInf, first_v = kInf, last_v = kInf;
    int bi = -1;
    bool need_cp = false;

    // Offset (halves) of octet 4c + gq of the group's union within a plane.
    // It is periodic in c with period P = lcm(4, OPR) / 4 chunks (P chunks
    // cover 4P / OPR whole union rows), so P lane-dependent bases plus
    // compile-time row offsets address every chunk.
    constexpr int P = (OPR == 3) ? 3 : 1;
    static_assert(OPR == 1 || OPR == 2 || OPR == 3 || OPR == 4, "octets per row");
    constexpr int kRowsPerPeriod = 4 * P / OPR;
    int a_base[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        const int o = 4 * c + gq;
        a_base[c] = (o / OPR) * LW + (o % OPR) * 8;
    }
    auto a_off = [&](int c) {
        const int o = 4 * c + gq;
        // octets past the union (zero weight) read a valid in-plane offset
        const int real_off = a_base[c % P] + (c / P) * kRowsPerPeriod * LW;
        return (4 * c + 3 < NOCT || o < NOCT) ? real_off : 0;
    };
    const int nslab = (nblk + nb - 1) / nb;
    constexpr int kOct = LW / 8;
    for (int s = 0; s < nslab; ++s) {
        const int b0 = s * nb;
        const int nbb = min(nb, nblk - b0);
        __syncthreads();  // every wave is done with the previous slab
        // cost planes: plane p = 16*bb + m, m = 4*gm + jm <-> disparity index
        // k = gm*Q + 4*(b0+bb) + jm; each item writes 8 consecutive positions
        const int items = nbb * 16 * LH * kOct;
#pragma unroll 1
        for (int it = tid; it < items; it += kThreads) {
            const int oc = it % kOct;
            const int t = it / kOct;
            const int row = t % LH;
            const int p = t / LH;
            const int m = p & 15;
            const int k = (m >> 2) * Q + 4 * (b0 + (p >> 4)) + (m & 3);
            const int d = g.dmin + min(k, D - 1);      // padded planes read in-bounds
            const int y = oy + row;
            const int x0 = ox + 8 * oc;
            const bool rowin = k < D && y >= 0 && y < g.H;
            const int lb = row * LW + 8 * oc;            // left bytes of this octet
            const int rb = row * RW + 8 * oc + (dmax - d);  // right bytes it is matched to
            h8 out;
            if (rowin && x0 >= 0 && x0 + 7 < g.W && x0 - d >= 0) {
                out = octet_cost<CH>(s_L + lb, s_R + rb, LH * LW, LH * RW, scap);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int x = x0 + j;
                    int sad = 0;
#pragma unroll
                    for (int ch = 0; ch < CH; ++ch)
                        sad += abs((int)s_L[ch * LH * LW + lb + j] - (int)s_R[ch * LH * RW + rb + j]);
                    float c = x - d < 0 ? scap : fminf((float)sad, scap);
                    c = (rowin && x >= 0 && x < g.W) ? c : 0.0f;
                    out[j] = (_Float16)c;
                }
            }
            *reinterpret_cast<h8*>(s_cost + (size_t)p * PS + row * LW + 8 * oc) = out;
        }
        __syncthreads();

#pragma unroll 1
        for (int bb = 0; bb < nbb; ++bb) {
            f4 acc_h = {0.f, 0.f, 0.f, 0.f};
            f4 acc_l = {0.f, 0.f, 0.f, 0.f};
            const _Float16* plane = s_cost + (size_t)(16 * bb + n) * PS + grow0 * LW + gcol0;
            // A operand of chunk c: this lane's disparity plane, octet 4c + gq;
            // loads run one chunk ahead of the MFMAs that consume them
            h8 a_cur = lds_h8<GW == 8>(plane + a_off(0));
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                h8 a_nxt = a_cur;
                if (c + 1 < NCH) a_nxt = lds_h8<GW == 8>(plane + a_off(c + 1));
                acc_h = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_cur, whi[c], acc_h, 0, 0, 0);
                acc_l = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_cur, wlo[c], acc_l, 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                a_cur = a_nxt;
            }
            // lane holds rows 4*gq + j of the 16x16 result: disparity index
            // k = gq*Q + 4*(b0+bb) + j of pixel n
            const int kb = gq * Q + 4 * (b0 + bb);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = kb + j;
                if (k < D) {
                    const float v = acc_h[j] + acc_l[j];
                    if (k == gq * Q) first_v = v;
                    last_v = v;
                    const bool lt = v < best;
                    if (lt) {
                        cm = prev;
                        best = v;
                        bi = k;
                    } else if (need_cp) {
                        cp = v;
                    }
                    need_cp = lt;
                    prev = v;
                    if (agg && pin)
                        agg[(size_t)k * g.W * g.H + (size_t)py * g.W + px] = (v / den) * inv_scale;
                }
            }
        }
    }

    // ---- merge the four quarters of pixel n (lanes n, n+16, n+32, n+48) ----
    // quarter t covers disparity indices [t*Q, (t+1)*Q); the first minimum is
    // the lowest quarter holding the smallest value
    float wv = __shfl(best, n), wm = __shfl(cm, n), wp = __shfl(cp, n);
    int wk = __shfl(bi, n), wc = __shfl((int)need_cp, n), wt = 0;
    float left_last = kInf;   // last value of the quarter before the winner
    float prev_last = __shfl(last_v, n);
#pragma unroll
    for (int t = 1; t < 4; ++t) {
        const int src = n + 16 * t;
        const float tv = __shfl(best, src);
        const int tk = __shfl(bi, src);
        const float tm = __shfl(cm, src), tp = __shfl(cp, src);
        const int tc = __shfl((int)need_cp, src);
        const bool take = tk >= 0 && tv < wv;
        if (take) {
            wv = tv; wk = tk; wm = tm; wp = tp; wc = tc; wt = t;
            left_last = prev_last;
        }
        prev_last = __shfl(last_v, src);
    }
    // first value of the quarter after the winner
    const float right_first = __shfl(first_v, n + 16 * min(wt + 1, 3));
    if (gq == 0 && pin) {
        float fm = wm, fp = wp;
        if (wk == wt * Q && wt > 0) fm = left_last;
        if (wc && wt < 3 && wk + 1 < D) fp = right_first;
        float ds = (float)(g.dmin + wk);
        if (wk > 0 && wk < D - 1) {
            const float dn = 2.0f * fm + 2.0f * fp - 4.0f * wv;
            if (dn > 0.0f) ds += (fm - fp) / dn;
        }
        const size_t o = (size_t)py * g.W + px;
        if (disp) disp[o] = g.dmin + wk;
        if (sub) sub[o] = ds;
    }
}

constexpr int kLdsLimit = 64 * 1024;

int pick_nb(int r, int ch, int D)
{
    const int nblk = (D + 15) >> 4;
    int nb = 1;
    while (nb < nblk && nb < 4 && mfma_layout(r, ch, D, nb + 1).bytes <= kLdsLimit) ++nb;
    return nb;
}

template <int R, int CH>
hipError_t launch_rc(const Geom& g, const Tables& t, float scap, const uint8_t* L,
                     const uint8_t* Rimg, int32_t* disp, float* sub, float* agg, hipStream_t s)
{
    const int nb = pick_nb(R, CH, g.D);
    const MfmaLayout lay = mfma_layout(R, CH, g.D, nb);
    if (lay.bytes > kLdsLimit) return hipErrorInvalidConfiguration;
    dim3 grid((g.W + kTileW - 1) / kTileW, (g.H + kTileH - 1) / kTileH);
    hipLaunchKernelGGL((k_fbs_mfma<R, CH>), grid, dim3(kThreads), lay.bytes, s, g, t, nb, scap, L,
                       Rimg, disp, sub, agg);
    return hipGetLastError();
}

template <int CH>
hipError_t launch_ch(const Geom& g, const Tables& t, float scap, const uint8_t* L,
                     const uint8_t* R, int32_t* disp, float* sub, float* agg, hipStream_t s)
{
    switch (g.r) {
    case 1: return launch_rc<1, CH>(g, t, scap, L, R, disp, sub, agg, s);
    case 2: return launch_rc<2, CH>(g, t, scap, L, R, disp, sub, agg, s);
    case 3: return launch_rc<3, CH>(g, t, scap, L, R, disp, sub, agg, s);
    case 4: return launch_rc<4, CH>(g, t, scap, L, R, disp, sub, agg, s);
    case 5: return launch_rc<5, CH>(g, t, scap, L, R, disp, sub, agg, s);
    case 6: return launch_rc<6, CH>(g, t, scap, L, R, disp, sub, agg, s);
    case 7: return launch_rc<7, CH>(g, t, scap, L, R, disp, sub, agg, s);
    case 8: return launch_rc<8, CH>(g, t, scap, L, R, disp, sub, agg, s);
    case 9: return launch_rc<9, CH>(g, t, scap, L, R, disp, sub, agg, s);
    case 10: return launch_rc<10, CH>(g, t, scap, L, R, disp, sub, agg, s);
    default: return hipErrorInvalidValue;
    }
}

// Cap as the kernel sees it: tau (gray) or 3 tau (RGB), which must be an
// exact fp16 value so every cost is exact in the A operand.
bool scaled_cap(const Geom& g, float* out)
{
    const double c = (g.C == 3 ? 3.0 : 1.0) * (double)g.tau;
    if (!(c > 0.0) || c > 2048.0) return false;
    const _Float16 h = (_Float16)(float)c;
    if ((double)(float)h != c) return false;
    *out = (float)c;
    return true;
}

}  // namespace

bool mfma_supported(const Geom& g)
{
    float scap;
    if (g.r < 1 || g.r > kMaxR) return false;
    if (g.C != 1 && g.C != 3) return false;
    if (!scaled_cap(g, &scap)) return false;
    return mfma_layout(g.r, g.C, g.D, 1).bytes <= kLdsLimit;
}

hipError_t launch_mfma(const Geom& g, const Tables& t, const uint8_t* L, const uint8_t* R,
                       int32_t* disp, float* sub, float* agg, hipStream_t s)
{
    float scap;
    if (!mfma_supported(g) || !scaled_cap(g, &scap)) return hipErrorInvalidValue;
    if (g.C == 3) return launch_ch<3>(g, t, scap, L, R, disp, sub, agg, s);
    return launch_ch<1>(g, t, scap, L, R, disp, sub, agg, s);
}

}  // namespace fbs
