// mfma_tile.h - fused TAD path with Eq. 6 on the matrix cores (gfx950): the
// tile code, its kernels and their launch helpers, shared by the per-frame,
// batched and surrogate-feature translation units.
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
// tile.  The left tile and the right strip it can match are staged in LDS once
// (gray: a byte per pixel; RGB: a dword per pixel, so every pixel access is
// aligned).  The disparity axis is walked in slabs of nb 16-disparity
// blocks: per slab all waves build the fp16 cost planes of the tile's window
// union in LDS (each cost computed once per workgroup), then every wave runs
// its MFMA chains.  Lane group g (lanes 16g..16g+15) of the 16x16 result holds
// disparities g*Q + 4b + j (Q = padded D / 4) of pixel lane%16, so each lane
// sees one contiguous quarter of the disparity range in ascending order and
// keeps a running first-minimum WTA with the Eq. 10 neighbours; the four
// quarters are merged with lane shuffles at the end.
#pragma once

#include <type_traits>

#include <algorithm>
#include <atomic>

#include "fbs_device.h"
#include "fbs_internal.h"

namespace fbs {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTileH = 8;         // tile rows; a tile is kTileH x (2 * waves) pixels
constexpr float kWScale = 16384.0f;  // 2^14: keeps small weights in fp16's normal range
constexpr int kMaxR = 10;
constexpr int kCoMax = 6;  // chunk-outer path: at most this many 16-disparity blocks
constexpr int kMaxNbAll = 64;  // bound on the 16-disparity blocks of one slab (FBS_MAX_DISP / 16)
// range factor by signed intensity difference -255..255 (no abs per weight),
// padded to a multiple of 4 floats
constexpr int kLutN = 512;

constexpr int n_chunks(int gh, int gw, int r) { return (((gh + 2 * r) * ((gw + 2 * r + 7) / 8)) + 3) / 4; }

// Geometry of one radius: group shape (the one with fewer K chunks), octets,
// chunks, and the LDS tile of a kTileH x tile_w workgroup tile.
struct Cfg {
    int GH, GW;  // group shape
    int OPR;     // 8-wide octets per union row
    int NOCT;    // octets of the group's union
    int NCH;     // K chunks of 32
    int GX, GY;  // groups across / down the tile
    int LH, LW;  // rows / padded columns of the tile's union
    // cost plane stride in halves: PS/2 = 4 (mod 64) dwords, i.e. 16 bytes
    // modulo 128, so 8 planes read at one offset (the 8 lanes of one cycle of
    // a 16-byte read) hit 8 distinct 4-bank groups; 8-byte reads serve 16
    // lanes per cycle, for which 4x4 groups also shift planes 8-15 (kShift)
    int PS;
};

__host__ __device__ constexpr Cfg cfg_of(int r, int tile_w)
{
    const bool wide = n_chunks(2, 8, r) <= n_chunks(4, 4, r);
    Cfg c{};
    c.GH = wide ? 2 : 4;
    c.GW = wide ? 8 : 4;
    c.OPR = (c.GW + 2 * r + 7) / 8;
    c.NOCT = (c.GH + 2 * r) * c.OPR;
    c.NCH = (c.NOCT + 3) / 4;
    c.GX = tile_w / c.GW;
    c.GY = kTileH / c.GH;
    c.LH = kTileH + 2 * r;
    c.LW = ((c.GX - 1) * c.GW + 8 * c.OPR + 7) / 8 * 8;
    c.PS = ((c.LH * c.LW + 127) / 128) * 128 + 8;
    return c;
}

__host__ __device__ constexpr int align16(int b) { return (b + 15) & ~15; }

struct MfmaLayout {
    int lwb, rwb;     // bytes per left-tile / right-strip row (pixel_bytes(ch) per pixel)
    int off_wx, off_wy, off_L, off_R, off_L4, off_cost;
    // NCC tiles only: the left tile and the right strip with a one-pixel
    // border (rows of nlw / nrw bytes), and per pixel the block sum (int) and
    // 1 / sqrt(n * sum I^2 - (sum I)^2) (double, 0 where that is not positive)
    // of the union positions (LH x LW) and of the strip columns (LH x SW)
    int nlw, nrw, sw;
    int off_nL, off_nR, off_sl, off_rl, off_sr, off_rr;
    int bytes;
};

// RGB: the left tile again as 16-bit words 4 * I per channel (R, G, B, 0),
// the byte offsets of the range factors, so that each of a weight's three
// factor addresses is one add.  (Gray keeps its byte tile: one address per
// weight, and small gray tiles stay within half the LDS.)
__host__ __device__ constexpr int pixel_words(int ch) { return ch == 3 ? 4 : 0; }

// Bytes per pixel in the LDS image rows: gray 1; RGB 4 (R, G, B, 0), so that a
// pixel is one aligned dword for the byte-wise SAD and the range weights.
__host__ __device__ constexpr int pixel_bytes(int ch) { return ch == 3 ? 4 : 1; }

__host__ __device__ constexpr MfmaLayout mfma_layout(int r, int ch, int D, int nb, int nw, bool ncc = false)
{
    const int tile_w = 2 * nw;
    const Cfg c = cfg_of(r, tile_w);
    MfmaLayout m{};
    m.lwb = pixel_bytes(ch) * c.LW;
    // +16: slack for the unaligned reads of the last octet of a row
    m.rwb = ncc ? 0 : (pixel_bytes(ch) * (c.LW + D - 1) + 16 + 3) & ~3;
    m.off_wx = (kLutN + 32) * 4;  // after the signed range LUT and the spatial factors
    m.off_wy = m.off_wx + tile_w * c.LW * 4;
    m.off_L = m.off_wy + align16(kTileH * c.LH * 4);
    m.off_R = m.off_L + align16(c.LH * m.lwb);
    m.off_L4 = m.off_R + align16(c.LH * m.rwb);
    m.off_cost = m.off_L4 + align16(c.LH * c.LW * pixel_words(ch) * 2);
    if (ncc) {
        m.sw = c.LW + D - 1;
        m.nlw = (c.LW + 2 + 3) & ~3;
        m.nrw = (m.sw + 2 + 16 + 3) & ~3;
        m.off_nL = m.off_cost;
        m.off_nR = m.off_nL + align16((c.LH + 2) * m.nlw);
        m.off_sl = m.off_nR + align16((c.LH + 2) * m.nrw);
        m.off_rl = m.off_sl + align16(c.LH * c.LW * 4);
        m.off_sr = m.off_rl + align16(c.LH * c.LW * 8);
        m.off_rr = m.off_sr + align16(c.LH * m.sw * 4);
        m.off_cost = m.off_rr + align16(c.LH * m.sw * 8);
    }
    // NCC costs are not integers: each block has hi and lo planes
    m.bytes = m.off_cost + (ncc ? 32 : 16) * nb * c.PS * 2;
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
typedef float f2 __attribute__((ext_vector_type(2)));

// v_perm_b32 picks bytes of the 64-bit {hi, lo} (selector 0-3: lo, 4-7: hi,
// 0x0c: zero).  With hi = 0x64646464, bytes b0, b1 of lo become the fp16 pair
// (1024 + b0, 1024 + b1): the byte fills the mantissa under the exponent of
// 1024, so differences of such pairs are exact.
__device__ __forceinline__ h2 bytes01_f16(uint32_t v)
{
    return __builtin_bit_cast(h2, __builtin_amdgcn_perm(0x64646464u, v, 0x04010400u));
}
__device__ __forceinline__ h2 bytes23_f16(uint32_t v)
{
    return __builtin_bit_cast(h2, __builtin_amdgcn_perm(0x64646464u, v, 0x04030402u));
}

// One tile's worth of work, shared by the per-frame and the batched kernels.
struct TileJob {
    Geom g;
    float scap;  // cap as the kernel sees it (tau, or 3 tau for RGB)
    int nb;      // 16-disparity blocks per LDS slab
    const uint8_t* L;
    const uint8_t* R;
    int32_t* disp;
    float* sub;
    float* agg;
    uint16_t* feat;  // FEAT tiles only: learned-surrogate features [H][W][32] BF16
    // Optional per-tile search ranges (lo, hi) [tiles_y][ranges_tx]: each tile
    // searches only its range (clipped to the job's; an empty range means the
    // whole one).  Only for disp / sub outputs (not agg or feat).
    const int2* ranges;
    int ranges_tx;
};

// The caller has put the range LUT by signed difference (kLutN floats, entry
// 255 + dI) at smem[0] and the spatial factors exp(-k^2/gd^2), k = 0..31 (0
// beyond the radius), right after it, and synchronised the workgroup.
// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// FEAT: besides the maps, write the learned surrogate's input features of
// each pixel: the 8 lowest aggregated costs (ascending, ties to the lower d)
// over the cost cap, their indices (d - d_min) / (D - 1), and the left
// intensity / 255, as BF16 in 32 channels (the rest zero).  The aggregated
// cost is formed exactly as for agg_out, so the features equal those of
// fbs_surrogate_features applied to agg_out bit for bit.
//
// Double-precision recheck of one pixel of the tile, from the definition:
// Eq. 6 with the weights of Eqs. 7-8 (exp in double) and the TAD cost from the
// staged left tile and right strip, WTA (ties to the lowest d) and Eq. 10.
// All 64 lanes of the wave take part; a pass gives lane l the aggregated
// costs at disparity indices base + l + 64 j (j < 4).  Every lane returns the
// pixel's disparity index and subpixel disparity.  Used only where the
// fp16-split weights cannot order near ties.
// NCC tiles: the bordered image tiles and the per-pixel block terms in LDS
// (layout in MfmaLayout), the union width and the block radius.
struct NccTile {
    const uint8_t* nL;
    const uint8_t* nR;
    const int* sl;
    const double* rl;
    const int* sr;
    const double* rr;
    int nlw, nrw, sw, lw, nr;
};

// NCC cost 1 - c of Eq. 1 at union position (row, col) and disparity d (the
// right pixel is strip column col + dmax - d), from the cross term and the
// block terms, in double
__device__ __forceinline__ double ncc_cost_lds(const NccTile& t, int row, int col, int sc)
{
    int slr = 0;
    for (int jr = 1 - t.nr; jr <= 1 + t.nr; ++jr)
        for (int jc = 1 - t.nr; jc <= 1 + t.nr; ++jc)
            slr += (int)t.nL[(row + jr) * t.nlw + col + jc] * (int)t.nR[(row + jr) * t.nrw + sc + jc];
    const int n = (2 * t.nr + 1) * (2 * t.nr + 1);
    const int num = n * slr - t.sl[row * t.lw + col] * t.sr[row * t.sw + sc];
    return 1.0 - (double)num * t.rl[row * t.lw + col] * t.rr[row * t.sw + sc];
}

template <int R, int CH, bool NCC = false, int PB = pixel_bytes(CH)>
__device__ __forceinline__ void recheck_pass(const Geom& g, const uint8_t* s_L, const uint8_t* s_R,
                                             int LWB, int RWB, int prow, int pcol, int x, int y,
                                             int base, int lane, double (&a)[4], const NccTile& nt)
{
    const int D = g.D, dmax = g.dmin + D - 1;
    const double igd = 1.0 / ((double)g.gd * (double)g.gd);
    const double igr = 1.0 / ((double)g.gr * (double)g.gr);
    const double tau = (double)g.tau;
    int lp[CH];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) lp[ch] = s_L[(prow + R) * LWB + (pcol + R) * PB + ch];
    double num[4] = {0.0, 0.0, 0.0, 0.0};
    double den = 0.0;
#pragma unroll 1
    for (int dy = -R; dy <= R; ++dy) {
        if (y + dy < 0 || y + dy >= g.H) continue;
        const int row = prow + R + dy;
#pragma unroll 1
        for (int dx = -R; dx <= R; ++dx) {
            const int qx = x + dx;
            if (qx < 0 || qx >= g.W) continue;
            const int col = pcol + R + dx;
            int lq[CH];
            double d2 = 0.0;
#pragma unroll
            for (int ch = 0; ch < CH; ++ch) {
                lq[ch] = s_L[row * LWB + col * PB + ch];
                const double t = (double)(lq[ch] - lp[ch]);
                d2 += t * t;
            }
            d2 /= (double)CH;
            const double w = exp(-(double)(dx * dx + dy * dy) * igd) * exp(-d2 * igr);
            den += w;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = base + lane + 64 * j;
                if (k >= 0 && k < D) {
                    const int d = g.dmin + k;
                    double c = NCC ? 2.0 : tau;
                    if (NCC) {
                        if (qx - d >= 0) c = ncc_cost_lds(nt, row, col, col + dmax - d);
                    } else if (qx - d >= 0) {
                        int sad = 0;
#pragma unroll
                        for (int ch = 0; ch < CH; ++ch)
                            sad += abs(lq[ch] - (int)s_R[row * RWB + (col + dmax - d) * PB + ch]);
                        const double m = (double)sad / (double)CH;
                        c = m < tau ? m : tau;
                    }
                    num[j] += w * c;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = num[j] / den;
}

template <int R, int CH, bool NCC>
__device__ __forceinline__ void recheck_pixel(const TileJob& job, const uint8_t* s_L, const uint8_t* s_R,
                                              int LWB, int RWB, int prow, int pcol, int X0, int Y0,
                                              int lane, int& k_out, float& ds_out, const NccTile& nt)
{
    const Geom& g = job.g;
    const int D = g.D;
    const int x = X0 + pcol, y = Y0 + prow;
    // lane-local first minimum over ascending k, pass by pass, then across the wave
    double bv = 0.0;
    int bk = -1;
#pragma unroll 1
    for (int base = 0; base < D; base += 256) {
        double a[4];
        recheck_pass<R, CH, NCC>(g, s_L, s_R, LWB, RWB, prow, pcol, x, y, base, lane, a, nt);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = base + lane + 64 * j;
            if (k < D && (bk < 0 || a[j] < bv)) {
                bv = a[j];
                bk = k;
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int ok = __shfl_xor(bk, off);
        if (ok >= 0 && (bk < 0 || ov < bv || (ov == bv && ok < bk))) {
            bv = ov;
            bk = ok;
        }
    }
    // the aggregated costs at bk - 1 (lane 0) and bk + 1 (lane 2) for Eq. 10
    double ds = (double)(g.dmin + bk);
    if (bk > 0 && bk < D - 1) {
        double a[4];
        recheck_pass<R, CH, NCC>(g, s_L, s_R, LWB, RWB, prow, pcol, x, y, bk - 1, lane, a, nt);
        const double cm = __shfl(a[0], 0), cp = __shfl(a[0], 2);
        const double dnm = 2.0 * cm + 2.0 * cp - 4.0 * bv;
        if (dnm > 0.0) ds += (cm - cp) / dnm;
    }
    k_out = bk;
    ds_out = (float)ds;
}

// CO (chunk-outer): the whole disparity range sits in one LDS slab (nb equal to
// the number of 16-disparity blocks, at most kCoMax); each K chunk's weights
// are formed and immediately applied to every block, so only one chunk of
// weights is live and the weight arithmetic of one chunk overlaps the matrix
// work of the previous.  Otherwise the weights of every chunk are formed once,
// held in registers, and applied slab by slab.  Both accumulate each block the
// same way - hi and lo products in two chains over the chunks in order, summed
// at the end - so the results do not depend on the path, the slab depth or
// the waves per workgroup.
template <int R, int CH, int NW, bool FEAT = false, bool CO = false, bool NCC = false>
__device__ __forceinline__ void mfma_tile(const TileJob& job_in, int tile_x, int tile_y,
                                          unsigned char* smem, int tid)
{
#pragma clang fp contract(off)
    TileJob job = job_in;
    if (job.ranges) {
        // this tile's search range: every step below sees it as the job's range
        const int2 rg = job.ranges[tile_y * job.ranges_tx + tile_x];
        const int lo = __builtin_amdgcn_readfirstlane(max(rg.x, job.g.dmin));
        const int hi = __builtin_amdgcn_readfirstlane(min(rg.y, job.g.dmin + job.g.D - 1));
        if (lo <= hi) {
            job.g.dmin = lo;
            job.g.D = hi - lo + 1;
        }
    }
    // Every floating-point operation here rounds as written: a fused
    // multiply-add in place of w - hi (w a product) would change lo, and the
    // compiler's choice could differ between kernels that share this code.
    constexpr int kThreads = 64 * NW, kTileW = 2 * NW;
    const Geom& g = job.g;
    const int nb = job.nb;
    const float scap = job.scap;
    const uint8_t* __restrict__ Lg = job.L;
    const uint8_t* __restrict__ Rg = job.R;
    int32_t* __restrict__ disp = job.disp;
    float* __restrict__ sub = job.sub;
    float* __restrict__ agg = job.agg;
    constexpr Cfg C = cfg_of(R, kTileW);
    constexpr int GH = C.GH, GW = C.GW, OPR = C.OPR, NOCT = C.NOCT, NCH = C.NCH;
    constexpr int LH = C.LH, LW = C.LW, PS = C.PS;
    // 4x4 groups read their A operands as two 8-byte halves, 16 lanes (rows
    // m = 0..15 of one K quarter) per LDS cycle; the plane stride is 16 bytes
    // modulo 128, so rows m and m + 8 would share banks.  Planes 8..15 of
    // every 16 therefore sit 4 halves (8 bytes) further in their slot (the
    // slot's pad holds them), and their stores are 8-byte pairs.  2x8 groups
    // read 16 bytes per lane, 8 lanes per cycle: no shift.
    constexpr int kShift = GW == 4 ? 4 : 0;
    constexpr int PB = pixel_bytes(CH);  // bytes per pixel in LDS
    constexpr int LWB = PB * LW;
    static_assert(C.GX * C.GY == NW, "one group per wave");

    const int D = g.D;
    const int nblk = (D + 15) >> 4;   // 16-disparity blocks
    const int Q = nblk * 4;           // disparities per lane group
    __builtin_assume(Q > 0 && Q <= 4 * kMaxNbAll);
    static_assert(!NCC || (CH == 1 && !FEAT && !CO), "NCC tiles: gray, slab path");
    const MfmaLayout lay = mfma_layout(R, CH, D, nb, NW, NCC);
    const int RWB = lay.rwb;
    __builtin_assume(RWB >= 0 && RWB < 65536);
    const float* s_gr = reinterpret_cast<const float*>(smem) + 255;  // index by I_q - I_p
    const float* s_gs = s_gr - 255 + kLutN;
    float* s_wx = reinterpret_cast<float*>(smem + lay.off_wx);
    float* s_wy = reinterpret_cast<float*>(smem + lay.off_wy);
    uint8_t* s_L = smem + lay.off_L;
    uint8_t* s_R = smem + lay.off_R;
    uint16_t* s_L4 = reinterpret_cast<uint16_t*>(smem + lay.off_L4);
    _Float16* s_cost = reinterpret_cast<_Float16*>(smem + lay.off_cost);
    NccTile nt{smem + lay.off_nL, smem + lay.off_nR,
               reinterpret_cast<const int*>(smem + lay.off_sl), reinterpret_cast<const double*>(smem + lay.off_rl),
               reinterpret_cast<const int*>(smem + lay.off_sr), reinterpret_cast<const double*>(smem + lay.off_rr),
               lay.nlw, lay.nrw, lay.sw, LW, g.ncc_r};

    const int lane = tid & 63, wave = tid >> 6;
    const int X0 = tile_x * kTileW, Y0 = tile_y * kTileH;
    const int ox = X0 - R, oy = Y0 - R;           // image position of LDS tile (0,0)
    const int dmax = g.dmin + D - 1;
    const int rox = ox - dmax;                    // image x of right-strip column 0

    // ---- stage: range LUT; spatial factor tables; left tile, right strip ----
    // s_wx[pc][U] = exp(-(U-R-pc)^2/gd^2) for union column U of pixel column pc,
    // 0 outside the window or the image; s_wy[pr][V] likewise along y, times
    // the 2^14 weight scale.  Image rows are copied as bytes with channels
    // interleaved; bytes off the image are staged as 0.
    for (int i = tid; i < kTileW * LW; i += kThreads) {
        const int pc = i / LW, u = i - pc * LW;
        const int dx = abs(u - R - pc), x = ox + u;
        s_wx[i] = (dx <= R && x >= 0 && x < g.W) ? s_gs[dx] : 0.0f;
    }
    for (int i = tid; i < kTileH * LH; i += kThreads) {
        const int pr = i / LH, v = i - pr * LH;
        const int dy = abs(v - R - pr), y = oy + v;
        s_wy[i] = (dy <= R && y >= 0 && y < g.H) ? s_gs[dy] * kWScale : 0.0f;
    }
    {
        // Pixels off the image are never weighted (their window positions have
        // zero weight, and right pixels left of the image are replaced by the
        // cap), so they only need to be finite: read them from clamped
        // in-bounds addresses instead of branching.  4 bytes per thread and
        // iteration (gray: 4 pixels; RGB: one pixel and a zero byte), all loads
        // issued before the LDS writes.  The left tile also goes to s_L4.
        auto stage = [&](uint8_t* dst, int wb, int nrows, int x0, int y0, const uint8_t* src, auto words_c) {
            const int n4 = nrows * wb / 4;
#pragma unroll 2
            for (int i = tid; i < n4; i += kThreads) {
                const int row = (4 * i) / wb, cb = 4 * i - row * wb;
                const size_t rbase = (size_t)min(max(y0 + row, 0), g.H - 1) * g.stride;
                uint32_t v = 0;
                if constexpr (CH == 1) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int xb = min(max(x0 + cb + e, 0), g.W - 1);
                        v |= (uint32_t)src[rbase + xb] << (8 * e);
                    }
                } else {
                    const size_t xb = (size_t)min(max(x0 + cb / 4, 0), g.W - 1) * 3;
#pragma unroll
                    for (int e = 0; e < 3; ++e) v |= (uint32_t)src[rbase + xb + e] << (8 * e);
                }
                reinterpret_cast<uint32_t*>(dst)[i] = v;
                if constexpr (decltype(words_c)::value) {
                    // the same pixel (R, G, B, 0) as 4 * byte in 16-bit words
                    const uint32_t w0 = ((v & 0xffu) | ((v & 0xff00u) << 8)) << 2;
                    const uint32_t w1 = ((v >> 16) & 0xffu) << 2;
                    reinterpret_cast<uint2*>(s_L4)[i] = make_uint2(w0, w1);
                }
            }
        };
        stage(s_L, LWB, LH, ox, oy, Lg, std::integral_constant<bool, CH == 3>{});
        if constexpr (NCC) {
            // NCC blocks reach one pixel past the union and the strip; clamped
            // reads give the clamp-to-edge block coordinates
            stage(smem + lay.off_nL, lay.nlw, LH + 2, ox - 1, oy - 1, Lg, std::false_type{});
            stage(smem + lay.off_nR, lay.nrw, LH + 2, rox - 1, oy - 1, Rg, std::false_type{});
        } else {
            stage(s_R, RWB, LH, rox, oy, Rg, std::false_type{});
        }
    }
    __syncthreads();
    if constexpr (NCC) {
        // block sum s and 1 / sqrt(n * sum I^2 - s^2) of every union position
        // and strip column (read after the barrier that opens the first slab)
        const int nr = g.ncc_r, nn = (2 * nr + 1) * (2 * nr + 1);
        auto terms = [&](const uint8_t* img, int wb, int w, int cnt, int* so, double* ro) {
            for (int i = tid; i < cnt; i += kThreads) {
                const int v = i / w, u = i - v * w;
                int s1 = 0, s2 = 0;
                for (int jr = 1 - nr; jr <= 1 + nr; ++jr)
                    for (int jc = 1 - nr; jc <= 1 + nr; ++jc) {
                        const int b = img[(v + jr) * wb + u + jc];
                        s1 += b;
                        s2 += b * b;
                    }
                const int var = nn * s2 - s1 * s1;
                so[i] = s1;
                ro[i] = var > 0 ? 1.0 / sqrt((double)var) : 0.0;
            }
        };
        terms(nt.nL, lay.nlw, LW, LH * LW, reinterpret_cast<int*>(smem + lay.off_sl),
              reinterpret_cast<double*>(smem + lay.off_rl));
        terms(nt.nR, lay.nrw, lay.sw, LH * lay.sw, reinterpret_cast<int*>(smem + lay.off_sr),
              reinterpret_cast<double*>(smem + lay.off_rr));
    }

    // ---- this wave's group and this lane's pixel / octet group ----
    const int gcol0 = (wave % C.GX) * GW, grow0 = (wave / C.GX) * GH;  // in the tile
    const int n = lane & 15, gq = lane >> 4;
    const int prow = grow0 + n / GW, pcol = gcol0 + n % GW;               // pixel in the tile
    const int px = X0 + pcol, py = Y0 + prow;
    const bool pin = px < g.W && py < g.H;

    // ---- support weights (Eqs. 7-8) for this lane's pixel, hi/lo fp16 ----
    // w = wx(dx) * wy(dy) * prod_ch gr(|dI_ch|) * 2^14, then w = hi + lo
    uint32_t lp[CH];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) lp[ch] = s_L[(prow + R) * LWB + (pcol + R) * PB + ch];
    // range factor of channel ch for a neighbour of intensity I: the float at
    // byte offset 4 * I from gb[ch] (RGB), s_gr[I - lp[0]] (gray)
    const uint8_t* gb[CH];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) gb[ch] = reinterpret_cast<const uint8_t*>(s_gr - (int)lp[ch]);
    auto chunk_weights = [&](int c, h8& whc, h8& wlc) {
#pragma clang fp contract(off)
        const int o = min(4 * c + gq, NOCT - 1);  // octets past the union: weight 0
        const bool real = 4 * c + gq < NOCT;
        const int V = grow0 + o / OPR;                          // tile union row
        const int U = gcol0 + (o % OPR) * 8;                    // tile union column
        const float wy = real ? s_wy[prow * LH + V] : 0.0f;
        const float4 wx0 = *reinterpret_cast<const float4*>(s_wx + pcol * LW + U);
        const float4 wx1 = *reinterpret_cast<const float4*>(s_wx + pcol * LW + U + 4);
        const float wx[8] = {wx0.x, wx0.y, wx0.z, wx0.w, wx1.x, wx1.y, wx1.z, wx1.w};
        // 8 pixels of the left image (U is a multiple of 8): RGB as words 4 * I,
        // gray as bytes
        constexpr int PW = pixel_words(CH);
        uint32_t lq[CH == 3 ? 4 * PW : 2];
        if constexpr (CH == 3) {
            const uint4* q = reinterpret_cast<const uint4*>(s_L4 + (V * LW + U) * PW);
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                const uint4 t = q[i];
                lq[4 * i] = t.x;
                lq[4 * i + 1] = t.y;
                lq[4 * i + 2] = t.z;
                lq[4 * i + 3] = t.w;
            }
        } else {
            const uint2 t = *reinterpret_cast<const uint2*>(s_L + V * LWB + U);
            lq[0] = t.x;
            lq[1] = t.y;
        }
        float wa[8], wb[8];  // w = wa * wb
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float wr = 1.0f;
#pragma unroll
            for (int ch = 0; ch < CH; ++ch) {
                float f;
                if constexpr (CH == 3) {
                    const int wi = PW * j + ch;  // word index
                    const uint32_t off = (wi & 1) ? lq[wi >> 1] >> 16 : lq[wi >> 1] & 0xffffu;
                    f = *reinterpret_cast<const float*>(gb[ch] + off);
                } else {
                    const int iv = (int)((lq[j >> 2] >> (8 * (j & 3))) & 0xffu);
                    f = s_gr[iv - (int)lp[0]];
                }
                wr = ch == 0 ? f : wr * f;
            }
            wa[j] = wx[j] * wy;
            wb[j] = wr;
        }
        h8 hv, lv;
#pragma unroll
        for (int j2 = 0; j2 < 4; ++j2) {
            // hi = w rounded to fp16, lo = the exact product's remainder
            // rounded to fp16 (an explicit fused multiply-add, so every kernel
            // forms the same bits)
            const int j0 = 2 * j2, j1 = j0 + 1;
            const f2 pw = {wa[j0] * wb[j0], wa[j1] * wb[j1]};
            const h2 hi = __builtin_convertvector(pw, h2);
            const f2 hf = __builtin_convertvector(hi, f2);
            const f2 rem = {__builtin_fmaf(wa[j0], wb[j0], -hf[0]), __builtin_fmaf(wa[j1], wb[j1], -hf[1])};
            const h2 lo = __builtin_convertvector(rem, h2);
            hv[2 * j2] = hi[0];
            hv[2 * j2 + 1] = hi[1];
            lv[2 * j2] = lo[0];
            lv[2 * j2 + 1] = lo[1];
        }
        if constexpr (!CO) {
            // Pin the packed chunk here.  Otherwise the conversions sink towards
            // their MFMA uses and all float weights of the tile stay live at once.
            // (The chunk-outer path uses each chunk at once and must stay free
            // to interleave it with the previous chunk's matrix work.)
            uint4 hu = __builtin_bit_cast(uint4, hv), lu = __builtin_bit_cast(uint4, lv);
            asm volatile("" : "+v"(hu.x), "+v"(hu.y), "+v"(hu.z), "+v"(hu.w), "+v"(lu.x),
                         "+v"(lu.y), "+v"(lu.z), "+v"(lu.w));
            whc = __builtin_bit_cast(h8, hu);
            wlc = __builtin_bit_cast(h8, lu);
        } else {
            whc = hv;
            wlc = lv;
        }
    };
    h8 whi[CO ? 1 : NCH], wlo[CO ? 1 : NCH];
    if constexpr (!CO) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) chunk_weights(c, whi[c], wlo[c]);
    }
    // Eq. 6's denominator (only for agg_out and features): an all-ones A
    // operand sums each weight column, giving sum_q (hi + lo)(p, q) for pixel
    // p in every lane of that pixel
    const bool want_den = FEAT || agg != nullptr;
    h8 ones;
#pragma unroll
    for (int j = 0; j < 8; ++j) ones[j] = (_Float16)1.0f;
    f4 dh = {0.f, 0.f, 0.f, 0.f}, dl = {0.f, 0.f, 0.f, 0.f};
    float rden = 0.0f;  // 1 / Eq. 6's denominator
    // the kernel's cost units: RGB sums 3 channels; NCC costs are scaled by 2^10
    const float inv_scale = NCC ? 1.0f / 1024.0f : 1.0f / (CH == 3 ? 3.0f : 1.0f);
    if constexpr (!CO) {
        if (want_den) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                dh = __builtin_amdgcn_mfma_f32_16x16x32_f16(ones, whi[c], dh, 0, 0, 0);
                dl = __builtin_amdgcn_mfma_f32_16x16x32_f16(ones, wlo[c], dl, 0, 0, 0);
            }
            rden = 1.0f / (dh[0] + dl[0]);
        }
    }

    // ---- running WTA over this lane's quarter of the disparity range ----
    const float kInf = __builtin_inff();
    float best = kInf, cm = kInf, cp = kInf, prev = kInf, first_v = kInf;
    float best2 = kInf;  // second-lowest value of this lane's quarter (near-tie check)
    int bi = -1;
    bool need_cp = false;
    // FEAT: this lane's 8 lowest aggregated costs of its quarter, ascending,
    // as 32-bit keys: the cost's bits with the low kbits (the width of D - 1)
    // replaced by the disparity index k.  Costs are >= 0, so the keys order by
    // cost at that resolution and then by disparity, and each key is unique.
    const int kbits = 32 - __builtin_clz((unsigned)max(D - 1, 1));
    const uint32_t kmask = (1u << kbits) - 1u;
    uint32_t tkey[FEAT ? 8 : 1];
    if constexpr (FEAT) {
#pragma unroll
        for (int i = 0; i < 8; ++i) tkey[i] = ~0u;
    }
    auto ce = [](uint32_t& a, uint32_t& b) {  // compare-exchange: a <= b after
        const uint32_t lo = min(a, b), hi = max(a, b);
        a = lo;
        b = hi;
    };

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
    auto a_off = [&](int c) -> int {
        if (4 * c + 3 < NOCT) return a_base[c % P] + (c / P) * kRowsPerPeriod * LW;
        // last chunk: octets past the union carry zero weight; read the last real one
        const int o = min(4 * c + gq, NOCT - 1);
        return (o / OPR) * LW + (o % OPR) * 8;
    };
    constexpr int kOct = LW / 8;
    const _Float16 hcap = (_Float16)scap;
    const h2 cap2 = {hcap, hcap};

    // Cost planes of blocks b0 .. b0+nbb-1: plane p = 16*bb + 4*gm + jm holds
    // disparity index k = gm*Q + 4*(b0+bb) + jm.  An item is one octet (8
    // positions of a tile row) of one quad (bb, gm) at the 4 consecutive
    // disparities d0 .. d0+3 (jm = 0..3), whose right pixels x - d are the 11
    // strip columns c = 8*oc + dmax - d0 - 3 + i, i = j - jm + 3.  Items are
    // spread evenly over the workgroup (octet index fastest), stepped without
    // divisions.  Costs of positions off the image or of padded disparities
    // (k >= D) are never weighted, so any finite value will do there: padded
    // disparities read up to 15 pixels before their strip row, which stays
    // inside the LDS tile (the left tile precedes the strip).
    constexpr int kPairs = LH * kOct;
    static_assert(kPairs <= kThreads, "a step covers every octet");
    const int b_q0 = tid / kPairs, b_p0 = tid - b_q0 * kPairs;
    auto build_slab = [&](int b0, int nbb) {
        const h2 off = {(_Float16)1024.0f, (_Float16)1024.0f};
        int pair = b_p0, quad = b_q0;
#pragma unroll 1
        while (quad < 4 * nbb) {
            // small ranges: lets the address arithmetic use 24-bit multiplies
            __builtin_assume(pair >= 0 && pair < kPairs);
            __builtin_assume(quad >= 0 && quad < 4 * kMaxNbAll);
            const int row = pair / kOct, oc = pair - row * kOct;
            const int x0 = ox + 8 * oc;
            const int k0 = (quad & 3) * Q + 4 * (b0 + (quad >> 2));
            const int d0 = g.dmin + k0;
            // planes 4 quad + jm (+ 16 k): bit 3 of the plane index is bit 1 of quad
            _Float16* dst = s_cost + (size_t)(4 * quad) * PS + ((quad & 2) ? kShift : 0) + row * LW + 8 * oc;
            auto put = [](_Float16* q, const h8& v) {
                if constexpr (kShift == 0) {
                    *reinterpret_cast<h8*>(q) = v;
                } else {
                    *reinterpret_cast<h4*>(q) = __builtin_shufflevector(v, v, 0, 1, 2, 3);
                    *reinterpret_cast<h4*>(q + 4) = __builtin_shufflevector(v, v, 4, 5, 6, 7);
                }
            };
            // a cost that pairs with a right pixel left of the image is the cap
            auto left_fill = [&](h8& out, int d) {
                const int thr = d - x0;  // positions j < thr: x - d < 0
                if (thr > 0) {
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (j < thr) out[j] = hcap;
                }
            };
            if constexpr (NCC) {
                // NCC (Eq. 1) at the 8 positions u = 8*oc + j and disparities d0 + jm:
                // cross terms by byte dot products over the block rows (bordered
                // tiles: position u is bordered column u + 1, and its block
                // columns u .. u + 2 are one dword with the fourth byte masked);
                // right block of (j, jm) at bordered strip columns rb + i .. + 2,
                // i = j - jm + 3.  Cost 1 - num * rl * rr in double, rounded to
                // float, scaled by 2^10 and split into fp16 hi + lo planes.
                const int nr = g.ncc_r, nn = (2 * nr + 1) * (2 * nr + 1);
                const uint32_t bmask = nr ? 0x00ffffffu : 0x0000ff00u;
                const int rb = 8 * oc + (dmax - d0 - 3);
                int slr[4][8];
#pragma unroll
                for (int jm = 0; jm < 4; ++jm)
#pragma unroll
                    for (int j = 0; j < 8; ++j) slr[jm][j] = 0;
#pragma unroll 1
                for (int jr = 1 - nr; jr <= 1 + nr; ++jr) {
                    const uint32_t* lw = reinterpret_cast<const uint32_t*>(nt.nL + (row + jr) * lay.nlw + 8 * oc);
                    const uint32_t a0 = lw[0], a1 = lw[1], a2 = lw[2];
                    uint32_t lb[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const uint32_t lo = j < 4 ? a0 : a1, hi = j < 4 ? a1 : a2;
                        lb[j] = ((j & 3) ? __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)(j & 3)) : lo) & bmask;
                    }
                    const int cb = (row + jr) * lay.nrw + rb;
                    const int ab = cb & ~3;
                    const uint32_t sh = (uint32_t)(cb - ab);
                    const uint32_t* wq = reinterpret_cast<const uint32_t*>(nt.nR + ab);
                    const uint32_t w0 = wq[0], w1 = wq[1], w2 = wq[2], w3 = wq[3];
                    const uint32_t u[4] = {__builtin_amdgcn_alignbyte(w1, w0, sh), __builtin_amdgcn_alignbyte(w2, w1, sh),
                                           __builtin_amdgcn_alignbyte(w3, w2, sh), w3 >> (8 * sh)};
                    uint32_t rw[11];
#pragma unroll
                    for (int i = 0; i < 11; ++i)
                        rw[i] = (i & 3) ? __builtin_amdgcn_alignbyte(u[(i >> 2) + 1], u[i >> 2], (uint32_t)(i & 3)) : u[i >> 2];
#pragma unroll
                    for (int jm = 0; jm < 4; ++jm)
#pragma unroll
                        for (int j = 0; j < 8; ++j)
                            slr[jm][j] = (int)__builtin_amdgcn_udot4(lb[j], rw[j - jm + 3], (uint32_t)slr[jm][j], false);
                }
                const int pbase = row * LW + 8 * oc, sbase = row * lay.sw + rb;
#pragma unroll
                for (int jm = 0; jm < 4; ++jm) {
                    const int d = d0 + jm;
                    h8 hv, lv;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int i = j - jm + 3;
                        // a right pixel left of the image (and a padded disparity) costs 2
                        const bool valid = x0 + j - d >= 0 && d <= dmax;
                        const int num = nn * slr[jm][j] - nt.sl[pbase + j] * nt.sr[sbase + i];
                        const double c = 1.0 - (double)num * nt.rl[pbase + j] * nt.rr[sbase + i];
                        const float cs = (valid ? (float)c : 2.0f) * 1024.0f;
                        const _Float16 h = (_Float16)cs;
                        hv[j] = h;
                        lv[j] = (_Float16)(cs - (float)h);
                    }
                    put(dst + (16 * (quad >> 2) + jm) * PS, hv);
                    put(dst + (16 * (quad >> 2) + 16 + jm) * PS, lv);
                }
            } else if constexpr (CH == 1) {
                const uint2 lv = *reinterpret_cast<const uint2*>(s_L + row * LWB + 8 * oc);
                const h2 l[4] = {bytes01_f16(lv.x), bytes23_f16(lv.x), bytes01_f16(lv.y), bytes23_f16(lv.y)};
                // bytes c0 .. c11 of strip columns from 8*oc + dmax - d0 - 3 on
                const int cb = row * RWB + 8 * oc + (dmax - d0 - 3);
                const int ab = cb & ~3;
                const uint32_t sh = (uint32_t)(cb - ab);
                const uint32_t* wq = reinterpret_cast<const uint32_t*>(s_R + ab);
                const uint32_t w0 = wq[0], w1 = wq[1], w2 = wq[2], w3 = wq[3];
                const uint32_t u0 = __builtin_amdgcn_alignbyte(w1, w0, sh);
                const uint32_t u1 = __builtin_amdgcn_alignbyte(w2, w1, sh);
                const uint32_t u2 = __builtin_amdgcn_alignbyte(w3, w2, sh);
                const uint32_t v0 = __builtin_amdgcn_alignbyte(u1, u0, 1u);
                const uint32_t v1 = __builtin_amdgcn_alignbyte(u2, u1, 1u);
                const uint32_t v2 = u2 >> 8;
                // E[k] = (c[2k], c[2k+1]), O[k] = (c[2k+1], c[2k+2]) as 1024 + byte
                const h2 E[5] = {bytes01_f16(u0), bytes23_f16(u0), bytes01_f16(u1), bytes23_f16(u1), bytes01_f16(u2)};
                const h2 O[5] = {bytes01_f16(v0), bytes23_f16(v0), bytes01_f16(v1), bytes23_f16(v1), bytes01_f16(v2)};
#pragma unroll
                for (int jm = 0; jm < 4; ++jm) {
                    // positions (2i, 2i+1) pair with c[2i - jm + 3], c[2i - jm + 4]
                    h8 out;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const h2 r = jm == 0 ? O[i + 1] : jm == 1 ? E[i + 1] : jm == 2 ? O[i] : E[i];
                        const h2 c = __builtin_elementwise_min(__builtin_elementwise_abs(l[i] - r), cap2);
                        out[2 * i] = c[0];
                        out[2 * i + 1] = c[1];
                    }
                    left_fill(out, d0 + jm);
                    put(dst + jm * PS, out);
                }
            } else {
                const uint4* lq = reinterpret_cast<const uint4*>(s_L + row * LWB + 32 * oc);
                const uint4 a0 = lq[0], a1 = lq[1];
                const uint32_t lpx[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
                // the 11 aligned pixel dwords of strip columns 8*oc + dmax - d0 - 3 on
                const uint32_t* rq = reinterpret_cast<const uint32_t*>(s_R + row * RWB + 32 * oc) + (dmax - d0 - 3);
                uint32_t rr[11];
#pragma unroll
                for (int i = 0; i < 11; ++i) rr[i] = rq[i];
#pragma unroll
                for (int jm = 0; jm < 4; ++jm) {
                    h8 out;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        // the two channel sums land on the fp16 exponent of 1024
                        // (sums <= 765), low and high half: the pair (1024 + s0, 1024 + s1)
                        const int j0 = 2 * i, j1 = j0 + 1;
                        uint32_t v = __builtin_amdgcn_sad_u8(lpx[j0], rr[j0 - jm + 3], 0x64006400u);
                        v = __builtin_amdgcn_sad_hi_u8(lpx[j1], rr[j1 - jm + 3], v);
                        const h2 c = __builtin_elementwise_min(__builtin_bit_cast(h2, v) - off, cap2);
                        out[2 * i] = c[0];
                        out[2 * i + 1] = c[1];
                    }
                    left_fill(out, d0 + jm);
                    put(dst + jm * PS, out);
                }
            }
            // next item: kThreads further in (quad, octet) order
            pair += kThreads % kPairs;
            quad += kThreads / kPairs;
            if (pair >= kPairs) {
                pair -= kPairs;
                ++quad;
            }
        }
    };

    // WTA (and agg_out / features) over the 4 rows j of one 16-disparity
    // block: lane holds rows 4*gq + j of the 16x16 result, i.e. disparity
    // index k = kb + j of pixel n; acc is the sum of the block's chains (TAD:
    // hi + lo weights; NCC: (hi + lo weights on hi costs) + hi weights on lo costs)
    auto wta_block = [&](int kb, const f4& acc) {
        if (agg && pin) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (kb + j < D)
                    agg[(size_t)(kb + j) * g.W * g.H + (size_t)py * g.W + px] = (acc[j] * rden) * inv_scale;
        }
        // The running first minimum as selects, no branches.  A padded
        // disparity (k >= D) enters as +inf: it never wins, leaves the second
        // lowest alone, and only ever follows the quarter's real values.
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kb + j;
            const float v = k < D ? acc[j] : kInf;
            if (j == 0 && kb == gq * Q) first_v = v;
            const bool lt = v < best;
            // best2 >= best always, so this is best when v < best, else
            // min(best2, v); and min(best, v) keeps best on a tie
            best2 = fminf(fmaxf(best, v), best2);
            best = fminf(best, v);
            cp = (!lt && need_cp) ? v : cp;
            cm = lt ? prev : cm;
            bi = lt ? k : bi;
            need_cp = lt;
            prev = v;  // after the last block: the quarter's last value
        }
        if constexpr (FEAT) {
            // the block's four keys, sorted, then merged into the running
            // list: the lowest 8 of list and block form a bitonic sequence
            // (list[0..3], min(list[4+i], blk[3-i])) that three
            // compare-exchange stages sort
            uint32_t bk[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = kb + j;
                const float a = (acc[j] * rden) * inv_scale;
                bk[j] = k < D ? (__float_as_uint(a) & ~kmask) | (uint32_t)k : ~0u;
            }
            ce(bk[0], bk[1]);
            ce(bk[2], bk[3]);
            ce(bk[0], bk[2]);
            ce(bk[1], bk[3]);
            ce(bk[1], bk[2]);
#pragma unroll
            for (int i = 0; i < 4; ++i) tkey[4 + i] = min(tkey[4 + i], bk[3 - i]);
#pragma unroll
            for (int i = 0; i < 4; ++i) ce(tkey[i], tkey[i + 4]);
#pragma unroll
            for (int i : {0, 1, 4, 5}) ce(tkey[i], tkey[i + 2]);
#pragma unroll
            for (int i : {0, 2, 4, 6}) ce(tkey[i], tkey[i + 1]);
        }
    };

    const _Float16* plane0 = s_cost + (size_t)n * PS + ((n & 8) ? kShift : 0) + grow0 * LW + gcol0;
    if constexpr (CO) {
        __syncthreads();
        build_slab(0, nblk);
        __syncthreads();
        // The chunk loop, with the block count and whether Sigma w is formed
        // fixed at compile time for the common cases (NBK = 0 / DEN = 2: read
        // at run time): then no branch separates the matrix instructions.
        auto co_chunks = [&](auto nbk_c, auto den_c) {
            constexpr int NBK = decltype(nbk_c)::value;
            constexpr int DEN = decltype(den_c)::value;
            const bool den_on = DEN == 2 ? want_den : DEN == 1;
            f4 ah[kCoMax], al[kCoMax];
#pragma unroll
            for (int b = 0; b < kCoMax; ++b) {
                ah[b] = f4{0.f, 0.f, 0.f, 0.f};
                al[b] = ah[b];
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                h8 wh, wl;
                chunk_weights(c, wh, wl);
                if (den_on) {
                    dh = __builtin_amdgcn_mfma_f32_16x16x32_f16(ones, wh, dh, 0, 0, 0);
                    dl = __builtin_amdgcn_mfma_f32_16x16x32_f16(ones, wl, dl, 0, 0, 0);
                }
                h8 a[kCoMax];
#pragma unroll
                for (int b = 0; b < kCoMax; ++b)
                    if (NBK ? b < NBK : b < nblk) a[b] = lds_h8<GW == 8>(plane0 + (size_t)(16 * b) * PS + a_off(c));
#pragma unroll
                for (int b = 0; b < kCoMax; ++b)
                    if (NBK ? b < NBK : b < nblk)
                        ah[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[b], wh, ah[b], 0, 0, 0);
#pragma unroll
                for (int b = 0; b < kCoMax; ++b)
                    if (NBK ? b < NBK : b < nblk)
                        al[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[b], wl, al[b], 0, 0, 0);
            }
            if (den_on) rden = 1.0f / (dh[0] + dl[0]);
#pragma unroll
            for (int b = 0; b < kCoMax; ++b)
                if (NBK ? b < NBK : b < nblk) wta_block(gq * Q + 4 * b, ah[b] + al[b]);
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        if constexpr (FEAT) {
            if (nblk == 6) co_chunks(std::integral_constant<int, 6>{}, I1{});
            else co_chunks(I0{}, I1{});
        } else {
            if (!want_den && nblk == 4) co_chunks(std::integral_constant<int, 4>{}, I0{});
            else if (!want_den && nblk == 6) co_chunks(std::integral_constant<int, 6>{}, I0{});
            else if (!want_den && nblk == 2) co_chunks(I2{}, I0{});
            else co_chunks(I0{}, I2{});
        }
    } else {
        const int nslab = (nblk + nb - 1) / nb;
        for (int s = 0; s < nslab; ++s) {
            const int b0 = s * nb;
            const int nbb = min(nb, nblk - b0);
            __syncthreads();  // every wave is done with the previous slab
            build_slab(b0, nbb);
            __syncthreads();
            // blocks in pairs: two independent hi and two lo chains, the
            // pair count fixed per call so that no branch separates the
            // matrix instructions; an odd last block runs alone
            auto blocks = [&](int bb, auto two_c) {
                constexpr bool TWO = decltype(two_c)::value;
                constexpr int kPlanes = NCC ? 32 : 16;  // planes per block (NCC: hi, then lo costs)
                f4 ah0 = {0.f, 0.f, 0.f, 0.f}, al0 = ah0, ah1 = ah0, al1 = ah0, am0 = ah0, am1 = ah0;
                const _Float16* p0 = plane0 + (size_t)(kPlanes * bb) * PS;
                const _Float16* p1 = p0 + (size_t)kPlanes * PS;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const h8 a0 = lds_h8<GW == 8>(p0 + a_off(c));
                    ah0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, whi[c], ah0, 0, 0, 0);
                    al0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, wlo[c], al0, 0, 0, 0);
                    if constexpr (NCC) {
                        const h8 m0 = lds_h8<GW == 8>(p0 + (size_t)16 * PS + a_off(c));
                        am0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(m0, whi[c], am0, 0, 0, 0);
                    }
                    if constexpr (TWO) {
                        const h8 a1 = lds_h8<GW == 8>(p1 + a_off(c));
                        ah1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, whi[c], ah1, 0, 0, 0);
                        al1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, wlo[c], al1, 0, 0, 0);
                        if constexpr (NCC) {
                            const h8 m1 = lds_h8<GW == 8>(p1 + (size_t)16 * PS + a_off(c));
                            am1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(m1, whi[c], am1, 0, 0, 0);
                        }
                    }
                }
                if constexpr (NCC) {
                    wta_block(gq * Q + 4 * (b0 + bb), (ah0 + al0) + am0);
                    if constexpr (TWO) wta_block(gq * Q + 4 * (b0 + bb + 1), (ah1 + al1) + am1);
                } else {
                    wta_block(gq * Q + 4 * (b0 + bb), ah0 + al0);
                    if constexpr (TWO) wta_block(gq * Q + 4 * (b0 + bb + 1), ah1 + al1);
                }
            };
            int bb = 0;
#pragma unroll 1
            for (; bb + 1 < nbb; bb += 2) blocks(bb, std::true_type{});
            if (bb < nbb) blocks(bb, std::false_type{});
        }
    }

    // ---- merge the four quarters of pixel n (lanes n, n+16, n+32, n+48) ----
    // quarter t covers disparity indices [t*Q, (t+1)*Q); the first minimum is
    // the lowest quarter holding the smallest value
    float wv = __shfl(best, n), wm = __shfl(cm, n), wp = __shfl(cp, n);
    int wk = __shfl(bi, n), wc = __shfl((int)need_cp, n), wt = 0;
    float left_last = kInf;   // last value of the quarter before the winner
    float prev_last = __shfl(prev, n);
    float qb[4], qs[4];       // each quarter's lowest and second-lowest value
    qb[0] = wv;
    qs[0] = __shfl(best2, n);
#pragma unroll
    for (int t = 1; t < 4; ++t) {
        const int src = n + 16 * t;
        const float tv = __shfl(best, src);
        qb[t] = tv;
        qs[t] = __shfl(best2, src);
        const int tk = __shfl(bi, src);
        const float tm = __shfl(cm, src), tp = __shfl(cp, src);
        const int tc = __shfl((int)need_cp, src);
        const bool take = tk >= 0 && tv < wv;
        if (take) {
            wv = tv; wk = tk; wm = tm; wp = tp; wc = tc; wt = t;
            left_last = prev_last;
        }
        prev_last = __shfl(prev, src);
    }
    // first value of the quarter after the winner
    const float right_first = __shfl(first_v, n + 16 * min(wt + 1, 3));
    // Near ties the weights' resolution cannot order.  Each weight below the
    // fp16 range of the split (w < 2^-38) is lost, so every numerator carries
    // an absolute error up to T * cap * 2^-25 (scaled units) besides its
    // relative 2^-22.  Where the lowest value is small enough that this
    // absolute error could exceed the 1e-5 relative tie zone, and the second
    // lowest lies within that error of it, the pixel is recomputed below in
    // double precision from the definition.
    float second = kInf;
#pragma unroll
    for (int t = 0; t < 4; ++t) second = fminf(second, t == wt ? qs[t] : qb[t]);
    constexpr float kTaps = (float)((2 * R + 1) * (2 * R + 1));
    const float abs_err = kTaps * scap * 0x1.0p-25f;
    const bool unsafe = pin && wv < kTaps * scap * 6e-3f &&
                        !(second - wv >= 4.0f * abs_err + 1e-6f * second);
    uint64_t recheck = __ballot(gq == 0 && unsafe);
    int fix_k = -1;
    float fix_ds = 0.0f;
    while (recheck) {
        const int n0 = __builtin_ctzll(recheck);
        recheck &= recheck - 1;
        int rk;
        float rds;
        recheck_pixel<R, CH, NCC>(job, s_L, s_R, LWB, RWB, grow0 + n0 / GW, gcol0 + n0 % GW, X0, Y0,
                             lane, rk, rds, nt);
        if (lane == n0) {
            fix_k = rk;
            fix_ds = rds;
        }
    }
    if (gq == 0 && pin) {
        float fm = wm, fp = wp;
        if (wk == wt * Q && wt > 0) fm = left_last;
        if (wc && wt < 3 && wk + 1 < D) fp = right_first;
        float ds = eq10_subpixel(g.dmin + wk, wk > 0 && wk < D - 1, fm, wv, fp);
        if (fix_k >= 0) {
            wk = fix_k;
            ds = fix_ds;
        }
        const size_t o = (size_t)py * g.W + px;
        if (disp) disp[o] = g.dmin + wk;
        if (sub) sub[o] = ds;
    }
    if constexpr (FEAT) {
        // merge the four quarters' sorted lists: 8 rounds, each taking the
        // smallest head key; keys are unique, so the lane holding it pops it
        uint32_t sel[8];
#pragma unroll
        for (int rnd = 0; rnd < 8; ++rnd) {
            uint32_t best_key = __shfl(tkey[0], n);
#pragma unroll
            for (int t = 1; t < 4; ++t) best_key = min(best_key, (uint32_t)__shfl(tkey[0], n + 16 * t));
            if (tkey[0] == best_key) {
#pragma unroll
                for (int i = 0; i < 7; ++i) tkey[i] = tkey[i + 1];
                tkey[7] = ~0u;
            }
            sel[rnd] = best_key;
        }
        // the pixel's four lanes share the conversions: quarter gq forms the
        // features of ranks 2gq and 2gq + 1 and stores its quarter of the
        // 64-byte record (dwords gq, 4 + gq, 8 + 2gq, 9 + 2gq)
        uint32_t s0 = sel[0], s1 = sel[1];
#pragma unroll
        for (int q = 1; q < 4; ++q)
            if (gq == q) {
                s0 = sel[2 * q];
                s1 = sel[2 * q + 1];
            }
        const float dn = (float)(D - 1);
        const uint32_t cw = bf16_bits(__uint_as_float(s0 & ~kmask) / g.tau) |
                            (bf16_bits(__uint_as_float(s1 & ~kmask) / g.tau) << 16);
        const uint32_t iw = bf16_bits((float)(int)(s0 & kmask) / dn) |
                            (bf16_bits((float)(int)(s1 & kmask) / dn) << 16);
        if (pin) {
            uint32_t* dst = reinterpret_cast<uint32_t*>(job.feat + ((size_t)py * g.W + px) * 32);
            dst[gq] = cw;
            dst[4 + gq] = iw;
            const uint32_t lb = gq == 0 ? bf16_bits((float)lp[0] / 255.0f) : 0u;
            *reinterpret_cast<uint2*>(dst + 8 + 2 * gq) = make_uint2(lb, 0u);
        }
    }
}

__device__ __forceinline__ void load_tables(const Tables& tb, int R, unsigned char* smem, int nthreads)
{
    float* s = reinterpret_cast<float*>(smem);
    for (int i = threadIdx.x; i < kLutN; i += nthreads) s[i] = i < 511 ? tb.gr[abs(i - 255)] : 0.0f;
    if (threadIdx.x < 32) s[kLutN + threadIdx.x] = (threadIdx.x <= R) ? tb.gs[threadIdx.x] : 0.0f;
}

// One workgroup per tile of one frame.
template <int R, int CH, int NW, bool CO>
__global__ __launch_bounds__(64 * NW) void k_fbs_mfma(TileJob job, Tables tb)
{
    extern __shared__ __align__(16) unsigned char smem[];
    load_tables(tb, R, smem, 64 * NW);
    __syncthreads();
    mfma_tile<R, CH, NW, false, CO>(job, blockIdx.x, blockIdx.y, smem, threadIdx.x);
}

// One workgroup per tile of one gray frame with the NCC cost (slab path).
template <int R, int NW>
__global__ __launch_bounds__(64 * NW) void k_fbs_mfma_ncc(TileJob job, Tables tb)
{
    extern __shared__ __align__(16) unsigned char smem[];
    load_tables(tb, R, smem, 64 * NW);
    __syncthreads();
    mfma_tile<R, 1, NW, false, false, true>(job, blockIdx.x, blockIdx.y, smem, threadIdx.x);
}

// One workgroup per tile of one gray frame, with the surrogate's features.
template <int R, int NW, bool CO>
// (8-wave tiles up to r = 4 are held to 128 registers: two workgroups per CU)
__global__ __launch_bounds__(64 * NW, NW == 8 && R <= 4 ? 4 : 1) void k_fbs_mfma_feat(TileJob job, Tables tb)
{
    extern __shared__ __align__(16) unsigned char smem[];
    load_tables(tb, R, smem, 64 * NW);
    __syncthreads();
    mfma_tile<R, 1, NW, true, CO>(job, blockIdx.x, blockIdx.y, smem, threadIdx.x);
}

// Persistent workgroups over a queue of (pair, tile) items of many frames of
// one class (radius, channels, waves, path and weight tables).  Every workgroup pops items until the queue is
// empty, so every wave reaches the end.
template <int R, int CH, int NW, bool CO>
__global__ __launch_bounds__(64 * NW) void k_fbs_mfma_batch(const BatchPair* __restrict__ pairs,
                                                            const int2* __restrict__ items,
                                                            int n_items, int* __restrict__ counter,
                                                            const uint8_t* const* __restrict__ Ls,
                                                            const uint8_t* const* __restrict__ Rs,
                                                            int32_t* const* __restrict__ disps,
                                                            float* const* __restrict__ subs,
                                                            Tables tb,
                                                            const int* __restrict__ n_dev,
                                                            int tiles_per_item)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_next[2];
    constexpr int kThreads = 64 * NW;
    // a queue whose length a previous kernel wrote on the device
    if (n_dev) n_items = __builtin_amdgcn_readfirstlane(*n_dev);
    load_tables(tb, R, smem, kThreads);   // the class shares its weight tables
    if (threadIdx.x == 0) s_next[0] = atomicAdd(counter, 1);
    int buf = 0;
    for (;;) {
        __syncthreads();   // s_next[buf] visible; every wave is done with the previous tile
        // uniform across the workgroup: keep the item, its pair and geometry
        // in scalar registers
        const int it = __builtin_amdgcn_readfirstlane(s_next[buf]);
        if (it >= n_items) break;
        // claim the next item now so the atomic's round trip overlaps this tile
        if (threadIdx.x == 0) s_next[buf ^ 1] = atomicAdd(counter, 1);
        buf ^= 1;
        // an item is tiles_per_item consecutive tiles of one pair (fewer at
        // the pair's end): the descriptor chain below is paid once for them
        const int2 w = items[it];
        const BatchPair& bp = pairs[w.x];
        TileJob job{bp.g, bp.scap, bp.nb, Ls[w.x], Rs[w.x], disps[w.x], subs[w.x], nullptr, nullptr};
        const int tend = min(w.y + tiles_per_item, bp.tiles_x * ((bp.g.H + kTileH - 1) / kTileH));
#pragma unroll 1
        for (int t = w.y; t < tend; ++t) {
            if (t > w.y) __syncthreads();  // every wave is done with the previous tile's LDS
            // an opaque copy of the thread index per tile keeps the compiler from
            // hoisting the tile's index arithmetic out of the loop (it would stay
            // live in registers across every tile)
            int tid;
            asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
            mfma_tile<R, CH, NW, false, CO>(job, t % bp.tiles_x, t / bp.tiles_x, smem, tid);
        }
    }
}

// One workgroup per (pair, tile) item of one class: the same tile code as
// the per-frame kernel, the item taken from blockIdx.
template <int R, int CH, int NW, bool CO>
__global__ __launch_bounds__(64 * NW) void k_fbs_mfma_items(const BatchPair* __restrict__ pairs,
                                                            const int2* __restrict__ items,
                                                            const uint8_t* const* __restrict__ Ls,
                                                            const uint8_t* const* __restrict__ Rs,
                                                            int32_t* const* __restrict__ disps,
                                                            float* const* __restrict__ subs,
                                                            Tables tb,
                                                            const int* __restrict__ n_dev)
{
    extern __shared__ __align__(16) unsigned char smem[];
    // a list whose length a previous kernel wrote on the device: the grid
    // covers its largest size and workgroups past the end leave at once
    if (n_dev && (int)blockIdx.x >= __builtin_amdgcn_readfirstlane(*n_dev)) return;
    load_tables(tb, R, smem, 64 * NW);   // the class shares its weight tables
    const int2 w = items[blockIdx.x];
    const BatchPair& bp = pairs[w.x];
    __syncthreads();
    TileJob job{bp.g, bp.scap, bp.nb, Ls[w.x], Rs[w.x], disps[w.x], subs[w.x], nullptr, nullptr};
    mfma_tile<R, CH, NW, false, CO>(job, w.y % bp.tiles_x, w.y / bp.tiles_x, smem, threadIdx.x);
}

constexpr int kLdsLimit = 160 * 1024;  // per workgroup and per CU on gfx950
constexpr int kMaxNb = 16;             // disparity blocks per slab
constexpr int kMaxR12 = 7;  // largest radius built with 12-wave workgroups

// deepest slab (>= 1) whose layout fits `budget` bytes
inline int deepest_nb(const Geom& g, int nw, int budget)
{
    const int nblk = (g.D + 15) >> 4;
    int nb = 1;
    while (nb < nblk && nb < kMaxNb && mfma_layout(g.r, g.C, g.D, nb + 1, nw).bytes <= budget) ++nb;
    return nb;
}

inline int max_nb(int r, int ch, int D, int nw, bool ncc = false)
{
    const int nblk = (D + 15) >> 4;
    int nb = 1;
    while (nb < nblk && nb < kMaxNb && mfma_layout(r, ch, D, nb + 1, nw, ncc).bytes <= kLdsLimit) ++nb;
    return nb;
}

// the chunk-outer path applies when one slab holds every disparity block
__host__ __device__ constexpr bool use_co(int D, int nb)
{
    return nb == ((D + 15) >> 4) && nb <= kCoMax;
}

template <int R, int CH, int NW>
hipError_t launch_frame(const TileJob& job, const Tables& t, hipStream_t s)
{
    const MfmaLayout lay = mfma_layout(R, CH, job.g.D, job.nb, NW);
    if (lay.bytes > kLdsLimit) return hipErrorInvalidConfiguration;
    dim3 grid((job.g.W + 2 * NW - 1) / (2 * NW), (job.g.H + kTileH - 1) / kTileH);
    if (use_co(job.g.D, job.nb))
        hipLaunchKernelGGL((k_fbs_mfma<R, CH, NW, true>), grid, dim3(64 * NW), lay.bytes, s, job, t);
    else
        hipLaunchKernelGGL((k_fbs_mfma<R, CH, NW, false>), grid, dim3(64 * NW), lay.bytes, s, job, t);
    return hipGetLastError();
}

// NCC frames: gray tiles of 4 waves, or of 8 up to r = kNccMaxR8 (at r = 10
// the 8-wave NCC tile spills: the weights and the cross terms of the cost
// build do not fit 256 registers together)
constexpr int kNccMaxR8 = 9;
template <int R, int CH, int NW>
struct NccLauncher {
    static hipError_t run(const TileJob& job, const Tables& t, hipStream_t s)
    {
        if constexpr (CH != 1 || NW == 12 || (NW == 8 && R > kNccMaxR8)) {
            return hipErrorInvalidValue;
        } else {
            const MfmaLayout lay = mfma_layout(R, 1, job.g.D, job.nb, NW, true);
            if (lay.bytes > kLdsLimit) return hipErrorInvalidConfiguration;
            dim3 grid((job.g.W + 2 * NW - 1) / (2 * NW), (job.g.H + kTileH - 1) / kTileH);
            hipLaunchKernelGGL((k_fbs_mfma_ncc<R, NW>), grid, dim3(64 * NW), lay.bytes, s, job, t);
            return hipGetLastError();
        }
    }
};

template <int R, int CH, int NW>
struct FeatOccupancy {
    static hipError_t run(int lds, bool co, int* blocks)
    {
        if constexpr (CH != 1 || NW == 4 || (NW == 12 && R > 6)) {
            return hipErrorInvalidValue;
        } else {
            if (co)
                return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    blocks, k_fbs_mfma_feat<R, NW, true>, 64 * NW, lds);
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                blocks, k_fbs_mfma_feat<R, NW, false>, 64 * NW, lds);
        }
    }
};

// FeatOccupancy through the (r, ch, nw) dispatcher: only gray tiles of 8 waves,
// or of 12 up to r = 6 (at r = 7 the 12-wave feature tile spills), exist
template <int R, int CH, int NW>
struct FeatOccupancyAny {
    static hipError_t run(int lds, bool co, int* blocks)
    {
        return FeatOccupancy<R, CH, NW>::run(lds, co, blocks);
    }
};

template <int R, int CH, int NW>
struct FeatLauncher {
    static hipError_t run(const TileJob& job, const Tables& t, hipStream_t s)
    {
        if constexpr (CH != 1 || NW == 4 || (NW == 12 && R > 6)) {
            return hipErrorInvalidValue;
        } else {
            const MfmaLayout lay = mfma_layout(R, 1, job.g.D, job.nb, NW);
            if (lay.bytes > kLdsLimit) return hipErrorInvalidConfiguration;
            dim3 grid((job.g.W + 2 * NW - 1) / (2 * NW), (job.g.H + kTileH - 1) / kTileH);
            if (use_co(job.g.D, job.nb))
                hipLaunchKernelGGL((k_fbs_mfma_feat<R, NW, true>), grid, dim3(64 * NW), lay.bytes,
                                   s, job, t);
            else
                hipLaunchKernelGGL((k_fbs_mfma_feat<R, NW, false>), grid, dim3(64 * NW), lay.bytes,
                                   s, job, t);
            return hipGetLastError();
        }
    }
};

template <int R, int CH, int NW, bool CO>
hipError_t launch_batch_co(const BatchClass& bc, hipStream_t s)
{
    if (bc.one_wg_per_item) {
        if (bc.n_items < 1) return hipSuccess;
        hipLaunchKernelGGL((k_fbs_mfma_items<R, CH, NW, CO>), dim3(bc.n_items), dim3(64 * NW),
                           bc.lds, s, bc.pairs, bc.items, bc.L, bc.R, bc.disp, bc.sub, bc.tb, bc.n_dev);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_fbs_mfma_batch<R, CH, NW, CO>), dim3(bc.grid), dim3(64 * NW), bc.lds, s,
                       bc.pairs, bc.items, bc.n_items, bc.counter, bc.L, bc.R, bc.disp, bc.sub,
                       bc.tb, bc.n_dev, std::max(1, bc.tiles_per_item));
    return hipGetLastError();
}

template <int R, int CH, int NW>
hipError_t launch_batch(const BatchClass& bc, hipStream_t s)
{
    if (bc.lds <= 0 || bc.lds > kLdsLimit) return hipErrorInvalidConfiguration;
    return bc.co ? launch_batch_co<R, CH, NW, true>(bc, s) : launch_batch_co<R, CH, NW, false>(bc, s);
}

// (R, CH, NW) dispatch; F<R, CH, NW>::run(args...)
template <template <int, int, int> class F, int CH, int NW, typename... A>
hipError_t dispatch_r(int r, A&&... a)
{
    switch (r) {
    case 1: return F<1, CH, NW>::run(a...);
    case 2: return F<2, CH, NW>::run(a...);
    case 3: return F<3, CH, NW>::run(a...);
    case 4: return F<4, CH, NW>::run(a...);
    case 5: return F<5, CH, NW>::run(a...);
    case 6: return F<6, CH, NW>::run(a...);
    case 7: return F<7, CH, NW>::run(a...);
    default: break;
    }
    // 12-wave workgroups cap a wave at 168 registers: above r = 7 the tile
    // spills, so those are not built
    if constexpr (NW != 12) {
        switch (r) {
        case 8: return F<8, CH, NW>::run(a...);
        case 9: return F<9, CH, NW>::run(a...);
        case 10: return F<10, CH, NW>::run(a...);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

template <template <int, int, int> class F, typename... A>
hipError_t dispatch(int r, int ch, int nw, A&&... a)
{
    if (ch == 3) {
        if (nw == 4) return dispatch_r<F, 3, 4>(r, a...);
        if (nw == 12) return dispatch_r<F, 3, 12>(r, a...);
        return dispatch_r<F, 3, 8>(r, a...);
    }
    if (nw == 4) return dispatch_r<F, 1, 4>(r, a...);
    if (nw == 12) return dispatch_r<F, 1, 12>(r, a...);
    return dispatch_r<F, 1, 8>(r, a...);
}

template <int R, int CH, int NW>
struct FrameLauncher {
    static hipError_t run(const TileJob& j, const Tables& t, hipStream_t s)
    {
        return launch_frame<R, CH, NW>(j, t, s);
    }
};

template <int R, int CH, int NW>
struct BatchLauncher {
    static hipError_t run(const BatchClass& bc, hipStream_t s) { return launch_batch<R, CH, NW>(bc, s); }
};

template <int R, int CH, int NW>
struct FrameOccupancy {
    static hipError_t run(int lds, bool co, int* blocks)
    {
        if (co)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_fbs_mfma<R, CH, NW, true>,
                                                                64 * NW, lds);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_fbs_mfma<R, CH, NW, false>,
                                                            64 * NW, lds);
    }
};

template <int R, int CH, int NW>
struct BatchOccupancy {
    static hipError_t run(int lds, bool co, int* blocks)
    {
        if (co)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                blocks, k_fbs_mfma_batch<R, CH, NW, true>, 64 * NW, lds);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            blocks, k_fbs_mfma_batch<R, CH, NW, false>, 64 * NW, lds);
    }
};

// Cap as the kernel sees it: tau (gray) or 3 tau (RGB), which must be an
// exact fp16 value so every cost is exact in the A operand.
inline bool scaled_cap(const Geom& g, float* out)
{
    const double c = (g.C == 3 ? 3.0 : 1.0) * (double)g.tau;
    if (!(c > 0.0) || c > 2048.0) return false;
    const _Float16 h = (_Float16)(float)c;
    if ((double)(float)h != c) return false;
    *out = (float)c;
    return true;
}

template <template <int, int, int> class Occ>
bool pick_cfg(const Geom& g, const int* cands, int ncands, MfmaCfg* out)
{
    const int nblk = (g.D + 15) >> 4;
    int best = -1;
    bool best_co = false;
    for (int i = 0; i < ncands; ++i) {
        const int cand = cands[i];
        if (!mfma_nw_valid(g, cand)) continue;
        int blocks = 0, nb = 0;
        bool co = false;
        if (nblk <= kCoMax && mfma_layout(g.r, g.C, g.D, nblk, cand).bytes <= kLdsLimit &&
            dispatch<Occ>(g.r, g.C, cand, mfma_layout(g.r, g.C, g.D, nblk, cand).bytes, true,
                          &blocks) == hipSuccess &&
            blocks >= 1) {
            nb = nblk;
            co = true;
        } else {
            blocks = 0;
            if (dispatch<Occ>(g.r, g.C, cand, mfma_layout(g.r, g.C, g.D, 1, cand).bytes, false,
                              &blocks) != hipSuccess ||
                blocks < 1)
                continue;
            nb = deepest_nb(g, cand, kLdsLimit / blocks);
            if (use_co(g.D, nb)) nb = std::max(1, nb - 1);   // that path was not chosen above
        }
        const int waves = blocks * cand;
        if (waves > best || (waves == best && co && !best_co)) {
            best = waves;
            best_co = co;
            *out = MfmaCfg{cand, nb};
        }
    }
    return best > 0;
}

}  // namespace
}  // namespace fbs
