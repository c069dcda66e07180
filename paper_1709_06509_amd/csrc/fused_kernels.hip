// Several consecutive half-steps of one scale in one launch, for scales small enough that a
// launch per half-step is bound by launch latency rather than by memory.
//
// The scale is cut into interior tiles.  A workgroup loads its tile plus a halo of h
// pixels on every side (clipped to the image) into LDS: the cost and the four incoming
// message volumes of every region pixel (and the freeze state).  It then runs h
// half-steps on the region with a workgroup barrier between them, and writes back the
// interior pixels only.  Half-step t reads, for every updated pixel, values that were
// final after half-step t-1 on the pixel and its four neighbours, so the set of region
// pixels whose values are exact shrinks by at most one pixel per half-step from the
// region's cut edges (image borders are exact: nothing lies beyond them).  After h
// half-steps the interior is exact, and equal bit for bit to h launches of k_halfstep.
//
// Per-pixel arithmetic is the same as the per-launch kernel (transform, freeze rule);
// only the storage differs: LDS holds the region row-major, [pixel][Dp] per volume.
#include <cstdlib>
#include <mutex>
#include <vector>

#include "bp_device.h"

namespace bpst {
namespace {

constexpr int kFusedThreads = 1024;

struct Region {
    int rx0, ry0, RW, RH;  // region origin and size (clipped to the image)
    int ix0, iy0, IW, IH;  // interior origin and size
};

__device__ __forceinline__ Region region_of(const FusedArgs& a)
{
    Region g;
    const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    g.ix0 = tx * a.TW;
    g.iy0 = ty * a.TH;
    const int ix1 = min(g.ix0 + a.TW, a.lv.W), iy1 = min(g.iy0 + a.TH, a.lv.H);
    g.IW = ix1 - g.ix0;
    g.IH = iy1 - g.iy0;
    g.rx0 = max(g.ix0 - a.halo, 0);
    g.ry0 = max(g.iy0 - a.halo, 0);
    g.RW = min(ix1 + a.halo, a.lv.W) - g.rx0;
    g.RH = min(iy1 + a.halo, a.lv.H) - g.ry0;
    return g;
}

template <int G, int MODE, bool NARROW>
__global__ __launch_bounds__(kFusedThreads) void k_fused(FusedArgs a)
{
    constexpr int Dp = 8 * G;
    extern __shared__ int4 lds4[];
    const Region g = region_of(a);
    const int W = a.lv.W, H = a.lv.H, Wh = a.lv.Wh;
    const long long cap = a.rmax;  // region pixels the LDS was sized for
    int* wsum = reinterpret_cast<int*>(lds4);           // per-wave counts (kFusedThreads / 64 of 64)
    int16_t* lc = reinterpret_cast<int16_t*>(lds4 + 16);  // after 256 bytes
    int16_t* lm = lc + cap * Dp;   // volume k at lm + k * cap * Dp
    uint8_t* lsa = reinterpret_cast<uint8_t*>(lm + 4 * cap * Dp);
    uint8_t* lsb = lsa + cap;
    int* llist = reinterpret_cast<int*>(lsb + ((cap + 3) & ~3LL));  // active pixels of a half-step
    const int R = g.RW * g.RH;

    // 0. Under the freeze rule, once pixels can be frozen (t0 >= 2): read the region's freeze
    //    state first.  A frozen pixel stays frozen for the rest of the scale, so a region
    //    with no active pixel cannot change during these half-steps: the workgroup leaves
    //    without loading anything else or writing anything back.  (The vote goes through the
    //    per-wave words of the dynamic LDS: a library reduction would add static LDS, which
    //    the largest regions have no room for.)
    const bool have_state = MODE == 1 && a.t0 >= 2;
    if (have_state) {
        int any = 0;
        for (int r = threadIdx.x; r < R; r += blockDim.x) {
            const int ry = r / g.RW, rx = r - ry * g.RW;
            const long long slot = slot_of(g.rx0 + rx, g.ry0 + ry, Wh);
            const uint8_t sa = a.state_a[slot];
            lsa[r] = sa;
            lsb[r] = a.state_b[slot];
            any |= sa != 0;
        }
        const unsigned long long vote = __ballot(any != 0);
        if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = vote != 0ull ? 1 : 0;
        __syncthreads();
        int live = 0;
        for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) live |= wsum[w];
        if (live == 0) return;  // the same for every thread of the workgroup
        // wsum is written again only after the barrier that ends the region load
    }

    // 1. load the region: cost, incoming messages (own, parent's or zero), and (before t0 = 2)
    //    the initial freeze state.  A thread takes two elements per round and issues all their
    //    global loads before any LDS store, so the round costs one memory latency, not two.
    //    Every load reads a valid address (the region's first pixel for a lane past the end,
    //    the pixel's own slot for a missing neighbour) and is masked afterwards: a load under
    //    a per-lane branch made the compiler wait for the first element's loads before it
    //    issued the second's.
    constexpr int kU = 2;
    for (int e0 = threadIdx.x; e0 < R * G; e0 += kU * blockDim.x) {
        int4 cv[kU], mv[kU][4];
        int rv[kU], keep[kU][4];
        const int4* pc[kU];
        const int4* pm[kU][4];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = e0 + u * (int)blockDim.x;
            const bool in = e < R * G;
            const int ee = in ? e : 0;
            const int r = ee / G, lane = ee - r * G;
            const int ry = r / g.RW, rx = r - ry * g.RW;
            const int x = g.rx0 + rx, y = g.ry0 + ry;
            const long long slot = slot_of(x, y, Wh);
            const int d0 = lane * 8;
            rv[u] = in ? r : -1;
            pc[u] = reinterpret_cast<const int4*>(a.cost + slot * Dp + d0);
            const bool has[4] = {x > 0, x < W - 1, y > 0, y < H - 1};
            // the source picks the volumes and the slot (no branch); zero messages read this
            // scale's own volumes and keep nothing
            const bool parent = a.source == kSrcParent;
            const int px = x >> 1, py = y >> 1;
            const bool phas[4] = {px > 0, px < a.plv.W - 1, py > 0, py < a.plv.H - 1};
            const int16_t* src = parent ? a.pmsgs : a.msgs;
            const long long vol = parent ? a.pvol : a.vol;
            const long long sl = parent ? slot_of(px, py, a.plv.Wh) : slot;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                pm[u][k] = reinterpret_cast<const int4*>(src + k * vol + sl * Dp + d0);
                keep[u][k] = a.source != kSrcZero && has[k] && (!parent || phas[k]) ? -1 : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            cv[u] = *pc[u];
#pragma unroll
            for (int k = 0; k < 4; ++k) mv[u][k] = *pm[u][k];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int r = rv[u];
            if (r < 0) continue;
            const int d0 = (e0 + u * (int)blockDim.x - r * G) * 8;
            *reinterpret_cast<int4*>(lc + (long long)r * Dp + d0) = cv[u];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int m = keep[u][k];
                *reinterpret_cast<int4*>(lm + k * cap * Dp + (long long)r * Dp + d0) =
                    make_int4(mv[u][k].x & m, mv[u][k].y & m, mv[u][k].z & m, mv[u][k].w & m);
            }
            if (MODE == 1 && !have_state && d0 == 0) {
                lsa[r] = 1;  // every pixel is active before its third half-step
                lsb[r] = 0;
            }
        }
    }
    __syncthreads();

    // 2. the half-steps, one colour each.  Thread e handles lane e % G of pixel e / G of the
    //    colour's row-major list (RWc a row), and every blockDim.x / G pixels after it; the
    //    (row, index) pair advances by a fixed step instead of being divided out each time.
    //    On the narrow path the pixel's lanes split its two message pairs (NarrowLane).
    const int RWc = (g.RW + 1) >> 1;  // pixels of one colour in a region row (at most)
    const int npix = g.RH * RWc;
    const int lane = threadIdx.x & (G - 1);
    constexpr int NV = NARROW ? NarrowLane<G>::NV : 1;  // label vectors a lane reads per volume
    constexpr int GL = NARROW ? NarrowLane<G>::GL : G;  // lanes that share one message
    const NarrowLane<G> nl(lane);
    const int d0 = NARROW ? nl.d0 : lane * 8;
    const bool hi = NARROW && G > 1 && nl.q != 0;  // the lane computes messages 2 and 3
    int4 lmask[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) lmask[v] = label_mask(d0 + 8 * v, a.D);
    const bool pad = a.D < Dp;
    const int pstep = blockDim.x / G, step_ry = pstep / RWc, step_i = pstep - step_ry * RWc;
    const int p_first = threadIdx.x / G;
    const int ry_first = p_first / RWc, i_first = p_first - ry_first * RWc;
    const int wave = threadIdx.x >> 6, nwaves = (blockDim.x + 63) >> 6;
    for (int s = 0; s < a.nsteps; ++s) {
        const int t = a.t0 + s, colour = t & 1;
        const bool check = MODE == 1 && t >= 2;
        // under the freeze rule, list the active pixels of this colour first (a ballot mask
        // per wave, ranks from mbcnt and the counts of the waves before), so that the update
        // loop below runs over active pixels only.  That pays where a compute unit holds more
        // waves than it has SIMDs (packing the active pixels onto fewer waves shortens the
        // longest SIMD queue); with a wave per SIMD or fewer it only adds two barriers, and
        // a wave whose pixels are all frozen skips the update anyway.
        const bool listed = check && a.compact;
        int count = npix;
        if (listed) {
            int total = 0;
            int ry = ry_first, i = i_first;
            for (int p0 = 0; p0 < npix; p0 += pstep) {
                const int p = p0 + p_first;
                bool active = false;
                int code = 0;
                if (p < npix && lane == 0) {
                    const int rx = 2 * i + ((colour ^ (g.rx0 + g.ry0 + ry)) & 1);
                    active = rx < g.RW && lsa[ry * g.RW + rx] != 0;
                    code = (ry << 16) | i;
                }
                const unsigned long long m = __ballot(active);
                const int rank =
                    (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                if ((threadIdx.x & 63) == 0) wsum[wave] = __popcll(m);
                __syncthreads();
                int base = 0, sum = 0;
                for (int w = 0; w < nwaves; ++w) {
                    base += w < wave ? wsum[w] : 0;
                    sum += wsum[w];
                }
                if (active) llist[total + base + rank] = code;
                total += sum;
                __syncthreads();
                i += step_i;
                ry += step_ry;
                if (i >= RWc) {
                    i -= RWc;
                    ++ry;
                }
            }
            count = total;
        }
        int ry = ry_first, i = i_first;
        for (int p = p_first; p < count; p += pstep) {
            if (listed) {
                const int code = llist[p];
                ry = code >> 16;
                i = code & 0xffff;
            }
            const int y = g.ry0 + ry;
            const int rx = 2 * i + ((colour ^ (g.rx0 + y)) & 1);
            const int x = g.rx0 + rx;
            const bool valid = rx < g.RW;
            const int r = ry * g.RW + rx;
            const bool has[4] = {x > 0, x < W - 1, y > 0, y < H - 1};
            const bool inreg[4] = {rx > 0, rx < g.RW - 1, ry > 0, ry < g.RH - 1};
            const int nbr[4] = {r - 1, r + 1, r - g.RW, r + g.RW};
            // incoming volumes in the lane's role order (identity unless the lane computes the
            // second pair on the narrow path): own pair first, then the other pair
            bool hr[4], ir[4];
            int nr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                hr[q] = hi ? has[(q + 2) & 3] : has[q];
                ir[q] = hi ? inreg[(q + 2) & 3] : inreg[q];
                nr[q] = hi ? nbr[(q + 2) & 3] : nbr[q];
            }
            // every LDS read is issued unconditionally from a valid address, so the loads of a
            // pixel overlap.  No mask is needed for a side with no neighbour: the region load
            // stored zeros there, and only that neighbour would ever write the slot.  (Zeroing
            // the loaded value instead made the compiler wait for each load in its own branch.)
            const long long rr = valid ? r : 0;
            int4 c4[NV], mp[4][NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) c4[v] = *reinterpret_cast<const int4*>(lc + rr * Dp + d0 + 8 * v);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    mp[q][v] = *reinterpret_cast<const int4*>(lm + role_msg(hi, q) * cap * Dp + rr * Dp + d0 + 8 * v);
            const bool act = valid && (!check || lsa[rr] != 0);
            const int sb = lsb[rr];  // the pixel's count of unchanged half-steps, read with the rest
            if (check && !listed && __ballot(act) == 0ull) {
                // every pixel of the wave is frozen (wave-uniform: no lane exchange is skipped
                // by part of a pixel's lanes)
                i += step_i;
                ry += step_ry;
                if (i >= RWc) {
                    i -= RWc;
                    ++ry;
                }
                continue;
            }
            int4 out[4][NV];
            if constexpr (NARROW) {
                narrow_update<G>(nl, c4, mp, a.D, pad, (unsigned)a.lambda, (unsigned)a.capv, out);
            } else {
                int Hs[8];
                unpack8u(c4[0], Hs);
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    Hs[j] = (d0 + j < a.D) ? Hs[j] + msg_at(mp[0][0], j) + msg_at(mp[1][0], j) +
                                                 msg_at(mp[2][0], j) + msg_at(mp[3][0], j)
                                           : kBig;
#pragma unroll
                for (int k = 0; k < 4; k += 2) {
                    int ha[8], hb[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        ha[j] = Hs[j] - msg_at(mp[k][0], j);
                        hb[j] = Hs[j] - msg_at(mp[k + 1][0], j);
                    }
                    transform2<G>(ha, hb, a.lambda, a.capv, lane, out[k][0], out[k + 1][0]);
                }
            }
            // The messages this lane sends: all four, or with the pairs split the two of its
            // pair (k = 2q + e; out[e] holds them).  Under the freeze rule the receivers'
            // previous values are read here, after the transform, so that they do not hold
            // registers through it.
            constexpr int NK = NARROW && G > 1 ? 2 : 4;
            int4 op[NK][NV];
#pragma unroll
            for (int e = 0; e < NK; ++e) {
                const bool tk = valid && hr[e] && ir[e];
#pragma unroll
                for (int v = 0; v < NV; ++v)  // (read whether or not compared: a valid address, no branch)
                    op[e][v] = *reinterpret_cast<const int4*>(lm + (role_msg(hi, e) ^ 1) * cap * Dp +
                                                              (tk ? (long long)nr[e] : rr) * Dp + d0 + 8 * v);
            }
            // every decision first, then every store (arithmetic after a store would wait for it)
            bool all_eq = true;
            bool stf[NK];
#pragma unroll
            for (int e = 0; e < NK; ++e) {
                bool store = act && hr[e] && ir[e];
                if (check) {
                    // a receiver outside the region is not held: its compare is skipped, which
                    // only affects pixels on the region's cut edge (never exact past step 0)
                    bool same = true;
#pragma unroll
                    for (int v = 0; v < NV; ++v) same = same && same_labels(op[e][v], out[e][v], lmask[v]);
                    const int eq = group_min<GL>(same ? 1 : 0);  // the GL lanes of the message
                    if (store && !eq) all_eq = false;
                    if (eq) store = false;
                }
                stf[e] = store;
            }
            // the freeze state needs all four messages: combine the pixel's lanes
            if (NARROW && G > 1 && check) all_eq = group_min<G>(all_eq ? 1 : 0) != 0;
            const int st = all_eq ? sb + 1 : 0;
#pragma unroll
            for (int e = 0; e < NK; ++e)
                if (stf[e]) {
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        *reinterpret_cast<int4*>(lm + (role_msg(hi, e) ^ 1) * cap * Dp + (long long)nr[e] * Dp + d0 +
                                                 8 * v) = out[e][v];
                }
            if (MODE == 1 && act && lane == 0) {
                if (t < 2) {
                    lsa[r] = 1;
                    lsb[r] = 0;
                } else {
                    lsb[r] = (uint8_t)st;
                    if (2 * st >= a.K) lsa[r] = 0;
                }
            }
            i += step_i;
            ry += step_ry;
            if (i >= RWc) {
                i -= RWc;
                ++ry;
            }
        }
        __syncthreads();
    }

    // 3. write back the interior: incoming messages on existing sides, and the state when
    //    later half-steps of this scale follow
    for (int e = threadIdx.x; e < g.IW * g.IH * G; e += blockDim.x) {
        const int q = e / G, lane = e - q * G;
        const int iy = q / g.IW, ix = q - iy * g.IW;
        const int x = g.ix0 + ix, y = g.iy0 + iy;
        const int r = (y - g.ry0) * g.RW + (x - g.rx0);
        const long long slot = slot_of(x, y, Wh);
        const int d0 = lane * 8;
        const bool has[4] = {x > 0, x < W - 1, y > 0, y < H - 1};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (has[k])
                *reinterpret_cast<int4*>(a.msgs + k * a.vol + slot * Dp + d0) =
                    *reinterpret_cast<const int4*>(lm + k * cap * Dp + (long long)r * Dp + d0);
        if (MODE == 1 && lane == 0 && a.keep_state) {
            a.state_a[slot] = lsa[r];
            a.state_b[slot] = lsb[r];
        }
    }
}

}  // namespace

size_t fused_lds_bytes(int G, long long rmax)
{
    const long long Dp = 8LL * G;
    // cost and 4 volumes, two state bytes (padded to 4) and an int of the active list per pixel
    return (size_t)(256 + 5 * rmax * Dp * 2 + ((2 * rmax + 3) & ~3LL) + 4 * rmax + 15) / 16 * 16;
}

int fused_threads(int G, long long rmax)
{
    const long long lanes = (rmax + 1) / 2 * G;  // one colour of the region, G lanes a pixel
    long long t = (lanes + 63) / 64 * 64;
    return (int)(t < 64 ? 64 : (t > kFusedThreads ? kFusedThreads : t));
}

// Estimated device time (us) of `iters` half-steps on scale lv: one launch per half-step,
// or fused launches of `steps` half-steps on TW x TH interior tiles.  The constants are
// measured on MI355X: a small launch costs about 4.5 us and a streaming one moves about
// 5 TB/s; a fused launch costs about 4 us plus its region loads and interior stores at
// 5 TB/s, and each of its half-steps about 0.9 us per 256 lanes a compute unit updates.
double per_launch_us(const Level& lv, int G, int iters)
{
    const double bytes = (double)lv.slots() / 2 * 8 * G * 2 * 9;  // one colour: cost, 4 in, 4 out
    const double t = bytes / 5.0e6;
    return iters * (t > 4.5 ? t : 4.5);
}

double fused_us(const Level& lv, int G, int iters, int steps, int TW, int TH)
{
    const int h = steps;
    const double rw = (double)(TW + 2 * h < lv.W ? TW + 2 * h : lv.W);
    const double rh = (double)(TH + 2 * h < lv.H ? TH + 2 * h : lv.H);
    const long long tiles = (long long)((lv.W + TW - 1) / TW) * ((lv.H + TH - 1) / TH);
    const long long lds = (long long)fused_lds_bytes(G, (long long)(TW + 2 * h) * (TH + 2 * h));
    long long per_cu = kFusedLdsBytes / (lds > 0 ? lds : 1);
    const long long threads = fused_threads(G, (long long)(TW + 2 * h) * (TH + 2 * h));
    const long long by_threads = 2048 / threads;
    if (per_cu > by_threads) per_cu = by_threads;
    if (per_cu < 1) per_cu = 1;
    const long long resident = 256 * per_cu;
    const double rounds = (double)((tiles + resident - 1) / resident);
    const long long in_round = tiles < resident ? tiles : resident;
    const double lanes_per_cu = (double)((in_round + 255) / 256) * (rw * rh / 2.0) * G;  // on a busy CU
    const double pass = 0.9 * (lanes_per_cu > 256.0 ? lanes_per_cu / 256.0 : 1.0);
    const double dp2 = 8.0 * G * 2;
    const double traffic = ((double)tiles * rw * rh * dp2 * 5 + (double)lv.W * lv.H * dp2 * 4) / 5.0e6;
    const int launches = (iters + steps - 1) / steps;
    return launches * (rounds * (4.0 + steps * pass) + traffic);
}

bool fused_narrow_pays(int G, long long rmax)
{
    (void)G;
    (void)rmax;
    return true;
}

namespace {
bool fused_search(const Level& lv, int G, int iters, int* steps, int* TW, int* TH, long long* rmax);
}

bool fused_geometry(const Level& lv, int G, int iters, int* steps, int* TW, int* TH, long long* rmax)
{
    // the search is memoised per (scale size, lanes, half-steps): solves repeat shapes
    struct Entry {
        int W, H, G, iters, ok, steps, TW, TH;
        long long rmax;
    };
    thread_local std::vector<Entry> memo;
    for (const Entry& e : memo)
        if (e.W == lv.W && e.H == lv.H && e.G == G && e.iters == iters) {
            *steps = e.steps;
            *TW = e.TW;
            *TH = e.TH;
            *rmax = e.rmax;
            return e.ok != 0;
        }
    Entry e{lv.W, lv.H, G, iters, 0, 0, 0, 0, 0};
    e.ok = fused_search(lv, G, iters, &e.steps, &e.TW, &e.TH, &e.rmax) ? 1 : 0;
    if (memo.size() > 256) memo.clear();
    memo.push_back(e);
    *steps = e.steps;
    *TW = e.TW;
    *TH = e.TH;
    *rmax = e.rmax;
    return e.ok != 0;
}

namespace {
bool fused_search(const Level& lv, int G, int iters, int* steps, int* TW, int* TH, long long* rmax)
{
    const long long per = 5LL * 8 * G * 2 + 6;                       // LDS bytes per region pixel
    const long long cap = (long long)(kFusedLdsBytes - 256 - 32) / per;  // wave counts, alignment
    double best = per_launch_us(lv, G, iters);
    bool found = false;
    for (int h = 1; h <= iters && h <= 12; ++h) {
        const int chunks = (iters + h - 1) / h;
        const int hs = (iters + chunks - 1) / chunks;  // equal chunks: the last is not shorter by much
        if (hs != h) continue;
        for (int tw = 2; tw <= lv.W + 1 && tw <= 256; tw += (tw < 16 ? 1 : 4)) {
            for (int th = 2; th <= lv.H + 1 && th <= 256; th += (th < 16 ? 1 : 4)) {
                const int ew = tw < lv.W ? tw : lv.W, eh = th < lv.H ? th : lv.H;
                if ((long long)(ew + 2 * h) * (eh + 2 * h) > cap) break;
                const double t = fused_us(lv, G, iters, h, ew, eh);
                if (t < best) {
                    best = t;
                    found = true;
                    *steps = h;
                    *TW = ew;
                    *TH = eh;
                    *rmax = (long long)(ew + 2 * h) * (eh + 2 * h);
                }
                if (th >= lv.H) break;
            }
            if (tw >= lv.W) break;
        }
    }
    return found;
}
}  // namespace

// Any tile: the widest interior whose region fits (used when fused launches are forced).
bool fused_geometry_max(const Level& lv, int G, int steps, int* TW, int* TH, long long* rmax)
{
    const long long per = 5LL * 8 * G * 2 + 6;
    const long long cap = (long long)(kFusedLdsBytes - 256 - 32) / per;
    const int h = steps;
    long long best_tiles = -1;
    for (int tw = 1; tw <= lv.W; ++tw) {
        if ((long long)(tw + 2 * h) * (1 + 2 * h) > cap) break;
        int th = (int)(cap / (tw + 2 * h)) - 2 * h;
        if (th > lv.H) th = lv.H;
        if (th < 1) break;
        const long long tiles = (long long)((lv.W + tw - 1) / tw) * ((lv.H + th - 1) / th);
        if (best_tiles < 0 || tiles < best_tiles) {
            best_tiles = tiles;
            *TW = tw;
            *TH = th;
            *rmax = (long long)(tw + 2 * h) * (th + 2 * h);
        }
    }
    return best_tiles > 0;
}

// Largest static LDS of the fused kernels (bytes): a launch needs it on top of its dynamic
// LDS, and the two together must fit the compute unit's 160 KB.
static size_t g_fused_static_lds = 0;

template <int G, int MODE>
void set_lds_attr()
{
    const void* fns[2] = {(const void*)k_fused<G, MODE, false>, (const void*)k_fused<G, MODE, true>};
    for (const void* fn : fns) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kFusedLdsBytes);
        hipFuncAttributes attr{};
        if (hipFuncGetAttributes(&attr, fn) == hipSuccess && attr.sharedSizeBytes > g_fused_static_lds)
            g_fused_static_lds = attr.sharedSizeBytes;
    }
}

void fused_prepare()
{
    // once per device (the attribute belongs to the device's copy of each kernel)
    static std::mutex mu;
    static std::vector<bool> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return;
    }
    std::lock_guard<std::mutex> lock(mu);
    if ((size_t)dev < done.size() && done[dev]) return;
    set_lds_attr<1, 0>(); set_lds_attr<1, 1>(); set_lds_attr<2, 0>(); set_lds_attr<2, 1>();
    set_lds_attr<4, 0>(); set_lds_attr<4, 1>(); set_lds_attr<8, 0>(); set_lds_attr<8, 1>();
    (void)hipGetLastError();
    if ((size_t)dev >= done.size()) done.resize(dev + 1, false);
    done[dev] = true;
}

hipError_t launch_fused(const FusedArgs& a, hipStream_t st)
{
    const int tiles = a.tiles_x * ((a.lv.H + a.TH - 1) / a.TH);
    const size_t lds = fused_lds_bytes(a.G, a.rmax);
    if (a.halo != a.nsteps || a.nsteps < 1) return hipErrorInvalidValue;
    if (a.narrow && (a.capv < 0 || a.capv > kNarrowCap)) return hipErrorInvalidValue;
    fused_prepare();
    if (lds + g_fused_static_lds > (size_t)kFusedLdsBytes) return hipErrorInvalidValue;
    const dim3 grid((unsigned)tiles), block((unsigned)fused_threads(a.G, a.rmax));
    // list active pixels only where a compute unit holds more than a wave per SIMD (a
    // workgroup per compute unit while the tiles fit the 256 units)
    FusedArgs b = a;
    b.compact = (long long)((tiles + 255) / 256) * ((block.x + 63) / 64) > 4 ? 1 : 0;
    if (a.compact == 0 || a.compact == 1) b.compact = a.compact;  // test hook: listing forced off / on
#define BPST_FUSED_G(GG)                                                                        \
    case GG:                                                                                    \
        if (a.narrow) {                                                                         \
            if (a.mode == 1) hipLaunchKernelGGL((k_fused<GG, 1, true>), grid, block, lds, st, b);  \
            else hipLaunchKernelGGL((k_fused<GG, 0, true>), grid, block, lds, st, b);              \
        } else {                                                                                \
            if (a.mode == 1) hipLaunchKernelGGL((k_fused<GG, 1, false>), grid, block, lds, st, b); \
            else hipLaunchKernelGGL((k_fused<GG, 0, false>), grid, block, lds, st, b);             \
        }                                                                                       \
        break;
    switch (b.G) {
        BPST_FUSED_G(1) BPST_FUSED_G(2) BPST_FUSED_G(4) BPST_FUSED_G(8)
        default: return hipErrorInvalidValue;
    }
#undef BPST_FUSED_G
    return hipGetLastError();
}

}  // namespace bpst
