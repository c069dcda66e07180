// Per-launch kernels of the hierarchical min-sum solve and their launchers.  The
// per-pixel arithmetic lives in bp_device.h, shared with the batched persistent solve.
#include "bp_device.h"

namespace bpst {
namespace {

__global__ void k_zero_stats(DevStats* s)
{
    int* w = reinterpret_cast<int*>(s);
    const int n = (int)(sizeof(DevStats) / sizeof(int));
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0;
}

template <int G, bool VEC>
__global__ __launch_bounds__(kThreads) void k_prep_level0(const int16_t* __restrict__ user,
                                                           int16_t* __restrict__ c0, Level lv, int D)
{
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const long long gi = t / G;
    const int lane = (int)(t & (G - 1));
    if (gi >= lv.slots()) return;
    ColourPix p = any_pixel(gi, lv);
    if (!p.valid) return;
    const int d0 = lane * 8;
    const int16_t* src = user + ((long long)p.y * lv.W + p.x) * D + d0;
    int v[8];
    if (VEC) {
        if (d0 < D) unpack8(*reinterpret_cast<const int4*>(src), v);
        else for (int j = 0; j < 8; ++j) v[j] = 0;
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (d0 + j < D) ? (int)src[j] : 0;
    }
    *reinterpret_cast<int4*>(c0 + gi * (8 * G) + d0) = finest_internal<G>(v, d0, D);
}

template <int G>
__global__ __launch_bounds__(kThreads) void k_pyramid(const int16_t* __restrict__ fine, Level lf,
                                                       int16_t* __restrict__ coarse, Level lc, int D)
{
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const long long gi = t / G;
    const int lane = (int)(t & (G - 1));
    const bool in = gi < lc.slots();
    ColourPix p = any_pixel(in ? gi : 0, lc);
    const bool valid = in && p.valid;
    const int d0 = lane * 8;
    int s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                int x = 2 * p.x + a, y = 2 * p.y + b;
                if (x < lf.W && y < lf.H) {
                    int v[8];
                    unpack8u(*reinterpret_cast<const int4*>(fine + slot_of(x, y, lf.Wh) * (8 * G) + d0), v);
#pragma unroll
                    for (int j = 0; j < 8; ++j) s[j] += v[j];
                }
            }
    }
    int mn = kBig;
#pragma unroll
    for (int j = 0; j < 8; ++j) if (d0 + j < D) mn = min(mn, s[j]);
    mn = group_min<G>(mn);
    int o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (d0 + j < D) ? min(s[j] - mn, 32767) : 0;
    if (valid) *reinterpret_cast<int4*>(coarse + gi * (8 * G) + d0) = pack8(o);
}

template <int G, bool VEC>
__global__ __launch_bounds__(kThreads) void k_pyramid_tree(const int16_t* __restrict__ user, PyramidArgs a)
{
    extern __shared__ int lds[];
    pyramid_tree_block<G, VEC>(user, a.c, a.lv, a.L, a.D, (int)blockIdx.x * tree_blocks(a.L, G, blockDim.x), lds,
                               a.skip_finest == 0);
}

// Start a scale: copy each pixel's parent messages (zero for a missing neighbour or for
// the coarsest scale) and reset the skip state.
template <int G, bool PACKED>
__global__ __launch_bounds__(kThreads) void k_init(const int16_t* __restrict__ parent, Level lp,
                                                    long long pvol, int16_t* __restrict__ msgs, Level lv,
                                                    long long vol, uint8_t* sa, uint8_t* sb, int mode)
{
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    init_pixel<G, PACKED>(parent, lp, pvol, msgs, lv, vol, sa, sb, mode, t / G, (int)(t & (G - 1)));
}

// Start scale s from caller-given messages [4][H][W][D].
template <int G>
__global__ __launch_bounds__(kThreads) void k_import(const int16_t* __restrict__ warm, int16_t* __restrict__ msgs,
                                                      Level lv, long long vol, int D, uint8_t* sa, uint8_t* sb,
                                                      int mode)
{
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const long long gi = t / G;
    const int lane = (int)(t & (G - 1));
    if (gi >= lv.slots()) return;
    ColourPix p = any_pixel(gi, lv);
    if (!p.valid) return;
    const int d0 = lane * 8;
    const bool has[4] = {p.x > 0, p.x < lv.W - 1, p.y > 0, p.y < lv.H - 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int v[8];
        const int16_t* src = warm + (((long long)k * lv.H + p.y) * lv.W + p.x) * D + d0;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (has[k] && d0 + j < D) ? (int)src[j] : 0;
        *reinterpret_cast<int4*>(msgs + k * vol + gi * (8 * G) + d0) = pack8(v);
    }
    if (lane == 0) {
        if (mode == 1) { sa[gi] = 1; sb[gi] = 0; }
        if (mode == 2) sa[gi] = 1;
    }
}

// One half-step over a whole scale (see halfstep_pixel), with optional per-block counters.
//
// Where pixels can be inactive (the freeze rule from its third half-step on, the exact
// skip always), a workgroup first compacts its tile: each wave forms the 64-bit mask of its
// active pixels with a ballot, each active pixel takes its rank from mbcnt plus the counts
// of the waves before it, and the active pixels are packed onto the first lanes.  Waves
// left without work leave at once (a tile with no active pixel loads nothing), the others
// update only active pixels.  Updates of one colour are independent, so the order does not
// change any result.
// Variant flags of k_halfstep.
// kHsUser: the finest scale's cost read from the caller's volume (12-bit messages only, D == Dp);
// kHsFull: D == Dp on the 12-bit path, so no label is masked.
constexpr int kHsCount = 1, kHsNarrow = 2, kHsStream = 4, kHsPacked = 8, kHsUser = 16, kHsFull = 32;

template <int G, int MODE, int SRC, int FL>
__global__ __launch_bounds__(kThreads) void k_halfstep(HalfstepArgs a)
{
    constexpr bool COUNT = (FL & kHsCount) != 0, NARROW = (FL & kHsNarrow) != 0, STREAM = (FL & kHsStream) != 0;
    constexpr bool PACKED = (FL & kHsPacked) != 0, USER = (FL & kHsUser) != 0, FULL_D = (FL & kHsFull) != 0;
    constexpr int kPix = kThreads / G;  // pixels of one tile
    const int lane = threadIdx.x & (G - 1);
    int gi = blockIdx.x * kPix + threadIdx.x / G;
    if (MODE == 2 || (MODE == 1 && a.t >= 2)) {
        __shared__ int list[kPix];
        __shared__ int wcount[kThreads / 64];
        const long long npix = (long long)a.lv.H * a.lv.Wh;
        bool active = false;
        if (lane == 0 && gi < npix) {
            const int y = gi / a.lv.Wh, xi = gi - y * a.lv.Wh;
            const int x = 2 * xi + ((a.colour ^ y) & 1);
            active = x < a.lv.W && a.state_a[(long long)(2 * y + a.colour) * a.lv.Wh + xi] != 0;
        }
        const unsigned long long m = __ballot(active);
        const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) wcount[wave] = __popcll(m);
        __syncthreads();
        int base = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            base += w < wave ? wcount[w] : 0;
            total += wcount[w];
        }
        if (active) list[base + rank] = threadIdx.x / G;
        __syncthreads();
        if (!COUNT && (threadIdx.x & ~63) >= total * G) return;  // the whole wave has no pixel
        gi = threadIdx.x < total * G ? blockIdx.x * kPix + list[threadIdx.x / G] : (int)npix;  // npix: no pixel
    }
    const PixOut r =
        halfstep_pixel<G, MODE, SRC, NARROW, STREAM, PACKED, USER, FULL_D>(a, gi, lane,
                                                                         MODE == 2 || (MODE == 1 && a.t >= 2));
    if (COUNT) {
        __shared__ int cnt[2];
        if (threadIdx.x == 0) { cnt[0] = 0; cnt[1] = 0; }
        __syncthreads();
        const bool lead = r.act && lane == 0;
        const int npix = __popcll(__ballot(lead));
        int nmsg = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) nmsg += __popcll(__ballot(lead && r.has[k]));
        if ((threadIdx.x & 63) == 0 && npix) {
            atomicAdd(&cnt[0], npix);
            atomicAdd(&cnt[1], nmsg);
        }
        __syncthreads();
        if (threadIdx.x == 0 && cnt[0]) {
            atomicAdd(&a.stats->pixel_updates, (unsigned long long)cnt[0]);
            atomicAdd(&a.stats->msg_updates, (unsigned long long)cnt[1]);
            if (a.t < kStatHalfsteps) atomicAdd(&a.stats->active[a.level][a.t], cnt[0]);
        }
    }
}

// colour < 0: every slot; otherwise the slots of one colour (index y * Wh + xi)
template <int G, bool PACKED, bool USER = false>
__global__ __launch_bounds__(kThreads) void k_wta(const int16_t* __restrict__ c0, const int16_t* __restrict__ msgs,
                                                   long long vol, Level lv, int D, int colour,
                                                   int16_t* __restrict__ disp)
{
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    long long gi = t / G;
    if (colour >= 0) {
        const long long y = gi / lv.Wh, xi = gi - y * lv.Wh;
        gi = y < lv.H ? (2 * y + colour) * lv.Wh + xi : lv.slots();  // slots(): no pixel
    }
    wta_pixel<G, PACKED, USER>(c0, msgs, vol, lv, D, disp, gi, (int)(t & (G - 1)));
}

template <int G, bool PACKED>
__global__ __launch_bounds__(kThreads) void k_export(const int16_t* __restrict__ msgs, long long vol, Level lv,
                                                      int D, int16_t* __restrict__ out)
{
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const long long gi = t / G;
    const int lane = (int)(t & (G - 1));
    if (gi >= lv.slots()) return;
    ColourPix p = any_pixel(gi, lv);
    if (!p.valid) return;
    const int d0 = lane * 8;
    const bool has[4] = {p.x > 0, p.x < lv.W - 1, p.y > 0, p.y < lv.H - 1};
    for (int k = 0; k < 4; ++k) {
        int16_t* dst = out + (((long long)k * lv.H + p.y) * lv.W + p.x) * D + d0;
        const int4 m = has[k] ? ldm<false, PACKED>(msgs, k * vol + gi * (8 * G) + d0) : make_int4(0, 0, 0, 0);
        if ((D & 7) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
            // whole 16-byte vectors (dst 16-byte aligned): a lane's 8 labels are all real or
            // all padding
            if (d0 < D) *reinterpret_cast<int4*>(dst) = m;
        } else {
            int v[8];
            unpack8u(m, v);
#pragma unroll
            for (int j = 0; j < 8; ++j) if (d0 + j < D) dst[j] = (int16_t)v[j];
        }
    }
}

// A scale's internal cost back to the caller's layout [H][W][D].
template <int G>
__global__ __launch_bounds__(kThreads) void k_export_cost(const int16_t* __restrict__ c, Level lv, int D,
                                                           int16_t* __restrict__ out)
{
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const long long gi = t / G;
    const int lane = (int)(t & (G - 1));
    if (gi >= lv.slots()) return;
    ColourPix p = any_pixel(gi, lv);
    if (!p.valid) return;
    const int d0 = lane * 8;
    int v[8];
    unpack8u(*reinterpret_cast<const int4*>(c + gi * (8 * G) + d0), v);
    int16_t* dst = out + ((long long)p.y * lv.W + p.x) * D + d0;
#pragma unroll
    for (int j = 0; j < 8; ++j) if (d0 + j < D) dst[j] = (int16_t)v[j];
}

constexpr int kEnergyBlocks = 1024;  // a multiple of kThreads (the final sum reads kEnergyBlocks / kThreads a lane)
static_assert(kEnergyBlocks % kThreads == 0, "energy blocks");

// Sum over the workgroup of e, and whether any lane saw an out-of-range disparity: a
// butterfly inside each wave, then one LDS word per wave (a single barrier).
__device__ __forceinline__ void block_sum(long long e, int bad, long long* wsum, int* wbad, long long* total,
                                          int* anybad)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    const bool wbad_any = __ballot(bad != 0) != 0ull;
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        wsum[wave] = e;
        wbad[wave] = wbad_any ? 1 : 0;
    }
    __syncthreads();
    long long t = 0;
    int b = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        t += wsum[w];
        b |= wbad[w];
    }
    *total = t;
    *anybad = b;
}

// Energy of a labelling over a grid-stride range of pixels: the data cost of each pixel and
// the smoothness cost of its right and lower edges.  The three disparities are loaded
// together, then the cost at the pixel's disparity (which depends on one of them).
__global__ __launch_bounds__(kThreads) void k_energy_partial(const int16_t* __restrict__ cost,
                                                              const int16_t* __restrict__ disp, int W, int H,
                                                              int D, int lam, int T, long long* part, int* bad)
{
    __shared__ long long wsum[kThreads / 64];
    __shared__ int wbad[kThreads / 64];
    long long e = 0;
    int mybad = 0;
    const long long n = (long long)W * H;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const int y = (int)(i / W), x = (int)(i - (long long)y * W);
        const bool right = x + 1 < W, down = y + 1 < H;
        const int dp = disp[i];
        const int dr = disp[right ? i + 1 : i];
        const int dd = disp[down ? i + W : i];
        const bool ok = dp >= 0 && dp < D;
        const int c = cost[i * D + (ok ? dp : 0)];
        // selects, not branches: a branch would pull the neighbours' loads in after dp's
        const int jr = right && dr >= 0 && dr < D ? min(abs(dp - dr), T) : 0;
        const int jd = down && dd >= 0 && dd < D ? min(abs(dp - dd), T) : 0;
        e += ok ? (long long)c + (long long)lam * (jr + jd) : 0;
        mybad |= ok ? 0 : 1;
    }
    long long t;
    int b;
    block_sum(e, mybad, wsum, wbad, &t, &b);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = t;
        bad[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(kThreads) void k_energy_final(const long long* part, const int* bad, int nb,
                                                            int64_t* out)
{
    __shared__ long long wsum[kThreads / 64];
    __shared__ int wbad[kThreads / 64];
    // nb <= kEnergyBlocks: a fixed number of loads a lane, all issued before any is used
    constexpr int kPer = kEnergyBlocks / kThreads;
    long long pv[kPer];
    int bv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = (int)threadIdx.x + u * kThreads;
        pv[u] = part[i < nb ? i : 0];
        bv[u] = bad[i < nb ? i : 0];
    }
    long long e = 0;
    int b = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const bool in = (int)threadIdx.x + u * kThreads < nb;
        e += in ? pv[u] : 0;
        b |= in ? bv[u] : 0;
    }
    long long t;
    int anybad;
    block_sum(e, b, wsum, wbad, &t, &anybad);
    if (threadIdx.x == 0) *out = anybad ? (int64_t)(-9223372036854775807LL - 1) : (int64_t)t;
}

// Left-right consistency: the left pixel (x, y) with disparity d matches the right pixel
// (x - d, y) and keeps d when that pixel's disparity (right view as reference) is within
// tol of it; otherwise -1.  Every lane loads its left disparity and, from a clamped column,
// the right one before either is used.
__global__ __launch_bounds__(kThreads) void k_lr_check(const int16_t* __restrict__ dl, const int16_t* __restrict__ dr,
                                                        int W, int H, int D, int tol, int16_t* __restrict__ out)
{
    const long long n = (long long)W * H;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const int y = (int)(i / W), x = (int)(i - (long long)y * W);
        const int d = dl[i];
        const bool in = d >= 0 && d < D && x - d >= 0;
        const int e = dr[(long long)y * W + (in ? x - d : x)];
        out[i] = (int16_t)(in && abs(e - d) <= tol ? d : -1);
    }
}

__global__ __launch_bounds__(kThreads) void k_luma(const uint8_t* __restrict__ rgb, long long n, uint8_t* __restrict__ y)
{
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        int r = rgb[3 * i], g = rgb[3 * i + 1], b = rgb[3 * i + 2];
        y[i] = (uint8_t)((77 * r + 150 * g + 29 * b + 128) >> 8);
    }
}

inline unsigned grid_for(long long items, int G)
{
    long long threads = items * G;
    return (unsigned)((threads + kThreads - 1) / kThreads);
}

}  // namespace

#define BPST_DISPATCH_G(G, CALL)                                 \
    switch (G) {                                                 \
    case 1: { constexpr int GG = 1; CALL; } break;               \
    case 2: { constexpr int GG = 2; CALL; } break;               \
    case 4: { constexpr int GG = 4; CALL; } break;               \
    case 8: { constexpr int GG = 8; CALL; } break;               \
    case 16: { constexpr int GG = 16; CALL; } break;             \
    case 32: { constexpr int GG = 32; CALL; } break;             \
    default: return hipErrorInvalidValue;                        \
    }

hipError_t launch_zero_stats(DevStats* s, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(kThreads), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_prep_level0(const int16_t* user, int16_t* c0, Level lv, int D, int G, hipStream_t st)
{
    const bool vec = (D % 8 == 0) && ((reinterpret_cast<uintptr_t>(user) & 15) == 0);
    const unsigned g = grid_for(lv.slots(), G);
    if (vec) {
        BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_prep_level0<GG, true>), dim3(g), dim3(kThreads), 0, st, user, c0, lv, D));
    } else {
        BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_prep_level0<GG, false>), dim3(g), dim3(kThreads), 0, st, user, c0, lv, D));
    }
    return hipGetLastError();
}

hipError_t launch_pyramid(const int16_t* fine, Level lf, int16_t* coarse, Level lc, int D, int G, hipStream_t st)
{
    const unsigned g = grid_for(lc.slots(), G);
    BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_pyramid<GG>), dim3(g), dim3(kThreads), 0, st, fine, lf, coarse, lc, D));
    return hipGetLastError();
}

hipError_t launch_pyramid_tree(const int16_t* user, const PyramidArgs& a, int G, bool* done, hipStream_t st)
{
    *done = false;
    if (a.L < 2) return hipSuccess;
    if (tree_block_lds(a.L, G) > 64 * 1024) return hipSuccess;
    const bool vec = (a.D % 8 == 0) && ((reinterpret_cast<uintptr_t>(user) & 15) == 0);
    // Workgroup width: whole waves, at least one block's lanes up to kThreads; then
    // narrower (fewer blocks per workgroup) while the grid would not give every CU two.
    const long long coarsest = (long long)a.lv[a.L - 1].W * a.lv[a.L - 1].H;
    const long long p1 = (1LL << (2 * (a.L - 2))) * G;
    long long threads = kThreads;
    while (threads > 64 && threads / 2 >= p1 &&
           (coarsest + tree_blocks(a.L, G, (int)threads) - 1) / tree_blocks(a.L, G, (int)threads) < 512)
        threads /= 2;
    const int nb = tree_blocks(a.L, G, (int)threads);
    const size_t lds = (size_t)nb * tree_block_lds(a.L, G);
    const dim3 grid((unsigned)((coarsest + nb - 1) / nb));
    if (vec) {
        BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_pyramid_tree<GG, true>), grid, dim3(threads), lds, st, user, a));
    } else {
        BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_pyramid_tree<GG, false>), grid, dim3(threads), lds, st, user, a));
    }
    *done = true;
    return hipGetLastError();
}

hipError_t launch_init(const int16_t* parent, Level lp, long long pvol, int16_t* msgs, Level lv, long long vol,
                       int G, uint8_t* sa, uint8_t* sb, int mode, hipStream_t st, bool packed)
{
    const unsigned g = grid_for(lv.slots(), G);
    if (packed) {
        BPST_DISPATCH_G(G, if constexpr (GG >= 16) hipLaunchKernelGGL((k_init<GG, true>), dim3(g), dim3(kThreads), 0,
                                                                      st, parent, lp, pvol, msgs, lv, vol, sa, sb, mode);
                           else return hipErrorInvalidValue);
    } else {
        BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_init<GG, false>), dim3(g), dim3(kThreads), 0, st, parent, lp, pvol,
                                              msgs, lv, vol, sa, sb, mode));
    }
    return hipGetLastError();
}

hipError_t launch_import(const int16_t* warm, int16_t* msgs, Level lv, long long vol, int D, int G, uint8_t* sa,
                         uint8_t* sb, int mode, hipStream_t st)
{
    const unsigned g = grid_for(lv.slots(), G);
    BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_import<GG>), dim3(g), dim3(kThreads), 0, st, warm, msgs, lv, vol, D, sa,
                                          sb, mode));
    return hipGetLastError();
}

template <int MODE, int SRC, int FL>
static hipError_t launch_halfstep_t(const HalfstepArgs& a, unsigned g, hipStream_t st)
{
    // the narrow variants exist for G <= kNarrowMaxG only, the 12-bit ones for G >= 16 only
    BPST_DISPATCH_G(a.G, if constexpr (((FL & kHsNarrow) == 0 || GG <= kNarrowMaxG) &&
                                       ((FL & kHsPacked) == 0 || GG >= 16)) hipLaunchKernelGGL(
                             (k_halfstep<GG, MODE, SRC, FL>), dim3(g), dim3(kThreads), 0, st, a);
                         else return hipErrorInvalidValue);
    return hipGetLastError();
}

template <int MODE, int SRC>
static hipError_t launch_halfstep_c(const HalfstepArgs& a, unsigned g, hipStream_t st)
{
    if (a.packed) {
        if (a.capv < 0 || a.capv > 4095 || a.narrow || a.out) return hipErrorInvalidValue;
        if (a.user_cost) {
            if (a.Dp != a.D || a.level != 0) return hipErrorInvalidValue;
            if constexpr (SRC == kSrcZero) {
                return hipErrorInvalidValue;  // the finest scale never starts from zero messages
            } else {
                if (a.count) return launch_halfstep_t<MODE, SRC, kHsCount | kHsPacked | kHsUser>(a, g, st);
                if (a.stream) return launch_halfstep_t<MODE, SRC, kHsStream | kHsPacked | kHsUser>(a, g, st);
                return launch_halfstep_t<MODE, SRC, kHsPacked | kHsUser>(a, g, st);
            }
        }
        if (a.Dp == a.D) {
            if (a.count) return launch_halfstep_t<MODE, SRC, kHsCount | kHsPacked | kHsFull>(a, g, st);
            if (a.stream) return launch_halfstep_t<MODE, SRC, kHsStream | kHsPacked | kHsFull>(a, g, st);
            return launch_halfstep_t<MODE, SRC, kHsPacked | kHsFull>(a, g, st);
        }
        if (a.count) return launch_halfstep_t<MODE, SRC, kHsCount | kHsPacked>(a, g, st);
        if (a.stream) return launch_halfstep_t<MODE, SRC, kHsStream | kHsPacked>(a, g, st);
        return launch_halfstep_t<MODE, SRC, kHsPacked>(a, g, st);
    }
    if (a.count) return launch_halfstep_t<MODE, SRC, kHsCount>(a, g, st);  // no narrow counting variant
    if (a.narrow) {
        if (a.capv < 0 || a.capv > kNarrowCap) return hipErrorInvalidValue;
        return launch_halfstep_t<MODE, SRC, kHsNarrow>(a, g, st);
    }
    if (a.stream) return launch_halfstep_t<MODE, SRC, kHsStream>(a, g, st);
    return launch_halfstep_t<MODE, SRC, 0>(a, g, st);
}

template <int MODE>
static hipError_t launch_halfstep_m(const HalfstepArgs& a, unsigned g, hipStream_t st)
{
    switch (a.source) {
    case kSrcOwn: return launch_halfstep_c<MODE, kSrcOwn>(a, g, st);
    case kSrcParent: return launch_halfstep_c<MODE, kSrcParent>(a, g, st);
    case kSrcZero: return launch_halfstep_c<MODE, kSrcZero>(a, g, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_halfstep(const HalfstepArgs& a, hipStream_t st)
{
    const unsigned g = grid_for((long long)a.lv.H * a.lv.Wh, a.G);
    switch (a.mode) {
    case 0: return launch_halfstep_m<0>(a, g, st);
    case 1: return launch_halfstep_m<1>(a, g, st);
    case 2: return a.source == kSrcOwn ? launch_halfstep_c<2, kSrcOwn>(a, g, st) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_wta(const int16_t* c0, const int16_t* msgs, long long vol, Level lv, int D, int G, int colour,
                      int16_t* disp, hipStream_t st, bool packed, bool user)
{
    const unsigned g = grid_for(colour < 0 ? lv.slots() : (long long)lv.H * lv.Wh, G);
    if (user) {
        if (!packed || D != 8 * G || (reinterpret_cast<uintptr_t>(c0) & 15) != 0) return hipErrorInvalidValue;
        BPST_DISPATCH_G(G, if constexpr (GG >= 16) hipLaunchKernelGGL((k_wta<GG, true, true>), dim3(g), dim3(kThreads),
                                                                      0, st, c0, msgs, vol, lv, D, colour, disp);
                           else return hipErrorInvalidValue);
    } else if (packed) {
        BPST_DISPATCH_G(G, if constexpr (GG >= 16) hipLaunchKernelGGL((k_wta<GG, true>), dim3(g), dim3(kThreads), 0,
                                                                      st, c0, msgs, vol, lv, D, colour, disp);
                           else return hipErrorInvalidValue);
    } else {
        BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_wta<GG, false>), dim3(g), dim3(kThreads), 0, st, c0, msgs, vol, lv, D,
                                              colour, disp));
    }
    return hipGetLastError();
}

hipError_t launch_export(const int16_t* msgs, long long vol, Level lv, int D, int G, int16_t* out, hipStream_t st,
                         bool packed)
{
    const unsigned g = grid_for(lv.slots(), G);
    if (packed) {
        BPST_DISPATCH_G(G, if constexpr (GG >= 16) hipLaunchKernelGGL((k_export<GG, true>), dim3(g), dim3(kThreads),
                                                                      0, st, msgs, vol, lv, D, out);
                           else return hipErrorInvalidValue);
    } else {
        BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_export<GG, false>), dim3(g), dim3(kThreads), 0, st, msgs, vol, lv, D,
                                              out));
    }
    return hipGetLastError();
}

hipError_t launch_export_cost(const int16_t* c, Level lv, int D, int G, int16_t* out, hipStream_t st)
{
    const unsigned g = grid_for(lv.slots(), G);
    BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_export_cost<GG>), dim3(g), dim3(kThreads), 0, st, c, lv, D, out));
    return hipGetLastError();
}

size_t energy_ws_bytes() { return (size_t)kEnergyBlocks * (sizeof(long long) + sizeof(int)); }

hipError_t launch_energy(const int16_t* cost, const int16_t* disp, int W, int H, int D, int lambda, int trunc,
                         int64_t* out, void* ws, hipStream_t st)
{
    long long* part = reinterpret_cast<long long*>(ws);
    int* bad = reinterpret_cast<int*>(part + kEnergyBlocks);
    const long long n = (long long)W * H;
    long long nb = (n + kThreads - 1) / kThreads;
    if (nb > kEnergyBlocks) nb = kEnergyBlocks;
    hipLaunchKernelGGL(k_energy_partial, dim3((unsigned)nb), dim3(kThreads), 0, st, cost, disp, W, H, D, lambda,
                       trunc, part, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kThreads), 0, st, part, bad, (int)nb, out);
    return hipGetLastError();
}

hipError_t launch_lr_check(const int16_t* dl, const int16_t* dr, int W, int H, int D, int tol, int16_t* out,
                           hipStream_t st)
{
    const long long n = (long long)W * H;
    long long nb = (n + kThreads - 1) / kThreads;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_lr_check, dim3((unsigned)nb), dim3(kThreads), 0, st, dl, dr, W, H, D, tol, out);
    return hipGetLastError();
}

hipError_t launch_luma(const uint8_t* rgb, int W, int H, uint8_t* y, hipStream_t st)
{
    const long long n = (long long)W * H;
    long long nb = (n + kThreads - 1) / kThreads;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_luma, dim3((unsigned)nb), dim3(kThreads), 0, st, rgb, n, y);
    return hipGetLastError();
}

}  // namespace bpst
