// Message-passing kernels of the hierarchical min-sum solve.
//
// Every kernel maps one pixel to G consecutive lanes of a wave64; lane g holds labels
// [8g, 8g + 8) of that pixel in registers as int32.  Cross-label work (minimum, prefix
// and suffix minima of the distance transform) runs across the G lanes with shuffles,
// so no LDS is needed and every global access is a coalesced 16-byte vector.
#include "internal.h"

namespace bpst {
namespace {

constexpr int kThreads = 256;
constexpr int kBig = 1 << 29;      // value of a padded label (d >= D): never the minimum
constexpr int kScanId = 1 << 30;   // identity of the min-scans

__device__ __forceinline__ void unpack8(const int4 v, int o[8])
{
    o[0] = (int)(short)(v.x & 0xffff); o[1] = v.x >> 16;
    o[2] = (int)(short)(v.y & 0xffff); o[3] = v.y >> 16;
    o[4] = (int)(short)(v.z & 0xffff); o[5] = v.z >> 16;
    o[6] = (int)(short)(v.w & 0xffff); o[7] = v.w >> 16;
}

__device__ __forceinline__ int4 pack8(const int o[8])
{
    int4 v;
    v.x = (o[0] & 0xffff) | (o[1] << 16);
    v.y = (o[2] & 0xffff) | (o[3] << 16);
    v.z = (o[4] & 0xffff) | (o[5] << 16);
    v.w = (o[6] & 0xffff) | (o[7] << 16);
    return v;
}

__device__ __forceinline__ long long slot_of(int x, int y, int Wh)
{
    return (long long)(2 * y + ((x + y) & 1)) * Wh + (x >> 1);
}

template <int G>
__device__ __forceinline__ int group_min(int v)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v = min(v, __shfl_xor(v, o, G));
    return v;
}

template <int G>
__device__ __forceinline__ int group_excl_prefix_min(int v, int lane)
{
    if (G == 1) return kScanId;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        int t = __shfl_up(v, o, G);
        if (lane >= o) v = min(v, t);
    }
    int e = __shfl_up(v, 1, G);
    return lane == 0 ? kScanId : e;
}

template <int G>
__device__ __forceinline__ int group_excl_suffix_min(int v, int lane)
{
    if (G == 1) return kScanId;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        int t = __shfl_down(v, o, G);
        if (lane + o < G) v = min(v, t);
    }
    int e = __shfl_down(v, 1, G);
    return lane == G - 1 ? kScanId : e;
}

// Min-sum message with truncated-linear jump cost, normalised:
//   m(d) = min( min_d' h(d') + lambda*|d - d'|,  min h + lambda*T ) - min h,
// saturated to int16.  The inner minimum is the classic two-pass lower envelope:
// forward f(d) = min(h(d), f(d-1) + lambda), then backward f(d) = min(f(d), f(d+1) + lambda).
// Each pass runs sequentially over a lane's 8 labels; the value carried into a lane from
// the lanes before it (after it) is a scan over the G lanes with the operator
// (a, b) -> min(b, a + 8*lambda*distance).  Integer min/+ are exact, so this association
// gives the same value as one sequential pass.  Padded labels hold kBig and never win.
template <int G>
__device__ __forceinline__ void transform(const int h[8], int lam, int capv, int lane, int out[8])
{
    int hm = min(min(min(h[0], h[1]), min(h[2], h[3])), min(min(h[4], h[5]), min(h[6], h[7])));
    hm = group_min<G>(hm);
    int f[8];
    // forward: carry = min over the lanes before of (their last forward value + lambda*gap)
    int last = h[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) last = min(h[j], last + lam);
    int cin = kScanId;
    if (G > 1) {
        int c = last;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            int t = __shfl_up(c, o, G);
            if (lane >= o) c = min(c, t + 8 * lam * o);
        }
        cin = __shfl_up(c, 1, G);
        if (lane == 0) cin = kScanId;
    }
    f[0] = min(h[0], cin + lam);
#pragma unroll
    for (int j = 1; j < 8; ++j) f[j] = min(h[j], f[j - 1] + lam);
    // backward on the forward result
    int first = f[7];
#pragma unroll
    for (int j = 6; j >= 0; --j) first = min(f[j], first + lam);
    int cb = kScanId;
    if (G > 1) {
        int c = first;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            int t = __shfl_down(c, o, G);
            if (lane + o < G) c = min(c, t + 8 * lam * o);
        }
        cb = __shfl_down(c, 1, G);
        if (lane == G - 1) cb = kScanId;
    }
    f[7] = min(f[7], cb + lam);
#pragma unroll
    for (int j = 6; j >= 0; --j) f[j] = min(f[j], f[j + 1] + lam);
#pragma unroll
    for (int j = 0; j < 8; ++j) out[j] = min(f[j] - hm, capv);
}

struct ColourPix {
    int x, y;
    long long slot;
    bool valid;
};

// Pixel of slot index gi over both colours (gi == its slot).
__device__ __forceinline__ ColourPix any_pixel(long long gi, const Level lv)
{
    ColourPix p;
    int r = (int)(gi / lv.Wh);
    int xi = (int)(gi - (long long)r * lv.Wh);
    p.y = r >> 1;
    p.x = 2 * xi + (((r & 1) ^ p.y) & 1);
    p.valid = p.y < lv.H && p.x < lv.W;
    p.slot = gi;
    return p;
}

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
    *reinterpret_cast<int4*>(c0 + gi * (8 * G) + d0) = pack8(v);
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
                    unpack8(*reinterpret_cast<const int4*>(fine + slot_of(x, y, lf.Wh) * (8 * G) + d0), v);
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

// The whole cost pyramid in one launch.  One workgroup per pixel (X, Y) of the coarsest
// scale: it re-lays the finest costs of the block of pixels under (X, Y) into the internal
// layout and builds every coarser scale of that block, handing each scale to the next in
// LDS.  Scale sizes halve with ceil, so the block's pixels at scale l are exactly
// [X s_l, (X+1) s_l) x [Y s_l, (Y+1) s_l) clipped to the scale, s_l = 2^(L-1-l).
template <int G, bool VEC>
__global__ __launch_bounds__(kThreads) void k_pyramid_tree(const int16_t* __restrict__ user, PyramidArgs a)
{
    constexpr int Dp = 8 * G;
    extern __shared__ int lds[];
    const int L = a.L, D = a.D;
    const int X = blockIdx.x, Y = blockIdx.y;
    const int s1 = 1 << (L - 2);
    int* cur = lds;                 // scale l-1 of the block, [s_{l-1}^2][Dp]
    int* nxt = lds + s1 * s1 * Dp;  // scale l
    // scale 1 from the caller's finest costs; also writes the internal finest layout
    {
        const Level l0 = a.lv[0], l1 = a.lv[1];
        const int tasks = s1 * s1 * G;
        for (int task = threadIdx.x; task < tasks; task += blockDim.x) {
            const int p = task / G, lane = task & (G - 1), d0 = lane * 8;
            const int px = X * s1 + (p % s1), py = Y * s1 + (p / s1);
            const bool valid = px < l1.W && py < l1.H;
            int s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (valid) {
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const int x = 2 * px + c, y = 2 * py + b;
                        if (x >= l0.W || y >= l0.H) continue;
                        const int16_t* src = user + ((long long)y * l0.W + x) * D + d0;
                        int v[8];
                        if (VEC) {
                            if (d0 < D) unpack8(*reinterpret_cast<const int4*>(src), v);
                            else for (int j = 0; j < 8; ++j) v[j] = 0;
                        } else {
#pragma unroll
                            for (int j = 0; j < 8; ++j) v[j] = (d0 + j < D) ? (int)src[j] : 0;
                        }
                        *reinterpret_cast<int4*>(a.c[0] + slot_of(x, y, l0.Wh) * Dp + d0) = pack8(v);
#pragma unroll
                        for (int j = 0; j < 8; ++j) s[j] += v[j];
                    }
            }
            int mn = kBig;
#pragma unroll
            for (int j = 0; j < 8; ++j) if (d0 + j < D) mn = min(mn, s[j]);
            mn = group_min<G>(mn);
            int o[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) o[j] = (d0 + j < D) ? min(s[j] - mn, 32767) : 0;
            if (valid) {
                *reinterpret_cast<int4*>(a.c[1] + slot_of(px, py, l1.Wh) * Dp + d0) = pack8(o);
#pragma unroll
                for (int j = 0; j < 8; ++j) cur[p * Dp + d0 + j] = o[j];
            }
        }
    }
    __syncthreads();
    for (int l = 2; l < L; ++l) {
        const Level lf = a.lv[l - 1], lc = a.lv[l];
        const int sl = 1 << (L - 1 - l), sf = 2 * sl;
        const int tasks = sl * sl * G;
        for (int task = threadIdx.x; task < tasks; task += blockDim.x) {
            const int p = task / G, lane = task & (G - 1), d0 = lane * 8;
            const int qx = p % sl, qy = p / sl;
            const int px = X * sl + qx, py = Y * sl + qy;
            const bool valid = px < lc.W && py < lc.H;
            int s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (valid) {
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        if (2 * px + c >= lf.W || 2 * py + b >= lf.H) continue;
                        const int* src = cur + ((2 * qy + b) * sf + (2 * qx + c)) * Dp + d0;
#pragma unroll
                        for (int j = 0; j < 8; ++j) s[j] += src[j];
                    }
            }
            int mn = kBig;
#pragma unroll
            for (int j = 0; j < 8; ++j) if (d0 + j < D) mn = min(mn, s[j]);
            mn = group_min<G>(mn);
            int o[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) o[j] = (d0 + j < D) ? min(s[j] - mn, 32767) : 0;
            if (valid) {
                *reinterpret_cast<int4*>(a.c[l] + slot_of(px, py, lc.Wh) * Dp + d0) = pack8(o);
#pragma unroll
                for (int j = 0; j < 8; ++j) nxt[p * Dp + d0 + j] = o[j];
            }
        }
        __syncthreads();
        int* t = cur;
        cur = nxt;
        nxt = t;
    }
}

// Start a scale: copy each pixel's parent messages (zero for a missing neighbour or for
// the coarsest scale) and reset the skip state.
template <int G>
__global__ __launch_bounds__(kThreads) void k_init(const int16_t* __restrict__ parent, Level lp,
                                                    long long pvol, int16_t* __restrict__ msgs, Level lv,
                                                    long long vol, uint8_t* sa, uint8_t* sb, int mode)
{
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const long long gi = t / G;
    const int lane = (int)(t & (G - 1));
    if (gi >= lv.slots()) return;
    ColourPix p = any_pixel(gi, lv);
    if (!p.valid) return;
    const int d0 = lane * 8;
    const bool has[4] = {p.x > 0, p.x < lv.W - 1, p.y > 0, p.y < lv.H - 1};
    const int px = p.x >> 1, py = p.y >> 1;
    const bool phas[4] = {px > 0, px < lp.W - 1, py > 0, py < lp.H - 1};
    const long long ps = parent ? slot_of(px, py, lp.Wh) : 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int4 v = make_int4(0, 0, 0, 0);
        // a slot is only ever read where its neighbour exists, on both scales
        if (parent && has[k] && phas[k]) v = *reinterpret_cast<const int4*>(parent + k * pvol + ps * (8 * G) + d0);
        *reinterpret_cast<int4*>(msgs + k * vol + gi * (8 * G) + d0) = v;
    }
    if (lane == 0) {
        if (mode == 1) { sa[gi] = 1; sb[gi] = 0; }
        if (mode == 2) sa[gi] = 1;
    }
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

// One half-step: every pixel of colour a.colour (that is still being updated) sends a
// new message to each of its neighbours.  Reads only slots of its own colour, writes only
// slots of the other colour, so the in-place update is race-free.
//   SRC == kSrcParent: first half-step of a scale; the incoming messages are read from the
//     parent's slots (the scale's own slots of this colour are never materialised);
//   SRC == kSrcZero: first half-step of the coarsest scale; incoming messages are zero.
// Skip mode 1 resets a pixel's state at its first update of the scale (t < 2).
template <int G, int MODE, int SRC, bool COUNT>
__global__ __launch_bounds__(kThreads) void k_halfstep(HalfstepArgs a)
{
    constexpr int Dp = 8 * G;
    const int t = blockIdx.x * kThreads + threadIdx.x;
    const int gi = t / G;
    const int lane = t & (G - 1);
    const int W = a.lv.W, H = a.lv.H, Wh = a.lv.Wh;
    const bool in = gi < H * Wh;
    const int y = in ? gi / Wh : 0;
    const int xi = gi - y * Wh;
    const int x = 2 * xi + ((a.colour ^ y) & 1);
    const bool valid = in && x < W;
    const long long slot = (long long)(2 * y + a.colour) * Wh + xi;
    const bool has[4] = {x > 0, x < W - 1, y > 0, y < H - 1};
    const long long nb[4] = {(long long)(2 * y + 1 - a.colour) * Wh + ((x - 1) >> 1),
                             (long long)(2 * y + 1 - a.colour) * Wh + ((x + 1) >> 1),
                             (long long)(2 * (y - 1) + 1 - a.colour) * Wh + (x >> 1),
                             (long long)(2 * (y + 1) + 1 - a.colour) * Wh + (x >> 1)};
    bool act = valid;
    if (MODE == 2 || (MODE == 1 && a.t >= 2)) act = act && a.state_a[slot] != 0;
    const int d0 = lane * 8;
    int Hs[8], m[4][8];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 8; ++j) m[k][j] = 0;
    if (act) {
        unpack8(*reinterpret_cast<const int4*>(a.cost + slot * Dp + d0), Hs);
        if (SRC == kSrcOwn) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (has[k]) unpack8(*reinterpret_cast<const int4*>(a.msgs + k * a.vol + slot * Dp + d0), m[k]);
        } else if (SRC == kSrcParent) {
            const int px = x >> 1, py = y >> 1;
            const bool phas[4] = {px > 0, px < a.plv.W - 1, py > 0, py < a.plv.H - 1};
            const long long ps = (long long)(2 * py + ((px + py) & 1)) * a.plv.Wh + (px >> 1);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (has[k] && phas[k])
                    unpack8(*reinterpret_cast<const int4*>(a.pmsgs + k * a.pvol + ps * Dp + d0), m[k]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) Hs[j] = 0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
        Hs[j] = (d0 + j < a.D) ? Hs[j] + m[0][j] + m[1][j] + m[2][j] + m[3][j] : kBig;
    if (MODE == 2 && act && lane == 0) a.state_a[slot] = 0;
    const bool check = (MODE == 2) || (MODE == 1 && a.t >= 2);
    bool all_eq = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int h[8], o[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) h[j] = Hs[j] - m[k][j];
        transform<G>(h, a.lambda, a.capv, lane, o);
        bool store = act && has[k];
        int16_t* dst = a.msgs + (k ^ 1) * a.vol + nb[k] * Dp + d0;
        if (check) {
            int old[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (store) unpack8(*reinterpret_cast<const int4*>(dst), old);
            int e = 1;
#pragma unroll
            for (int j = 0; j < 8; ++j) if (d0 + j < a.D && old[j] != o[j]) e = 0;
            e = group_min<G>(e);
            if (store && !e) all_eq = false;
            if (e) store = false;
            if (MODE == 2 && store && lane == 0) a.state_a[nb[k]] = 1;
        }
        if (store) *reinterpret_cast<int4*>(dst) = pack8(o);
    }
    if (MODE == 1 && act && lane == 0) {
        if (a.t < 2) {
            a.state_a[slot] = 1;
            a.state_b[slot] = 0;
        } else {
            int s = all_eq ? (int)a.state_b[slot] + 1 : 0;
            a.state_b[slot] = (uint8_t)s;
            if (2 * s >= a.K) a.state_a[slot] = 0;
        }
    }
    if (COUNT) {
        __shared__ int cnt[2];
        if (threadIdx.x == 0) { cnt[0] = 0; cnt[1] = 0; }
        __syncthreads();
        const bool lead = act && lane == 0;
        const int npix = __popcll(__ballot(lead));
        int nmsg = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) nmsg += __popcll(__ballot(lead && has[k]));
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

template <int G>
__global__ __launch_bounds__(kThreads) void k_wta(const int16_t* __restrict__ c0, const int16_t* __restrict__ msgs,
                                                   long long vol, Level lv, int D, int16_t* __restrict__ disp)
{
    constexpr int Dp = 8 * G;
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    const long long gi = t / G;
    const int lane = (int)(t & (G - 1));
    const bool in = gi < lv.slots();
    ColourPix p = any_pixel(in ? gi : 0, lv);
    const bool valid = in && p.valid;
    const int d0 = lane * 8;
    const bool has[4] = {p.x > 0, p.x < lv.W - 1, p.y > 0, p.y < lv.H - 1};
    int b[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
        unpack8(*reinterpret_cast<const int4*>(c0 + gi * Dp + d0), b);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (has[k]) {
                int v[8];
                unpack8(*reinterpret_cast<const int4*>(msgs + k * vol + gi * Dp + d0), v);
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] += v[j];
            }
    }
    // key = belief * 256 + d: the minimum key is the smallest d among the minimal beliefs
    int key = 0x7fffffff;
#pragma unroll
    for (int j = 0; j < 8; ++j) if (d0 + j < D) key = min(key, b[j] * 256 + d0 + j);
    key = group_min<G>(key);
    if (valid && lane == 0) disp[(long long)p.y * lv.W + p.x] = (int16_t)(key & 255);
}

template <int G>
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
        int v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (has[k]) unpack8(*reinterpret_cast<const int4*>(msgs + k * vol + gi * (8 * G) + d0), v);
        int16_t* dst = out + (((long long)k * lv.H + p.y) * lv.W + p.x) * D + d0;
#pragma unroll
        for (int j = 0; j < 8; ++j) if (d0 + j < D) dst[j] = (int16_t)v[j];
    }
}

constexpr int kEnergyBlocks = 1024;

__global__ __launch_bounds__(kThreads) void k_energy_partial(const int16_t* __restrict__ cost,
                                                              const int16_t* __restrict__ disp, int W, int H,
                                                              int D, int lam, int T, long long* part, int* bad)
{
    __shared__ long long red[kThreads];
    __shared__ int anybad;
    if (threadIdx.x == 0) anybad = 0;
    __syncthreads();
    long long e = 0;
    int mybad = 0;
    const long long n = (long long)W * H;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const int y = (int)(i / W), x = (int)(i - (long long)y * W);
        const int dp = disp[i];
        if (dp < 0 || dp >= D) { mybad = 1; continue; }
        e += cost[i * D + dp];
        if (x + 1 < W) {
            int dq = disp[i + 1];
            if (dq >= 0 && dq < D) e += (long long)lam * min(abs(dp - dq), T);
        }
        if (y + 1 < H) {
            int dq = disp[i + W];
            if (dq >= 0 && dq < D) e += (long long)lam * min(abs(dp - dq), T);
        }
    }
    red[threadIdx.x] = e;
    if (mybad) anybad = 1;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) { part[blockIdx.x] = red[0]; bad[blockIdx.x] = anybad; }
}

__global__ __launch_bounds__(kThreads) void k_energy_final(const long long* part, const int* bad, int nb,
                                                            int64_t* out)
{
    __shared__ long long red[kThreads];
    __shared__ int anybad;
    if (threadIdx.x == 0) anybad = 0;
    __syncthreads();
    long long e = 0;
    int b = 0;
    for (int i = threadIdx.x; i < nb; i += kThreads) { e += part[i]; b |= bad[i]; }
    red[threadIdx.x] = e;
    if (b) anybad = 1;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = anybad ? (int64_t)(-9223372036854775807LL - 1) : (int64_t)red[0];
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
    const long long s1 = 1LL << (a.L - 2), s2 = s1 / 2;
    const size_t lds = (size_t)(s1 * s1 + s2 * s2) * 8 * G * sizeof(int);
    if (lds > 64 * 1024) return hipSuccess;
    const bool vec = (a.D % 8 == 0) && ((reinterpret_cast<uintptr_t>(user) & 15) == 0);
    const long long tasks = s1 * s1 * G;
    const unsigned threads = (unsigned)(tasks >= kThreads ? kThreads : ((tasks + 63) / 64) * 64);
    const dim3 grid((unsigned)a.lv[a.L - 1].W, (unsigned)a.lv[a.L - 1].H);
    if (vec) {
        BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_pyramid_tree<GG, true>), grid, dim3(threads), lds, st, user, a));
    } else {
        BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_pyramid_tree<GG, false>), grid, dim3(threads), lds, st, user, a));
    }
    *done = true;
    return hipGetLastError();
}

hipError_t launch_init(const int16_t* parent, Level lp, long long pvol, int16_t* msgs, Level lv, long long vol,
                       int G, uint8_t* sa, uint8_t* sb, int mode, hipStream_t st)
{
    const unsigned g = grid_for(lv.slots(), G);
    BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_init<GG>), dim3(g), dim3(kThreads), 0, st, parent, lp, pvol, msgs, lv,
                                          vol, sa, sb, mode));
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

template <int MODE, int SRC, bool COUNT>
static hipError_t launch_halfstep_t(const HalfstepArgs& a, unsigned g, hipStream_t st)
{
    BPST_DISPATCH_G(a.G, hipLaunchKernelGGL((k_halfstep<GG, MODE, SRC, COUNT>), dim3(g), dim3(kThreads), 0, st, a));
    return hipGetLastError();
}

template <int MODE, int SRC>
static hipError_t launch_halfstep_c(const HalfstepArgs& a, unsigned g, hipStream_t st)
{
    return a.count ? launch_halfstep_t<MODE, SRC, true>(a, g, st) : launch_halfstep_t<MODE, SRC, false>(a, g, st);
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

hipError_t launch_wta(const int16_t* c0, const int16_t* msgs, long long vol, Level lv, int D, int G, int16_t* disp,
                      hipStream_t st)
{
    const unsigned g = grid_for(lv.slots(), G);
    BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_wta<GG>), dim3(g), dim3(kThreads), 0, st, c0, msgs, vol, lv, D, disp));
    return hipGetLastError();
}

hipError_t launch_export(const int16_t* msgs, long long vol, Level lv, int D, int G, int16_t* out, hipStream_t st)
{
    const unsigned g = grid_for(lv.slots(), G);
    BPST_DISPATCH_G(G, hipLaunchKernelGGL((k_export<GG>), dim3(g), dim3(kThreads), 0, st, msgs, vol, lv, D, out));
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

hipError_t launch_luma(const uint8_t* rgb, int W, int H, uint8_t* y, hipStream_t st)
{
    const long long n = (long long)W * H;
    long long nb = (n + kThreads - 1) / kThreads;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_luma, dim3((unsigned)nb), dim3(kThreads), 0, st, rgb, n, y);
    return hipGetLastError();
}

}  // namespace bpst
