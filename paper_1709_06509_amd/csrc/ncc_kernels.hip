// Correlation volume: zero-mean NCC of window x window patches, quantised to an int16 cost.
//
// One workgroup produces one image row y and a tile of TX columns for every
// disparity.  The window rows y-r..y+r of both views are staged in LDS as packed byte
// columns (4 dwords = up to 16 rows), so every window sum is a handful of 4-way byte
// dot products (v_dot4_u32_u8), all in exact integer arithmetic:
//   V[u][d]  = sum_rows  left(u, .) * right(u - d, .)     (column products)
//   S_IJ     = sum_{i=-r..r} V[x + i][d]
//   S_I, S_II, S_J, S_JJ from per-column byte sums and squares.
// With n = w^2, num = n S_IJ - S_I S_J, vI = n S_II - S_I^2, vJ = n S_JJ - S_J^2 the
// correlation is num / sqrt(vI vJ).  The quantised cost round-half-up(scale (1 - ncc))
// is taken from a float estimate and, when that estimate lies within a margin of a
// rounding boundary (several times its worst-case error), settled exactly by comparing
// squares in 128-bit integers, so the result never depends on floating-point rounding.
#include "internal.h"

namespace bpst {
namespace {

// Columns per workgroup: about 2048 outputs a workgroup, at least 32 columns.
__host__ __device__ inline int ncc_tile_x(int D) { return D <= 16 ? 128 : (D <= 32 ? 64 : 32); }
constexpr int kThreads = 256;
constexpr int kMaxR = 6;  // window <= 13 rows: fits 4 packed dwords per column

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Is B <= A * sqrt(P) exactly?  (P > 0)
__device__ bool le_times_sqrt(long long B, long long A, unsigned long long P)
{
    typedef unsigned __int128 u128;
    const unsigned long long ab = (unsigned long long)(B < 0 ? -B : B);
    const unsigned long long aa = (unsigned long long)(A < 0 ? -A : A);
    const u128 b2 = (u128)ab * ab;
    const u128 a2p = (u128)(aa * aa) * P;
    if (A >= 0) return B <= 0 ? true : (b2 <= a2p);
    return B >= 0 ? false : (b2 >= a2p);
}

// One tile: image row y, columns x0 .. x0 + TX - 1 (clipped), every disparity.  WIN is
// the window size (odd, <= 13), known at compile time so every window loop unrolls.
// Element loops walk (column, disparity) pairs with an incremental index, not a division.
template <int WIN>
__device__ __forceinline__ void ncc_tile(const uint8_t* __restrict__ L, const uint8_t* __restrict__ R, int W, int H,
                                         int D, int TX, int scale, int trunc, float margin,
                                         int16_t* __restrict__ cost, float* __restrict__ ncc_out, int y, int x0,
                                         unsigned* smem)
{
    constexpr int r = WIN >> 1;
    const int nI = TX + 2 * r;          // left columns  x0-r .. x0+TX-1+r
    const int nJ = TX + 2 * r + D - 1;  // right columns x0-r-(D-1) .. x0+TX-1+r
    const int uI0 = x0 - r, uJ0 = x0 - r - (D - 1);
    uint4* colI = reinterpret_cast<uint4*>(smem);
    uint4* colJ = colI + nI;
    // per left column x: {window sum S_I, n S_II - S_I^2, its reciprocal square root (0 for a
    // flat window), 0}; the same per right column u = x0-(D-1) ..: TX and TX + D - 1 entries,
    // one 16-byte read each in the finishing loop
    int4* QI = reinterpret_cast<int4*>(colJ + nJ);
    int4* QJ = QI + TX;
    int* cI = reinterpret_cast<int*>(QJ + TX + D - 1);  // per-column sums
    int* cII = cI + nI;
    int* cJ = cII + nI;
    int* cJJ = cJ + nJ;
    int* V = cJJ + nJ;  // [nI][D]

    // 1. packed byte columns of the window rows (clamped), zero beyond the window.  A thread
    //    takes two columns a round and issues all their loads before using any (a lane past
    //    the last column reads column 0 and drops it): one memory latency a round.
    constexpr int kU = 2;
    for (int c0 = threadIdx.x; c0 < nI + nJ; c0 += kU * kThreads) {
        unsigned bytes[kU][WIN];
#pragma unroll
        for (int q = 0; q < kU; ++q) {
            const int c = c0 + q * kThreads < nI + nJ ? c0 + q * kThreads : 0;
            const bool left = c < nI;
            const uint8_t* img = left ? L : R;
            const int xx = clampi(left ? uI0 + c : uJ0 + (c - nI), 0, W - 1);
#pragma unroll
            for (int j = 0; j < WIN; ++j) bytes[q][j] = img[(long long)clampi(y - r + j, 0, H - 1) * W + xx];
        }
        // keeps the scheduler from packing the first column, and waiting for it, before the
        // second column's loads are issued
        __builtin_amdgcn_sched_barrier(0);
        unsigned w4[kU][4];
#pragma unroll
        for (int q = 0; q < kU; ++q) {
#pragma unroll
            for (int k = 0; k < 4; ++k) w4[q][k] = 0u;
#pragma unroll
            for (int j = 0; j < WIN; ++j) w4[q][j >> 2] |= bytes[q][j] << (8 * (j & 3));
        }
#pragma unroll
        for (int q = 0; q < kU; ++q) {
            const int c = c0 + q * kThreads;
            if (c >= nI + nJ) continue;
            const uint4 pk = make_uint4(w4[q][0], w4[q][1], w4[q][2], w4[q][3]);
            unsigned s = 0, ss = 0;
#pragma unroll
            for (int k = 0; k < (WIN + 3) / 4; ++k) {
                s = __builtin_amdgcn_udot4(w4[q][k], 0x01010101u, s, false);
                ss = __builtin_amdgcn_udot4(w4[q][k], w4[q][k], ss, false);
            }
            if (c < nI) { colI[c] = pk; cI[c] = (int)s; cII[c] = (int)ss; }
            else { colJ[c - nI] = pk; cJ[c - nI] = (int)s; cJJ[c - nI] = (int)ss; }
        }
    }
    __syncthreads();

    // 2. horizontal window sums of the left columns and the right columns, and their
    //    variances (window <= 13: n S_II - S_I^2 fits in int32) with reciprocal roots
    constexpr int n = WIN * WIN;
    for (int i = threadIdx.x; i < TX; i += kThreads) {
        int s = 0, ss = 0;
#pragma unroll
        for (int k = 0; k < WIN; ++k) { s += cI[i + k]; ss += cII[i + k]; }
        const int v = n * ss - s * s;
        QI[i] = make_int4(s, v, __float_as_int(v > 0 ? rsqrtf((float)v) : 0.0f), 0);
    }
    for (int i = threadIdx.x; i < TX + D - 1; i += kThreads) {
        int s = 0, ss = 0;
#pragma unroll
        for (int k = 0; k < WIN; ++k) { s += cJ[i + k]; ss += cJJ[i + k]; }
        const int v = n * ss - s * s;
        QJ[i] = make_int4(s, v, __float_as_int(v > 0 ? rsqrtf((float)v) : 0.0f), 0);
    }
    // 3. column products V[u][d] = sum over the window rows of left(u) * right(u - d)
    const int du = kThreads / D, dd = kThreads - du * D;  // step of (u, d) per kThreads elements
    {
        int u = threadIdx.x / D, d = threadIdx.x - u * D;
        for (int e = threadIdx.x; e < nI * D; e += kThreads) {
            const uint4 a = colI[u];
            const uint4 b = colJ[u - d + (D - 1)];  // right column uI0 + u - d
            unsigned s = __builtin_amdgcn_udot4(a.x, b.x, 0u, false);
            if (WIN > 4) s = __builtin_amdgcn_udot4(a.y, b.y, s, false);
            if (WIN > 8) s = __builtin_amdgcn_udot4(a.z, b.z, s, false);
            if (WIN > 12) s = __builtin_amdgcn_udot4(a.w, b.w, s, false);
            V[e] = (int)s;
            u += du;
            d += dd;
            if (d >= D) { d -= D; ++u; }
        }
    }
    __syncthreads();

    // 4. finish every (x, d) of the tile.  Thread t takes disparity d = t mod D and a run of
    //    XR consecutive columns, sliding the horizontal window sum along the run (two LDS
    //    reads per column instead of WIN); consecutive threads write consecutive d.  The
    //    loop body has no branch but the exact settle, which the wave takes only when one of
    //    its lanes lies near a rounding boundary.
    const int tileW = min(TX, W - x0);
    const int tpd = D >= kThreads ? 1 : kThreads / D;  // runs per disparity
    const int XR = (TX + tpd - 1) / tpd;
    const int d = threadIdx.x % D, run = threadIdx.x / D;
    if (run < tpd) {
        const int i0 = run * XR, i1 = min(i0 + XR, tileW);
        // the window's first WIN - 1 columns; each step adds its last column before use and
        // drops its first after
        int sij = 0;
        if (i0 < i1) {
#pragma unroll
            for (int k = 0; k < WIN - 1; ++k) sij += V[(i0 + k) * D + d];
        }
        long long o = ((long long)y * W + x0 + i0) * D + d;
        const float fscale = (float)scale;
        // the columns entering and leaving the window advance by a row of V a step (no index
        // products in the loop)
        const int* vin = V + (i0 + WIN - 1) * D + d;
        const int* vout = V + i0 * D + d;
        for (int i = i0; i < i1; ++i, o += D, vin += D, vout += D) {
            const int x = x0 + i;
            const bool outside = x - d < 0;  // no right pixel: the truncation cost
            const int u = outside ? 0 : i - d + (D - 1);
            // all four LDS reads first, so that they overlap
            const int4 qi = QI[i], qj = QJ[u];
            const int add = *vin, drop = *vout;
            __builtin_amdgcn_sched_barrier(0);
            sij += add;
            // window <= 13: every product and difference below fits in int32, and the factors
            // (n, S_IJ <= 169 * 255^2, S_I, S_J <= 169 * 255) fit the 24-bit multiplier
            const int num = (int)(__umul24((unsigned)n, (unsigned)sij) - __umul24((unsigned)qi.x, (unsigned)qj.x));
            const bool flat = qi.y == 0 || qj.y == 0;
            // fp32 estimate: c carries at most about 4 units of rounding (two conversions,
            // two reciprocal roots of 1 ulp, two products), relative error below 5e-7, so
            // |error of v| < 5e-7 * scale; within `margin` (>= 4e-6 * scale) of a rounding
            // boundary the exact test decides
            const float c = (float)num * (__int_as_float(qi.z) * __int_as_float(qj.z));
            const float v = fscale * (1.0f - c) + 0.5f;
            int k = (int)floorf(v);
            const float fr = v - (float)k;
            const bool settle = !outside && !flat && (fr < margin || fr > 1.0f - margin);
            if (settle) {
                const unsigned long long P = (unsigned long long)qi.y * (unsigned long long)qj.y;
                const long long B = 2LL * scale * num;
                while (!le_times_sqrt(B, 2LL * scale - 2LL * k + 1, P)) --k;
                while (le_times_sqrt(B, 2LL * scale - 2LL * (k + 1) + 1, P)) ++k;
            }
            k = flat ? scale : k;
            k = k < 0 ? 0 : (k > trunc ? trunc : k);
            cost[o] = (int16_t)(outside ? trunc : k);
            if (ncc_out) ncc_out[o] = outside ? -2.0f : (flat ? 0.0f : c);
            sij -= drop;
        }
    }
}

template <int WIN>
__global__ __launch_bounds__(kThreads) void k_ncc(const uint8_t* __restrict__ L, const uint8_t* __restrict__ R,
                                                   int W, int H, int D, int TX, int scale, int trunc, float margin,
                                                   int16_t* __restrict__ cost, float* __restrict__ ncc_out)
{
    extern __shared__ unsigned smem[];
    ncc_tile<WIN>(L, R, W, H, D, TX, scale, trunc, margin, cost, ncc_out, blockIdx.y, blockIdx.x * TX, smem);
}

// Every tile of every pair of a batch in one launch; tile_start[p] is the first tile of
// pair p (prefix sums, tile_start[n] = total), a pair's tiles run row-major over
// (row, column tile).
template <int WIN>
__global__ __launch_bounds__(kThreads) void k_ncc_batched(const NccPair* __restrict__ pairs, const int* tile_start,
                                                           int n, int scale, int trunc, float margin)
{
    extern __shared__ unsigned smem[];
    const int tile = blockIdx.x;
    int lo = 0, hi = n;  // find p with tile_start[p] <= tile < tile_start[p + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= tile) lo = mid;
        else hi = mid;
    }
    const NccPair P = pairs[lo];
    const int local = tile - tile_start[lo];
    const int TX = ncc_tile_x(P.D);
    const int tx = (P.W + TX - 1) / TX;
    const int y = local / tx, x0 = (local - y * tx) * TX;
    ncc_tile<WIN>(P.left, P.right, P.W, P.H, P.D, TX, scale, trunc, margin, P.cost, nullptr, y, x0, smem);
}

size_t ncc_lds_bytes(int D, int win, int TX)
{
    const int r = win >> 1;
    const int nI = TX + 2 * r, nJ = TX + 2 * r + D - 1;
    return (size_t)(nI + nJ) * 16 + (size_t)(TX + TX + D - 1) * 16 + (size_t)(2 * nI + 2 * nJ) * 4 +
           (size_t)nI * D * 4;
}

// Tile width of a single image: the batched width, halved (down to 32 columns) while the
// image would give fewer than 2048 workgroups, so that a small image still spreads over
// many compute units and each workgroup's serial part stays short.
int ncc_single_tile_x(int W, int H, int D)
{
    int TX = ncc_tile_x(D);
    while (TX > 32 && (long long)((W + TX - 1) / TX) * H < 2048) TX /= 2;
    return TX;
}

float ncc_margin(int scale) { return 1e-4f + 2e-6f * (float)(2 * scale + 1); }

}  // namespace

int ncc_tiles(int W, int H, int D) { return H * ((W + ncc_tile_x(D) - 1) / ncc_tile_x(D)); }

size_t ncc_lds_max(int max_d, int win)
{
    size_t m = 0;
    for (int D = 1; D <= max_d; ++D) m = ncc_lds_bytes(D, win, ncc_tile_x(D)) > m ? ncc_lds_bytes(D, win, ncc_tile_x(D)) : m;
    return m;
}

hipError_t launch_ncc(const uint8_t* L, const uint8_t* R, int W, int H, int D, int win, int scale, int trunc,
                      int16_t* cost, float* ncc, hipStream_t st)
{
    if ((win >> 1) > kMaxR) return hipErrorInvalidValue;
    const int TX = ncc_single_tile_x(W, H, D);
    dim3 grid((unsigned)((W + TX - 1) / TX), (unsigned)H);
    const size_t lds = ncc_lds_bytes(D, win, TX);
    const float m = ncc_margin(scale);
#define BPST_NCC(WV) \
    case WV: hipLaunchKernelGGL(k_ncc<WV>, grid, dim3(kThreads), lds, st, L, R, W, H, D, TX, scale, trunc, m, cost, ncc); \
        break;
    switch (win) {
        BPST_NCC(1) BPST_NCC(3) BPST_NCC(5) BPST_NCC(7) BPST_NCC(9) BPST_NCC(11) BPST_NCC(13)
        default: return hipErrorInvalidValue;
    }
#undef BPST_NCC
    return hipGetLastError();
}

hipError_t launch_ncc_batched(const NccPair* pairs, const int* tile_start, int n, int total_tiles, int max_d, int win,
                              int scale, int trunc, hipStream_t st)
{
    if ((win >> 1) > kMaxR) return hipErrorInvalidValue;
    if (total_tiles <= 0) return hipSuccess;
    const size_t lds = ncc_lds_max(max_d, win);  // the tile width, hence the LDS, depends on D
    const float m = ncc_margin(scale);
    const dim3 grid((unsigned)total_tiles);
#define BPST_NCCB(WV) \
    case WV: hipLaunchKernelGGL(k_ncc_batched<WV>, grid, dim3(kThreads), lds, st, pairs, tile_start, n, scale, trunc, m); \
        break;
    switch (win) {
        BPST_NCCB(1) BPST_NCCB(3) BPST_NCCB(5) BPST_NCCB(7) BPST_NCCB(9) BPST_NCCB(11) BPST_NCCB(13)
        default: return hipErrorInvalidValue;
    }
#undef BPST_NCCB
    return hipGetLastError();
}

}  // namespace bpst
