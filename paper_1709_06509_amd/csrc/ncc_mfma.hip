// Correlation volume on the matrix cores: the window sums of left x right products as int8
// MFMA tiles, everything else exact integer or guarded float arithmetic on the vector units.
//
// For one image row y and a left column x, the window product sum with the right column
// k = x - d is a dot product over the window's samples m = (channel, row j, column i):
//   S_IJ(x, k) = sum_m I(x + i - r, y + j - r)_c * J(k + i - r, y + j - r)_c.
// Over a 16 x 16 block of (k, x) that is one small matrix product, A[k][m] B[m][x], with the
// right view's window samples as the rows of A and the left view's as the columns of B.  The
// bytes enter as signed values v - 128 (v_mfma_i32_16x16x64_i8, int32 accumulation, exact);
// the offsets are put back with the window sums S_I, S_J:
//   sum I J = sum I'J' + 128 (S_I + S_J) - 128^2 N,      N = samples in the window.
// With n = window^2, a channel's zero-mean numerator is n S_IJc - S_Ic S_Jc, and pooled over
// the channels
//   num = n acc + P_x + sum_c S_Jc R_xc,   P_x = 128 n S_I - 128^2 n N,  R_xc = 128 n - S_Ic,
// two multiply-adds a channel per output.  ncc = num / sqrt(vI vJ) (vI = n sum_c S_IIc -
// sum_c S_Ic^2, likewise vJ); the quantised cost round-half-up(scale (1 - ncc)) comes from a
// float estimate and, within a margin of a rounding boundary, from an exact 128-bit test.
//
// K is laid out in 16-byte slots (channel, window column i): the window's rows of one image
// column, row j in byte j, zero past the window.  The views are staged in LDS the same way,
// one slot per image column (a transposed tile), so every operand of a lane is one aligned
// 16-byte read.  Lane l of v_mfma_i32_16x16x64_i8 supplies row / column l mod 16 and slot
// l / 16 of a K-step of four slots; its 4 results are rows 4 (l / 16) + v, column l mod 16.
//
// A workgroup takes row y and 64 left columns x0 .. x0 + 63 for every disparity; wave w owns
// the 16 columns xb = x0 + 16 w .. and runs nb blocks of 16 right columns kb = xb - 16 b
// (b = 0 .. nb - 1, nb = ceil((D - 1) / 16) + 1), which between them give every d in [0, D).
// Results go to LDS as [x][d] (rows padded against bank conflicts) and leave as one
// contiguous stretch of the cost volume.
#include <mutex>
#include <vector>

#include "internal.h"

namespace bpst {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kMThreads = 256;  // 4 waves
constexpr int kMTX = 64;        // left columns per workgroup (16 per wave)

__device__ __forceinline__ int clampm(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Is B <= A * sqrt(P) exactly?  (P > 0)
__device__ bool le_sqrt(long long B, long long A, unsigned long long P)
{
    typedef unsigned __int128 u128;
    const unsigned long long ab = (unsigned long long)(B < 0 ? -B : B);
    const unsigned long long aa = (unsigned long long)(A < 0 ? -A : A);
    const u128 b2 = (u128)ab * ab;
    const u128 a2p = (u128)(aa * aa) * P;
    if (A >= 0) return B <= 0 ? true : (b2 <= a2p);
    return B >= 0 ? false : (b2 >= a2p);
}

// The exact quantised cost next to a rounding boundary.  The cost is the largest k with
// k <= scale (1 - ncc) + 1/2, i.e. 2 scale num <= (2 scale - 2 k + 1) sqrt(vI vJ).  The float
// estimate kq lies within the margin (far below one) of it: with its fractional part near 0
// the cost is kq or kq - 1, near 1 it is kq + 1 or kq, so one exact comparison of the
// candidate decides.  vI, vJ > 0.
__device__ __noinline__ int settle_cost(int kq, bool up, int num, int vI, int vJ, int scale)
{
    const int kc = up ? kq + 1 : kq;
    // the comparison in double first: lhs = 2 scale num and A are exact, and A sqrt(vI vJ)
    // carries at most 3.5 * 2^-53 relative error (the product, the square root, the
    // multiplication), so a difference larger than 2^-49 of it has the exact sign; closer
    // calls (ties included) go to the 128-bit integer test
    const double A = 2.0 * (double)scale - 2.0 * (double)kc + 1.0;
    const double rhs = A * __builtin_sqrt((double)vI * (double)vJ);
    const double diff = rhs - 2.0 * (double)scale * (double)num;
    const double tol = __builtin_fabs(rhs) * 0x1p-49;
    if (diff > tol) return kc;
    if (diff < -tol) return kc - 1;
    const unsigned long long P = (unsigned long long)vI * (unsigned long long)vJ;
    return le_sqrt(2LL * scale * num, 2LL * scale - 2LL * kc + 1, P) ? kc : kc - 1;
}

__host__ __device__ inline int mfma_nb(int D) { return (D - 1 + 15) / 16 + 1; }

template <int WIN, int CH>
struct Shape {
    static constexpr int r = WIN / 2;
    static constexpr int NQ = CH * WIN;        // 16-byte slots of the K dimension
    static constexpr int KS = (NQ + 3) / 4;     // K-steps of 64 bytes (4 slots)
    static constexpr int n = WIN * WIN;
    static constexpr int NL = kMTX + 16;        // staged left columns x0 - r .. x0 - r + NL - 1
};

// Row pitch (int16) of the [x][d] results in LDS.  D a multiple of 8: D + 8, rows 16-byte
// aligned for the copy-out, and the 16 columns a wave writes at once land in at least 8
// banks; otherwise an odd number of dwords (all in different banks).
__host__ __device__ inline int out_pitch(int D) { return (D & 7) == 0 ? D + 8 : ((D & 1) ? D + 1 : D + 2); }

// LDS layout of one workgroup (bytes), for D disparities.
struct MLayout {
    int NR, NK;  // staged right columns, right columns with per-column data
    int stL, stR, colS, colQ, kS, kR, kV, out, total;
};

template <int WIN, int CH>
__host__ __device__ inline MLayout mlayout(int D)
{
    typedef Shape<WIN, CH> S;
    MLayout m;
    const int nb = mfma_nb(D);
    m.NK = 16 * (nb - 1) + kMTX;
    m.NR = m.NK + 16;
    int o = 0;
    m.stL = o; o += 16 * CH * S::NL;          // [channel][column][16] slots
    m.stR = o; o += 16 * CH * m.NR;
    const int ncol = S::NL + m.NR;
    m.colS = o; o += 4 * CH * ncol;          // per staged column: window-row sums of each channel
    m.colQ = o; o += 4 * ncol;               // and of the squares, channels pooled
    m.kS = o; o += 4 * CH * m.NK;             // per right column k: S_Jc
    m.kR = o; o += 4 * m.NK;                  // 1 / sqrt(vJ) (0 for a flat window)
    m.kV = o; o += 4 * m.NK;                  // vJ
    o = (o + 15) & ~15;
    m.out = o; o += 2 * kMTX * out_pitch(D);  // [x][d] results of the tile
    m.total = (o + 15) & ~15;
    return m;
}

template <int WIN, int CH>
__device__ __forceinline__ void ncc_mfma_tile(const uint8_t* __restrict__ L, const uint8_t* __restrict__ R, int W,
                                              int H, int D, int scale, int trunc, float margin,
                                              int16_t* __restrict__ cost, float* __restrict__ ncc_out, int y, int x0,
                                              unsigned char* smem)
{
    typedef Shape<WIN, CH> S;
    constexpr int r = S::r, NL = S::NL, n = S::n;
    static_assert(WIN <= 16, "a window column fills at most one 16-byte slot");
    const MLayout m = mlayout<WIN, CH>(D);
    const int nb = mfma_nb(D);
    const int kR0 = x0 - 16 * (nb - 1);  // first right column with per-column data
    const int uR0 = kR0 - r;            // first staged right column
    const int uL0 = x0 - r;             // first staged left column
    const int NR = m.NR, NK = m.NK, ncol = NL + NR;
    unsigned char* stL = smem + m.stL;
    unsigned char* stR = smem + m.stR;
    int* colS = reinterpret_cast<int*>(smem + m.colS);
    int* colQ = reinterpret_cast<int*>(smem + m.colQ);
    int* kS = reinterpret_cast<int*>(smem + m.kS);
    float* kR = reinterpret_cast<float*>(smem + m.kR);
    int* kV = reinterpret_cast<int*>(smem + m.kV);
    int16_t* out = reinterpret_cast<int16_t*>(smem + m.out);
    const int OP = out_pitch(D);

    // 1. stage the views (clamped to the image) as slots of signed v - 128, and each staged
    //    column's window-row sums of every channel and of the squares (pooled).  A thread
    //    takes whole columns and issues all of a column's loads before using any; the two
    //    views go in separate passes, so image and row addresses stay wave-uniform.
    //    Loads go through a buffer resource of the image (byte offsets below 2^31: at most
    //    16384 x 16384 x 3), the row's offset in a scalar register and the column's in a
    //    vector one, so addressing costs no vector arithmetic.
    auto stage = [&](const uint8_t* __restrict__ img, int u0, int ncols, unsigned char* st, int pitch, int t0) {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(img), (short)0, W * H * CH, 0x00020000);
        for (int tt = threadIdx.x; tt < ncols; tt += kMThreads) {
            const int off = clampm(u0 + tt, 0, W - 1) * CH;
            int vals[CH * WIN];
#pragma unroll
            for (int j = 0; j < WIN; ++j) {
                const int rowoff = clampm(y - r + j, 0, H - 1) * W * CH;
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    vals[c * WIN + j] = __builtin_amdgcn_raw_buffer_load_b8(rs, off + c, rowoff, 0);
            }
            int q = 0;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                unsigned wd[4] = {0u, 0u, 0u, 0u};
                int sum = 0;
#pragma unroll
                for (int j = 0; j < WIN; ++j) {
                    const int v = vals[c * WIN + j];
                    wd[j >> 2] |= (unsigned)(v ^ 0x80) << (8 * (j & 3));
                    sum += v;
                    q += v * v;
                }
                *reinterpret_cast<uint4*>(st + (c * pitch + tt) * 16) = make_uint4(wd[0], wd[1], wd[2], wd[3]);
                colS[c * ncol + t0 + tt] = sum;
            }
            colQ[t0 + tt] = q;
        }
    };
    stage(L, uL0, NL, stL, NL, 0);
    stage(R, uR0, NR, stR, NR, NL);
    __syncthreads();
    // 2. window sums, variance and reciprocal root of every right column k
    for (int kk = threadIdx.x; kk < NK; kk += kMThreads) {
        const int t0 = NL + kk;  // first staged column of the window
        int sc[CH];
        int q = 0;
#pragma unroll
        for (int c = 0; c < CH; ++c) sc[c] = 0;
#pragma unroll
        for (int i = 0; i < WIN; ++i) {
#pragma unroll
            for (int c = 0; c < CH; ++c) sc[c] += colS[c * ncol + t0 + i];
            q += colQ[t0 + i];
        }
        int v = n * q;
#pragma unroll
        for (int c = 0; c < CH; ++c) v -= sc[c] * sc[c];
#pragma unroll
        for (int c = 0; c < CH; ++c) kS[c * NK + kk] = sc[c];
        kR[kk] = v > 0 ? rsqrtf((float)v) : 0.0f;
        kV[kk] = v;
    }
    __syncthreads();

    // 3. per wave: 16 left columns, nb blocks of 16 right columns
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int lc = l & 15, g = l >> 4;
    const int xl = 16 * w + lc;  // this lane's left column, relative to x0
    const int x = x0 + xl;
    // this column's window sums (every lane of the column computes them)
    int SI[CH], RX[CH];
    int sI = 0, qI = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) SI[c] = 0;
#pragma unroll
    for (int i = 0; i < WIN; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) SI[c] += colS[c * ncol + xl + i];
        qI += colQ[xl + i];
    }
    int vI = n * qI;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        vI -= SI[c] * SI[c];
        sI += SI[c];
        RX[c] = 128 * n - SI[c];
    }
    const float rI = vI > 0 ? rsqrtf((float)vI) : 0.0f;
    // num is assembled in unsigned (wrap-around) arithmetic: its final value fits in int32
    // (|num| <= n * sum_c S_IJc < 2^31 for the supported windows), partial sums may not
    const unsigned Px = 128u * (unsigned)n * (unsigned)sI - 16384u * (unsigned)n * (unsigned)(CH * n);
    // the left view's operands, kept for every block: slot q = 4 s + g of the K-step s
    v4i bf[S::KS];
#pragma unroll
    for (int s = 0; s < S::KS; ++s) {
        const int q = 4 * s + g;
        v4i v = {0, 0, 0, 0};
        if (q < S::NQ) {
            const int c = q / WIN, i = q - c * WIN;
            v = *reinterpret_cast<const v4i*>(stL + (c * NL + xl + i) * 16);
        }
        bf[s] = v;
    }
    int16_t* o16 = out + (16 * w) * OP;  // this wave's [16][OP] results
    const float fscale = (float)scale, fbase = (float)scale + 0.5f;
    // The blocks are software-pipelined: the MFMAs of block b + 1 are issued before block b's
    // results are finished, so their latency hides under the vector work.
    auto block_mfma = [&](int b) {
        const int kkA = x0 + 16 * w - 16 * b - kR0 + lc;  // this lane's A row, relative to kR0
        v4i acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < S::KS; ++s) {
            const int q = 4 * s + g;
            v4i a = {0, 0, 0, 0};
            if (q < S::NQ) {
                const int c = q / WIN, i = q - c * WIN;
                a = *reinterpret_cast<const v4i*>(stR + (c * NR + kkA + i) * 16);
            }
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bf[s], acc, 0, 0, 0);
        }
        return acc;
    };
    v4i acc = block_mfma(0);
    for (int b = 0; b < nb; ++b) {
        const v4i cur = acc;
        if (b + 1 < nb) acc = block_mfma(b + 1);
        // results: rows k = kb + 4 g + v (v = 0..3), column x; kk0 is a multiple of 4, so the
        // four rows' per-column data are one 16-byte read per array
        const int kk0 = x0 + 16 * w - 16 * b - kR0 + 4 * g;
        int4 sj[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) sj[c] = *reinterpret_cast<const int4*>(kS + c * NK + kk0);
        const float4 rj = *reinterpret_cast<const float4*>(kR + kk0);
        const int4 vj = *reinterpret_cast<const int4*>(kV + kk0);
        int kqv[4], numv[4];
        unsigned near = 0;  // bit v: output v lies within the margin of a rounding boundary
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            // every factor fits the 24-bit multiplier: |acc| <= CH n 128^2, S_J <= n 255,
            // |R_x| <= 128 n; each product fits 32 bits
            unsigned un = Px + (unsigned)__mul24(n, cur[v]);
#pragma unroll
            for (int c = 0; c < CH; ++c) un += (unsigned)__mul24(sj[c][v], RX[c]);
            const int num = (int)un;
            const float cf = (float)num * (rI * rj[v]);
            const float vv = __builtin_fmaf(-fscale, cf, fbase);
            kqv[v] = (int)vv;  // vv > 0: truncation is the floor
            numv[v] = num;
            // within `margin` of a rounding boundary: fract(vv) near 0 or 1
            near |= __builtin_fabsf(__builtin_amdgcn_fractf(vv) - 0.5f) > 0.5f - margin ? 1u << v : 0u;
            if (ncc_out) {
                const bool flat = vI == 0 || vj[v] == 0;
                const bool outside = kR0 + kk0 + v < 0;
                const int d = x - (kR0 + kk0 + v);
                if (d >= 0 && d < D && x < W)
                    ncc_out[((long long)y * W + x) * D + d] = outside ? -2.0f : (flat ? 0.0f : cf);
            }
        }
        if (near) {
            // rare: settle the outputs next to a boundary exactly (a flat window's estimate
            // is exact, and a column with no right pixel takes the truncation cost below)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if ((near >> v) & 1u && vI > 0 && vj[v] > 0 && kR0 + kk0 + v >= 0) {
                    // the estimate again, for the side of the boundary it lies on
                    const float vv = __builtin_fmaf(-fscale, (float)numv[v] * (rI * rj[v]), fbase);
                    const bool up = __builtin_amdgcn_fractf(vv) > 0.5f;
                    kqv[v] = settle_cost(kqv[v], up, numv[v], vI, vj[v], scale);
                }
        }
        // a block whose 16 columns are all in the image, whose 16 right columns are all >= 0
        // and whose disparities d = x - k all lie in [0, D) stores without per-lane tests
        const int kb = x0 + 16 * w - 16 * b;
        const bool plain = kb >= 0 && x0 + 16 * w + 15 < W && 16 * b - 15 >= 0 && 16 * b + 15 < D;
        int16_t* orow = o16 + lc * OP + (lc + 16 * b - 4 * g - 3);  // d of v = 3; v = 0 is 3 above
        if (plain) {
#pragma unroll
            for (int v = 0; v < 4; ++v) orow[3 - v] = (int16_t)min(kqv[v], trunc);
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = kR0 + kk0 + v;
                const int d = x - k;
                int kq = kqv[v];
                kq = kq < 0 ? 0 : (kq > trunc ? trunc : kq);
                if (d >= 0 && d < D) o16[lc * OP + d] = (int16_t)(k < 0 ? trunc : kq);
            }
        }
    }
    __syncthreads();
    // 4. the tile's results are one contiguous stretch of the cost volume, x0 .. x0 + nx - 1
    const int nx = min(kMTX, W - x0);
    int16_t* dst = cost + ((long long)y * W + x0) * D;
    if ((D & 7) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        // 16-byte vectors: a row is D / 8 of them
        const int vr = D >> 3, op = OP >> 3;
        const uint4* src16 = reinterpret_cast<const uint4*>(out);
        uint4* dst16 = reinterpret_cast<uint4*>(dst);
        if ((vr & (vr - 1)) == 0) {
            const int sh = __builtin_ctz(vr);
            for (int e = threadIdx.x; e < nx * vr; e += kMThreads)
                dst16[e] = src16[(e >> sh) * op + (e & (vr - 1))];
        } else {
            for (int e = threadIdx.x; e < nx * vr; e += kMThreads) {
                const int row = e / vr, c16 = e - row * vr;
                dst16[e] = src16[row * op + c16];
            }
        }
    } else if ((D & 1) == 0 && (reinterpret_cast<uintptr_t>(dst) & 3) == 0) {
        // dwords: each wave copies rows, a row's dwords across the lanes
        const int dw = D >> 1, ow = OP >> 1;
        const unsigned* src32 = reinterpret_cast<const unsigned*>(out);
        unsigned* dst32 = reinterpret_cast<unsigned*>(dst);
        for (int row = w; row < nx; row += kMThreads / 64)
            for (int c2 = l; c2 < dw; c2 += 64) dst32[row * dw + c2] = src32[row * ow + c2];
    } else {
        for (int row = w; row < nx; row += kMThreads / 64)
            for (int c2 = l; c2 < D; c2 += 64) dst[row * D + c2] = out[row * OP + c2];
    }
}

// Every tile of every pair of a batch (grey views) in one launch; tile_start[p] is the first
// tile of pair p (prefix sums, tile_start[n] = total), a pair's tiles run row-major over
// (row, block of 64 columns).  The LDS is sized for the largest D; each tile lays out its own.
template <int WIN>
__global__ __launch_bounds__(kMThreads) void k_ncc_mfma_batched(const NccPair* __restrict__ pairs,
                                                                const int* __restrict__ tile_start, int n, int scale,
                                                                int trunc, float margin)
{
    extern __shared__ __align__(16) unsigned char msmem[];
    const int tile = blockIdx.x;
    int lo = 0, hi = n;  // find p with tile_start[p] <= tile < tile_start[p + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= tile) lo = mid;
        else hi = mid;
    }
    const NccPair P = pairs[lo];
    const int local = tile - tile_start[lo];
    const int tx = (P.W + kMTX - 1) / kMTX;
    const int y = local / tx, x0 = (local - y * tx) * kMTX;
    ncc_mfma_tile<WIN, 1>(P.left, P.right, P.W, P.H, P.D, scale, trunc, margin, P.cost, nullptr, y, x0, msmem);
}

template <int WIN, int CH>
__global__ __launch_bounds__(kMThreads) void k_ncc_mfma(const uint8_t* __restrict__ L, const uint8_t* __restrict__ R,
                                                        int W, int H, int D, int scale, int trunc, float margin,
                                                        int16_t* __restrict__ cost, float* __restrict__ ncc_out)
{
    extern __shared__ __align__(16) unsigned char msmem[];
    ncc_mfma_tile<WIN, CH>(L, R, W, H, D, scale, trunc, margin, cost, ncc_out, blockIdx.y, blockIdx.x * kMTX, msmem);
}

// Launches whose dynamic LDS exceeds 64 KB (colour views with D above about 250) need the
// kernel's limit raised, once per device (the attribute belongs to the device's copy).
template <int WIN, int CH>
hipError_t raise_lds_limit()
{
    static std::mutex mu;
    static std::vector<bool> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((size_t)dev < done.size() && done[dev]) return hipSuccess;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ncc_mfma<WIN, CH>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    if ((size_t)dev >= done.size()) done.resize(dev + 1, false);
    done[dev] = true;
    return hipSuccess;
}

template <int WIN, int CH>
hipError_t launch_mfma_t(const uint8_t* L, const uint8_t* R, int W, int H, int D, int scale, int trunc, float margin,
                         int16_t* cost, float* ncc, hipStream_t st)
{
    const MLayout m = mlayout<WIN, CH>(D);
    if (m.total > 160 * 1024) return hipErrorInvalidValue;  // never for D <= 256 (at most about 66 KB)
    if (m.total > 64 * 1024) {
        const hipError_t e = raise_lds_limit<WIN, CH>();
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)((W + kMTX - 1) / kMTX), (unsigned)H);
    hipLaunchKernelGGL((k_ncc_mfma<WIN, CH>), grid, dim3(kMThreads), (size_t)m.total, st, L, R, W, H, D, scale, trunc,
                       margin, cost, ncc);
    return hipGetLastError();
}

}  // namespace

// Margin of the float estimate v = scale (1 - c) + 1/2 around a rounding boundary.  The
// estimate c = float(num) (rsq(vI) rsq(vJ)) carries two conversions and three products
// (half an ulp each, 2^-24 relative) and two reciprocal roots (1 ulp each, 2^-23), so
// |c - ncc| <= |ncc| (4 * 2^-24 + 2 * 2^-23) < 4.8e-7; the fused multiply-add adds half an
// ulp of v <= 2 scale + 1/2.  Hence |v - exact| <= scale * 7.2e-7 + 1.2e-7 for every
// scale <= 4096.  The margin is about three times that (reciprocal roots up to three ulps
// off would still be caught); inside it the exact 128-bit test decides.
float ncc_margin_of(int scale) { return 2e-6f * (float)scale + 2e-5f; }

hipError_t launch_ncc_mfma(const uint8_t* L, const uint8_t* R, int W, int H, int D, int win, int channels, int scale,
                           int trunc, int16_t* cost, float* ncc, hipStream_t st)
{
    const float mg = ncc_margin_of(scale);
    if (channels == 1) {
        switch (win) {
            case 1: return launch_mfma_t<1, 1>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 3: return launch_mfma_t<3, 1>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 5: return launch_mfma_t<5, 1>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 7: return launch_mfma_t<7, 1>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 9: return launch_mfma_t<9, 1>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 11: return launch_mfma_t<11, 1>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 13: return launch_mfma_t<13, 1>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (channels == 3) {
        switch (win) {
            case 1: return launch_mfma_t<1, 3>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 3: return launch_mfma_t<3, 3>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 5: return launch_mfma_t<5, 3>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 7: return launch_mfma_t<7, 3>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            case 9: return launch_mfma_t<9, 3>(L, R, W, H, D, scale, trunc, mg, cost, ncc, st);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

int ncc_mfma_tiles(int W, int H) { return H * ((W + kMTX - 1) / kMTX); }

hipError_t launch_ncc_mfma_batched(const NccPair* pairs, const int* tile_start, int n, int total_tiles, int max_d,
                                   int win, int scale, int trunc, hipStream_t st)
{
    if (total_tiles <= 0) return hipSuccess;
    const float mg = ncc_margin_of(scale);
    const dim3 grid((unsigned)total_tiles);
#define BPST_NCCMB(WV)                                                                                         \
    case WV: {                                                                                                 \
        const size_t lds = (size_t)mlayout<WV, 1>(max_d).total;                                               \
        if (lds > 64 * 1024) return hipErrorInvalidValue;                                                     \
        hipLaunchKernelGGL(k_ncc_mfma_batched<WV>, grid, dim3(kMThreads), lds, st, pairs, tile_start, n, scale, \
                           trunc, mg);                                                                         \
        break;                                                                                                 \
    }
    switch (win) {
        BPST_NCCMB(1) BPST_NCCMB(3) BPST_NCCMB(5) BPST_NCCMB(7) BPST_NCCMB(9) BPST_NCCMB(11) BPST_NCCMB(13)
        default: return hipErrorInvalidValue;
    }
#undef BPST_NCCMB
    return hipGetLastError();
}

size_t ncc_mfma_lds(int D, int win, int channels)
{
#define BPST_ML(WV, CV) \
    if (win == WV && channels == CV) return (size_t)mlayout<WV, CV>(D).total;
    BPST_ML(1, 1) BPST_ML(3, 1) BPST_ML(5, 1) BPST_ML(7, 1) BPST_ML(9, 1) BPST_ML(11, 1) BPST_ML(13, 1)
    BPST_ML(1, 3) BPST_ML(3, 3) BPST_ML(5, 3) BPST_ML(7, 3) BPST_ML(9, 3)
#undef BPST_ML
    return 0;
}

}  // namespace bpst
