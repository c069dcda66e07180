// Learned warm start: a small CNN (3x3 convolutions, bf16 weights and activations, fp32
// accumulation on MFMA) that predicts the initial messages of the second-coarsest scale.
//
// Activations are NHWC bf16 [H][W][C_p] with C_p a multiple of 16 (padded channels hold 0);
// weights are bf16 [Cout_p][9][Cin_p] (tap t = 3*dy + dx).  A convolution is an implicit
// GEMM: D[pixel][co] = sum over (tap, ci) of A[pixel][(tap, ci)] * B[(tap, ci)][co], run on
// v_mfma_f32_16x16x32_bf16 with K = (tap, ci) flattened (k = tap * cin_p + ci) and walked 32
// at a time, zero past 9 cin_p.  Operand layout of that instruction (64 lanes, checked on the
// GPU): A[i][k] sits in lane i + 16*(k/8), element k%8; B[k][j] in lane j + 16*(k/8), element
// k%8; D[i][j] in lane j + 16*(i/4), element i%4.  cin_p is a multiple of 16, so a lane's 8
// consecutive k never straddle two taps.
//
// Reductions over pixels (weight and bias gradients, the loss) are split into fixed pixel
// chunks whose partial sums are added in chunk order, so results are deterministic.
#include <mutex>
#include <vector>

#include "internal.h"

namespace bpst {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kCT = 256;  // threads per workgroup

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// The same rounding (to nearest even) by the hardware conversion: the layers' activations,
// where it saves the integer sequence above on every output.
__device__ __forceinline__ uint16_t to_bf16_hw(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

typedef short v8s __attribute__((ext_vector_type(8)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_u16x2(unsigned v) { return __builtin_bit_cast(u16x2, v); }

// 8 bf16 at a 16-byte-aligned address (global or LDS)
__device__ __forceinline__ v8s load8(const uint16_t* p) { return *reinterpret_cast<const v8s*>(p); }

// K-steps of 32 over a 3x3 layer's flattened (tap, channel) dimension of 9 cin_p
__host__ __device__ constexpr int ksteps(int cin_p) { return (9 * cin_p + 31) / 32; }

// Weights of one workgroup's 32 output channels in LDS: row co holds [9][cin_p] plus 8
// elements of padding (rows stay 16-byte aligned, and the 16 rows one operand reads move
// across the banks).
constexpr int kLdsMaxCin = 112;
__host__ __device__ constexpr int wrow(int cin_p) { return 9 * cin_p + 8; }

// Forward convolution (also the data gradient, with flipped weights and a ReLU mask).
// One workgroup: 64 pixels x 32 output channels; wave w owns pixels 16w..16w+15.
//   out_bf16 [P][Cout_p] = bf16( act(acc + bias) ) where act = ReLU if relu, or
//                         acc * (mask[p][co] > 0) if mask (the ReLU derivative)
//   out_f32  [P][Cout_p] = the same value before bf16 rounding (nullable)
// K-step s covers k = 32 s .. 32 s + 31 of the flattened (tap, channel) dimension; lane group
// g = lane / 16 supplies k0 = 32 s + 8 g .. + 7: channels c .. c + 7 of tap k0 / cin_p.
// CS = cin_p / 16 when it is at most kLdsMaxCin / 16: the K loop is unrolled (its loads are
// in flight together) and the weights come from LDS; CS = 0: any cin_p, weights read from
// global memory.
template <int CS>
__global__ __launch_bounds__(kCT) void k_conv_fwd(const uint16_t* __restrict__ in, int H, int W, int cin_p,
                                                  const uint16_t* __restrict__ w, const float* __restrict__ bias,
                                                  int cout, int cout_p, int relu, const uint16_t* __restrict__ mask,
                                                  uint16_t* __restrict__ out_bf16, float* __restrict__ out_f32)
{
    extern __shared__ __align__(16) uint16_t wl[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int P = H * W;
    const int p = blockIdx.x * 64 + wave * 16 + (lane & 15);  // this lane's A row (pixel)
    const int py = p / W, px = p - py * W;
    const int g = lane >> 4;
    const int co0 = blockIdx.y * 32;
    const int cp = CS ? 16 * CS : cin_p;
    const int K = 9 * cp, NS = (K + 31) / 32;
    const int rs = CS ? wrow(16 * CS) : K;  // element stride between output channels
    const uint16_t* wb;
    if (CS) {
        // stage [32][9][cin_p] (contiguous in global memory) into padded LDS rows, 8 B at a time
        const uint16_t* src = w + (long long)co0 * K;
        const int per = K / 4;  // 8-byte pieces per row
        for (int e = threadIdx.x; e < 32 * per; e += kCT) {
            const int r = e / per, q = e - r * per;
            *reinterpret_cast<uint2*>(wl + r * rs + 4 * q) = *reinterpret_cast<const uint2*>(src + (long long)r * K + 4 * q);
        }
        __syncthreads();
        wb = wl;
    } else {
        wb = w + (long long)co0 * K;
    }
    const uint16_t* b0 = wb + (long long)(lane & 15) * rs;
    const uint16_t* b1 = wb + (long long)(16 + (lane & 15)) * rs;
    const v8s zero = {0, 0, 0, 0, 0, 0, 0, 0};
    v4f acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int s = 0; s < (CS ? ksteps(16 * CS) : 1); ++s) {
        for (int ss = s; ss < NS; ss += (CS ? NS : 1)) {  // CS: one pass; otherwise the runtime loop
            const int k0 = 32 * ss + 8 * g;
            const bool kv = k0 < K;
            const int tap = kv ? k0 / cp : 0, c = kv ? k0 - tap * cp : 0;
            const int ys = py + tap / 3 - 1, xs = px + tap % 3 - 1;
            const bool ok = kv && p < P && ys >= 0 && ys < H && xs >= 0 && xs < W;
            // out-of-image taps and k past the end read valid addresses and use zero
            const v8s av = load8(in + (ok ? ((long long)ys * W + xs) * cin_p + c : 0LL));
            const v8s bv0 = load8(b0 + (kv ? k0 : 0));
            const v8s bv1 = load8(b1 + (kv ? k0 : 0));
            const v8s a = ok ? av : zero;
            acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, kv ? bv0 : zero, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, kv ? bv1 : zero, acc[1], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int co = co0 + 16 * t + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = blockIdx.x * 64 + wave * 16 + (lane >> 4) * 4 + i;
            if (q >= P) continue;
            float v = 0.f;
            if (co < cout) {
                v = acc[t][i] + (bias ? bias[co] : 0.f);
                if (relu) v = fmaxf(v, 0.f);
                if (mask && from_bf16(mask[(long long)q * cout_p + co]) <= 0.f) v = 0.f;
            }
            if (out_bf16) out_bf16[(long long)q * cout_p + co] = to_bf16_hw(v);
            if (out_f32) out_f32[(long long)q * cout_p + co] = v;
        }
    }
}

// w' [Cin_p][9][Cout_p] with w'[ci][8 - t][co] = w[co][t][ci]: the data gradient of a 3x3
// convolution with zero padding is the convolution of the output gradient with w'.
__global__ void k_flip(const uint16_t* __restrict__ w, int cin_p, int cout_p, uint16_t* __restrict__ wf)
{
    const long long n = (long long)cout_p * 9 * cin_p;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int ci = (int)(i % cin_p);
        const int t = (int)((i / cin_p) % 9);
        const int co = (int)(i / ((long long)cin_p * 9));
        wf[((long long)ci * 9 + (8 - t)) * cout_p + co] = w[i];
    }
}

// Weight gradient partials: dW[co][t][ci] = sum_p g[p][co] * in[p + tap offset][ci] over pixel
// chunk s; one workgroup per (chunk, tap, 32 output channels, 16 input channels).  The four
// waves take interleaved 16-pixel steps and are summed in a fixed order at the end.
__global__ __launch_bounds__(kCT) void k_conv_wgrad(const uint16_t* __restrict__ in, const uint16_t* __restrict__ g,
                                                    int H, int W, int cin_p, int cout_p, int chunk,
                                                    float* __restrict__ part)
{
    __shared__ float red[4][32][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int s = blockIdx.x, tap = blockIdx.y % 9;
    const int co0 = (blockIdx.y / 9) * 32, ci0 = blockIdx.z * 16;
    const int P = H * W;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int pbeg = s * chunk, pend = min(P, pbeg + chunk);
    v4f acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    const int kq = (lane >> 4) * 4;
    for (int p0 = pbeg + wave * 16; p0 < pend; p0 += 64) {
        // A[co][k = pixel], B[k = pixel][ci]
        v4s a0, a1, b;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = p0 + kq + v;
            short ga0 = 0, ga1 = 0, bx = 0;
            if (p < pend) {
                ga0 = (short)g[(long long)p * cout_p + co0 + (lane & 15)];
                ga1 = (short)g[(long long)p * cout_p + co0 + 16 + (lane & 15)];
                const int py = p / W, px = p - py * W;
                const int ys = py + dy, xs = px + dx;
                if (ys >= 0 && ys < H && xs >= 0 && xs < W)
                    bx = (short)in[((long long)ys * W + xs) * cin_p + ci0 + (lane & 15)];
            }
            a0[v] = ga0;
            a1[v] = ga1;
            b[v] = bx;
        }
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b, acc[1], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wave][16 * t + (lane >> 4) * 4 + i][lane & 15] = acc[t][i];
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 16; e += kCT) {
        const int r = e / 16, c = e % 16;
        const float v = ((red[0][r][c] + red[1][r][c]) + red[2][r][c]) + red[3][r][c];
        part[(((long long)s * cout_p + co0 + r) * 9 + tap) * cin_p + ci0 + c] = v;
    }
}

// Bias gradient partials: sum over pixel chunk s of g[p][co].  Workgroup (s, 64 channels):
// wave w adds the pixels p = w (mod 4) of the chunk with four independent accumulators (so
// four loads are in flight), then the four waves' sums are added in wave order.
__global__ __launch_bounds__(kCT) void k_bgrad(const uint16_t* __restrict__ g, int P, int cout_p, int chunk,
                                               float* __restrict__ part)
{
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int s = blockIdx.x, co = blockIdx.y * 64 + lane;
    const int pbeg = s * chunk, pend = min(P, pbeg + chunk);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (co < cout_p) {
        int p = pbeg + wave;
        for (; p + 12 < pend; p += 16) {
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] += from_bf16(g[(long long)(p + 4 * j) * cout_p + co]);
        }
        for (; p < pend; p += 4) acc[0] += from_bf16(g[(long long)p * cout_p + co]);
    }
    red[wave][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (wave == 0 && co < cout_p)
        part[(long long)s * cout_p + co] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// out[i] = sum over s (in order) of part[s][i]
__global__ void k_reduce_chunks(const float* __restrict__ part, int S, long long n, float* __restrict__ out)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int s = 0; s < S; ++s) acc += part[(long long)s * n + i];
        out[i] = acc;
    }
}

// Mean L1 loss of y*lamT against the label messages over the slots with a neighbour, and its
// gradient with respect to y (bf16, the last layer's output gradient) into g [P][cout_p].
__global__ void k_l1(const float* __restrict__ y, const int16_t* __restrict__ label, int H, int W, int D, int cout_p,
                     float lam_t, float inv_n, uint16_t* __restrict__ g, float* __restrict__ part)
{
    __shared__ float red[kCT];
    const int P = H * W;
    float acc = 0.f;
    for (long long i = (long long)blockIdx.x * kCT + threadIdx.x; i < (long long)P * cout_p;
         i += (long long)gridDim.x * kCT) {
        const int c = (int)(i % cout_p);
        const int p = (int)(i / cout_p);
        float grad = 0.f;
        if (c < 4 * D) {
            const int k = c / D, d = c - k * D;
            const int py = p / W, px = p - py * W;
            const bool has = k == 0 ? px > 0 : k == 1 ? px < W - 1 : k == 2 ? py > 0 : py < H - 1;
            if (has) {
                // fused: r is y*lam_t - label rounded once, so its sign is the exact one
                const float r = fmaf(y[i], lam_t, -(float)label[(((long long)k * H + py) * W + px) * D + d]);
                acc += fabsf(r);
                grad = (r > 0.f ? lam_t : (r < 0.f ? -lam_t : 0.f)) * inv_n;
            }
        }
        g[i] = to_bf16(grad);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kCT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv_n;
}

// *out = sum of part[0..n), in fp64 and in a fixed order: thread t adds t, t + 256, ...,
// then a fixed halving tree over the threads.  One workgroup of kCT threads.
__global__ __launch_bounds__(kCT) void k_sum_ordered(const float* __restrict__ part, int n, float* __restrict__ out)
{
    __shared__ double red[kCT];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kCT) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kCT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)red[0];
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       uint16_t* __restrict__ w16, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        w16[i] = to_bf16(wi);
    }
}

__global__ void k_to_bf16(const float* __restrict__ x, long long n, uint16_t* __restrict__ out)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = to_bf16(x[i]);
}

// CNN input at scale s: views box-averaged over 2^s x 2^s blocks / 255, and the coarsest
// cost (internal layout of scale s+1, Dp labels) of the pixel's parent / 1024; bf16.  One
// thread per output channel, so writes (and the cost reads) are contiguous.
__global__ void k_warm_input(const uint8_t* __restrict__ L, const uint8_t* __restrict__ R, int W, int H, int s,
                             const int16_t* __restrict__ coarse, Level lc, int Dp, int D, int Ws, int Hs, int cin_p,
                             uint16_t* __restrict__ out)
{
    const long long n = (long long)Ws * Hs * cin_p;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % cin_p);
        const long long pix = i / cin_p;
        const int Y = (int)(pix / Ws), X = (int)(pix - (long long)Y * Ws);
        float v = 0.f;
        if (ch < 2) {
            const uint8_t* img = ch == 0 ? L : R;
            const int B = 1 << s;
            int sum = 0, cnt = 0;
            for (int y = Y * B; y < (Y + 1) * B && y < H; ++y)
                for (int x = X * B; x < (X + 1) * B && x < W; ++x) {
                    sum += img[(long long)y * W + x];
                    ++cnt;
                }
            v = (float)sum / ((float)cnt * 255.0f);
        } else if (ch < 2 + D) {
            const int cx = X >> 1, cy = Y >> 1;
            v = (float)coarse[((long long)(2 * cy + ((cx + cy) & 1)) * lc.Wh + (cx >> 1)) * Dp + (ch - 2)] / 1024.0f;
        }
        out[i] = to_bf16(v);
    }
}

// Messages [4][Hs][Ws][D] from the CNN output y [Hs][Ws][ystride] (channel k*D + d).  One
// message (side k of one pixel) per group of GS lanes (GS = D rounded up to a power of two,
// at most 64); lane j of a group takes the labels j, j + GS, ..., so reads and writes are
// contiguous, and the group's minimum comes from a butterfly of lane exchanges.
template <int GS>
__global__ __launch_bounds__(kCT) void k_warm_messages(const float* __restrict__ y, int Ws, int Hs, int D, int ystride,
                                                       int lam_t, int16_t* __restrict__ out)
{
    constexpr int kMaxPer = GS < 64 ? 1 : 4;  // labels per lane (D <= GS below 64, D <= 256)
    const long long n = 4LL * Ws * Hs;
    const int j = threadIdx.x & (GS - 1);
    const long long first = ((long long)blockIdx.x * kCT + threadIdx.x) / GS;
    const long long step = (long long)gridDim.x * (kCT / GS);
    for (long long i = first; i < n; i += step) {  // uniform per group: GS divides 64
        const int k = (int)(i / ((long long)Ws * Hs));
        const long long pix = i - (long long)k * Ws * Hs;
        const int Y = (int)(pix / Ws), X = (int)(pix - (long long)Y * Ws);
        const bool has = k == 0 ? X > 0 : k == 1 ? X < Ws - 1 : k == 2 ? Y > 0 : Y < Hs - 1;
        int16_t* o = out + i * D;
        const float* yy = y + pix * ystride + k * D;
        int q[kMaxPer];
        int mn = 0x7fffffff;
#pragma unroll
        for (int t = 0; t < kMaxPer; ++t) {
            const int d = j + t * GS;
            q[t] = 0;
            if (d < D && has) {
                const float r = rintf(yy[d] * (float)lam_t);
                q[t] = r < 0.f ? 0 : (r > (float)lam_t ? lam_t : (int)r);
                mn = min(mn, q[t]);
            }
        }
#pragma unroll
        for (int w = 1; w < GS; w <<= 1) mn = min(mn, __shfl_xor(mn, w, GS));
        if (!has) mn = 0;
#pragma unroll
        for (int t = 0; t < kMaxPer; ++t) {
            const int d = j + t * GS;
            if (d < D) o[d] = (int16_t)(q[t] - mn);
        }
    }
}

// ---- the whole warm start of one scale in one launch ----
//
// A workgroup of 8 waves takes a tile of kWTW x kWTH pixels of scale s.  A 3x3 layer's output
// over a region needs its input over the region grown by one pixel a side, so the six layers
// run over regions that shrink from the tile plus a 5-pixel border (layer 1) to the tile
// itself (layer 6), and the network input is needed over the tile plus 6.  Nothing but the
// messages leaves the workgroup:
//   - the input is formed in LDS, one [pixel][channel] row per pixel of the input region:
//     the views' box averages per pixel and the parent's coarse cost (both bf16, rounded as
//     the input kernel rounds them) written to each of the parent's pixels;
//   - hidden activations (32 channels, bf16) ping-pong between two LDS buffers;
//   - a layer stores its outputs as computed; where its region reaches outside the image,
//     those positions are then cleared to 0, the zero padding the next layer reads there, so
//     no operand needs a bounds test;
//   - the last layer's outputs are quantised in registers and staged in LDS; the copy-out
//     takes each message's minimum over d (DPP across the lanes holding its pieces) and
//     subtracts it as it stores 16-byte vectors into the scale's message volumes
//     (colour-split slots, Dp labels), with the state bytes a warm-started scale begins with.
// Every output is computed as the layer-by-layer path computes it: the same MFMA, the same
// K order (32-wide steps of the flattened (tap, channel) dimension), the same bias, ReLU and
// bf16 rounding, the same quantisation, so the messages are bit-identical.  A wave keeps the
// weight fragments it needs for a layer in registers (every workgroup reads the same
// weights: they stay in the caches).
constexpr int kWT = 512;             // threads per workgroup (8 waves)
constexpr int kWWaves = kWT / 64;
constexpr int kWTW = 10, kWTH = 8;   // tile of scale s (240 workgroups at 160 x 120)
constexpr int kWIW = kWTW + 12, kWIH = kWTH + 12;          // network input region
constexpr int kWPW = kWIW / 2, kWPH = kWIH / 2;            // parents of the input region (2 x 2 pixels each)
constexpr int kWAS = 40;             // bf16 per pixel of an activation buffer: 32 channels + 8 (16-byte rows, banks)
constexpr int kWN = kWTW * kWTH;     // pixels of the tile
static_assert(kWTW % 2 == 0 && kWTH % 2 == 0, "even tiles: the parent region starts at an exact half");

__host__ __device__ constexpr int warm_act_pixels(int halo) { return (kWTW + 2 * halo) * (kWTH + 2 * halo); }
// Rows of an activation buffer: the region's pixels rounded up to whole 16-pixel blocks (the
// rows past the region take a block's unused results, so stores need no bounds test).
__host__ __device__ constexpr int warm_act_rows(int halo) { return (warm_act_pixels(halo) + 15) / 16 * 16; }
// Pitch (bf16) of a pixel's row of network input: 16 NC1 channels + 8 (16-byte rows; the
// 16 pixels one operand reads spread over the banks).
__host__ __device__ constexpr int warm_in_pitch(int cin0) { return cin0 + 8; }

// Staged messages of one tile pixel (int16 elements): 4 D, padded so that the rows four pixels
// apart fall on different banks.
__host__ __device__ constexpr int warm_msg_stride(int D) { return 4 * D + 8; }
// Labels per message slot in the solve's volumes for the D the network supports (8 times the
// power of two of lanes per pixel: 16, 32, 64, 64 for D = 16, 32, 48, 64).
__host__ __device__ constexpr int warm_dp(int D) { return D <= 16 ? 16 : (D <= 32 ? 32 : 64); }

// LDS: region 1 holds the activations of layers 1, 3, 5; region 2 holds the network input,
// then the activations of layers 2 and 4, then the last layer's staged messages.
__host__ __device__ inline size_t warm_r1(int)
{
    return ((size_t)warm_act_rows(5) * kWAS * 2 + 15) / 16 * 16;  // region 2 starts 16-byte aligned
}
__host__ __device__ inline size_t warm_r2(int cin0, int D)
{
    const size_t inp = (size_t)kWIW * kWIH * warm_in_pitch(cin0) * 2;
    const size_t act = (size_t)warm_act_rows(4) * kWAS * 2;
    const size_t last = (size_t)kWN * warm_msg_stride(D) * 2;  // staged messages
    size_t m = inp > act ? inp : act;
    return m > last ? m : last;
}
__host__ __device__ inline size_t warm_cnn_lds(int cin0, int D) { return warm_r1(cin0) + warm_r2(cin0, D); }


// The weight fragments (B operands) of one wave for a 3x3 layer of cin_p = 16 NC input
// channels: output channel co, every K-step (zero past 9 cin_p), lane layout of the MFMA.
template <int NC>
__device__ __forceinline__ void warm_frags(const WarmCnnArgs& a, int layer, int co, v8s (&bf)[ksteps(16 * NC)])
{
    constexpr int K = 9 * 16 * NC;
    const int g = (threadIdx.x & 63) >> 4;
    const uint16_t* bw = a.w16 + a.w_off[layer] + (long long)co * K;
#pragma unroll
    for (int s = 0; s < ksteps(16 * NC); ++s) {
        const int k0 = 32 * s + 8 * g;
        const v8s v = load8(bw + (k0 < K ? k0 : 0));
        bf[s] = k0 < K ? v : v8s{0, 0, 0, 0, 0, 0, 0, 0};
    }
}

// Offset (bf16) of lane group g's operand at K-step s in a region whose pixel rows are PITCH
// apart and IWl pixels wide, relative to the pixel's row at tap (0, 0); -1 past 9 cin_p.
template <int NC, int PITCH>
__device__ __forceinline__ int warm_koff(int s, int g, int IWl)
{
    constexpr int cp = 16 * NC;
    const int k0 = 32 * s + 8 * g;
    if (k0 >= 9 * cp) return -1;
    const int tap = k0 / cp, c = k0 - tap * cp;
    return ((tap / 3) * IWl + (tap % 3)) * PITCH + c;
}

// NP blocks of 16 region pixels (b0, b0 + 4, ...) of one 3x3 layer, 32 output channels, over
// the region of halo HO around the tile: output pixel q of the region (row-major, width
// kWTW + 2 HO) from the input region of halo HO + 1 (rows of PITCH bf16 per pixel).  The
// caller's fragments bf and bias are those of output channel 16 t + i (t = wave / 4); the NP
// accumulation chains share each weight fragment.
template <int NC, int PITCH, int HO, int NP>
__device__ __forceinline__ void warm_blocks(const WarmCnnArgs& a, const v8s (&bf)[ksteps(16 * NC)], float bias, int x0,
                                            int y0, const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int b0)
{
    constexpr int OW = kWTW + 2 * HO, N = OW * (kWTH + 2 * HO), IWl = OW + 2;
    constexpr int NS = ksteps(16 * NC);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4, t = wave >> 2;
    const v8s zero = {0, 0, 0, 0, 0, 0, 0, 0};
    // this lane's A row in each block: its input row at tap (0, 0) (rows past the region read
    // row 0; their results go to the buffer's padding rows)
    const uint16_t* arow[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int q = 16 * (b0 + 4 * p) + i;
        const int ry = q < N ? q / OW : 0, rx = q < N ? q - (q / OW) * OW : 0;
        arow[p] = in + (ry * IWl + rx) * PITCH;
    }
    v4f acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = v4f{0.f, 0.f, 0.f, 0.f};
    // operands are read PD K-steps ahead of their use (a ring of PD + 1 slots)
    constexpr int PD = 3;
    v8s ring[PD + 1][NP];
    auto fetch = [&](int s) {
        const int off = warm_koff<NC, PITCH>(s, g, IWl);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const v8s av = load8(arow[p] + (off < 0 ? 0 : off));
            ring[s % (PD + 1)][p] = off < 0 ? zero : av;
        }
    };
#pragma unroll
    for (int s = 0; s < PD && s < NS; ++s) fetch(s);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (s + PD < NS) fetch(s + PD);
#pragma unroll
        for (int p = 0; p < NP; ++p)
            acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ring[s % (PD + 1)][p], bf[s], acc[p], 0, 0, 0);
    }
    // results: rows 4 g + e of block p (region pixels), column i (channel 16 t + i), stored as
    // computed (rows past the region go to the buffer's padding rows; region positions outside
    // the image are cleared afterwards, warm_clear_outside)
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            out[(16 * (b0 + 4 * p) + 4 * g + e) * kWAS + 16 * t + i] = to_bf16_hw(fmaxf(acc[p][e] + bias, 0.f));
}

// Whether the region of halo HO around the tile reaches outside the image (uniform over the
// workgroup).
template <int HO>
__device__ __forceinline__ bool warm_edge(int x0, int y0, int Ws, int Hs)
{
    return x0 - HO < 0 || y0 - HO < 0 || x0 + kWTW + HO > Ws || y0 + kWTH + HO > Hs;
}

// Zero the positions of the region of halo HO that lie outside the image (the next layer's
// zero padding there), 32 channels as four 16-byte pieces; after the layer's stores.
template <int HO>
__device__ __forceinline__ void warm_clear_outside(int x0, int y0, int Ws, int Hs, uint16_t* __restrict__ out)
{
    constexpr int OW = kWTW + 2 * HO, N = OW * (kWTH + 2 * HO);
    for (int e = threadIdx.x; e < N * 4; e += kWT) {
        const int q = e >> 2, c = e & 3;
        const int oy = q / OW, ox = q - oy * OW;
        const int Yo = y0 - HO + oy, Xo = x0 - HO + ox;
        if (Yo < 0 || Yo >= Hs || Xo < 0 || Xo >= Ws)
            *reinterpret_cast<uint4*>(out + q * kWAS + 8 * c) = make_uint4(0u, 0u, 0u, 0u);
    }
}

// One 3x3 layer over the region of halo HO.  Waves 0-3 compute output channels 0-15, waves
// 4-7 channels 16-31; wave w takes blocks w % 4, w % 4 + 4, ... in pairs (the last one alone
// when the count is odd).
template <int NC, int PITCH, int HO>
__device__ __forceinline__ void warm_layer(const WarmCnnArgs& a, const v8s (&bf)[ksteps(16 * NC)], float bias, int x0,
                                           int y0, const uint16_t* __restrict__ in, uint16_t* __restrict__ out)
{
    constexpr int NBLK = (warm_act_pixels(HO) + 15) / 16;
    const int wq = (threadIdx.x >> 6) & 3;
    for (int b0 = wq; b0 < NBLK; b0 += 8) {
        if (b0 + 4 < NBLK)
            warm_blocks<NC, PITCH, HO, 2>(a, bf, bias, x0, y0, in, out, b0);
        else
            warm_blocks<NC, PITCH, HO, 1>(a, bf, bias, x0, y0, in, out, b0);
    }
}

// Layer 1 (the region of halo 5, 16 NC input channels) with every wave computing all 32
// output channels for its blocks (w, w + 8, w + 16), so each operand read from LDS feeds two
// MFMAs (channels i and 16 + i) and the layer reads its operands once, not once per channel
// half.  The weights of both halves stream through registers in chunks of kW1Chunk K-steps,
// the next chunk's loads in flight while a chunk runs.  Every output still accumulates its
// K-steps in order, as warm_blocks does.
constexpr int kW1Chunk = 6;

// The weight fragments of K-steps kW1Chunk c .. of output channels i and 16 + i (zero past the
// last step and past 9 cin_p).
template <int NC>
__device__ __forceinline__ void warm_l1_chunk(const WarmCnnArgs& a, int c, v8s (&dst)[2][kW1Chunk])
{
    constexpr int K = 9 * 16 * NC;
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    const uint16_t* bw = a.w16 + a.w_off[0] + (long long)i * K;
    const v8s zero = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < kW1Chunk; ++j) {
        const int k0 = 32 * (c * kW1Chunk + j) + 8 * g;
        const bool ok = k0 < K;
        const v8s v0 = load8(bw + (ok ? k0 : 0)), v1 = load8(bw + 16LL * K + (ok ? k0 : 0));
        dst[0][j] = ok ? v0 : zero;
        dst[1][j] = ok ? v1 : zero;
    }
}

template <int NC, int PITCH>
__device__ __forceinline__ void warm_layer1(const WarmCnnArgs& a, v8s (&wb)[2][2][kW1Chunk], int x0, int y0,
                                            const uint16_t* __restrict__ in, uint16_t* __restrict__ out)
{
    constexpr int HO = 5, OW = kWTW + 2 * HO, N = OW * (kWTH + 2 * HO), IWl = OW + 2;
    constexpr int NS = ksteps(16 * NC), NBLK = (N + 15) / 16, MB = (NBLK + kWWaves - 1) / kWWaves;
    constexpr int NCH = (NS + kW1Chunk - 1) / kW1Chunk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    const v8s zero = {0, 0, 0, 0, 0, 0, 0, 0};
    const float bias0 = a.params[a.b_off[0] + i], bias1 = a.params[a.b_off[0] + 16 + i];
    // this lane's A row in each of its blocks (rows past the region read row 0; their results
    // go to the buffer's padding rows)
    const uint16_t* arow[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        const int q = 16 * (wave + kWWaves * m) + i;
        const int ry = q < N ? q / OW : 0, rx = q < N ? q - (q / OW) * OW : 0;
        arow[m] = in + (ry * IWl + rx) * PITCH;
    }
    v4f acc[MB][2];
#pragma unroll
    for (int m = 0; m < MB; ++m) acc[m][0] = acc[m][1] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (c + 1 < NCH) warm_l1_chunk<NC>(a, c + 1, wb[(c + 1) & 1]);
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            if (wave + kWWaves * m >= NBLK) continue;  // uniform over the wave
            // the chunk's operands of the block, all read before the first product
            v8s av[kW1Chunk];
#pragma unroll
            for (int j = 0; j < kW1Chunk; ++j) {
                const int off = warm_koff<NC, PITCH>(c * kW1Chunk + j, g, IWl);
                const v8s v = load8(arow[m] + (off < 0 ? 0 : off));
                av[j] = off < 0 ? zero : v;
            }
#pragma unroll
            for (int j = 0; j < kW1Chunk; ++j) {
                if (c * kW1Chunk + j >= NS) break;
                acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[j], wb[c & 1][0][j], acc[m][0], 0, 0, 0);
                acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[j], wb[c & 1][1][j], acc[m][1], 0, 0, 0);
            }
        }
    }
    // results: rows 4 g + e of each block, channels i and 16 + i, stored as computed (region
    // positions outside the image are cleared afterwards, warm_clear_outside)
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        if (wave + kWWaves * m >= NBLK) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            uint16_t* o = out + (16 * (wave + kWWaves * m) + 4 * g + e) * kWAS;
            o[i] = to_bf16_hw(fmaxf(acc[m][0][e] + bias0, 0.f));
            o[16 + i] = to_bf16_hw(fmaxf(acc[m][1][e] + bias1, 0.f));
        }
    }
}

template <int NC1, int T>
__global__ __launch_bounds__(kWT) void k_warm_cnn(WarmCnnArgs a)
{
    extern __shared__ __align__(16) uint16_t wsm[];
    constexpr int cin0 = 16 * NC1, D = 16 * T, IP = warm_in_pitch(cin0);
    uint16_t* r1 = wsm;
    uint16_t* r2 = wsm + warm_r1(cin0) / 2;
    uint16_t* inp = r2;                              // [kWIH][kWIW][IP]
    uint16_t* actA = r1;                             // layers 1, 3, 5
    uint16_t* actB = r2;                             // layers 2, 4
    const int x0 = blockIdx.x * kWTW, y0 = blockIdx.y * kWTH;
    const int px0 = (x0 - 6) / 2, py0 = (y0 - 6) / 2;  // exact: x0, y0 are even
    const int Ws = a.lv.W, Hs = a.lv.H;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    const int co = 16 * (wave >> 2) + i;  // this lane's output channel in layers 1-5

    v8s w1[2][2][kW1Chunk];  // the first layer's weights, chunk by chunk (warm_layer1)

    // the network input, one row of cin0 channels per pixel of the input region, 0 at pixels
    // outside the image: channels 0 and 1 the views averaged over the 2^s x 2^s block of each
    // pixel (clipped at the image), / 255, bf16; channels 2 .. D + 1 the parent's cost at
    // scale s + 1, / 1024, bf16 (four channels an item, written to each of the parent's
    // pixels); the padding channels 0.  Every global load of the phase is issued before any
    // is used: the views' bytes (up to 4 x 4 blocks, each from a valid address, masked), then
    // the parents' costs.
    const int Bs = 1 << a.s;
    {
        constexpr int NI = 2 * kWIW * kWIH, NIT = (NI + kWT - 1) / kWT;
        constexpr int NP = kWPW * kWPH * (cin0 / 4), NPT = (NP + kWT - 1) / kWT;
        unsigned d0[NIT][4], d1[NIT][4];  // up to 4 x 4 blocks: per row, the aligned words holding its bytes
        int ny[NIT], nx[NIT], bsum[NIT];
        bool in_img[NIT];
#pragma unroll
        for (int j = 0; j < NIT; ++j) {
            const int e = threadIdx.x + j * kWT;
            const int v = e / (kWIW * kWIH), r = e - v * (kWIW * kWIH);
            const int ry = r / kWIW, rx = r - ry * kWIW;
            const int Y = y0 - 6 + ry, X = x0 - 6 + rx;
            in_img[j] = e < NI && Y >= 0 && Y < Hs && X >= 0 && X < Ws;
            ny[j] = in_img[j] ? min(Bs, a.H - Y * Bs) : 0;  // >= 1 in the image: (Y, X) is in scale s
            nx[j] = in_img[j] ? min(Bs, a.W - X * Bs) : 0;
            const uint8_t* base = (v == 0 ? a.left : a.right) + (in_img[j] ? (long long)(Y * Bs) * a.W + X * Bs : 0);
            bsum[j] = 0;
            if (Bs <= 4) {
                // a row's nx bytes from the one or two 4-byte-aligned words that hold them (each
                // word holds a byte of the view, so it lies in the view's pages); rows past ny
                // read row 0
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const uintptr_t ra = reinterpret_cast<uintptr_t>(base) + (jj < ny[j] ? (uintptr_t)jj * a.W : 0);
                    const unsigned sh = (unsigned)(ra & 3u);
                    const unsigned* wp = reinterpret_cast<const unsigned*>(ra - sh);
                    d0[j][jj] = wp[0];
                    d1[j][jj] = wp[sh + nx[j] > 4 ? 1 : 0];
                }
            } else {
                for (int jj = 0; jj < ny[j]; ++jj)
                    for (int k = 0; k < nx[j]; ++k) bsum[j] += base[(long long)jj * a.W + k];
            }
        }
        unsigned lo[NPT], hi[NPT];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int e = threadIdx.x + j * kWT;
            const int c4 = e % (cin0 / 4), pp = e / (cin0 / 4);
            const int pr = pp / kWPW, pc = pp - pr * kWPW;
            const int cy = py0 + pr, cx = px0 + pc;
            const bool inside = e < NP && cy >= 0 && cy < a.lc.H && cx >= 0 && cx < a.lc.W;
            const int16_t* src =
                a.coarse + (inside ? ((long long)(2 * cy + ((cx + cy) & 1)) * a.lc.Wh + (cx >> 1)) * a.Dp : 0);
            // labels 4 c4 - 2, 4 c4 - 1 (channels 4 c4, 4 c4 + 1) and 4 c4, 4 c4 + 1: pairs of
            // labels are wholly inside [0, D) or outside it (D is even)
            const bool lo_ok = inside && c4 >= 1 && 4 * c4 <= D;
            const bool hi_ok = inside && 4 * c4 < D;
            const unsigned lv = *reinterpret_cast<const unsigned*>(src + (lo_ok ? 4 * c4 - 2 : 0));
            const unsigned hv = *reinterpret_cast<const unsigned*>(src + (hi_ok ? 4 * c4 : 0));
            lo[j] = lo_ok ? lv : 0u;
            hi[j] = hi_ok ? hv : 0u;
        }
#pragma unroll
        for (int j = 0; j < NIT; ++j) {
            const int e = threadIdx.x + j * kWT;
            if (e >= NI) break;
            unsigned sum = (unsigned)bsum[j];
            if (Bs <= 4) {
                const int v = e / (kWIW * kWIH), r = e - v * (kWIW * kWIH);
                const int ry = r / kWIW, rx = r - ry * kWIW;
                const uint8_t* base = (v == 0 ? a.left : a.right) +
                                      (in_img[j] ? (long long)((y0 - 6 + ry) * Bs) * a.W + (x0 - 6 + rx) * Bs : 0);
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const uintptr_t ra = reinterpret_cast<uintptr_t>(base) + (jj < ny[j] ? (uintptr_t)jj * a.W : 0);
                    const unsigned x = __builtin_amdgcn_alignbyte(d1[j][jj], d0[j][jj], (unsigned)(ra & 3u));
                    const unsigned m = jj < ny[j] ? (nx[j] >= 4 ? ~0u : (1u << (8 * nx[j])) - 1u) : 0u;
                    sum = __builtin_amdgcn_udot4(x & m, 0x01010101u, sum, false);
                }
            }
            const int v = e / (kWIW * kWIH), r = e - v * (kWIW * kWIH);
            inp[r * IP + v] = in_img[j] ? to_bf16((float)sum / ((float)(ny[j] * nx[j]) * 255.0f)) : (uint16_t)0;
        }
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int e = threadIdx.x + j * kWT;
            if (e >= NP) break;
            const int c4 = e % (cin0 / 4), pp = e / (cin0 / 4);
            const bool lo_ok = c4 >= 1 && 4 * c4 <= D, hi_ok = 4 * c4 < D;
            auto cv = [](unsigned w, int half) {
                return to_bf16((float)(int16_t)(half ? (w >> 16) : (w & 0xffffu)) / 1024.0f);
            };
            const unsigned w01 = lo_ok ? ((unsigned)cv(lo[j], 0) | ((unsigned)cv(lo[j], 1) << 16)) : 0u;
            const unsigned w23 = hi_ok ? ((unsigned)cv(hi[j], 0) | ((unsigned)cv(hi[j], 1) << 16)) : 0u;
            // straight into the rows of the parent's four pixels of the input region;
            // 0 at pixels outside the image; channels 0, 1 belong to the box averages above
            const int pr = pp / kWPW, pc = pp - pr * kWPW;
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    const int ry = 2 * pr + dy, rx = 2 * pc + dx;
                    const int Y = y0 - 6 + ry, X = x0 - 6 + rx;
                    const bool img = Y >= 0 && Y < Hs && X >= 0 && X < Ws;
                    uint16_t* row = inp + (ry * kWIW + rx) * IP + 4 * c4;
                    if (c4 == 0)
                        *reinterpret_cast<unsigned*>(row + 2) = img ? w23 : 0u;
                    else
                        *reinterpret_cast<uint2*>(row) = img ? make_uint2(w01, w23) : make_uint2(0u, 0u);
                }
        }
    }
    // the first layer's first weight chunk (issued after the views' and parents' loads have
    // returned, which they would otherwise delay)
    warm_l1_chunk<NC1>(a, 0, w1[0]);
    __syncthreads();
    // each layer's weights are loaded while the layer before it runs
    v8s w2[ksteps(32)], w3[ksteps(32)], w4[ksteps(32)], w5[ksteps(32)];
    warm_frags<2>(a, 1, co, w2);
    const float b2 = a.params[a.b_off[1] + co];
    warm_layer1<NC1, IP>(a, w1, x0, y0, inp, actA);
    __syncthreads();
    if (warm_edge<5>(x0, y0, Ws, Hs)) {
        warm_clear_outside<5>(x0, y0, Ws, Hs, actA);
        __syncthreads();
    }
    warm_frags<2>(a, 2, co, w3);
    const float b3 = a.params[a.b_off[2] + co];
    warm_layer<2, kWAS, 4>(a, w2, b2, x0, y0, actA, actB);
    __syncthreads();
    if (warm_edge<4>(x0, y0, Ws, Hs)) {
        warm_clear_outside<4>(x0, y0, Ws, Hs, actB);
        __syncthreads();
    }
    warm_frags<2>(a, 3, co, w4);
    const float b4 = a.params[a.b_off[3] + co];
    warm_layer<2, kWAS, 3>(a, w3, b3, x0, y0, actB, actA);
    __syncthreads();
    if (warm_edge<3>(x0, y0, Ws, Hs)) {
        warm_clear_outside<3>(x0, y0, Ws, Hs, actA);
        __syncthreads();
    }
    warm_frags<2>(a, 4, co, w5);
    const float b5 = a.params[a.b_off[4] + co];
    warm_layer<2, kWAS, 2>(a, w4, b4, x0, y0, actA, actB);
    __syncthreads();
    if (warm_edge<2>(x0, y0, Ws, Hs)) {
        warm_clear_outside<2>(x0, y0, Ws, Hs, actB);
        __syncthreads();
    }

    // last layer: 4D outputs over the tile in 4T blocks of 16 channels (T per side k).  Wave w
    // takes channel blocks w and w + 8 and runs every 16-pixel block of the tile; each output
    // is quantised in registers and staged in LDS as it is (pixel rows padded so that the rows
    // four pixels apart that one store writes fall on different banks); the copy-out takes
    // each message's minimum over d and subtracts it as it stores the messages as 16-byte
    // vectors.
    constexpr int NT = 4 * T, TPW = (NT + kWWaves - 1) / kWWaves, NB = (kWN + 15) / 16, MS = warm_msg_stride(D);
    constexpr int DP = warm_dp(D), P8 = DP / 8;
    v8s w6[TPW][ksteps(32)];
    float bc[TPW];
#pragma unroll
    for (int m = 0; m < TPW; ++m) {
        const int t = wave + kWWaves * m;
        const int c6 = 16 * (t < NT ? t : 0) + i;
        warm_frags<2>(a, kCnnLayers - 1, c6, w6[m]);
        bc[m] = a.params[a.b_off[kCnnLayers - 1] + c6];
    }
    warm_layer<2, kWAS, 1>(a, w5, b5, x0, y0, actB, actA);
    __syncthreads();
    if (warm_edge<1>(x0, y0, Ws, Hs)) {
        warm_clear_outside<1>(x0, y0, Ws, Hs, actA);
        __syncthreads();
    }

    int16_t* msg = reinterpret_cast<int16_t*>(r2);  // [kWN][MS]
    const float lamf = (float)a.lam_t;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int q = 16 * b + i;
        const int ry = q < kWN ? q / kWTW : 0, rx = q < kWN ? q - (q / kWTW) * kWTW : 0;
        const uint16_t* arow = actA + (ry * (kWTW + 2) + rx) * kWAS;
        v4f acc[TPW];
#pragma unroll
        for (int m = 0; m < TPW; ++m) acc[m] = v4f{0.f, 0.f, 0.f, 0.f};
        // 32 input channels: K-step s is tap s, channels 8 g .. 8 g + 7; the block's nine
        // operands are read before the first product
        v8s av[ksteps(32)];
#pragma unroll
        for (int s = 0; s < ksteps(32); ++s) av[s] = load8(arow + ((s / 3) * (kWTW + 2) + (s % 3)) * kWAS + 8 * g);
#pragma unroll
        for (int s = 0; s < ksteps(32); ++s)
#pragma unroll
            for (int m = 0; m < TPW; ++m)
                if (NT % kWWaves == 0 || wave + kWWaves * m < NT)  // uniform over the wave
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[s], w6[m][s], acc[m], 0, 0, 0);
#pragma unroll
        for (int m = 0; m < TPW; ++m) {
            const int t = wave + kWWaves * m;
            if (NT % kWWaves != 0 && t >= NT) continue;
            const int k = t / T, u = t - k * T;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int qq = (int)fminf(fmaxf(rintf((acc[m][e] + bc[m]) * lamf), 0.f), lamf);
                const int qo = 16 * b + 4 * g + e;
                if (kWN % 16 == 0 || qo < kWN) msg[qo * MS + k * D + 16 * u + i] = (int16_t)qq;
            }
        }
    }
    __syncthreads();
    // copy-out: 16-byte pieces of 8 labels, the P8 pieces of a message on consecutive lanes,
    // which take the message's minimum over its D labels through DPP and subtract it (every
    // label is at least the minimum, so one 32-bit subtraction takes it off both halves);
    // labels D .. Dp - 1 and sides without a neighbour are 0.  Every lane of the workgroup
    // runs every iteration (the exchanges need them); the stores are predicated.
    {
        constexpr int NI = kWN * 4 * P8, NIT = (NI + kWT - 1) / kWT;
#pragma unroll
        for (int j = 0; j < NIT; ++j) {
            const int e = threadIdx.x + j * kWT;
            const int c = e % P8, qk = e < NI ? e / P8 : 0, k = qk & 3, qo = qk >> 2;
            const bool lab = 8 * c < D;
            const uint4 r = *reinterpret_cast<const uint4*>(msg + qo * MS + k * D + 8 * (lab ? c : 0));
            const u16x2 m2 = __builtin_elementwise_min(__builtin_elementwise_min(as_u16x2(r.x), as_u16x2(r.y)),
                                                       __builtin_elementwise_min(as_u16x2(r.z), as_u16x2(r.w)));
            int mn = lab ? min((int)m2[0], (int)m2[1]) : INT_MAX;
            mn = min(mn, __builtin_amdgcn_update_dpp(INT_MAX, mn, 0xB1, 0xf, 0xf, false));  // quad_perm [1,0,3,2]
            if constexpr (P8 >= 4)
                mn = min(mn, __builtin_amdgcn_update_dpp(INT_MAX, mn, 0x4E, 0xf, 0xf, false));  // quad_perm [2,3,0,1]
            if constexpr (P8 >= 8)
                mn = min(mn, __builtin_amdgcn_update_dpp(INT_MAX, mn, 0x141, 0xf, 0xf, false));  // row_half_mirror
            const int oy = qo / kWTW, ox = qo - oy * kWTW;
            const int Yo = y0 + oy, Xo = x0 + ox;
            if (e >= NI || Yo >= Hs || Xo >= Ws) continue;
            const bool has = k == 0 ? Xo > 0 : k == 1 ? Xo < Ws - 1 : k == 2 ? Yo > 0 : Yo < Hs - 1;
            const unsigned mm = (unsigned)mn * 0x10001u;
            const uint4 v = has && lab ? make_uint4(r.x - mm, r.y - mm, r.z - mm, r.w - mm) : make_uint4(0u, 0u, 0u, 0u);
            const long long gi = (long long)(2 * Yo + ((Xo + Yo) & 1)) * a.lv.Wh + (Xo >> 1);
            *reinterpret_cast<uint4*>(a.msgs + k * a.vol + gi * DP + 8 * c) = v;
            if (k == 0 && c == 0) {
                if (a.mode == 1) {
                    a.state_a[gi] = 1;
                    a.state_b[gi] = 0;
                }
                if (a.mode == 2) a.state_a[gi] = 1;
            }
        }
    }
}

inline unsigned blocks_for(long long n, int t = kCT, long long cap = 8192)
{
    long long b = (n + t - 1) / t;
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

hipError_t launch_conv_fwd(const uint16_t* in, int H, int W, int cin_p, const uint16_t* w, const float* bias, int cout,
                           int cout_p, int relu, const uint16_t* mask, uint16_t* out_bf16, float* out_f32, hipStream_t st)
{
    const dim3 grid((unsigned)((H * W + 63) / 64), (unsigned)(cout_p / 32));
    const int cs = cin_p <= kLdsMaxCin ? cin_p / 16 : 0;
    const size_t lds = cs ? (size_t)32 * wrow(cin_p) * sizeof(uint16_t) : 0;
#define BPST_CONV(CSV) \
    case CSV: hipLaunchKernelGGL(k_conv_fwd<CSV>, grid, dim3(kCT), lds, st, in, H, W, cin_p, w, bias, cout, cout_p, relu, \
                                 mask, out_bf16, out_f32); break;
    switch (cs) {
        BPST_CONV(0) BPST_CONV(1) BPST_CONV(2) BPST_CONV(3) BPST_CONV(4) BPST_CONV(5) BPST_CONV(6) BPST_CONV(7)
        default: return hipErrorInvalidValue;
    }
#undef BPST_CONV
    return hipGetLastError();
}

hipError_t launch_flip(const uint16_t* w, int cin_p, int cout_p, uint16_t* wf, hipStream_t st)
{
    hipLaunchKernelGGL(k_flip, dim3(blocks_for((long long)cout_p * 9 * cin_p)), dim3(kCT), 0, st, w, cin_p, cout_p, wf);
    return hipGetLastError();
}

int wgrad_chunks(int P, int chunk) { return (P + chunk - 1) / chunk; }

hipError_t launch_conv_wgrad(const uint16_t* in, const uint16_t* g, int H, int W, int cin_p, int cout_p, int chunk,
                             float* part_w, float* part_b, float* dw, float* db, hipStream_t st)
{
    const int P = H * W, S = wgrad_chunks(P, chunk);
    hipLaunchKernelGGL(k_conv_wgrad, dim3((unsigned)S, (unsigned)(9 * (cout_p / 32)), (unsigned)(cin_p / 16)),
                       dim3(kCT), 0, st, in, g, H, W, cin_p, cout_p, chunk, part_w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long nw = (long long)cout_p * 9 * cin_p;
    hipLaunchKernelGGL(k_reduce_chunks, dim3(blocks_for(nw)), dim3(kCT), 0, st, part_w, S, nw, dw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bgrad, dim3((unsigned)S, (unsigned)((cout_p + 63) / 64)), dim3(kCT), 0, st, g, P, cout_p,
                       chunk, part_b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_chunks, dim3(blocks_for(cout_p)), dim3(kCT), 0, st, part_b, S, (long long)cout_p, db);
    return hipGetLastError();
}

int l1_blocks(int P, int cout_p) { return (int)blocks_for((long long)P * cout_p, kCT, 1024); }

hipError_t launch_l1(const float* y, const int16_t* label, int H, int W, int D, int cout_p, float lam_t, float inv_n,
                     uint16_t* g, float* part, float* loss, hipStream_t st)
{
    const int nb = l1_blocks(H * W, cout_p);
    hipLaunchKernelGGL(k_l1, dim3((unsigned)nb), dim3(kCT), 0, st, y, label, H, W, D, cout_p, lam_t, inv_n, g, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(kCT), 0, st, part, nb, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, float* m, float* v, const float* g, uint16_t* w16, long long n, int step, float lr,
                       float b1, float b2, float eps, hipStream_t st)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(kCT), 0, st, w, m, v, g, w16, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* x, long long n, uint16_t* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(kCT), 0, st, x, n, out);
    return hipGetLastError();
}

hipError_t launch_warm_input(const uint8_t* L, const uint8_t* R, int W, int H, int s, const int16_t* coarse, Level lc,
                             int Dp, int D, int Ws, int Hs, int cin_p, uint16_t* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_warm_input, dim3(blocks_for((long long)Ws * Hs * cin_p)), dim3(kCT), 0, st, L, R, W, H, s,
                       coarse, lc, Dp, D, Ws, Hs, cin_p, out);
    return hipGetLastError();
}

hipError_t launch_warm_messages(const float* y, int Ws, int Hs, int D, int ystride, int lam_t, int16_t* out,
                                hipStream_t st)
{
    const long long n = 4LL * Ws * Hs;
    int gs = 1;
    while (gs < D && gs < 64) gs <<= 1;
    const unsigned nb = blocks_for(n * gs);
#define BPST_WARM(GS) \
    case GS: hipLaunchKernelGGL(k_warm_messages<GS>, dim3(nb), dim3(kCT), 0, st, y, Ws, Hs, D, ystride, lam_t, out); break;
    switch (gs) {
        BPST_WARM(1) BPST_WARM(2) BPST_WARM(4) BPST_WARM(8) BPST_WARM(16) BPST_WARM(32) BPST_WARM(64)
        default: return hipErrorInvalidValue;
    }
#undef BPST_WARM
    return hipGetLastError();
}

bool warm_cnn_supported(int D) { return D >= 16 && D <= 64 && D % 16 == 0; }

// The kernel's LDS limit raised above the 64 KB default, once per device (the attribute
// belongs to the device's copy of the kernel).
template <int NC1, int T>
hipError_t warm_lds_limit()
{
    static std::mutex mu;
    static std::vector<bool> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((size_t)dev < done.size() && done[dev]) return hipSuccess;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_warm_cnn<NC1, T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)warm_cnn_lds(16 * NC1, 16 * T));
    if (e != hipSuccess) return e;
    if ((size_t)dev >= done.size()) done.resize(dev + 1, false);
    done[dev] = true;
    return hipSuccess;
}

template <int NC1, int T>
hipError_t launch_warm_cnn_t(const WarmCnnArgs& a, hipStream_t st)
{
    const size_t lds = warm_cnn_lds(16 * NC1, 16 * T);
    if (lds > 64 * 1024) {
        const hipError_t e = warm_lds_limit<NC1, T>();
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)((a.lv.W + kWTW - 1) / kWTW), (unsigned)((a.lv.H + kWTH - 1) / kWTH));
    hipLaunchKernelGGL((k_warm_cnn<NC1, T>), grid, dim3(kWT), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_warm_cnn(const WarmCnnArgs& a, hipStream_t st)
{
    if (!warm_cnn_supported(a.D) || a.lv.W < 1 || a.lv.H < 1 || a.Dp != warm_dp(a.D)) return hipErrorInvalidValue;
    switch (a.D) {
    case 16: return launch_warm_cnn_t<2, 1>(a, st);
    case 32: return launch_warm_cnn_t<3, 2>(a, st);
    case 48: return launch_warm_cnn_t<4, 3>(a, st);
    default: return launch_warm_cnn_t<5, 4>(a, st);
    }
}

}  // namespace bpst
