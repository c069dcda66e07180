// Internal declarations shared by the host runtime (api.cpp) and the kernel files.
//
// Device data layout of one scale (W x H pixels, D labels):
//  - Labels are padded to Dp = 8 * G, G = lanes per pixel (a power of two with
//    8 * G >= D); lane g of a pixel owns labels [8g, 8g + 8) as one 16-byte vector.
//  - Pixels are stored colour-split: the pixels of colour c = (x + y) & 1 in row y
//    are contiguous, slot(x, y) = (2y + c) * Wh + (x >> 1), Wh = ceil(W / 2).  A
//    half-step touches one colour, so its reads and writes are dense streams.
//  - The four message volumes of a scale are consecutive, each slots * Dp int16.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bpst {

constexpr int kMaxScales = 8;
constexpr int kStatHalfsteps = 64;

inline int lanes_for(int D)
{
    int g = 1;
    while (8 * g < D) g <<= 1;
    return g;
}

struct Level {
    int W, H, Wh;
    __host__ __device__ long long slots() const { return 2LL * H * Wh; }
};

inline Level make_level(int W, int H) { return Level{W, H, (W + 1) / 2}; }

// Device counters of one solve (kept in the workspace).
struct DevStats {
    unsigned long long msg_updates;
    unsigned long long pixel_updates;
    int active[kMaxScales][kStatHalfsteps];
};

// Where the first half-step of a scale reads its incoming messages from.
enum MsgSource { kSrcOwn = 0, kSrcParent = 1, kSrcZero = 2 };

struct HalfstepArgs {
    const int16_t* cost;     // this scale's cost, colour-split, Dp labels
    int16_t* msgs;           // 4 volumes
    long long vol;           // elements per volume
    const int16_t* pmsgs;    // parent scale's volumes (source kSrcParent)
    long long pvol;
    Level plv;
    uint8_t* state_a;        // skip 1: active; skip 2: dirty
    uint8_t* state_b;        // skip 1: stable count
    Level lv;
    int D, Dp, G;
    int lambda;
    int capv;                // min(lambda * min(T, D), 32767): clamp of a normalised message
    int colour, t, K, mode, source, count;
    int narrow;              // packed 16-bit sums (no counters): see the narrow path in bp_device.h
    int stream;              // nontemporal loads and stores (the scale's volumes exceed the caches)
    int packed;              // messages stored in 12 bits (G >= 16, capv <= 4095; see bp_device.h)
    int user_cost;           // cost is the caller's finest volume [H][W][D] (D == Dp, 16-byte aligned,
                             // 12-bit messages only), read at pixel (y W + x), not the colour-split slot
    DevStats* stats;
    int level;
    int16_t* disp;           // non-null (plain BP, int32 path, last half-step of the finest scale):
                             // also write each updated pixel's winner-take-all disparity
    int16_t* out;            // non-null: outgoing messages go to these 4 volumes (the Jacobi
                             // schedule's second set), not in place
};

// Coarsest pixels that one workgroup of `threads` lanes takes in the one-launch cost
// pyramid.  The block under one coarsest pixel needs s1^2 G lanes on scale 1
// (s1 = 2^(L-2)); blocks smaller than the workgroup are packed side by side.
__host__ __device__ inline int tree_blocks(int L, int G, int threads)
{
    const int p1 = (1 << (2 * (L - 2))) * G;
    return p1 >= threads ? 1 : threads / p1;
}

// LDS of one block of the cost pyramid: scales 1 and 2 of the block, int per label.
inline size_t tree_block_lds(int L, int G)
{
    const long long s1 = 1LL << (L - 2), s2 = s1 / 2;
    return (size_t)(s1 * s1 + s2 * s2) * 8 * G * sizeof(int);
}

struct PyramidArgs {
    int16_t* c[kMaxScales];  // internal cost of every scale
    Level lv[kMaxScales];
    int L, D;
    int skip_finest;         // the solve reads the caller's finest cost itself: c[0] is not written
};

// ---- batched solve ----
struct NccPair {
    const uint8_t* left;
    const uint8_t* right;
    int16_t* cost;
    int W, H, D, pad_;
};

// One pair of a batch as the persistent kernel sees it.
struct PairDev {
    const int16_t* cost;      // caller's finest cost [H][W][D]
    int16_t* disparity;       // caller's output [H][W]
    int16_t* c[kMaxScales];   // internal cost of every scale
    int16_t* m[2];            // message buffers (even scales in 0, odd in 1)
    uint8_t* sa;
    uint8_t* sb;
    Level lv[kMaxScales];
    long long vol[kMaxScales];
    int D, G, vec, pad_;      // vec: the caller's cost allows 16-byte loads
};

enum PhaseType { kPhPyramid = 0, kPhInit = 1, kPhHalfstep = 2, kPhWta = 3 };

// One phase of the batched solve; all pairs run it before any pair starts the next.
struct PhaseDesc {
    int type, level, t, source;
    int table;   // offset in BatchArgs::tiles of this phase's prefix sums (npairs + 1 ints)
    int stream;  // half-step: the pairs' working sets at this scale together exceed the caches;
                 // WTA: the same flag of the last half-step of the finest scale
    int wta;     // half-step: plain BP's last at the finest scale, which also writes the winners
                 // of the pixels it updates on the int32 path; WTA: the colour of those pixels
                 // (-1: none), skipped wherever that half-step ran on the int32 path
};

struct BatchArgs {
    const PairDev* pairs;
    const PhaseDesc* phases;
    const int* tiles;
    int npairs, nphases, L;
    int lambda, capv, K, mode;
    int order;                // 0: chunk = workgroup index; 1: the workgroups of one XCD take adjacent chunks
    int narrow;               // half-steps on the narrow path (pairs with G <= kNarrowMaxG; capv <= kNarrowCap)
    int packed;               // every message volume stored in 12 bits (capv <= 4095; never with narrow)
    int gmax;                 // largest lanes-per-pixel among the pairs (selects a leaner kernel when <= 8)
    unsigned* barrier;        // 10 words: per-XCD-group arrivals, group arrivals, generation
    int* error;               // set when a grid barrier times out
    long long timeout_ticks;  // of the wall clock
};

// Several half-steps of one scale in one launch (fused_kernels.hip).
struct FusedArgs {
    const int16_t* cost;     // this scale's cost, colour-split, Dp labels
    int16_t* msgs;           // 4 volumes
    long long vol;
    const int16_t* pmsgs;    // parent scale's volumes (source kSrcParent)
    long long pvol;
    Level plv;
    uint8_t* state_a;        // freeze rule: active, stable count
    uint8_t* state_b;
    Level lv;
    int D, G, lambda, capv, K, mode;
    int source;              // incoming messages at t0: kSrcOwn, kSrcParent or kSrcZero
    int t0, nsteps;          // half-steps t0 .. t0 + nsteps - 1
    int TW, TH, halo, tiles_x;
    long long rmax;          // region pixels the LDS holds: (TW + 2 halo) (TH + 2 halo)
    int keep_state;          // write the freeze state back (later half-steps of the scale follow)
    int narrow;              // packed 16-bit sums: incoming messages in [0, capv], capv <= kNarrowCap
    int compact;             // list the active pixels of each freeze-rule half-step: -1 launch_fused
                             // decides (the default), 0 / 1 forced off / on (a test hook)
};
constexpr int kFusedLdsBytes = 160 * 1024;
// Largest capv for which the packed 16-bit message sums are exact: with every cost
// min-normalised per pixel, a sum that saturates at 65535 is still at least capv above the
// minimum (at most 3 capv), so it clips to capv as its true value would.
constexpr int kNarrowCap = 16383;
// Widest pixel (lanes) a one-per-half-step launch takes the narrow path for.  Wider pixels
// are large disparity ranges, whose half-steps stream far more memory than they compute:
// there the narrow path's doubled vector loads per lane cost more than its arithmetic saves.
constexpr int kNarrowMaxG = 8;
// Half-steps whose working set (the cost and the four message volumes) is larger than the
// 256 MB Infinity Cache stream it with nontemporal loads and stores: it cannot stay cached
// from one half-step to the next, and plain accesses would only evict what could.  (A
// 197 MB working set, 640x480 at D = 64, is 2 % faster with plain accesses.)
constexpr double kStreamBytes = 256e6;
inline bool stream_scale(const Level& lv, int G) { return 5.0 * (double)lv.slots() * 8 * G * 2 > kStreamBytes; }
// Whether the narrow path is expected to be faster in a fused launch whose region holds
// rmax pixels (it lowers the work per lane; small regions are bound by other costs).
bool fused_narrow_pays(int G, long long rmax);
// Half-steps per fused launch and interior tile for `iters` half-steps on scale lv, chosen
// by a cost model; false if one launch per half-step is estimated to be faster.
bool fused_geometry(const Level& lv, int G, int iters, int* steps, int* TW, int* TH, long long* rmax);
// The widest interior tile whose region (halo = steps) fits the LDS.
bool fused_geometry_max(const Level& lv, int G, int steps, int* TW, int* TH, long long* rmax);
size_t fused_lds_bytes(int G, long long rmax);
hipError_t launch_fused(const FusedArgs& a, hipStream_t st);
// Lets the fused kernels use the whole LDS; called once outside graph capture (errors ignored).
void fused_prepare();

constexpr int kXcds = 8;
constexpr int kThreadsPerTile = 256;  // workgroup size of every pixel kernel: a tile is 256 / G pixels

hipError_t launch_export_cost(const int16_t* c, Level lv, int D, int G, int16_t* out, hipStream_t st);

// Sets the calling thread's last-error message (cleared for BP_OK); returns code.
int32_t report(int32_t code, const char* msg);

// ---- learned warm start (cnn_kernels.hip) ----
hipError_t launch_conv_fwd(const uint16_t* in, int H, int W, int cin_p, const uint16_t* w, const float* bias, int cout,
                           int cout_p, int relu, const uint16_t* mask, uint16_t* out_bf16, float* out_f32,
                           hipStream_t st);
hipError_t launch_flip(const uint16_t* w, int cin_p, int cout_p, uint16_t* wf, hipStream_t st);
int wgrad_chunks(int P, int chunk);
hipError_t launch_conv_wgrad(const uint16_t* in, const uint16_t* g, int H, int W, int cin_p, int cout_p, int chunk,
                             float* part_w, float* part_b, float* dw, float* db, hipStream_t st);
int l1_blocks(int P, int cout_p);
hipError_t launch_l1(const float* y, const int16_t* label, int H, int W, int D, int cout_p, float lam_t, float inv_n,
                     uint16_t* g, float* part, float* loss, hipStream_t st);
hipError_t launch_adam(float* w, float* m, float* v, const float* g, uint16_t* w16, long long n, int step, float lr,
                       float b1, float b2, float eps, hipStream_t st);
hipError_t launch_to_bf16(const float* x, long long n, uint16_t* out, hipStream_t st);
hipError_t launch_warm_input(const uint8_t* L, const uint8_t* R, int W, int H, int s, const int16_t* coarse, Level lc,
                             int Dp, int D, int Ws, int Hs, int cin_p, uint16_t* out, hipStream_t st);
hipError_t launch_warm_messages(const float* y, int Ws, int Hs, int D, int ystride, int lam_t, int16_t* out,
                                hipStream_t st);

// The network's layer count, and the offsets of each layer's weights and biases in the
// parameter vector (bf16 weights use the same offsets); false if D is outside 1..256.
constexpr int kCnnLayers = 6;
bool cnn_offsets(int D, long long w_off[kCnnLayers], long long b_off[kCnnLayers]);

// The whole warm start of one scale in one launch (cnn_kernels.hip): network input, the six
// convolutions and the quantisation, written straight into the scale's message volumes and
// state bytes in the solve's internal layout.  Bit-identical to launch_warm_input +
// launch_conv_fwd x 6 + launch_warm_messages + launch_import.
struct WarmCnnArgs {
    const uint8_t* left;     // finest views, uint8 [H][W]
    const uint8_t* right;
    int W, H;
    int s;                   // the warm scale (views averaged over 2^s x 2^s blocks)
    const int16_t* coarse;   // internal cost of scale s + 1
    Level lc;
    int D, Dp, G;
    const uint16_t* w16;     // bf16 weights; biases are read from params (fp32)
    const float* params;
    long long w_off[kCnnLayers], b_off[kCnnLayers];
    int lam_t;               // quantisation range: min(lambda * min(trunc, D), 32767)
    int16_t* msgs;           // scale s: four volumes of vol elements, colour-split slots of Dp labels
    Level lv;
    long long vol;
    uint8_t* state_a;
    uint8_t* state_b;
    int mode;                // skip mode: the state bytes a scale starts with
};
// D must be a multiple of 16 and at most 64 (else hipErrorInvalidValue, nothing launched).
bool warm_cnn_supported(int D);
hipError_t launch_warm_cnn(const WarmCnnArgs& a, hipStream_t st);

// The batch's correlation volumes in one launch (ncc_mfma.hip): tiles of one row and 64
// columns, listed by per-pair prefix sums of ncc_mfma_tiles.
int ncc_mfma_tiles(int W, int H);
hipError_t launch_ncc_mfma_batched(const NccPair* pairs, const int* tile_start, int n, int total_tiles, int max_d,
                                   int win, int scale, int trunc, hipStream_t st);
hipError_t launch_batch_reset(unsigned* barrier, int* error, hipStream_t st);
// Largest co-resident grid of the persistent kernel for `lds` bytes of LDS per workgroup.
hipError_t batch_max_blocks_per_cu(int mode, int gmax, size_t lds, int* blocks);
hipError_t launch_batch_solve(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
// One phase of the batch as its own launch: `tiles` workgroups, one per tile.
// Half-step variant bits of a one-phase launch: the narrow path, streamed volumes.
constexpr int kHvNarrow = 1, kHvStream = 2, kHvPacked = 4;  // kHvPacked: message volumes in 12 bits
hipError_t launch_batch_phase(const BatchArgs& a, int phase, int type, int src, int tiles, size_t lds, int hv,
                              hipStream_t st);

// Launchers (return hipError_t of the launch).
// launch_pyramid_tree: re-layout of the finest scale plus every coarser scale in one launch;
// sets *done = false (and launches nothing) when the block of one coarsest pixel does not
// fit in LDS, in which case the caller uses launch_prep_level0 + launch_pyramid.
hipError_t launch_pyramid_tree(const int16_t* user, const PyramidArgs& a, int G, bool* done, hipStream_t st);
hipError_t launch_zero_stats(DevStats* s, hipStream_t st);
hipError_t launch_prep_level0(const int16_t* user, int16_t* c0, Level lv, int D, int G, hipStream_t st);
hipError_t launch_pyramid(const int16_t* fine, Level lf, int16_t* coarse, Level lc, int D, int G,
                          hipStream_t st);
// packed: the scale's messages are stored in 12 bits (see bp_device.h; G >= 16 only)
hipError_t launch_init(const int16_t* parent, Level lp, long long pvol, int16_t* msgs, Level lv,
                       long long vol, int G, uint8_t* state_a, uint8_t* state_b, int mode, hipStream_t st,
                       bool packed = false);
hipError_t launch_import(const int16_t* warm, int16_t* msgs, Level lv, long long vol, int D, int G,
                         uint8_t* state_a, uint8_t* state_b, int mode, hipStream_t st);
hipError_t launch_halfstep(const HalfstepArgs& a, hipStream_t st);
// colour -1: every pixel; 0 or 1: only the pixels with (x + y) & 1 == colour.  user: c0 is the
// caller's finest volume [H][W][D] (packed only, D == 8 G, 16-byte aligned), not the internal layout.
hipError_t launch_wta(const int16_t* c0, const int16_t* msgs, long long vol, Level lv, int D, int G, int colour,
                      int16_t* disparity, hipStream_t st, bool packed = false, bool user = false);
hipError_t launch_export(const int16_t* msgs, long long vol, Level lv, int D, int G, int16_t* out,
                         hipStream_t st, bool packed = false);
hipError_t launch_energy(const int16_t* cost, const int16_t* disp, int W, int H, int D, int lambda,
                         int trunc, int64_t* out, void* ws, hipStream_t st);
size_t energy_ws_bytes();

// Static device scratch of the solve that allocates nothing (noalloc.hip): its size, and its
// device address on the current device (looked up once per device).
constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;
hipError_t noalloc_scratch(void** ptr);
hipError_t launch_lr_check(const int16_t* dl, const int16_t* dr, int W, int H, int D, int tol, int16_t* out,
                           hipStream_t st);
hipError_t launch_luma(const uint8_t* rgb, int W, int H, uint8_t* y, hipStream_t st);
// The correlation volume with the window sums on the matrix cores (ncc_mfma.hip): views of
// `channels` (1, or 3 interleaved) bytes a pixel; channels 3 needs win <= 9.
hipError_t launch_ncc_mfma(const uint8_t* L, const uint8_t* R, int W, int H, int D, int win, int channels, int scale,
                           int trunc, int16_t* cost, float* ncc, hipStream_t st);

}  // namespace bpst
