// Batched solve: many stereo pairs of uneven sizes and disparity ranges in one persistent
// launch.
//
// The batch runs as a fixed sequence of phases (the cost pyramid, then for each scale from
// the coarsest its start and half-steps, then the winner-take-all).  Every pair has the
// same sequence, so a phase covers the same step of all pairs at once: its tiles (256
// lanes of one pair each) are dealt to the resident workgroups, which then meet at a
// grid-wide barrier before the next phase.  Per-pixel work is the same code as the
// per-launch kernels (bp_device.h), so each pair's result is bit-identical to its solo
// solve.
//
// The grid never exceeds the co-resident capacity the occupancy query reports.  A barrier
// wait is bounded: past the timeout a workgroup raises the error flag and every workgroup
// leaves, so the launch always drains.
#include "bp_device.h"

namespace bpst {
namespace {

// barrier words: [0..7] arrivals per XCD group, [8] group arrivals, [9] generation
constexpr int kBarGroup = 8, kBarGen = 9, kBarWords = 10;
constexpr int kLdsPairs = 1024;  // pair tables up to this size are searched in LDS

__global__ void k_batch_reset(unsigned* barrier, int* error)
{
    if (threadIdx.x < kBarWords) barrier[threadIdx.x] = 0u;
    if (threadIdx.x == 0) *error = 0;
}

__device__ __forceinline__ bool error_raised(const BatchArgs& a)
{
    return __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Grid-wide barrier: release this workgroup's writes, count in, wait for the generation
// to advance, acquire everyone's writes.  Arrivals are counted in two levels: workgroups
// b with equal b % 8 (the workgroups of one XCD) share a counter, and the last arrival of
// each group counts in at the group counter, so no single address takes every atomic.
// Returns false (for the whole workgroup) on error.
__device__ __forceinline__ bool grid_barrier(const BatchArgs& a, int* s_ok)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned* gen = a.barrier + kBarGen;
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned x = blockIdx.x % kXcds;
        const unsigned nx = (gridDim.x - x + kXcds - 1) / kXcds;              // workgroups in group x
        const unsigned ngroups = gridDim.x < (unsigned)kXcds ? gridDim.x : (unsigned)kXcds;
        bool last = false;
        if (__hip_atomic_fetch_add(a.barrier + x, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == nx - 1) {
            __hip_atomic_store(a.barrier + x, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(a.barrier + kBarGroup, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
                ngroups - 1) {
                __hip_atomic_store(a.barrier + kBarGroup, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                last = true;
            }
        }
        if (!last) {
            const long long t0 = (long long)wall_clock64();
            while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (error_raised(a)) { ok = 0; break; }
                if ((long long)wall_clock64() - t0 > a.timeout_ticks) {
                    __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// One tile of a phase whose type (and half-step message source) is known at compile time.
// HV: the variant, fixed at compile time for one-phase launches (bit 0 narrow path, bit 1
// streamed volumes, bit 2 messages in 12 bits) or -1 to read it from the arguments
// (persistent launch).
constexpr int kHvRuntime = -1;

template <int G, int MODE, int TYPE, int SRC, int HV = kHvRuntime>
__device__ __forceinline__ void run_tile_t(const BatchArgs& a, const PhaseDesc& ph, const PairDev& Q, int lt,
                                           int* lds)
{
    if constexpr (HV == kHvRuntime) {
        // the persistent launch: the storage of the messages from the arguments
        if (a.packed) {
            run_tile_t<G, MODE, TYPE, SRC, kHvRuntime - 1>(a, ph, Q, lt, lds);
            return;
        }
    }
    // kHvRuntime - 1: the persistent launch's 12-bit variant
    constexpr bool RT = HV == kHvRuntime || HV == kHvRuntime - 1;
    constexpr bool PK = HV == kHvRuntime - 1 || (!RT && (HV & kHvPacked) != 0);
    constexpr int kPix = kThreads / G;  // pixels per tile
    const int lane = threadIdx.x & (G - 1);
    const long long gi = (long long)lt * kPix + threadIdx.x / G;
    const int l = ph.level;
    if (TYPE == kPhPyramid) {
        const int c0 = lt * tree_blocks(a.L, G, kThreads);
        if (Q.vec) pyramid_tree_block<G, true>(Q.cost, Q.c, Q.lv, a.L, Q.D, c0, lds);
        else pyramid_tree_block<G, false>(Q.cost, Q.c, Q.lv, a.L, Q.D, c0, lds);
    } else if (TYPE == kPhInit) {
        const bool top = l == a.L - 1;
        init_pixel<G, PK>(top ? nullptr : Q.m[(l + 1) & 1], Q.lv[top ? l : l + 1], top ? 0 : Q.vol[l + 1],
                          Q.m[l & 1], Q.lv[l], Q.vol[l], Q.sa, Q.sb, a.mode, gi, lane);
    } else if (TYPE == kPhHalfstep) {
        HalfstepArgs h{};
        h.cost = Q.c[l];
        h.msgs = Q.m[l & 1];
        h.vol = Q.vol[l];
        if (l + 1 < a.L) {
            h.pmsgs = Q.m[(l + 1) & 1];
            h.pvol = Q.vol[l + 1];
            h.plv = Q.lv[l + 1];
        }
        h.state_a = Q.sa;
        h.state_b = Q.sb;
        h.lv = Q.lv[l];
        h.D = Q.D;
        h.Dp = 8 * G;
        h.G = G;
        h.lambda = a.lambda;
        h.capv = a.capv;
        h.colour = ph.t & 1;
        h.t = ph.t;
        h.K = a.K;
        h.mode = MODE;
        if (MODE == 0 && ph.wta) h.disp = Q.disparity;  // written on the int32 path only
        if constexpr (RT) {
            if constexpr (G <= kNarrowMaxG && !PK) {
                if (a.narrow && !ph.stream) {
                    halfstep_pixel<G, MODE, SRC, true>(h, (int)gi, lane);
                    return;
                }
            }
            if (ph.stream) halfstep_pixel<G, MODE, SRC, false, true, PK>(h, (int)gi, lane);
            else halfstep_pixel<G, MODE, SRC, false, false, PK>(h, (int)gi, lane);
        } else {
            // pixels wider than kNarrowMaxG lanes stay on the int32 path, as do 12-bit messages
            constexpr bool N = (HV & kHvNarrow) != 0 && G <= kNarrowMaxG && !PK;
            halfstep_pixel<G, MODE, SRC, N, (HV & kHvStream) != 0, PK>(h, (int)gi, lane);
        }
    } else {
        // the colour the last half-step already decided, where it ran on the int32 path (the
        // same rule as the half-step's own choice above)
        const bool narrow = G <= kNarrowMaxG && a.narrow && !ph.stream && !PK;
        if (MODE == 0 && ph.wta >= 0 && !narrow && gi < Q.lv[0].slots()) {
            const long long row = gi / Q.lv[0].Wh;  // 2 y + colour
            if ((int)(row & 1) == ph.wta) return;
        }
        wta_pixel<G, PK>(Q.c[0], Q.m[0], Q.vol[0], Q.lv[0], Q.D, Q.disparity, gi, lane);
    }
}

// One tile of any phase (type and source read at run time).
template <int G, int MODE>
__device__ __forceinline__ void run_tile(const BatchArgs& a, const PhaseDesc& ph, const PairDev& Q, int lt, int* lds)
{
    switch (ph.type) {
    case kPhPyramid: run_tile_t<G, MODE, kPhPyramid, kSrcOwn>(a, ph, Q, lt, lds); break;
    case kPhInit: run_tile_t<G, MODE, kPhInit, kSrcOwn>(a, ph, Q, lt, lds); break;
    case kPhHalfstep:
        if (ph.source == kSrcParent) run_tile_t<G, MODE, kPhHalfstep, kSrcParent>(a, ph, Q, lt, lds);
        else if (ph.source == kSrcZero) run_tile_t<G, MODE, kPhHalfstep, kSrcZero>(a, ph, Q, lt, lds);
        else run_tile_t<G, MODE, kPhHalfstep, kSrcOwn>(a, ph, Q, lt, lds);
        break;
    default: run_tile_t<G, MODE, kPhWta, kSrcOwn>(a, ph, Q, lt, lds); break;
    }
}

// Each workgroup takes one contiguous chunk of a phase's tiles (mostly one pair, neighbouring
// rows).  Order 0: chunk = workgroup index.  Order 1: the workgroups of one XCD (b % 8) take
// adjacent chunks, so neighbouring rows share that XCD's L2.
__device__ __forceinline__ void chunk_of(const BatchArgs& a, int total, int* lo, int* hi)
{
    const int nb = (int)gridDim.x;
    int c = (int)blockIdx.x;
    if (a.order == 1 && nb % kXcds == 0) c = (int)(blockIdx.x % kXcds) * (nb / kXcds) + (int)(blockIdx.x / kXcds);
    *lo = (int)((long long)total * c / nb);
    *hi = (int)((long long)total * (c + 1) / nb);
}

// The same for at most kWavePairs - 1 pairs in one memory round trip instead of a chain of
// dependent loads: every lane of the wave loads eight of the n + 1 prefix sums, and the
// number of sums <= tile (they are non-decreasing, so these form a prefix) is one more than
// the pair.  Each wave computes it on its own, so no barrier is needed.
constexpr int kWavePairs = 512;
__device__ __forceinline__ int pair_of_wave(const int* ts, int n, int tile)
{
    const int l = (int)(threadIdx.x & 63);
    int v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = 64 * k + l <= n ? ts[64 * k + l] : 0x7fffffff;
    int count = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) count += __popcll(__ballot(v[k] <= tile));
    return count - 1;
}

// Pair p with ts[p] <= tile < ts[p + 1].
__device__ __forceinline__ int pair_of(const int* ts, int n, int tile)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ts[mid] <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int MODE, int GMAX>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_solve(BatchArgs a)
{
    extern __shared__ int lds[];
    __shared__ int s_ok;
    __shared__ int s_ts[kLdsPairs + 1];
    const bool in_lds = a.npairs <= kLdsPairs;
    for (int p = 0; p < a.nphases; ++p) {
        const PhaseDesc ph = a.phases[p];
        const int* gts = a.tiles + ph.table;
        if (in_lds) {
            for (int i = threadIdx.x; i <= a.npairs; i += blockDim.x) s_ts[i] = gts[i];
            __syncthreads();
        }
        const int* ts = in_lds ? s_ts : gts;
        int lo, hi;
        chunk_of(a, ts[a.npairs], &lo, &hi);
        int q = lo < hi ? pair_of(ts, a.npairs, lo) : 0;
        for (int tile = lo; tile < hi; ++tile) {
            while (tile >= ts[q + 1]) ++q;
            const PairDev& Q = a.pairs[q];
            const int lt = tile - ts[q];
            switch (Q.G) {
            case 1: run_tile<1, MODE>(a, ph, Q, lt, lds); break;
            case 2: run_tile<2, MODE>(a, ph, Q, lt, lds); break;
            case 4: run_tile<4, MODE>(a, ph, Q, lt, lds); break;
            case 8: run_tile<8, MODE>(a, ph, Q, lt, lds); break;
            case 16: if (GMAX >= 16) run_tile<16, MODE>(a, ph, Q, lt, lds); break;
            default: if (GMAX >= 32) run_tile<32, MODE>(a, ph, Q, lt, lds); break;
            }
        }
        if (!grid_barrier(a, &s_ok)) return;
    }
}

// The other schedule: one launch per phase, one workgroup per tile of every pair.  The
// kernel boundary orders the phases, so no grid barrier is needed.
template <int MODE, int GMAX, int TYPE, int SRC, int HV>
__global__ __launch_bounds__(kThreads) void k_batch_phase(BatchArgs a, int phase)
{
    extern __shared__ int lds[];
    const PhaseDesc ph = a.phases[phase];
    const int* ts = a.tiles + ph.table;
    const int tile = blockIdx.x;
    const int q = a.npairs < kWavePairs ? pair_of_wave(ts, a.npairs, tile) : pair_of(ts, a.npairs, tile);
    const PairDev& Q = a.pairs[q];
    const int lt = tile - ts[q];
    switch (Q.G) {
    case 1: run_tile_t<1, MODE, TYPE, SRC, HV>(a, ph, Q, lt, lds); break;
    case 2: run_tile_t<2, MODE, TYPE, SRC, HV>(a, ph, Q, lt, lds); break;
    case 4: run_tile_t<4, MODE, TYPE, SRC, HV>(a, ph, Q, lt, lds); break;
    case 8: run_tile_t<8, MODE, TYPE, SRC, HV>(a, ph, Q, lt, lds); break;
    case 16: if (GMAX >= 16) run_tile_t<16, MODE, TYPE, SRC, HV>(a, ph, Q, lt, lds); break;
    default: if (GMAX >= 32) run_tile_t<32, MODE, TYPE, SRC, HV>(a, ph, Q, lt, lds); break;
    }
}

template <int MODE, int GMAX, int HV>
static void launch_phase_v(const BatchArgs& a, int phase, int type, int src, int tiles, size_t lds, hipStream_t st)
{
    const dim3 g((unsigned)tiles), b(kThreads);
    switch (type) {
    case kPhPyramid:
        hipLaunchKernelGGL((k_batch_phase<MODE, GMAX, kPhPyramid, kSrcOwn, 0>), g, b, lds, st, a, phase);
        break;
    case kPhInit:
        hipLaunchKernelGGL((k_batch_phase<MODE, GMAX, kPhInit, kSrcOwn, HV & kHvPacked>), g, b, 0, st, a, phase);
        break;
    case kPhHalfstep:
        if (src == kSrcParent)
            hipLaunchKernelGGL((k_batch_phase<MODE, GMAX, kPhHalfstep, kSrcParent, HV>), g, b, 0, st, a, phase);
        else if (src == kSrcZero)
            hipLaunchKernelGGL((k_batch_phase<MODE, GMAX, kPhHalfstep, kSrcZero, HV>), g, b, 0, st, a, phase);
        else
            hipLaunchKernelGGL((k_batch_phase<MODE, GMAX, kPhHalfstep, kSrcOwn, HV>), g, b, 0, st, a, phase);
        break;
    default:
        hipLaunchKernelGGL((k_batch_phase<MODE, GMAX, kPhWta, kSrcOwn, HV & kHvPacked>), g, b, 0, st, a, phase);
        break;
    }
}

// hv: the variant (kHvNarrow | kHvStream | kHvPacked bits, never narrow with packed), fixed per
// launch
template <int MODE, int GMAX>
static void launch_phase_m(const BatchArgs& a, int phase, int type, int src, int tiles, size_t lds, int hv,
                           hipStream_t st)
{
    switch (hv) {
    case kHvNarrow: launch_phase_v<MODE, GMAX, kHvNarrow>(a, phase, type, src, tiles, lds, st); break;
    case kHvStream: launch_phase_v<MODE, GMAX, kHvStream>(a, phase, type, src, tiles, lds, st); break;
    case kHvPacked: launch_phase_v<MODE, GMAX, kHvPacked>(a, phase, type, src, tiles, lds, st); break;
    case kHvPacked | kHvStream:
        launch_phase_v<MODE, GMAX, kHvPacked | kHvStream>(a, phase, type, src, tiles, lds, st);
        break;
    default: launch_phase_v<MODE, GMAX, 0>(a, phase, type, src, tiles, lds, st); break;
    }
}

}  // namespace

hipError_t launch_batch_phase(const BatchArgs& a, int phase, int type, int src, int tiles, size_t lds, int hv,
                              hipStream_t st)
{
    if (tiles <= 0) return hipSuccess;
    if (a.gmax <= 8) {
        switch (a.mode) {
        case 0: launch_phase_m<0, 8>(a, phase, type, src, tiles, lds, hv, st); break;
        case 1: launch_phase_m<1, 8>(a, phase, type, src, tiles, lds, hv, st); break;
        default: launch_phase_m<2, 8>(a, phase, type, src, tiles, lds, hv, st); break;
        }
    } else {
        switch (a.mode) {
        case 0: launch_phase_m<0, 32>(a, phase, type, src, tiles, lds, hv, st); break;
        case 1: launch_phase_m<1, 32>(a, phase, type, src, tiles, lds, hv, st); break;
        default: launch_phase_m<2, 32>(a, phase, type, src, tiles, lds, hv, st); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_batch_reset(unsigned* barrier, int* error, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, barrier, error);
    return hipGetLastError();
}

template <int GMAX>
static hipError_t max_blocks_g(int mode, size_t lds, int* blocks)
{
    switch (mode) {
    case 0: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_solve<0, GMAX>, kThreads, lds);
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_solve<1, GMAX>, kThreads, lds);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_solve<2, GMAX>, kThreads, lds);
    default: return hipErrorInvalidValue;
    }
}

hipError_t batch_max_blocks_per_cu(int mode, int gmax, size_t lds, int* blocks)
{
    *blocks = 0;
    return gmax <= 8 ? max_blocks_g<8>(mode, lds, blocks) : max_blocks_g<32>(mode, lds, blocks);
}

template <int GMAX>
static void launch_g(const BatchArgs& a, int blocks, size_t lds, hipStream_t st)
{
    switch (a.mode) {
    case 0: hipLaunchKernelGGL((k_batch_solve<0, GMAX>), dim3(blocks), dim3(kThreads), lds, st, a); break;
    case 1: hipLaunchKernelGGL((k_batch_solve<1, GMAX>), dim3(blocks), dim3(kThreads), lds, st, a); break;
    default: hipLaunchKernelGGL((k_batch_solve<2, GMAX>), dim3(blocks), dim3(kThreads), lds, st, a); break;
    }
}

hipError_t launch_batch_solve(const BatchArgs& a, int blocks, size_t lds, hipStream_t st)
{
    if (a.mode < 0 || a.mode > 2) return hipErrorInvalidValue;
    if (a.gmax <= 8) launch_g<8>(a, blocks, lds, st);
    else launch_g<32>(a, blocks, lds, st);
    return hipGetLastError();
}

}  // namespace bpst
