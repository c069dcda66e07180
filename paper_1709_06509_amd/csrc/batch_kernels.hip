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

__global__ void k_batch_reset(unsigned* barrier, int* error)
{
    if (threadIdx.x == 0) {
        barrier[0] = 0u;
        barrier[1] = 0u;
        *error = 0;
    }
}

__device__ __forceinline__ bool error_raised(const BatchArgs& a)
{
    return __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Grid-wide barrier: release this workgroup's writes, count in, wait for the generation
// to advance, acquire everyone's writes.  Returns false (for the whole workgroup) on error.
__device__ __forceinline__ bool grid_barrier(const BatchArgs& a, int* s_ok)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned* count = a.barrier;
        unsigned* gen = a.barrier + 1;
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned arrived = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
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

template <int G, int MODE>
__device__ __forceinline__ void run_tile(const BatchArgs& a, const PhaseDesc& ph, const PairDev& Q, int lt, int* lds)
{
    constexpr int kPix = kThreads / G;  // pixels per tile
    const int lane = threadIdx.x & (G - 1);
    const long long gi = (long long)lt * kPix + threadIdx.x / G;
    const int l = ph.level;
    switch (ph.type) {
    case kPhPyramid: {
        const int Wc = Q.lv[a.L - 1].W;
        if (Q.vec) pyramid_tree_block<G, true>(Q.cost, Q.c, Q.lv, a.L, Q.D, lt % Wc, lt / Wc, lds);
        else pyramid_tree_block<G, false>(Q.cost, Q.c, Q.lv, a.L, Q.D, lt % Wc, lt / Wc, lds);
        break;
    }
    case kPhInit: {
        const bool top = l == a.L - 1;
        init_pixel<G>(top ? nullptr : Q.m[(l + 1) & 1], Q.lv[top ? l : l + 1], top ? 0 : Q.vol[l + 1], Q.m[l & 1],
                      Q.lv[l], Q.vol[l], Q.sa, Q.sb, a.mode, gi, lane);
        break;
    }
    case kPhHalfstep: {
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
        if (ph.source == kSrcParent) halfstep_pixel<G, MODE, kSrcParent>(h, (int)gi, lane);
        else if (ph.source == kSrcZero) halfstep_pixel<G, MODE, kSrcZero>(h, (int)gi, lane);
        else halfstep_pixel<G, MODE, kSrcOwn>(h, (int)gi, lane);
        break;
    }
    case kPhWta:
        wta_pixel<G>(Q.c[0], Q.m[0], Q.vol[0], Q.lv[0], Q.D, Q.disparity, gi, lane);
        break;
    }
}

// Tile i of this workgroup within a phase of `total` tiles, or -1 when it has no more.
__device__ __forceinline__ int tile_of(const BatchArgs& a, int i, int total)
{
    if (a.order == 0) {
        const long long t = (long long)blockIdx.x + (long long)i * gridDim.x;
        return t < total ? (int)t : -1;
    }
    // workgroup b runs on XCD b % 8: give every XCD one contiguous eighth of the tiles
    const int per = (int)(gridDim.x / kXcds);
    const int x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    const int lo = (int)((long long)total * x / kXcds), hi = (int)((long long)total * (x + 1) / kXcds);
    const long long t = (long long)lo + j + (long long)i * per;
    return t < hi ? (int)t : -1;
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_batch_solve(BatchArgs a)
{
    extern __shared__ int lds[];
    __shared__ int s_ok;
    for (int p = 0; p < a.nphases; ++p) {
        const PhaseDesc ph = a.phases[p];
        const int* ts = a.tiles + ph.table;
        const int total = ts[a.npairs];
        for (int i = 0;; ++i) {
            const int tile = tile_of(a, i, total);
            if (tile < 0) break;
            int lo = 0, hi = a.npairs;  // ts[lo] <= tile < ts[lo + 1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (ts[mid] <= tile) lo = mid;
                else hi = mid;
            }
            const PairDev& Q = a.pairs[lo];
            const int lt = tile - ts[lo];
            switch (Q.G) {
            case 1: run_tile<1, MODE>(a, ph, Q, lt, lds); break;
            case 2: run_tile<2, MODE>(a, ph, Q, lt, lds); break;
            case 4: run_tile<4, MODE>(a, ph, Q, lt, lds); break;
            case 8: run_tile<8, MODE>(a, ph, Q, lt, lds); break;
            case 16: run_tile<16, MODE>(a, ph, Q, lt, lds); break;
            default: run_tile<32, MODE>(a, ph, Q, lt, lds); break;
            }
        }
        if (!grid_barrier(a, &s_ok)) return;
    }
}

}  // namespace

hipError_t launch_batch_reset(unsigned* barrier, int* error, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, barrier, error);
    return hipGetLastError();
}

hipError_t batch_max_blocks_per_cu(int mode, size_t lds, int* blocks)
{
    *blocks = 0;
    switch (mode) {
    case 0: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_solve<0>, kThreads, lds);
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_solve<1>, kThreads, lds);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_solve<2>, kThreads, lds);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_solve(const BatchArgs& a, int blocks, size_t lds, hipStream_t st)
{
    switch (a.mode) {
    case 0: hipLaunchKernelGGL(k_batch_solve<0>, dim3(blocks), dim3(kThreads), lds, st, a); break;
    case 1: hipLaunchKernelGGL(k_batch_solve<1>, dim3(blocks), dim3(kThreads), lds, st, a); break;
    case 2: hipLaunchKernelGGL(k_batch_solve<2>, dim3(blocks), dim3(kThreads), lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bpst
