// Host runtime of the C ABI declared in include/bpstereo.h: argument validation,
// workspace carving, the per-scale launch sequence and optional event timing.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bpstereo.h"
#include "internal.h"

#define BP_API extern "C" __attribute__((visibility("default")))

namespace {

thread_local std::string g_last_error;

int32_t fail(int32_t code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int32_t fail(int32_t code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int32_t ok()
{
    g_last_error.clear();
    return BP_OK;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(BP_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Workspace layout of one solve; offsets in bytes from the workspace base.
struct Plan {
    int L, D, G, Dp;
    bpst::Level lv[bpst::kMaxScales];
    long long vol[bpst::kMaxScales];  // elements of one message volume at scale l
    size_t off_stats, off_cost[bpst::kMaxScales], off_msgs[2], off_sa, off_sb, total;
};

bool params_valid(int W, int H, const bp_params* p, std::string* why)
{
    char b[256];
    auto bad = [&](const char* m) { if (why) *why = m; return false; };
    if (!p) return bad("params is NULL");
    if (W < 1 || H < 1 || W > 16384 || H > 16384) return bad("width/height must be in 1..16384");
    if (p->num_disp < 1 || p->num_disp > 256) return bad("num_disp must be in 1..256");
    if (p->num_scales < 1 || p->num_scales > bpst::kMaxScales) return bad("num_scales must be in 1..8");
    for (int l = 0; l < p->num_scales; ++l)
        if (p->iters[l] < 0 || p->iters[l] > 1024) {
            snprintf(b, sizeof b, "iters[%d] = %d outside 0..1024", l, p->iters[l]);
            if (why) *why = b;
            return false;
        }
    if (p->lambda < 0 || p->lambda > 65535) return bad("lambda must be in 0..65535");
    if (p->trunc < 0) return bad("trunc must be >= 0");
    if (p->skip_mode < 0 || p->skip_mode > 2) return bad("skip_mode must be 0, 1 or 2");
    if (p->skip_mode == 1 && (p->converge_iters < 2 || p->converge_iters > 64 || (p->converge_iters & 1)))
        return bad("converge_iters must be even and in 2..64");
    if (p->warm_msgs && p->num_scales < 2) return bad("warm_msgs needs num_scales >= 2");
    return true;
}

Plan make_plan(int W, int H, const bp_params* p)
{
    Plan pl{};
    pl.L = p->num_scales;
    pl.D = p->num_disp;
    pl.G = bpst::lanes_for(pl.D);
    pl.Dp = 8 * pl.G;
    pl.lv[0] = bpst::make_level(W, H);
    for (int l = 1; l < pl.L; ++l) pl.lv[l] = bpst::make_level((pl.lv[l - 1].W + 1) / 2, (pl.lv[l - 1].H + 1) / 2);
    size_t o = 0;
    pl.off_stats = o;
    o = align_up(o + sizeof(bpst::DevStats));
    for (int l = 0; l < pl.L; ++l) {
        pl.vol[l] = pl.lv[l].slots() * pl.Dp;
        pl.off_cost[l] = o;
        o = align_up(o + (size_t)pl.vol[l] * sizeof(int16_t));
    }
    // scales alternate between two message buffers: even scales in 0, odd scales in 1
    for (int b = 0; b < 2; ++b) {
        pl.off_msgs[b] = o;
        if (b < pl.L) o = align_up(o + 4 * (size_t)pl.vol[b] * sizeof(int16_t));
    }
    pl.off_sa = o;
    o = align_up(o + (size_t)pl.lv[0].slots());
    pl.off_sb = o;
    o = align_up(o + (size_t)pl.lv[0].slots());
    pl.total = o;
    return pl;
}

}  // namespace

// Everything that determines the launch sequence of a solve, pointers included.
struct SolveKey {
    int32_t width, height;
    bp_params params;
    const void *cost, *workspace, *disparity, *final_msgs;
    size_t workspace_bytes;
};

struct bp_context {
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t used = 0;
    long long pixels_max = 0;
    bool graphs = false;
    std::vector<std::pair<SolveKey, hipGraphExec_t>> cache;  // oldest first
    long long graph_hits = 0, graph_captures = 0, graph_fallbacks = 0;
};

namespace {
constexpr size_t kMaxGraphs = 32;

SolveKey make_key(int32_t W, int32_t H, const bp_params* p, const void* cost, const void* ws, size_t wsb,
                  const void* disp, const void* msgs)
{
    SolveKey k;
    std::memset(&k, 0, sizeof k);  // padding too: keys are compared bytewise
    k.width = W;
    k.height = H;
    k.params.num_disp = p->num_disp;
    k.params.num_scales = p->num_scales;
    for (int l = 0; l < p->num_scales; ++l) k.params.iters[l] = p->iters[l];
    k.params.lambda = p->lambda;
    k.params.trunc = p->trunc;
    k.params.skip_mode = p->skip_mode;
    k.params.converge_iters = p->skip_mode == 1 ? p->converge_iters : 0;
    k.params.warm_msgs = p->warm_msgs;
    k.cost = cost;
    k.workspace = ws;
    k.workspace_bytes = wsb;
    k.disparity = disp;
    k.final_msgs = msgs;
    return k;
}
}  // namespace

BP_API const char* bp_last_error(void) { return g_last_error.c_str(); }

BP_API int32_t bp_context_create(bp_context** out)
{
    if (!out) return fail(BP_E_INVAL, "out is NULL");
    bp_context* c = new (std::nothrow) bp_context();
    if (!c) return fail(BP_E_NOMEM, "cannot allocate a context");
    *out = c;
    return ok();
}

BP_API int32_t bp_context_destroy(bp_context* ctx)
{
    if (!ctx) return fail(BP_E_INVAL, "ctx is NULL");
    for (auto& e : ctx->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto& e : ctx->cache) (void)hipGraphExecDestroy(e.second);
    delete ctx;
    return ok();
}

BP_API int32_t bp_context_set_graphs(bp_context* ctx, int32_t on)
{
    if (!ctx) return fail(BP_E_INVAL, "ctx is NULL");
    ctx->graphs = on != 0;
    return ok();
}

BP_API int32_t bp_context_graph_counts(bp_context* ctx, int64_t* counts)
{
    if (!ctx || !counts) return fail(BP_E_INVAL, "ctx/counts is NULL");
    counts[0] = ctx->graph_captures;
    counts[1] = ctx->graph_hits;
    counts[2] = ctx->graph_fallbacks;
    return ok();
}

BP_API int32_t bp_context_set_timing(bp_context* ctx, int32_t on)
{
    if (!ctx) return fail(BP_E_INVAL, "ctx is NULL");
    ctx->timing = on != 0;
    return ok();
}

BP_API int32_t bp_context_take_timing(bp_context* ctx, bp_timing* out)
{
    if (!ctx || !out) return fail(BP_E_INVAL, "ctx/out is NULL");
    double ms = 0.0;
    for (size_t i = 0; i < ctx->used; ++i) {
        HIP_TRY(hipEventSynchronize(ctx->events[i].second));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, ctx->events[i].first, ctx->events[i].second));
        ms += t;
    }
    out->halfstep_ms = ms;
    out->halfstep_launches = (int64_t)ctx->used;
    out->halfstep_pixel_updates_max = ctx->pixels_max;
    ctx->used = 0;
    ctx->pixels_max = 0;
    return ok();
}

BP_API int32_t stereo_luma(const uint8_t* rgb, int32_t width, int32_t height, uint8_t* luma, void* stream)
{
    if (!rgb || !luma) return fail(BP_E_INVAL, "rgb/luma is NULL");
    if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(BP_E_INVAL, "bad image size");
    HIP_TRY(bpst::launch_luma(rgb, width, height, luma, (hipStream_t)stream));
    return ok();
}

BP_API int32_t stereo_cost_volume(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                                  int32_t num_disp, int32_t window, int32_t cost_scale, int32_t cost_trunc,
                                  int16_t* cost, float* ncc_or_null, void* stream)
{
    if (!left || !right || !cost) return fail(BP_E_INVAL, "left/right/cost is NULL");
    if (width < 1 || height < 1 || width > 16384 || height > 16384)
        return fail(BP_E_INVAL, "width/height must be in 1..16384");
    if (num_disp < 1 || num_disp > 256) return fail(BP_E_INVAL, "num_disp must be in 1..256");
    if (window < 1 || window > 13 || (window & 1) == 0) return fail(BP_E_INVAL, "window must be odd, 1..13");
    if (cost_scale < 1 || cost_scale > 4096) return fail(BP_E_INVAL, "cost_scale must be in 1..4096");
    if (cost_trunc < 0 || cost_trunc > 32767) return fail(BP_E_INVAL, "cost_trunc must be in 0..32767");
    HIP_TRY(bpst::launch_ncc(left, right, width, height, num_disp, window, cost_scale, cost_trunc, cost, ncc_or_null,
                             (hipStream_t)stream));
    return ok();
}

BP_API size_t bp_workspace_bytes(int32_t width, int32_t height, const bp_params* params)
{
    if (!params_valid(width, height, params, nullptr)) return 0;
    return make_plan(width, height, params).total;
}

// Enqueue every launch of one solve on `st` (no synchronisation, no allocation).
static int32_t enqueue_solve(bp_context* ctx, const Plan& pl, const int16_t* cost, const bp_params* params,
                             void* workspace, int16_t* disparity, int16_t* final_msgs_or_null, bool count,
                             hipStream_t st)
{
    char* ws = static_cast<char*>(workspace);
    auto* stats = reinterpret_cast<bpst::DevStats*>(ws + pl.off_stats);
    int16_t* C[bpst::kMaxScales];
    for (int l = 0; l < pl.L; ++l) C[l] = reinterpret_cast<int16_t*>(ws + pl.off_cost[l]);
    int16_t* M[2] = {reinterpret_cast<int16_t*>(ws + pl.off_msgs[0]), reinterpret_cast<int16_t*>(ws + pl.off_msgs[1])};
    uint8_t* sa = reinterpret_cast<uint8_t*>(ws + pl.off_sa);
    uint8_t* sb = reinterpret_cast<uint8_t*>(ws + pl.off_sb);
    const int mode = params->skip_mode;
    const int tq = params->trunc < pl.D ? params->trunc : pl.D;
    const int capv = params->lambda * tq < 32767 ? params->lambda * tq : 32767;

    if (count) HIP_TRY(bpst::launch_zero_stats(stats, st));
    {
        bpst::PyramidArgs pa{};
        for (int l = 0; l < pl.L; ++l) {
            pa.c[l] = C[l];
            pa.lv[l] = pl.lv[l];
        }
        pa.L = pl.L;
        pa.D = pl.D;
        bool done = false;
        HIP_TRY(bpst::launch_pyramid_tree(cost, pa, pl.G, &done, st));
        if (!done) {
            HIP_TRY(bpst::launch_prep_level0(cost, C[0], pl.lv[0], pl.D, pl.G, st));
            for (int l = 0; l + 1 < pl.L; ++l)
                HIP_TRY(bpst::launch_pyramid(C[l], pl.lv[l], C[l + 1], pl.lv[l + 1], pl.D, pl.G, st));
        }
    }

    const int start = params->warm_msgs ? pl.L - 2 : pl.L - 1;
    for (int l = start; l >= 0; --l) {
        int16_t* msgs = M[l & 1];
        const int iters = params->iters[l];
        // The first half-step reads the parent's (or zero) messages directly, unless the
        // scale needs its initial messages materialised: fewer than two half-steps (the
        // colour-0 slots would never be written), a warm start, or the exact dirty-skip,
        // whose change test compares against the initial messages.
        const bool fuse = iters >= 2 && mode != 2 && !(l == start && params->warm_msgs);
        int source = bpst::kSrcOwn;
        if (fuse) {
            source = (l == start) ? bpst::kSrcZero : bpst::kSrcParent;
        } else if (l == start && params->warm_msgs) {
            HIP_TRY(bpst::launch_import(params->warm_msgs, msgs, pl.lv[l], pl.vol[l], pl.D, pl.G, sa, sb, mode, st));
        } else if (l == start) {
            HIP_TRY(bpst::launch_init(nullptr, pl.lv[l], 0, msgs, pl.lv[l], pl.vol[l], pl.G, sa, sb, mode, st));
        } else {
            HIP_TRY(bpst::launch_init(M[(l + 1) & 1], pl.lv[l + 1], pl.vol[l + 1], msgs, pl.lv[l], pl.vol[l], pl.G, sa,
                                      sb, mode, st));
        }
        bpst::HalfstepArgs a{};
        a.cost = C[l];
        a.msgs = msgs;
        a.vol = pl.vol[l];
        if (l + 1 < pl.L) {
            a.pmsgs = M[(l + 1) & 1];
            a.pvol = pl.vol[l + 1];
            a.plv = pl.lv[l + 1];
        }
        a.state_a = sa;
        a.state_b = sb;
        a.lv = pl.lv[l];
        a.D = pl.D;
        a.Dp = pl.Dp;
        a.G = pl.G;
        a.lambda = params->lambda;
        a.capv = capv;
        a.K = params->converge_iters;
        a.mode = mode;
        a.count = count ? 1 : 0;
        a.stats = stats;
        a.level = l;
        for (int t = 0; t < iters; ++t) {
            a.t = t;
            a.colour = t & 1;
            a.source = (t == 0) ? source : bpst::kSrcOwn;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (ctx && ctx->timing) {
                if (ctx->used == ctx->events.size()) {
                    hipEvent_t x, y;
                    HIP_TRY(hipEventCreate(&x));
                    HIP_TRY(hipEventCreate(&y));
                    ctx->events.emplace_back(x, y);
                }
                e0 = ctx->events[ctx->used].first;
                e1 = ctx->events[ctx->used].second;
                ctx->used++;
                ctx->pixels_max += (long long)pl.lv[l].H * pl.lv[l].Wh;
                HIP_TRY(hipEventRecord(e0, st));
            }
            HIP_TRY(bpst::launch_halfstep(a, st));
            if (e1) HIP_TRY(hipEventRecord(e1, st));
        }
    }
    HIP_TRY(bpst::launch_wta(C[0], M[0], pl.vol[0], pl.lv[0], pl.D, pl.G, disparity, st));
    if (final_msgs_or_null)
        HIP_TRY(bpst::launch_export(M[0], pl.vol[0], pl.lv[0], pl.D, pl.G, final_msgs_or_null, st));
    return BP_OK;
}

BP_API int32_t bp_hierarchical_solve(bp_context* ctx, const int16_t* cost, int32_t width, int32_t height,
                                     const bp_params* params, void* workspace, size_t workspace_bytes,
                                     int16_t* disparity, int16_t* final_msgs_or_null, bp_stats* stats_or_null,
                                     void* stream)
{
    std::string why;
    if (!params_valid(width, height, params, &why)) return fail(BP_E_INVAL, "%s", why.c_str());
    if (!cost || !disparity) return fail(BP_E_INVAL, "cost/disparity is NULL");
    const Plan pl = make_plan(width, height, params);
    if (!workspace || workspace_bytes < pl.total)
        return fail(BP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, pl.total);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(BP_E_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    hipStream_t st = (hipStream_t)stream;
    const bool count = stats_or_null != nullptr;
    if (ctx && ctx->graphs && !count && !ctx->timing && st != nullptr) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(st, &cs));
        if (cs == hipStreamCaptureStatusNone) {
            const SolveKey key = make_key(width, height, params, cost, workspace, workspace_bytes, disparity,
                                          final_msgs_or_null);
            for (auto& e : ctx->cache)
                if (std::memcmp(&e.first, &key, sizeof key) == 0) {
                    HIP_TRY(hipGraphLaunch(e.second, st));
                    ctx->graph_hits++;
                    return ok();
                }
            const char* force = getenv("BPSTEREO_GRAPH_FORCE_FAIL");
            if (!(force && force[0] == '1') &&
                hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                const int32_t rc = enqueue_solve(ctx, pl, cost, params, workspace, disparity, final_msgs_or_null,
                                                 false, st);
                hipGraph_t g = nullptr;
                const hipError_t ee = hipStreamEndCapture(st, &g);
                hipGraphExec_t ex = nullptr;
                const bool good = rc == BP_OK && ee == hipSuccess && g &&
                                  hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
                if (g) (void)hipGraphDestroy(g);
                if (good) {
                    if (ctx->cache.size() >= kMaxGraphs) {
                        (void)hipGraphExecDestroy(ctx->cache.front().second);
                        ctx->cache.erase(ctx->cache.begin());
                    }
                    ctx->cache.emplace_back(key, ex);
                    ctx->graph_captures++;
                    HIP_TRY(hipGraphLaunch(ex, st));
                    return ok();
                }
            }
            (void)hipGetLastError();  // a failed capture leaves nothing enqueued: run eagerly
            ctx->graph_fallbacks++;
        }
    }
    {
        const int32_t rc = enqueue_solve(ctx, pl, cost, params, workspace, disparity, final_msgs_or_null, count, st);
        if (rc != BP_OK) return rc;
    }
    auto* stats = reinterpret_cast<bpst::DevStats*>(static_cast<char*>(workspace) + pl.off_stats);
    if (stats_or_null) {
        bpst::DevStats hs;
        HIP_TRY(hipMemcpyAsync(&hs, stats, sizeof hs, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        std::memset(stats_or_null, 0, sizeof *stats_or_null);
        stats_or_null->msg_updates = (int64_t)hs.msg_updates;
        stats_or_null->pixel_updates = (int64_t)hs.pixel_updates;
        for (int l = 0; l < pl.L; ++l) {
            stats_or_null->n_halfsteps[l] = (params->warm_msgs && l == pl.L - 1) ? 0 : params->iters[l];
            for (int t = 0; t < bpst::kStatHalfsteps; ++t) stats_or_null->active[l][t] = hs.active[l][t];
        }
    }
    return ok();
}

BP_API size_t bp_energy_workspace_bytes(int32_t width, int32_t height)
{
    (void)width;
    (void)height;
    return bpst::energy_ws_bytes();
}

BP_API int32_t bp_energy(const int16_t* cost, const int16_t* disparity, int32_t width, int32_t height,
                         int32_t num_disp, int32_t lambda, int32_t trunc, int64_t* energy, void* workspace,
                         size_t workspace_bytes, void* stream)
{
    if (!cost || !disparity || !energy) return fail(BP_E_INVAL, "cost/disparity/energy is NULL");
    if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(BP_E_INVAL, "bad image size");
    if (num_disp < 1 || num_disp > 256) return fail(BP_E_INVAL, "num_disp must be in 1..256");
    if (lambda < 0 || lambda > 65535 || trunc < 0) return fail(BP_E_INVAL, "lambda/trunc out of range");
    if (!workspace || workspace_bytes < bpst::energy_ws_bytes())
        return fail(BP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, bpst::energy_ws_bytes());
    if (reinterpret_cast<uintptr_t>(workspace) % 8 != 0) return fail(BP_E_WORKSPACE, "workspace must be 8-byte aligned");
    HIP_TRY(bpst::launch_energy(cost, disparity, width, height, num_disp, lambda, trunc, energy, workspace,
                                (hipStream_t)stream));
    return ok();
}
