// Host runtime of the C ABI declared in include/bpstereo.h: argument validation,
// workspace carving, the per-scale launch sequence and optional event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
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

}  // namespace

namespace bpst {
int32_t report(int32_t code, const char* msg)
{
    if (code == BP_OK) g_last_error.clear();
    else g_last_error = msg ? msg : "";
    return code;
}
}  // namespace bpst

namespace {

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
    bool packed;  // the solve's messages are stored in 12 bits (see bp_device.h)
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
    // 12-bit messages where every message fits (its clamp min(lambda min(T, D), 32767) is at
    // most 4095; caller-given warm messages can be larger) and a pixel spans 16 or more lanes
    // (D > 64: there the half-steps are bound by memory, not by their instruction count)
    const long long capv = std::min((long long)p->lambda * std::min(p->trunc, p->num_disp), 32767LL);
    pl.packed = pl.G >= 16 && capv <= 4095 && !p->warm_msgs;
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
    int32_t fused;
};

struct bp_context {
    int timing = 0;  // 0 off; 1 an event pair per message-update launch; 2 one per scale's launches
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    std::vector<int> event_scale;     // scale of the launches each event pair brackets
    std::vector<int> event_launches;  // and how many launches it brackets
    size_t used = 0;
    long long pixels_max = 0;
    bool graphs = false;
    int fused = 2;  // several half-steps per launch on small scales: 0 never, 1 wherever it fits, 2 by size
    std::vector<std::pair<SolveKey, hipGraphExec_t>> cache;  // oldest first
    long long graph_hits = 0, graph_captures = 0, graph_fallbacks = 0;
    // batched solve: pinned staging for the per-batch tables (two, each guarded by the event
    // of its last upload), tuned launch shapes and captured graphs
    void* staging[2] = {nullptr, nullptr};
    size_t staging_bytes[2] = {0, 0};
    hipEvent_t staging_done[2] = {nullptr, nullptr};
    int staging_next = 0;
    struct Tuned {
        std::vector<int32_t> sig;
        int bpc, order, sched;
    };
    std::vector<Tuned> tuned;
    int forced_sched = -1, forced_bpc = 1, forced_order = 0;
    std::vector<std::pair<std::vector<char>, hipGraphExec_t>> batch_graphs;
};

namespace {
// Event pair for timed launches on ctx (timing mode): `launches` consecutive launches of
// one scale.  Returns the pair's index in *slot.
int32_t timing_events(bp_context* ctx, int scale, int launches, hipEvent_t* e0, hipEvent_t* e1,
                      size_t* slot = nullptr)
{
    if (ctx->used == ctx->events.size()) {
        hipEvent_t x, y;
        HIP_TRY(hipEventCreate(&x));
        HIP_TRY(hipEventCreate(&y));
        ctx->events.emplace_back(x, y);
        ctx->event_scale.push_back(0);
        ctx->event_launches.push_back(0);
    }
    *e0 = ctx->events[ctx->used].first;
    *e1 = ctx->events[ctx->used].second;
    ctx->event_scale[ctx->used] = scale;
    ctx->event_launches[ctx->used] = launches;
    if (slot) *slot = ctx->used;
    ctx->used++;
    return BP_OK;
}
}  // namespace

BP_API int32_t bp_context_set_batch_schedule(bp_context* ctx, int32_t schedule, int32_t blocks_per_cu, int32_t order)
{
    if (!ctx) return fail(BP_E_INVAL, "ctx is NULL");
    if (schedule < -1 || schedule > 2 || (schedule == 0 && (blocks_per_cu < 1 || order < 0 || order > 1)))
        return fail(BP_E_INVAL, "schedule must be -1, 0 (with blocks_per_cu >= 1, order 0/1), 1 or 2");
    ctx->forced_sched = schedule;
    ctx->forced_bpc = blocks_per_cu;
    ctx->forced_order = order;
    g_last_error.clear();
    return BP_OK;
}

namespace {
constexpr size_t kMaxGraphs = 32;
constexpr int kFusedMaxSteps = 5;  // half-steps (and halo pixels) per fused launch when forced

SolveKey make_key(int32_t W, int32_t H, const bp_params* p, const void* cost, const void* ws, size_t wsb,
                  const void* disp, const void* msgs, int32_t fused)
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
    k.fused = fused;
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
    bpst::fused_prepare();
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
    for (auto& e : ctx->batch_graphs) (void)hipGraphExecDestroy(e.second);
    for (int i = 0; i < 2; ++i) {
        if (ctx->staging_done[i]) {
            (void)hipEventSynchronize(ctx->staging_done[i]);
            (void)hipEventDestroy(ctx->staging_done[i]);
        }
        if (ctx->staging[i]) (void)hipHostFree(ctx->staging[i]);
    }
    delete ctx;
    return ok();
}

BP_API int32_t bp_context_set_fused(bp_context* ctx, int32_t mode)
{
    if (!ctx) return fail(BP_E_INVAL, "ctx is NULL");
    if (mode < 0 || mode > 2) return fail(BP_E_INVAL, "mode must be 0, 1 or 2");
    ctx->fused = mode;
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
    if (on < 0 || on > 2) return fail(BP_E_INVAL, "timing mode must be 0, 1 or 2");
    ctx->timing = on;
    return ok();
}

BP_API int32_t bp_context_take_timing(bp_context* ctx, bp_timing* out)
{
    if (!ctx || !out) return fail(BP_E_INVAL, "ctx/out is NULL");
    double ms = 0.0;
    int64_t launches = 0;
    std::memset(out, 0, sizeof *out);
    for (size_t i = 0; i < ctx->used; ++i) {
        HIP_TRY(hipEventSynchronize(ctx->events[i].second));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, ctx->events[i].first, ctx->events[i].second));
        ms += t;
        launches += ctx->event_launches[i];
        const int l = ctx->event_scale[i];
        if (l >= 0 && l < bpst::kMaxScales) {
            out->scale_ms[l] += t;
            out->scale_launches[l] += ctx->event_launches[i];
        }
    }
    out->halfstep_ms = ms;
    out->halfstep_launches = launches;
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

BP_API int32_t bp_lr_check(const int16_t* disp_left, const int16_t* disp_right, int32_t width, int32_t height,
                           int32_t num_disp, int32_t tol, int16_t* out, void* stream)
{
    if (!disp_left || !disp_right || !out) return fail(BP_E_INVAL, "disp_left/disp_right/out is NULL");
    if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(BP_E_INVAL, "bad image size");
    if (num_disp < 1 || num_disp > 256) return fail(BP_E_INVAL, "num_disp must be in 1..256");
    if (tol < 0) return fail(BP_E_INVAL, "tol must be >= 0");
    HIP_TRY(bpst::launch_lr_check(disp_left, disp_right, width, height, num_disp, tol, out, (hipStream_t)stream));
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
    HIP_TRY(bpst::launch_ncc_mfma(left, right, width, height, num_disp, window, 1, cost_scale, cost_trunc, cost,
                                  ncc_or_null, (hipStream_t)stream));
    return ok();
}

BP_API int32_t stereo_cost_volume_rgb(const uint8_t* left_rgb, const uint8_t* right_rgb, int32_t width, int32_t height,
                                      int32_t num_disp, int32_t window, int32_t cost_scale, int32_t cost_trunc,
                                      int16_t* cost, float* ncc_or_null, void* stream)
{
    if (!left_rgb || !right_rgb || !cost) return fail(BP_E_INVAL, "left_rgb/right_rgb/cost is NULL");
    if (width < 1 || height < 1 || width > 16384 || height > 16384)
        return fail(BP_E_INVAL, "width/height must be in 1..16384");
    if (num_disp < 1 || num_disp > 256) return fail(BP_E_INVAL, "num_disp must be in 1..256");
    if (window < 1 || window > 9 || (window & 1) == 0) return fail(BP_E_INVAL, "window must be odd, 1..9");
    if (cost_scale < 1 || cost_scale > 4096) return fail(BP_E_INVAL, "cost_scale must be in 1..4096");
    if (cost_trunc < 0 || cost_trunc > 32767) return fail(BP_E_INVAL, "cost_trunc must be in 0..32767");
    HIP_TRY(bpst::launch_ncc_mfma(left_rgb, right_rgb, width, height, num_disp, window, 3, cost_scale, cost_trunc, cost,
                                  ncc_or_null, (hipStream_t)stream));
    return ok();
}

BP_API size_t bp_workspace_bytes(int32_t width, int32_t height, const bp_params* params)
{
    if (!params_valid(width, height, params, nullptr)) return 0;
    return make_plan(width, height, params).total;
}

// Test and tuning hooks (environment variables), read once per solve: none changes a result,
// only how the same arithmetic is cut into launches.
struct Hooks {
    int fused_steps = 0;        // BPSTEREO_FUSED_STEPS=n: fused launches of n half-steps
    int tile_w = 0, tile_h = 0; // BPSTEREO_FUSED_TILE=WxH: smaller interior tiles of fused launches
    int fused_tail = 0;         // BPSTEREO_FUSED_TAIL=k: freeze rule, one launch a half-step up to t = k
    int compact = -1;           // BPSTEREO_FUSED_COMPACT=0/1: force the active-pixel listing off/on
    bool graph_fail = false;    // BPSTEREO_GRAPH_FORCE_FAIL=1: make graph capture fail
};

static Hooks read_hooks()
{
    Hooks h;
    if (const char* v = getenv("BPSTEREO_FUSED_STEPS")) h.fused_steps = atoi(v);
    if (const char* v = getenv("BPSTEREO_FUSED_TILE")) {
        if (sscanf(v, "%dx%d", &h.tile_w, &h.tile_h) != 2) h.tile_w = h.tile_h = 0;
    }
    if (const char* v = getenv("BPSTEREO_FUSED_TAIL")) h.fused_tail = atoi(v);
    if (const char* v = getenv("BPSTEREO_FUSED_COMPACT")) {
        if ((v[0] == '0' || v[0] == '1') && v[1] == 0) h.compact = v[0] - '0';
    }
    if (const char* v = getenv("BPSTEREO_GRAPH_FORCE_FAIL")) h.graph_fail = v[0] == '1';
    return h;
}

// The learned warm start computed inside a solve (bp_warmstart_solve): the views the cost
// volume was built from and the network's parameters.
struct WarmNet {
    const uint8_t* left;
    const uint8_t* right;
    int width, height;
    const float* params;
    const uint16_t* w16;
};

// Enqueue every launch of one solve on `st` (no synchronisation, no allocation).  With `net`,
// the solve starts at scale L - 2 from the network's messages, as with params->warm_msgs.
static int32_t enqueue_solve(bp_context* ctx, const Plan& pl, const int16_t* cost, const bp_params* params,
                             void* workspace, int16_t* disparity, int16_t* final_msgs_or_null, bool count,
                             hipStream_t st, bool timing_allowed = true, const WarmNet* net = nullptr)
{
    const Hooks hk = read_hooks();
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
    // With 12-bit messages (int32 sums, no narrow or fused launches) and a caller's volume laid
    // out as the kernels read it (D == Dp, 16-byte aligned), the finest scale's half-steps and
    // winner-take-all read the caller's cost directly: the pyramid then writes no internal copy
    // of it, a full cost volume of writes saved.  Messages and winners are unchanged, since the
    // internal copy differs only by a per-pixel shift.
    bool user0 = pl.packed && pl.Dp == pl.D && (reinterpret_cast<uintptr_t>(cost) & 15) == 0;
    {
        bpst::PyramidArgs pa{};
        for (int l = 0; l < pl.L; ++l) {
            pa.c[l] = C[l];
            pa.lv[l] = pl.lv[l];
        }
        pa.L = pl.L;
        pa.D = pl.D;
        pa.skip_finest = user0 ? 1 : 0;
        bool done = false;
        HIP_TRY(bpst::launch_pyramid_tree(cost, pa, pl.G, &done, st));
        if (!done) {
            user0 = false;  // the per-scale pyramid builds the coarser scales from the internal copy
            HIP_TRY(bpst::launch_prep_level0(cost, C[0], pl.lv[0], pl.D, pl.G, st));
            for (int l = 0; l + 1 < pl.L; ++l)
                HIP_TRY(bpst::launch_pyramid(C[l], pl.lv[l], C[l + 1], pl.lv[l + 1], pl.D, pl.G, st));
        }
    }

    const bool warm = params->warm_msgs || net;
    const int start = warm ? pl.L - 2 : pl.L - 1;
    // Half-step t of scale l may use packed 16-bit sums (bp_device.h, the narrow path) when
    // every incoming message it reads is a transform output, in [0, capv], and capv is small
    // enough.  Raw warm messages (any value up to 32767) are read by the warm scale's first
    // half-step, and reach finer scales when the warm scale runs fewer than two half-steps
    // (then some slots are never rewritten).
    auto narrow_ok = [&](int l, int t) {
        if (capv > bpst::kNarrowCap) return false;
        if (!warm) return true;
        if (l == start) return t > 0;
        return params->iters[start] >= 2;
    };
    int wta_colour = -1;  // the pixels the WTA launch covers: -1 all, else one colour
    for (int l = start; l >= 0; --l) {
        int16_t* msgs = M[l & 1];
        const int iters = params->iters[l];
        // The first half-step reads the parent's (or zero) messages directly, unless the
        // scale needs its initial messages materialised: fewer than two half-steps (the
        // colour-0 slots would never be written), a warm start, or the exact dirty-skip,
        // whose change test compares against the initial messages.
        const bool fuse = iters >= 2 && mode != 2 && !(l == start && warm);
        // Several half-steps per launch from LDS (fused_kernels.hip): no counters, freeze
        // rule or plain, and (by default) only where a half-step moves little enough memory
        // that one launch per half-step would be bound by launch latency.
        int ftw = 0, fth = 0, fsteps = 0;
        long long frmax = 0;
        const int fmode = ctx ? ctx->fused : 2;
        if (fmode != 0 && !count && mode != 2 && iters >= 1 && pl.G <= 8) {
            // test and tuning hook: a fixed number of half-steps per fused launch
            const int forced_steps = hk.fused_steps;
            if (forced_steps > 0) {
                fsteps = forced_steps < iters ? forced_steps : iters;
                if (!bpst::fused_geometry_max(pl.lv[l], pl.G, fsteps, &ftw, &fth, &frmax)) fsteps = 0;
            } else if (fmode == 2) {
                if (!bpst::fused_geometry(pl.lv[l], pl.G, iters, &fsteps, &ftw, &fth, &frmax)) fsteps = 0;
            } else {
                const int chunks = (iters + kFusedMaxSteps - 1) / kFusedMaxSteps;
                fsteps = (iters + chunks - 1) / chunks;
                if (!bpst::fused_geometry_max(pl.lv[l], pl.G, fsteps, &ftw, &fth, &frmax)) fsteps = 0;
            }
            {
                // test hook: smaller interior tiles, so that small images are cut into many
                const int fw = hk.tile_w, fh = hk.tile_h;
                if (fsteps > 0 && fw >= 1 && fh >= 1 && fw <= ftw && fh <= fth) {
                    ftw = fw;
                    fth = fh;
                    frmax = (long long)(fw + 2 * fsteps) * (fh + 2 * fsteps);
                }
            }
        }
        // The scale's half-steps as consecutive segments, each run one launch per half-step
        // (steps == 0) or in fused launches of `steps` half-steps on its own tile.
        struct Seg {
            int t0, t1, steps, tw, th;
            long long rmax;
        };
        Seg segs[2];  // a fixed array: planning a solve allocates nothing
        int nsegs = 0;
        if (hk.fused_tail >= 2 && hk.fused_tail < iters && fsteps == 0 && fmode != 0 && mode == 1 && !count &&
            pl.G <= 8) {
            // tuning hook: one launch per half-step up to t = k, then fused launches
            const int k = hk.fused_tail;
            const int chunks = (iters - k + kFusedMaxSteps * 2 - 1) / (kFusedMaxSteps * 2);
            const int steps = (iters - k + chunks - 1) / chunks;
            Seg b{k, iters, steps, 0, 0, 0};
            if (bpst::fused_geometry_max(pl.lv[l], pl.G, steps, &b.tw, &b.th, &b.rmax)) {
                segs[nsegs++] = {0, k, 0, 0, 0, 0};
                segs[nsegs++] = b;
            }
        }
        if (nsegs == 0) segs[nsegs++] = {0, iters, fsteps, ftw, fth, frmax};
        int source = bpst::kSrcOwn;
        if (fuse) {
            source = (l == start) ? bpst::kSrcZero : bpst::kSrcParent;
        } else if (l == start && net) {
            bpst::WarmCnnArgs w{};
            w.left = net->left;
            w.right = net->right;
            w.W = net->width;
            w.H = net->height;
            w.s = l;
            w.coarse = C[l + 1];
            w.lc = pl.lv[l + 1];
            w.D = pl.D;
            w.Dp = pl.Dp;
            w.G = pl.G;
            w.w16 = net->w16;
            w.params = net->params;
            if (!bpst::cnn_offsets(pl.D, w.w_off, w.b_off)) return fail(BP_E_INVAL, "num_disp outside the network's range");
            w.lam_t = capv;
            w.msgs = msgs;
            w.lv = pl.lv[l];
            w.vol = pl.vol[l];
            w.state_a = sa;
            w.state_b = sb;
            w.mode = mode;
            HIP_TRY(bpst::launch_warm_cnn(w, st));
        } else if (l == start && params->warm_msgs) {
            HIP_TRY(bpst::launch_import(params->warm_msgs, msgs, pl.lv[l], pl.vol[l], pl.D, pl.G, sa, sb, mode, st));
        } else if (l == start) {
            HIP_TRY(bpst::launch_init(nullptr, pl.lv[l], 0, msgs, pl.lv[l], pl.vol[l], pl.G, sa, sb, mode, st,
                                      pl.packed));
        } else {
            HIP_TRY(bpst::launch_init(M[(l + 1) & 1], pl.lv[l + 1], pl.vol[l + 1], msgs, pl.lv[l], pl.vol[l], pl.G, sa,
                                      sb, mode, st, pl.packed));
        }
        bpst::HalfstepArgs a{};
        a.cost = (l == 0 && user0) ? cost : C[l];
        a.user_cost = (l == 0 && user0) ? 1 : 0;
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
        a.packed = pl.packed ? 1 : 0;
        // timing mode 2: one event pair around all of this scale's message-update launches
        const bool time_each = ctx && ctx->timing == 1 && timing_allowed;
        hipEvent_t s0 = nullptr, s1 = nullptr;
        size_t sslot = 0;
        int scale_launches = 0;
        if (ctx && ctx->timing == 2 && timing_allowed && iters > 0) {
            const int32_t rc = timing_events(ctx, l, 0, &s0, &s1, &sslot);
            if (rc != BP_OK) return rc;
            HIP_TRY(hipEventRecord(s0, st));
        }
        for (int si = 0; si < nsegs; ++si) {
            const Seg& sg = segs[si];
            for (int t = sg.t0; sg.steps == 0 && t < sg.t1; ++t) {
                a.t = t;
                a.colour = t & 1;
                a.source = (t == 0) ? source : bpst::kSrcOwn;
                // Scales too large for the caches stream their volumes (nontemporal accesses) on
                // the int32 path; the narrow path's lower arithmetic pays where memory does not
                // bound the launch.
                a.stream = bpst::stream_scale(pl.lv[l], pl.G) ? 1 : 0;
                a.narrow = narrow_ok(l, t) && !count && pl.G <= bpst::kNarrowMaxG && !a.stream ? 1 : 0;
                // plain BP's last half-step at the finest scale also writes the winner of the
                // pixels it updates (their incoming messages are final): the WTA launch then
                // covers the other colour only
                a.disp = nullptr;
                if (l == 0 && mode == 0 && !a.narrow && t == iters - 1) {
                    a.disp = disparity;
                    wta_colour = 1 - (t & 1);
                }
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (time_each) {
                    const int32_t rc = timing_events(ctx, l, 1, &e0, &e1);
                    if (rc != BP_OK) return rc;
                    HIP_TRY(hipEventRecord(e0, st));
                }
                if (ctx && ctx->timing && timing_allowed) ctx->pixels_max += (long long)pl.lv[l].H * pl.lv[l].Wh;
                HIP_TRY(bpst::launch_halfstep(a, st));
                ++scale_launches;
                if (e1) HIP_TRY(hipEventRecord(e1, st));
            }
            if (sg.steps > 0) {
                // the fused kernel reads the parent's (or zero) messages itself at t = 0, as the
                // first half-step does; where an init kernel ran, it reads its own volumes
                bpst::FusedArgs f{};
                f.cost = C[l];
                f.msgs = msgs;
                f.vol = pl.vol[l];
                f.pmsgs = a.pmsgs;
                f.pvol = a.pvol;
                f.plv = a.plv;
                f.state_a = sa;
                f.state_b = sb;
                f.lv = pl.lv[l];
                f.D = pl.D;
                f.G = pl.G;
                f.lambda = params->lambda;
                f.capv = capv;
                f.K = params->converge_iters;
                f.mode = mode;
                f.TW = sg.tw;
                f.TH = sg.th;
                f.tiles_x = (pl.lv[l].W + sg.tw - 1) / sg.tw;
                f.rmax = sg.rmax;
                for (int t0 = sg.t0; t0 < sg.t1; t0 += sg.steps) {
                    f.t0 = t0;
                    f.nsteps = sg.t1 - t0 < sg.steps ? sg.t1 - t0 : sg.steps;
                    f.halo = f.nsteps;  // a shorter last chunk keeps the tile: its smaller halo fits the LDS
                    f.source = t0 == 0 ? source : bpst::kSrcOwn;
                    f.keep_state = t0 + f.nsteps < iters ? 1 : 0;
                    f.narrow = narrow_ok(l, t0) && bpst::fused_narrow_pays(pl.G, sg.rmax) ? 1 : 0;
                    f.compact = hk.compact;
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    if (time_each) {
                        const int32_t rc = timing_events(ctx, l, 1, &e0, &e1);
                        if (rc != BP_OK) return rc;
                        HIP_TRY(hipEventRecord(e0, st));
                    }
                    if (ctx && ctx->timing && timing_allowed)
                        ctx->pixels_max += (long long)pl.lv[l].H * pl.lv[l].Wh * f.nsteps;
                    HIP_TRY(bpst::launch_fused(f, st));
                    ++scale_launches;
                    if (e1) HIP_TRY(hipEventRecord(e1, st));
                }
            }
        }
        if (s1) {
            HIP_TRY(hipEventRecord(s1, st));
            ctx->event_launches[sslot] = scale_launches;
        }
    }
    HIP_TRY(bpst::launch_wta(user0 ? cost : C[0], M[0], pl.vol[0], pl.lv[0], pl.D, pl.G, wta_colour, disparity, st,
                             pl.packed, user0));
    if (final_msgs_or_null)
        HIP_TRY(bpst::launch_export(M[0], pl.vol[0], pl.lv[0], pl.D, pl.G, final_msgs_or_null, st, pl.packed));
    return BP_OK;
}

// The solve after argument checks: graph replay or capture when the context asks for it,
// else eager launches; then the counters, if requested.  `noalloc`: eager launches only and
// no timing events (the context's graph and timing modes are ignored), so the call creates
// no runtime object.
static int32_t run_solve(bp_context* ctx, const Plan& pl, const int16_t* cost, int32_t width, int32_t height,
                         const bp_params* params, void* workspace, size_t workspace_bytes, int16_t* disparity,
                         int16_t* final_msgs_or_null, bp_stats* stats_or_null, bool noalloc, hipStream_t st,
                         const WarmNet* net = nullptr)
{
    const bool count = stats_or_null != nullptr;
    // (the context's graphs are keyed by the solve's buffers; a network-warmed solve runs eagerly)
    if (!noalloc && !net && ctx && ctx->graphs && !count && !ctx->timing && st != nullptr) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(st, &cs));
        if (cs == hipStreamCaptureStatusNone) {
            const SolveKey key = make_key(width, height, params, cost, workspace, workspace_bytes, disparity,
                                          final_msgs_or_null, ctx->fused);
            for (auto& e : ctx->cache)
                if (std::memcmp(&e.first, &key, sizeof key) == 0) {
                    HIP_TRY(hipGraphLaunch(e.second, st));
                    ctx->graph_hits++;
                    return ok();
                }
            if (!read_hooks().graph_fail &&
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
        const int32_t rc = enqueue_solve(ctx, pl, cost, params, workspace, disparity, final_msgs_or_null, count, st,
                                         !noalloc, net);
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
            stats_or_null->n_halfsteps[l] = ((params->warm_msgs || net) && l == pl.L - 1) ? 0 : params->iters[l];
            for (int t = 0; t < bpst::kStatHalfsteps; ++t) stats_or_null->active[l][t] = hs.active[l][t];
        }
    }
    return ok();
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
    return run_solve(ctx, pl, cost, width, height, params, workspace, workspace_bytes, disparity,
                     final_msgs_or_null, stats_or_null, false, (hipStream_t)stream);
}

BP_API int32_t bp_warmstart_solve(bp_context* ctx, const uint8_t* left, const uint8_t* right, const int16_t* cost,
                                  int32_t width, int32_t height, const bp_params* params, const float* cnn_params,
                                  const uint16_t* cnn_weights, void* workspace, size_t workspace_bytes,
                                  int16_t* disparity, int16_t* final_msgs_or_null, bp_stats* stats_or_null,
                                  void* stream)
{
    std::string why;
    if (!params_valid(width, height, params, &why)) return fail(BP_E_INVAL, "%s", why.c_str());
    if (!left || !right || !cost || !disparity || !cnn_params || !cnn_weights)
        return fail(BP_E_INVAL, "a pointer is NULL");
    if (reinterpret_cast<uintptr_t>(cnn_weights) % 16 != 0) return fail(BP_E_INVAL, "cnn_weights must be 16-byte aligned");
    if (params->warm_msgs) return fail(BP_E_INVAL, "warm_msgs must be NULL: the network provides the start");
    if (params->num_scales < 2) return fail(BP_E_INVAL, "the warm start needs num_scales >= 2");
    if (!bpst::warm_cnn_supported(params->num_disp))
        return fail(BP_E_UNSUPPORTED, "the one-launch network needs num_disp a multiple of 16 in 16..64 (the "
                                      "layer-level calls take any num_disp)");
    const Plan pl = make_plan(width, height, params);
    if (!workspace || workspace_bytes < pl.total)
        return fail(BP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, pl.total);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(BP_E_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    const WarmNet net{left, right, width, height, cnn_params, cnn_weights};
    return run_solve(ctx, pl, cost, width, height, params, workspace, workspace_bytes, disparity,
                     final_msgs_or_null, stats_or_null, false, (hipStream_t)stream, &net);
}

BP_API int32_t bp_message_bits(int32_t width, int32_t height, const bp_params* params)
{
    std::string why;
    if (!params_valid(width, height, params, &why)) return 0;
    return make_plan(width, height, params).packed ? 12 : 16;
}

BP_API size_t bp_noalloc_scratch_bytes(void) { return bpst::kNoallocScratchBytes; }

BP_API int32_t bp_hierarchical_solve_noalloc(bp_context* ctx, const int16_t* cost, int32_t width, int32_t height,
                                             const bp_params* params, int16_t* disparity,
                                             int16_t* final_msgs_or_null, bp_stats* stats_or_null, void* stream)
{
    std::string why;
    if (!params_valid(width, height, params, &why)) return fail(BP_E_INVAL, "%s", why.c_str());
    if (!cost || !disparity) return fail(BP_E_INVAL, "cost/disparity is NULL");
    const Plan pl = make_plan(width, height, params);
    if (pl.total > bpst::kNoallocScratchBytes)
        return fail(BP_E_WORKSPACE,
                    "this shape needs %zu bytes of scratch; the static scratch of the allocation-free solve holds "
                    "%zu (use bp_hierarchical_solve with a workspace)",
                    pl.total, bpst::kNoallocScratchBytes);
    void* scratch = nullptr;
    HIP_TRY(bpst::noalloc_scratch(&scratch));
    return run_solve(ctx, pl, cost, width, height, params, scratch, bpst::kNoallocScratchBytes, disparity,
                     final_msgs_or_null, stats_or_null, true, (hipStream_t)stream);
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

// ---------------------------------------------------------------------------------------
// Batched solve
// ---------------------------------------------------------------------------------------
namespace {

constexpr size_t kBatchHeader = 256;    // barrier words (u32) at 0, error flag (i32) at kBatchErrorOff
constexpr size_t kBatchErrorOff = 64;

struct BatchPlan {
    int n = 0, L = 0, nphases = 0, ncc_total = 0, max_d = 0, gmax = 1;
    size_t off_ncc = 0, off_pairs = 0, off_phases = 0, off_tiles = 0, off_ncc_tiles = 0;
    size_t table_end = 0, total = 0, lds = 0;
    std::vector<size_t> pair_off;
    std::vector<Plan> plans;
    std::vector<bpst::PhaseDesc> phases;
    std::vector<int> tiles;      // nphases x (n + 1)
    std::vector<int> ncc_tiles;  // n + 1
};

bp_params pair_params(const bp_pair_desc& d, const bp_batch_params* p)
{
    bp_params q{};
    q.num_disp = d.num_disp;
    q.num_scales = p->num_scales;
    for (int l = 0; l < 8; ++l) q.iters[l] = p->iters[l];
    q.lambda = p->lambda;
    q.trunc = p->trunc;
    q.skip_mode = p->skip_mode;
    q.converge_iters = p->converge_iters;
    q.warm_msgs = nullptr;
    return q;
}

// LDS of a pyramid workgroup of the batched solve (kThreadsPerTile lanes).
size_t tree_lds_bytes(int L, int G)
{
    return (size_t)bpst::tree_blocks(L, G, bpst::kThreadsPerTile) * bpst::tree_block_lds(L, G);
}

// Validates the batch and lays out its workspace; returns 0 or a BP_E_* code.
int32_t plan_batch(const bp_pair_desc* pairs, int32_t n, const bp_batch_params* p, BatchPlan* bp, bool check_ptrs)
{
    if (!pairs || !p) return fail(BP_E_INVAL, "pairs/params is NULL");
    if (n < 1 || n > 65536) return fail(BP_E_INVAL, "n must be in 1..65536");
    if (p->window < 1 || p->window > 13 || (p->window & 1) == 0) return fail(BP_E_INVAL, "window must be odd, 1..13");
    if (p->cost_scale < 1 || p->cost_scale > 4096) return fail(BP_E_INVAL, "cost_scale must be in 1..4096");
    if (p->cost_trunc < 0 || p->cost_trunc > 32767) return fail(BP_E_INVAL, "cost_trunc must be in 0..32767");
    if (p->num_scales < 2) return fail(BP_E_UNSUPPORTED, "a batch needs num_scales >= 2");
    BatchPlan& b = *bp;
    b.n = n;
    b.L = p->num_scales;
    b.plans.resize(n);
    b.pair_off.resize(n);
    std::string why;
    for (int i = 0; i < n; ++i) {
        const bp_pair_desc& d = pairs[i];
        const bp_params q = pair_params(d, p);
        if (!params_valid(d.width, d.height, &q, &why)) return fail(BP_E_INVAL, "pair %d: %s", i, why.c_str());
        if (check_ptrs && (!d.left || !d.right || !d.cost || !d.disparity))
            return fail(BP_E_INVAL, "pair %d: a pointer is NULL", i);
        b.plans[i] = make_plan(d.width, d.height, &q);
        if (bpst::tree_block_lds(b.L, b.plans[i].G) > 64 * 1024)
            return fail(BP_E_UNSUPPORTED, "pair %d: D=%d with %d scales exceeds the pyramid's LDS", i, d.num_disp, b.L);
        b.lds = std::max(b.lds, tree_lds_bytes(b.L, b.plans[i].G));
        b.max_d = std::max(b.max_d, d.num_disp);
        b.gmax = std::max(b.gmax, b.plans[i].G);
    }
    // half-steps of a scale stream their volumes when all pairs' working sets together exceed
    // the caches (see stream_scale)
    int stream[bpst::kMaxScales] = {0};
    for (int l = 0; l < b.L; ++l) {
        double bytes = 0;
        for (int i = 0; i < n; ++i) bytes += 5.0 * (double)b.plans[i].lv[l].slots() * 8 * b.plans[i].G * 2;
        stream[l] = bytes > bpst::kStreamBytes ? 1 : 0;
    }
    // phase sequence (the same as a single solve without a warm start)
    b.phases.push_back({bpst::kPhPyramid, 0, 0, 0, 0, 0, 0});
    for (int l = b.L - 1; l >= 0; --l) {
        const bool fuse = p->iters[l] >= 2 && p->skip_mode != 2;
        if (!fuse) b.phases.push_back({bpst::kPhInit, l, 0, bpst::kSrcOwn, 0, 0, 0});
        for (int t = 0; t < p->iters[l]; ++t) {
            int src = bpst::kSrcOwn;
            if (t == 0 && fuse) src = (l == b.L - 1) ? bpst::kSrcZero : bpst::kSrcParent;
            // plain BP's last half-step of the finest scale also writes the winners of the
            // pixels it updates (their incoming messages are final)
            const int wta = l == 0 && t == p->iters[0] - 1 && p->skip_mode == 0 ? 1 : 0;
            b.phases.push_back({bpst::kPhHalfstep, l, t, src, 0, stream[l], wta});
        }
    }
    const int wta_colour = p->iters[0] >= 1 && p->skip_mode == 0 ? (p->iters[0] - 1) & 1 : -1;
    b.phases.push_back({bpst::kPhWta, 0, 0, 0, 0, stream[0], wta_colour});
    b.nphases = (int)b.phases.size();
    b.tiles.assign((size_t)b.nphases * (n + 1), 0);
    for (int ph = 0; ph < b.nphases; ++ph) {
        bpst::PhaseDesc& d = b.phases[ph];
        d.table = ph * (n + 1);
        int* ts = &b.tiles[(size_t)ph * (n + 1)];
        long long acc = 0;
        for (int i = 0; i < n; ++i) {
            ts[i] = (int)acc;
            const Plan& pl = b.plans[i];
            const long long px = bpst::kThreadsPerTile / pl.G;
            const bpst::Level& lv = pl.lv[d.level];
            long long nt = 0;
            switch (d.type) {
            case bpst::kPhPyramid: {
                const long long nb = bpst::tree_blocks(b.L, pl.G, bpst::kThreadsPerTile);
                nt = ((long long)pl.lv[b.L - 1].W * pl.lv[b.L - 1].H + nb - 1) / nb;
                break;
            }
            case bpst::kPhInit:
            case bpst::kPhWta: nt = (lv.slots() + px - 1) / px; break;
            case bpst::kPhHalfstep: nt = ((long long)lv.H * lv.Wh + px - 1) / px; break;
            }
            acc += nt;
            if (acc > 2000000000LL) return fail(BP_E_UNSUPPORTED, "batch too large for one launch");
        }
        ts[n] = (int)acc;
    }
    b.ncc_tiles.assign(n + 1, 0);
    long long acc = 0;
    for (int i = 0; i < n; ++i) {
        b.ncc_tiles[i] = (int)acc;
        acc += bpst::ncc_mfma_tiles(pairs[i].width, pairs[i].height);
    }
    b.ncc_tiles[n] = (int)acc;
    b.ncc_total = (int)acc;
    // workspace: header | NccPair[n] | PairDev[n] | PhaseDesc[] | tiles | ncc tiles | pair regions
    size_t o = kBatchHeader;
    b.off_ncc = o;
    o = align_up(o + sizeof(bpst::NccPair) * n);
    b.off_pairs = o;
    o = align_up(o + sizeof(bpst::PairDev) * n);
    b.off_phases = o;
    o = align_up(o + sizeof(bpst::PhaseDesc) * b.nphases);
    b.off_tiles = o;
    o = align_up(o + sizeof(int) * b.tiles.size());
    b.off_ncc_tiles = o;
    o = align_up(o + sizeof(int) * b.ncc_tiles.size());
    b.table_end = o;
    for (int i = 0; i < n; ++i) {
        b.pair_off[i] = o;
        o = align_up(o + b.plans[i].total);
    }
    b.total = o;
    return BP_OK;
}

// Host image of the table region [kBatchHeader, table_end) for workspace base ws.
void fill_tables(const BatchPlan& b, const bp_pair_desc* pairs, char* ws, std::vector<char>* img)
{
    img->assign(b.table_end - kBatchHeader, 0);
    char* base = img->data() - kBatchHeader;  // so that base + off matches workspace offsets
    auto* ncc = reinterpret_cast<bpst::NccPair*>(base + b.off_ncc);
    auto* pd = reinterpret_cast<bpst::PairDev*>(base + b.off_pairs);
    for (int i = 0; i < b.n; ++i) {
        const bp_pair_desc& d = pairs[i];
        const Plan& pl = b.plans[i];
        char* r = ws + b.pair_off[i];
        ncc[i] = bpst::NccPair{d.left, d.right, d.cost, d.width, d.height, d.num_disp, 0};
        bpst::PairDev q{};
        q.cost = d.cost;
        q.disparity = d.disparity;
        for (int l = 0; l < pl.L; ++l) {
            q.c[l] = reinterpret_cast<int16_t*>(r + pl.off_cost[l]);
            q.lv[l] = pl.lv[l];
            q.vol[l] = pl.vol[l];
        }
        q.m[0] = reinterpret_cast<int16_t*>(r + pl.off_msgs[0]);
        q.m[1] = reinterpret_cast<int16_t*>(r + pl.off_msgs[1]);
        q.sa = reinterpret_cast<uint8_t*>(r + pl.off_sa);
        q.sb = reinterpret_cast<uint8_t*>(r + pl.off_sb);
        q.D = pl.D;
        q.G = pl.G;
        q.vec = (pl.D % 8 == 0) && ((reinterpret_cast<uintptr_t>(d.cost) & 15) == 0);
        pd[i] = q;
    }
    std::memcpy(base + b.off_phases, b.phases.data(), sizeof(bpst::PhaseDesc) * b.nphases);
    std::memcpy(base + b.off_tiles, b.tiles.data(), sizeof(int) * b.tiles.size());
    std::memcpy(base + b.off_ncc_tiles, b.ncc_tiles.data(), sizeof(int) * b.ncc_tiles.size());
}

std::vector<int32_t> batch_signature(const bp_pair_desc* pairs, int32_t n, const bp_batch_params* p)
{
    std::vector<int32_t> s;
    s.reserve(3 * n + 32);
    s.push_back(n);
    const int32_t* pp = reinterpret_cast<const int32_t*>(p);
    for (size_t i = 0; i < sizeof(bp_batch_params) / 4; ++i) s.push_back(pp[i]);
    for (int i = 0; i < n; ++i) {
        s.push_back(pairs[i].width);
        s.push_back(pairs[i].height);
        s.push_back(pairs[i].num_disp);
    }
    return s;
}

int32_t device_limits(int mode, int gmax, size_t lds, int* cus, int* max_bpc, long long* ticks_per_s)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev));
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    *ticks_per_s = (long long)(khz > 0 ? khz : 100000) * 1000LL;
    HIP_TRY(bpst::batch_max_blocks_per_cu(mode, gmax, lds, max_bpc));
    if (*max_bpc < 1) return fail(BP_E_UNSUPPORTED, "the persistent kernel cannot be resident");
    return BP_OK;
}

// Upload the tables through a pinned staging buffer, stream-ordered.
int32_t upload_tables(bp_context* ctx, const std::vector<char>& img, char* ws, hipStream_t st)
{
    const int i = ctx->staging_next;
    ctx->staging_next ^= 1;
    if (ctx->staging_done[i]) HIP_TRY(hipEventSynchronize(ctx->staging_done[i]));  // previous copy finished
    else HIP_TRY(hipEventCreateWithFlags(&ctx->staging_done[i], hipEventDisableTiming));
    if (ctx->staging_bytes[i] < img.size()) {
        if (ctx->staging[i]) HIP_TRY(hipHostFree(ctx->staging[i]));
        ctx->staging[i] = nullptr;
        ctx->staging_bytes[i] = 0;
        HIP_TRY(hipHostMalloc(&ctx->staging[i], img.size(), hipHostMallocDefault));
        ctx->staging_bytes[i] = img.size();
    }
    std::memcpy(ctx->staging[i], img.data(), img.size());
    HIP_TRY(hipMemcpyAsync(ws + kBatchHeader, ctx->staging[i], img.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(ctx->staging_done[i], st));
    return BP_OK;
}

// A batch keeps its messages in 12 bits wherever every message fits (min(lambda * T, 32767)
// <= 4095, as in the solo solve, whatever D): a quarter fewer message bytes on the streamed
// half-step phases, which hold most of a batch's time.
bool batch_packed(const bp_batch_params* p) { return (long long)p->lambda * p->trunc <= 4095; }

bpst::BatchArgs batch_args(const BatchPlan& b, const bp_batch_params* p, char* ws, int order, long long ticks,
                           bool narrow)
{
    bpst::BatchArgs a{};
    a.pairs = reinterpret_cast<const bpst::PairDev*>(ws + b.off_pairs);
    a.phases = reinterpret_cast<const bpst::PhaseDesc*>(ws + b.off_phases);
    a.tiles = reinterpret_cast<const int*>(ws + b.off_tiles);
    a.npairs = b.n;
    a.nphases = b.nphases;
    a.L = b.L;
    a.lambda = p->lambda;
    // min(T, D) differs per pair only when T exceeds some pair's D; the clamp value is
    // min(lambda * T, 32767) either way unless T >= D, where the clamp never binds
    const long long lt = (long long)p->lambda * p->trunc;
    a.capv = (int)(lt < 32767 ? lt : 32767);
    a.packed = batch_packed(p) ? 1 : 0;  // the narrow path does not take 12-bit messages
    a.narrow = narrow && a.capv <= bpst::kNarrowCap && !a.packed ? 1 : 0;
    a.K = p->converge_iters;
    a.mode = p->skip_mode;
    a.order = order;
    a.gmax = b.gmax;
    a.barrier = reinterpret_cast<unsigned*>(ws);
    a.error = reinterpret_cast<int*>(ws + kBatchErrorOff);
    a.timeout_ticks = ticks * 10;  // 10 s
    return a;
}

// The solve part of a batch: schedule 0 is one persistent launch of bpc workgroups per
// compute unit; schedule 1 is one launch per phase; schedule 2 is schedule 1 with packed
// 16-bit message sums where lambda * trunc allows them.

int32_t enqueue_batch_solve(bp_context* ctx, const BatchPlan& b, const bp_batch_params* p, char* ws, int sched, int bpc,
                            int order, int cus, long long ticks, hipStream_t st)
{
    // schedules: 0 one persistent launch, 1 one launch per phase, 2 the same on the narrow path
    const bpst::BatchArgs a = batch_args(b, p, ws, order, ticks, sched == 2);
    HIP_TRY(bpst::launch_batch_reset(a.barrier, a.error, st));
    if (sched == 1 || sched == 2) {
        for (int ph = 0; ph < b.nphases; ++ph) {
            const bpst::PhaseDesc& d = b.phases[ph];
            // timing mode: an event pair around every half-step phase
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (ctx && ctx->timing && d.type == bpst::kPhHalfstep) {
                const int32_t rc = timing_events(ctx, d.level, 1, &e0, &e1);
                if (rc != BP_OK) return rc;
                HIP_TRY(hipEventRecord(e0, st));
            }
            // streamed phases stay on the int32 path (the narrow path pays only off the memory bound)
            const int hv = (d.stream ? bpst::kHvStream : (a.narrow ? bpst::kHvNarrow : 0)) | (a.packed ? bpst::kHvPacked : 0);
            HIP_TRY(bpst::launch_batch_phase(a, ph, d.type, d.source, b.tiles[(size_t)ph * (b.n + 1) + b.n],
                                             b.lds, hv, st));
            if (e1) HIP_TRY(hipEventRecord(e1, st));
        }
        return BP_OK;
    }
    int blocks = bpc * cus;
    if (order == 1) blocks = std::max(bpst::kXcds, blocks / bpst::kXcds * bpst::kXcds);
    HIP_TRY(bpst::launch_batch_solve(a, blocks, b.lds, st));
    return BP_OK;
}

int32_t enqueue_batch(bp_context* ctx, const BatchPlan& b, const bp_batch_params* p, char* ws, int sched, int bpc,
                      int order, int cus, long long ticks, hipStream_t st)
{
    HIP_TRY(bpst::launch_ncc_mfma_batched(reinterpret_cast<const bpst::NccPair*>(ws + b.off_ncc),
                                          reinterpret_cast<const int*>(ws + b.off_ncc_tiles), b.n, b.ncc_total,
                                          b.max_d, p->window, p->cost_scale, p->cost_trunc, st));
    return enqueue_batch_solve(ctx, b, p, ws, sched, bpc, order, cus, ticks, st);
}

}  // namespace

BP_API size_t bp_batch_workspace_bytes(const bp_pair_desc* pairs, int32_t n, const bp_batch_params* params)
{
    BatchPlan b;
    if (plan_batch(pairs, n, params, &b, false) != BP_OK) return 0;
    return b.total;
}

BP_API int32_t bp_batch_message_bits(const bp_pair_desc* pairs, int32_t n, const bp_batch_params* params)
{
    BatchPlan b;
    if (plan_batch(pairs, n, params, &b, false) != BP_OK) return 0;
    return batch_packed(params) ? 12 : 16;
}

BP_API int32_t bp_solve_batched(bp_context* ctx, const bp_pair_desc* pairs, int32_t n, const bp_batch_params* params,
                                void* workspace, size_t workspace_bytes, void* stream)
{
    if (!ctx) return fail(BP_E_INVAL, "a batched solve needs a context");
    BatchPlan b;
    int32_t rc = plan_batch(pairs, n, params, &b, true);
    if (rc != BP_OK) return rc;
    if (!workspace || workspace_bytes < b.total)
        return fail(BP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, b.total);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(BP_E_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    char* ws = static_cast<char*>(workspace);
    hipStream_t st = (hipStream_t)stream;
    int cus = 0, max_bpc = 0;
    long long ticks = 0;
    rc = device_limits(params->skip_mode, b.gmax, b.lds, &cus, &max_bpc, &ticks);
    if (rc != BP_OK) return rc;
    // untuned: one launch per phase with packed sums where they apply (schedule 2, which runs
    // as schedule 1 when lambda * trunc > 16383): measured faster than the persistent launch
    int bpc = std::min(2, max_bpc), order = 0, sched = 2;
    const std::vector<int32_t> sig = batch_signature(pairs, n, params);
    for (const auto& t : ctx->tuned)
        if (t.sig == sig) {
            bpc = std::min(t.bpc, max_bpc);
            order = t.order;
            sched = t.sched;
        }
    if (ctx->forced_sched >= 0) {
        sched = ctx->forced_sched;
        bpc = std::min(ctx->forced_bpc, max_bpc);
        order = ctx->forced_order;
    }
    std::vector<char> img;
    fill_tables(b, pairs, ws, &img);
    rc = upload_tables(ctx, img, ws, st);
    if (rc != BP_OK) return rc;
    if (ctx->graphs && !ctx->timing && st != nullptr) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(st, &cs));
        if (cs == hipStreamCaptureStatusNone) {
            // graph key: the table image (pointers and shapes), the workspace and the launch shape
            std::vector<char> key(img);
            const char* extra = reinterpret_cast<const char*>(&ws);
            key.insert(key.end(), extra, extra + sizeof(ws));
            key.insert(key.end(), reinterpret_cast<const char*>(params),
                       reinterpret_cast<const char*>(params) + sizeof(*params));
            const int shape[3] = {bpc, order, sched};
            key.insert(key.end(), reinterpret_cast<const char*>(shape), reinterpret_cast<const char*>(shape) + 12);
            for (auto& e : ctx->batch_graphs)
                if (e.first == key) {
                    HIP_TRY(hipGraphLaunch(e.second, st));
                    ctx->graph_hits++;
                    return ok();
                }
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                const int32_t r2 = enqueue_batch(nullptr, b, params, ws, sched, bpc, order, cus, ticks, st);
                hipGraph_t g = nullptr;
                const hipError_t ee = hipStreamEndCapture(st, &g);
                hipGraphExec_t ex = nullptr;
                const bool good = r2 == BP_OK && ee == hipSuccess && g &&
                                  hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
                if (g) (void)hipGraphDestroy(g);
                if (good) {
                    if (ctx->batch_graphs.size() >= kMaxGraphs) {
                        (void)hipGraphExecDestroy(ctx->batch_graphs.front().second);
                        ctx->batch_graphs.erase(ctx->batch_graphs.begin());
                    }
                    ctx->batch_graphs.emplace_back(std::move(key), ex);
                    ctx->graph_captures++;
                    HIP_TRY(hipGraphLaunch(ex, st));
                    return ok();
                }
            }
            (void)hipGetLastError();
            ctx->graph_fallbacks++;
        }
    }
    rc = enqueue_batch(ctx, b, params, ws, sched, bpc, order, cus, ticks, st);
    if (rc != BP_OK) return rc;
    return ok();
}

BP_API int32_t bp_batch_status(const void* workspace, void* stream, int32_t* status)
{
    if (!workspace || !status) return fail(BP_E_INVAL, "workspace/status is NULL");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int32_t e = 0;
    HIP_TRY(hipMemcpy(&e, static_cast<const char*>(workspace) + kBatchErrorOff, sizeof e, hipMemcpyDeviceToHost));
    *status = e;
    return ok();
}

BP_API int32_t bp_autotune_batched(bp_context* ctx, const bp_pair_desc* pairs, int32_t n,
                                   const bp_batch_params* params, void* workspace, size_t workspace_bytes,
                                   void* stream, bp_batch_tuning* out)
{
    if (!ctx || !out) return fail(BP_E_INVAL, "ctx/out is NULL");
    BatchPlan b;
    int32_t rc = plan_batch(pairs, n, params, &b, true);
    if (rc != BP_OK) return rc;
    if (!workspace || workspace_bytes < b.total)
        return fail(BP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, b.total);
    char* ws = static_cast<char*>(workspace);
    hipStream_t st = (hipStream_t)stream;
    int cus = 0, max_bpc = 0;
    long long ticks = 0;
    rc = device_limits(params->skip_mode, b.gmax, b.lds, &cus, &max_bpc, &ticks);
    if (rc != BP_OK) return rc;
    std::vector<char> img;
    fill_tables(b, pairs, ws, &img);
    rc = upload_tables(ctx, img, ws, st);
    if (rc != BP_OK) return rc;
    std::memset(out, 0, sizeof *out);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // candidates: the per-phase schedule, then the persistent launch at each shape
    struct Cand {
        int sched, bpc, order;
    };
    std::vector<Cand> cands{{1, 0, 0}};
    if ((long long)params->lambda * params->trunc <= bpst::kNarrowCap) cands.push_back({2, 0, 0});
    for (int bpc = 1; bpc <= max_bpc; bpc = (bpc < 4 ? bpc + 1 : bpc * 2))
        for (int order = 0; order < 2; ++order) cands.push_back({0, bpc, order});
    int k = 0;
    for (const Cand& c : cands) {
        if (k >= 16) break;
        out->schedule[k] = c.sched;
        out->blocks_per_cu[k] = c.bpc;
        out->order[k] = c.order;
        float best = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {  // the first run warms caches and code
            HIP_TRY(hipEventRecord(e0, st));
            rc = enqueue_batch_solve(nullptr, b, params, ws, c.sched, c.bpc, c.order, cus, ticks, st);
            if (rc != BP_OK) return rc;
            HIP_TRY(hipEventRecord(e1, st));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        int32_t err = 0;
        HIP_TRY(hipMemcpy(&err, ws + kBatchErrorOff, sizeof err, hipMemcpyDeviceToHost));
        out->ms[k] = err ? 1e30f : best;
        ++k;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    out->n_candidates = k;
    int bi = 0;
    for (int i = 1; i < k; ++i)
        if (out->ms[i] < out->ms[bi]) bi = i;
    out->best = bi;
    const std::vector<int32_t> sig = batch_signature(pairs, n, params);
    bool found = false;
    for (auto& t : ctx->tuned)
        if (t.sig == sig) {
            t.bpc = out->blocks_per_cu[bi];
            t.order = out->order[bi];
            t.sched = out->schedule[bi];
            found = true;
        }
    if (!found) ctx->tuned.push_back({sig, out->blocks_per_cu[bi], out->order[bi], out->schedule[bi]});
    // leave the workspace holding a complete solve of the batch
    rc = enqueue_batch(nullptr, b, params, ws, out->schedule[bi], out->blocks_per_cu[bi], out->order[bi], cus, ticks,
                       st);
    if (rc != BP_OK) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    return ok();
}

// ---------------------------------------------------------------------------------------
// Pieces of the solve used by the learned warm start
// ---------------------------------------------------------------------------------------
namespace {
// Enqueue the cost pyramid of a solve into its workspace (the internal cost of every scale).
int32_t enqueue_pyramid(const Plan& pl, const int16_t* cost, char* ws, hipStream_t st)
{
    int16_t* C[bpst::kMaxScales];
    for (int l = 0; l < pl.L; ++l) C[l] = reinterpret_cast<int16_t*>(ws + pl.off_cost[l]);
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
    return BP_OK;
}

int32_t check_solve_args(int32_t W, int32_t H, const bp_params* p, void* ws, size_t wsb, Plan* pl)
{
    std::string why;
    if (!params_valid(W, H, p, &why)) return fail(BP_E_INVAL, "%s", why.c_str());
    *pl = make_plan(W, H, p);
    if (!ws || wsb < pl->total) return fail(BP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", wsb, pl->total);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0)
        return fail(BP_E_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    return BP_OK;
}
}  // namespace

BP_API int32_t bp_pyramid_level(const int16_t* cost, int32_t width, int32_t height, const bp_params* params,
                                int32_t level, void* workspace, size_t workspace_bytes, int16_t* out, void* stream)
{
    Plan pl;
    int32_t rc = check_solve_args(width, height, params, workspace, workspace_bytes, &pl);
    if (rc != BP_OK) return rc;
    if (!cost || !out) return fail(BP_E_INVAL, "cost/out is NULL");
    if (level < 0 || level >= pl.L) return fail(BP_E_INVAL, "level must be in 0..num_scales-1");
    hipStream_t st = (hipStream_t)stream;
    if (level == 0) {
        // the finest scale is the caller's cost itself (internally it is kept shifted by each
        // pixel's minimum)
        if (out != cost)
            HIP_TRY(hipMemcpyAsync(out, cost, (size_t)width * height * params->num_disp * sizeof(int16_t),
                                   hipMemcpyDeviceToDevice, st));
        return ok();
    }
    char* ws = static_cast<char*>(workspace);
    rc = enqueue_pyramid(pl, cost, ws, st);
    if (rc != BP_OK) return rc;
    // export scale `level` from the internal layout (its message buffers are free scratch here)
    HIP_TRY(bpst::launch_export_cost(reinterpret_cast<const int16_t*>(ws + pl.off_cost[level]), pl.lv[level], pl.D,
                                     pl.G, out, st));
    return ok();
}

namespace {
// Workspace of the Jacobi schedule: the internal cost, then two sets of four message volumes.
struct JacobiPlan {
    int G, Dp;
    bpst::Level lv;
    long long vol;
    size_t off_cost, off_msgs[2], total;
};

bool jacobi_valid(int W, int H, int D, std::string* why)
{
    if (W < 1 || H < 1 || W > 16384 || H > 16384) return *why = "width/height must be in 1..16384", false;
    if (D < 1 || D > 256) return *why = "num_disp must be in 1..256", false;
    return true;
}

JacobiPlan make_jacobi_plan(int W, int H, int D)
{
    JacobiPlan p{};
    p.G = bpst::lanes_for(D);
    p.Dp = 8 * p.G;
    p.lv = bpst::make_level(W, H);
    p.vol = p.lv.slots() * p.Dp;
    size_t o = 0;
    p.off_cost = o;
    o = align_up(o + (size_t)p.vol * sizeof(int16_t));
    for (int b = 0; b < 2; ++b) {
        p.off_msgs[b] = o;
        o = align_up(o + 4 * (size_t)p.vol * sizeof(int16_t));
    }
    p.total = o;
    return p;
}
}  // namespace

BP_API size_t bp_jacobi_workspace_bytes(int32_t width, int32_t height, int32_t num_disp)
{
    std::string why;
    if (!jacobi_valid(width, height, num_disp, &why)) return 0;
    return make_jacobi_plan(width, height, num_disp).total;
}

BP_API int32_t bp_jacobi_iterations(const int16_t* cost, int32_t width, int32_t height, int32_t num_disp,
                                    int32_t lambda, int32_t trunc, int32_t iterations,
                                    const int16_t* init_msgs_or_null, int16_t* msgs_out, void* workspace,
                                    size_t workspace_bytes, void* stream)
{
    std::string why;
    if (!jacobi_valid(width, height, num_disp, &why)) return fail(BP_E_INVAL, "%s", why.c_str());
    if (lambda < 0 || lambda > 65535 || trunc < 0) return fail(BP_E_INVAL, "lambda/trunc out of range");
    if (iterations < 0 || iterations > 65536) return fail(BP_E_INVAL, "iterations must be in 0..65536");
    if (!cost || !msgs_out) return fail(BP_E_INVAL, "cost/msgs_out is NULL");
    const JacobiPlan jp = make_jacobi_plan(width, height, num_disp);
    if (!workspace || workspace_bytes < jp.total)
        return fail(BP_E_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes, jp.total);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(BP_E_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    hipStream_t st = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    int16_t* C = reinterpret_cast<int16_t*>(ws + jp.off_cost);
    int16_t* M[2] = {reinterpret_cast<int16_t*>(ws + jp.off_msgs[0]), reinterpret_cast<int16_t*>(ws + jp.off_msgs[1])};
    HIP_TRY(bpst::launch_prep_level0(cost, C, jp.lv, num_disp, jp.G, st));
    // the initial set: the caller's messages (zero where a pixel has no neighbour), or zeros
    if (init_msgs_or_null)
        HIP_TRY(bpst::launch_import(init_msgs_or_null, M[0], jp.lv, jp.vol, num_disp, jp.G, nullptr, nullptr, 0, st));
    else
        HIP_TRY(bpst::launch_init(nullptr, jp.lv, 0, M[0], jp.lv, jp.vol, jp.G, nullptr, nullptr, 0, st));
    const int tq = trunc < num_disp ? trunc : num_disp;
    bpst::HalfstepArgs a{};
    a.cost = C;
    a.vol = jp.vol;
    a.lv = jp.lv;
    a.D = num_disp;
    a.Dp = jp.Dp;
    a.G = jp.G;
    a.lambda = lambda;
    a.capv = lambda * tq < 32767 ? lambda * tq : 32767;
    a.mode = 0;
    a.source = bpst::kSrcOwn;
    a.stream = bpst::stream_scale(jp.lv, jp.G) ? 1 : 0;
    // Each iteration reads one set and writes the other: both colours send from the same
    // (previous) messages.  A colour's update writes only the other colour's slots, so the
    // two launches of an iteration do not read what the other writes.
    for (int it = 0; it < iterations; ++it) {
        a.msgs = M[it & 1];
        a.out = M[(it + 1) & 1];
        for (int c = 0; c < 2; ++c) {
            a.colour = c;
            a.t = c;
            HIP_TRY(bpst::launch_halfstep(a, st));
        }
    }
    HIP_TRY(bpst::launch_export(M[iterations & 1], jp.vol, jp.lv, num_disp, jp.G, msgs_out, st));
    return ok();
}

BP_API int32_t bp_warmstart_input(const uint8_t* left, const uint8_t* right, const int16_t* cost, int32_t width,
                                  int32_t height, const bp_params* params, void* workspace, size_t workspace_bytes,
                                  uint16_t* input, void* stream)
{
    Plan pl;
    int32_t rc = check_solve_args(width, height, params, workspace, workspace_bytes, &pl);
    if (rc != BP_OK) return rc;
    if (!left || !right || !cost || !input) return fail(BP_E_INVAL, "a pointer is NULL");
    if (pl.L < 2) return fail(BP_E_INVAL, "the warm start needs num_scales >= 2");
    hipStream_t st = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    rc = enqueue_pyramid(pl, cost, ws, st);
    if (rc != BP_OK) return rc;
    const int s = pl.L - 2;
    const int cin_p = (2 + pl.D + 15) / 16 * 16;
    HIP_TRY(bpst::launch_warm_input(left, right, width, height, s,
                                    reinterpret_cast<const int16_t*>(ws + pl.off_cost[pl.L - 1]), pl.lv[pl.L - 1],
                                    pl.Dp, pl.D, pl.lv[s].W, pl.lv[s].H, cin_p, input, st));
    return ok();
}
