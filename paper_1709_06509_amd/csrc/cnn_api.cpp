// Host side of the learned warm start: the network's layer geometry and parameter layout,
// its forward and backward passes composed from the convolution kernels, Adam, and the
// conversion of its output into initial messages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/bpstereo.h"
#include "internal.h"

#define BP_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kLayers = 6;
constexpr int kHidden = 32;
constexpr int kChunk = 512;  // pixels per partial sum of the weight gradient

struct LayerGeo {
    int cin, cin_p, cout, cout_p, relu;
    long long w_off, b_off;
};

bool geometry(int D, LayerGeo g[kLayers], long long* total)
{
    if (D < 1 || D > 256) return false;
    long long o = 0;
    for (int l = 0; l < kLayers; ++l) {
        LayerGeo& L = g[l];
        L.cin = l == 0 ? 2 + D : kHidden;
        L.cout = l == kLayers - 1 ? 4 * D : kHidden;
        L.cin_p = (L.cin + 15) / 16 * 16;
        L.cout_p = (L.cout + 31) / 32 * 32;
        L.relu = l < kLayers - 1;
        L.w_off = o;
        o += (long long)L.cout_p * 9 * L.cin_p;
        L.b_off = o;
        o += L.cout_p;
    }
    *total = o;
    return true;
}

size_t a256(size_t v) { return (v + 255) / 256 * 256; }

static_assert(kLayers == bpst::kCnnLayers, "one layer count");

struct CnnWs {
    size_t act[kLayers];  // act[l], l >= 1: bf16 [P][32], the input of layer l
    size_t gy, gh[2], wflip, part_w, part_b, part_loss, total;
};

CnnWs ws_layout(long long P, const LayerGeo g[kLayers])
{
    CnnWs w{};
    size_t o = 0;
    for (int l = 1; l < kLayers; ++l) {
        w.act[l] = o;
        o = a256(o + (size_t)P * kHidden * 2);
    }
    w.gy = o;
    o = a256(o + (size_t)P * g[kLayers - 1].cout_p * 2);
    for (int i = 0; i < 2; ++i) {
        w.gh[i] = o;
        o = a256(o + (size_t)P * kHidden * 2);
    }
    size_t maxw = 0, maxc = 0;
    for (int l = 0; l < kLayers; ++l) {
        maxw = std::max(maxw, (size_t)g[l].cout_p * 9 * g[l].cin_p);
        maxc = std::max(maxc, (size_t)g[l].cout_p);
    }
    const size_t S = (size_t)bpst::wgrad_chunks((int)P, kChunk);
    w.wflip = o;
    o = a256(o + maxw * 2);
    w.part_w = o;
    o = a256(o + S * maxw * 4);
    w.part_b = o;
    o = a256(o + S * maxc * 4);
    w.part_loss = o;
    o = a256(o + (size_t)bpst::l1_blocks((int)P, g[kLayers - 1].cout_p) * 4);
    w.total = o;
    return w;
}

int32_t fail(int32_t code, const char* msg) { return bpst::report(code, msg); }

int32_t hip_fail(hipError_t e, const char* what)
{
    char b[256];
    snprintf(b, sizeof b, "%s: %s", what, hipGetErrorString(e));
    return bpst::report(BP_E_HIP, b);
}

#define CNN_TRY(expr)                                        \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

bool size_ok(int32_t Ws, int32_t Hs) { return Ws >= 1 && Hs >= 1 && Ws <= 4096 && Hs <= 4096; }

// The convolutions read activations and weights 16 bytes (8 bf16) at a time.
bool a16(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

}  // namespace

bool bpst::cnn_offsets(int D, long long w_off[kCnnLayers], long long b_off[kCnnLayers])
{
    LayerGeo g[kLayers];
    long long n = 0;
    if (!geometry(D, g, &n)) return false;
    for (int l = 0; l < kLayers; ++l) {
        w_off[l] = g[l].w_off;
        b_off[l] = g[l].b_off;
    }
    return true;
}

BP_API int64_t bp_cnn_param_count(int32_t num_disp)
{
    LayerGeo g[kLayers];
    long long n = 0;
    if (!geometry(num_disp, g, &n)) return -1;
    return n;
}

BP_API int32_t bp_cnn_layer(int32_t num_disp, int32_t layer, int32_t* dims, int64_t* offsets)
{
    LayerGeo g[kLayers];
    long long n = 0;
    if (!geometry(num_disp, g, &n) || layer < 0 || layer >= kLayers || !dims || !offsets)
        return fail(BP_E_INVAL, "num_disp must be in 1..256, layer in 0..5, dims/offsets non-NULL");
    const LayerGeo& L = g[layer];
    dims[0] = L.cin;
    dims[1] = L.cin_p;
    dims[2] = L.cout;
    dims[3] = L.cout_p;
    dims[4] = L.relu;
    offsets[0] = L.w_off;
    offsets[1] = L.b_off;
    return fail(BP_OK, nullptr);
}

BP_API size_t bp_cnn_workspace_bytes(int32_t Ws, int32_t Hs, int32_t num_disp)
{
    LayerGeo g[kLayers];
    long long n = 0;
    if (!size_ok(Ws, Hs) || !geometry(num_disp, g, &n)) return 0;
    return ws_layout((long long)Ws * Hs, g).total;
}

BP_API int32_t bp_conv3x3_forward(const uint16_t* in, int32_t H, int32_t W, int32_t cin_p, const uint16_t* weights,
                                  const float* bias, int32_t cout, int32_t cout_p, int32_t relu, const uint16_t* mask,
                                  uint16_t* out_bf16, float* out_f32, void* stream)
{
    if (!in || !weights || (!out_bf16 && !out_f32)) return fail(BP_E_INVAL, "in/weights/outputs are NULL");
    if (!a16(in) || !a16(weights)) return fail(BP_E_INVAL, "in and weights must be 16-byte aligned");
    if (!size_ok(W, H) || cin_p < 16 || cin_p % 16 || cout < 1 || cout_p < cout || cout_p % 32)
        return fail(BP_E_INVAL, "bad sizes: cin_p must be a multiple of 16, cout_p a multiple of 32 >= cout");
    CNN_TRY(bpst::launch_conv_fwd(in, H, W, cin_p, weights, bias, cout, cout_p, relu, mask, out_bf16, out_f32,
                                  (hipStream_t)stream));
    return fail(BP_OK, nullptr);
}

BP_API int32_t bp_conv3x3_data_grad(const uint16_t* g, int32_t H, int32_t W, int32_t cout_p, const uint16_t* weights,
                                    int32_t cin, int32_t cin_p, const uint16_t* mask, uint16_t* flip_scratch,
                                    uint16_t* out_bf16, float* out_f32, void* stream)
{
    if (!g || !weights || !flip_scratch || (!out_bf16 && !out_f32)) return fail(BP_E_INVAL, "a pointer is NULL");
    if (!a16(g) || !a16(flip_scratch)) return fail(BP_E_INVAL, "g and flip_scratch must be 16-byte aligned");
    if (!size_ok(W, H) || cout_p < 32 || cout_p % 32 || cin < 1 || cin_p < cin || cin_p % 32)
        return fail(BP_E_INVAL, "bad sizes: cout_p and cin_p must be multiples of 32");
    hipStream_t st = (hipStream_t)stream;
    CNN_TRY(bpst::launch_flip(weights, cin_p, cout_p, flip_scratch, st));
    CNN_TRY(bpst::launch_conv_fwd(g, H, W, cout_p, flip_scratch, nullptr, cin, cin_p, 0, mask, out_bf16, out_f32, st));
    return fail(BP_OK, nullptr);
}

BP_API size_t bp_conv3x3_wgrad_workspace_bytes(int32_t H, int32_t W, int32_t cin_p, int32_t cout_p)
{
    if (!size_ok(W, H) || cin_p < 16 || cout_p < 32) return 0;
    const size_t S = (size_t)bpst::wgrad_chunks(H * W, kChunk);
    return a256(S * (size_t)cout_p * 9 * cin_p * 4) + a256(S * (size_t)cout_p * 4);
}

BP_API int32_t bp_conv3x3_weight_grad(const uint16_t* in, const uint16_t* g, int32_t H, int32_t W, int32_t cin_p,
                                      int32_t cout_p, void* workspace, size_t workspace_bytes, float* dw, float* db,
                                      void* stream)
{
    if (!in || !g || !dw || !db || !workspace) return fail(BP_E_INVAL, "a pointer is NULL");
    if (!size_ok(W, H) || cin_p < 16 || cin_p % 16 || cout_p < 32 || cout_p % 32)
        return fail(BP_E_INVAL, "bad sizes: cin_p multiple of 16, cout_p multiple of 32");
    const size_t need = bp_conv3x3_wgrad_workspace_bytes(H, W, cin_p, cout_p);
    if (workspace_bytes < need) return fail(BP_E_WORKSPACE, "weight-gradient workspace too small");
    const size_t S = (size_t)bpst::wgrad_chunks(H * W, kChunk);
    char* ws = static_cast<char*>(workspace);
    float* pw = reinterpret_cast<float*>(ws);
    float* pb = reinterpret_cast<float*>(ws + a256(S * (size_t)cout_p * 9 * cin_p * 4));
    CNN_TRY(bpst::launch_conv_wgrad(in, g, H, W, cin_p, cout_p, kChunk, pw, pb, dw, db, (hipStream_t)stream));
    return fail(BP_OK, nullptr);
}

BP_API int32_t bp_cnn_forward(const uint16_t* input, int32_t Ws, int32_t Hs, int32_t num_disp, const float* params,
                              const uint16_t* weights_bf16, void* workspace, size_t workspace_bytes, float* y,
                              void* stream)
{
    LayerGeo g[kLayers];
    long long n = 0;
    if (!size_ok(Ws, Hs) || !geometry(num_disp, g, &n)) return fail(BP_E_INVAL, "bad size or num_disp");
    if (!input || !params || !weights_bf16 || !y || !workspace) return fail(BP_E_INVAL, "a pointer is NULL");
    if (!a16(input) || !a16(weights_bf16) || !a16(workspace))
        return fail(BP_E_INVAL, "input, weights_bf16 and workspace must be 16-byte aligned");
    const long long P = (long long)Ws * Hs;
    const CnnWs wl = ws_layout(P, g);
    if (workspace_bytes < wl.total) return fail(BP_E_WORKSPACE, "CNN workspace too small");
    hipStream_t st = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    const uint16_t* a = input;
    for (int l = 0; l < kLayers; ++l) {
        const LayerGeo& L = g[l];
        const bool last = l == kLayers - 1;
        uint16_t* out = last ? nullptr : reinterpret_cast<uint16_t*>(ws + wl.act[l + 1]);
        CNN_TRY(bpst::launch_conv_fwd(a, Hs, Ws, L.cin_p, weights_bf16 + L.w_off, params + L.b_off, L.cout, L.cout_p,
                                      L.relu, nullptr, out, last ? y : nullptr, st));
        a = out;
    }
    return fail(BP_OK, nullptr);
}

BP_API int32_t bp_cnn_backward(const uint16_t* input, int32_t Ws, int32_t Hs, int32_t num_disp,
                               const uint16_t* weights_bf16, void* workspace, size_t workspace_bytes, const float* y,
                               const int16_t* label, int32_t lam_t, float* grads, float* loss, void* stream)
{
    LayerGeo g[kLayers];
    long long n = 0;
    if (!size_ok(Ws, Hs) || !geometry(num_disp, g, &n)) return fail(BP_E_INVAL, "bad size or num_disp");
    if (!input || !weights_bf16 || !y || !label || !grads || !loss || !workspace)
        return fail(BP_E_INVAL, "a pointer is NULL");
    if (lam_t < 1) return fail(BP_E_INVAL, "lam_t must be >= 1");
    if (!a16(workspace)) return fail(BP_E_INVAL, "workspace must be 16-byte aligned");
    const long long P = (long long)Ws * Hs;
    const CnnWs wl = ws_layout(P, g);
    if (workspace_bytes < wl.total) return fail(BP_E_WORKSPACE, "CNN workspace too small");
    hipStream_t st = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    const int D = num_disp;
    // slots with a neighbour: D labels each
    const long long valid = (long long)D * (2LL * (Ws - 1) * Hs + 2LL * Ws * (Hs - 1));
    const float inv_n = valid > 0 ? 1.0f / (float)valid : 0.0f;
    uint16_t* gcur = reinterpret_cast<uint16_t*>(ws + wl.gy);
    CNN_TRY(bpst::launch_l1(y, label, Hs, Ws, D, g[kLayers - 1].cout_p, (float)lam_t, inv_n, gcur,
                            reinterpret_cast<float*>(ws + wl.part_loss), loss, st));
    float* pw = reinterpret_cast<float*>(ws + wl.part_w);
    float* pb = reinterpret_cast<float*>(ws + wl.part_b);
    uint16_t* wflip = reinterpret_cast<uint16_t*>(ws + wl.wflip);
    for (int l = kLayers - 1; l >= 0; --l) {
        const LayerGeo& L = g[l];
        const uint16_t* a = l == 0 ? input : reinterpret_cast<const uint16_t*>(ws + wl.act[l]);
        CNN_TRY(bpst::launch_conv_wgrad(a, gcur, Hs, Ws, L.cin_p, L.cout_p, kChunk, pw, pb, grads + L.w_off,
                                        grads + L.b_off, st));
        if (l == 0) break;
        uint16_t* gnext = reinterpret_cast<uint16_t*>(ws + wl.gh[l & 1]);
        CNN_TRY(bpst::launch_flip(weights_bf16 + L.w_off, L.cin_p, L.cout_p, wflip, st));
        CNN_TRY(bpst::launch_conv_fwd(gcur, Hs, Ws, L.cout_p, wflip, nullptr, L.cin, L.cin_p, 0, a, gnext, nullptr,
                                      st));
        gcur = gnext;
    }
    return fail(BP_OK, nullptr);
}

BP_API int32_t bp_adam_step(float* params, float* m, float* v, const float* grads, uint16_t* weights_bf16, int64_t n,
                            int32_t step, float lr, float beta1, float beta2, float eps, void* stream)
{
    if (!params || !m || !v || !grads || !weights_bf16 || n < 1 || step < 1)
        return fail(BP_E_INVAL, "a pointer is NULL, n < 1 or step < 1");
    CNN_TRY(bpst::launch_adam(params, m, v, grads, weights_bf16, n, step, lr, beta1, beta2, eps, (hipStream_t)stream));
    return fail(BP_OK, nullptr);
}

BP_API int32_t bp_cnn_to_bf16(const float* params, int64_t n, uint16_t* weights_bf16, void* stream)
{
    if (!params || !weights_bf16 || n < 1) return fail(BP_E_INVAL, "a pointer is NULL or n < 1");
    CNN_TRY(bpst::launch_to_bf16(params, n, weights_bf16, (hipStream_t)stream));
    return fail(BP_OK, nullptr);
}

BP_API int32_t bp_warmstart_messages(const float* y, int32_t Ws, int32_t Hs, int32_t num_disp, int32_t lambda,
                                     int32_t trunc, int16_t* msgs, void* stream)
{
    LayerGeo g[kLayers];
    long long n = 0;
    if (!size_ok(Ws, Hs) || !geometry(num_disp, g, &n)) return fail(BP_E_INVAL, "bad size or num_disp");
    if (!y || !msgs) return fail(BP_E_INVAL, "y/msgs is NULL");
    if (lambda < 0 || lambda > 65535 || trunc < 0) return fail(BP_E_INVAL, "lambda/trunc out of range");
    const long long lt = (long long)lambda * std::min(trunc, num_disp);
    const int lam_t = (int)std::min(lt, 32767LL);
    CNN_TRY(bpst::launch_warm_messages(y, Ws, Hs, num_disp, g[kLayers - 1].cout_p, lam_t, msgs, (hipStream_t)stream));
    return fail(BP_OK, nullptr);
}
