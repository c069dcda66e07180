// Device-side building blocks shared by the per-launch kernels (bp_kernels.hip) and the
// batched persistent solve (batch_kernels.hip): the data layout helpers, the min-sum
// message transform and the per-pixel bodies of the pyramid, half-step and
// winner-take-all.  Every kernel maps one pixel to G consecutive lanes of a wave64; lane g
// holds labels [8g, 8g + 8) of that pixel in int32 registers, and cross-label work runs
// across the G lanes with shuffles, so every global access is a coalesced 16-byte vector.
#pragma once

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

// The same for the internal costs and messages, which are never negative: zero-extended
// (the finest scale's internal cost uses the whole u16 range).
__device__ __forceinline__ void unpack8u(const int4 v, int o[8])
{
    o[0] = v.x & 0xffff; o[1] = (int)((unsigned)v.x >> 16);
    o[2] = v.y & 0xffff; o[3] = (int)((unsigned)v.y >> 16);
    o[4] = v.z & 0xffff; o[5] = (int)((unsigned)v.z >> 16);
    o[6] = v.w & 0xffff; o[7] = (int)((unsigned)v.w >> 16);
}

__device__ __forceinline__ int4 pack8u(const unsigned o[8])
{
    return make_int4((int)((o[0] & 0xffffu) | (o[1] << 16)), (int)((o[2] & 0xffffu) | (o[3] << 16)),
                     (int)((o[4] & 0xffffu) | (o[5] << 16)), (int)((o[6] & 0xffffu) | (o[7] << 16)));
}

// Label j of a packed vector of 8 non-negative int16 values.
__device__ __forceinline__ int msg_at(const int4 v, int j)
{
    const int w = (j >> 1) == 0 ? v.x : (j >> 1) == 1 ? v.y : (j >> 1) == 2 ? v.z : v.w;
    return (j & 1) ? (int)((unsigned)w >> 16) : (w & 0xffff);
}

__device__ __forceinline__ long long slot_of(int x, int y, int Wh)
{
    return (long long)(2 * y + ((x + y) & 1)) * Wh + (x >> 1);
}

// Lane exchanges inside an aligned group of G lanes, through DPP (a VALU operand modifier,
// no LDS round trip) for groups of up to 8 lanes: quad permutations for exchanges inside a
// quad, row shifts for the scans' "lane - O" and "lane + O", and mirrors for exchanges
// between the quads of a half row.  Groups of 16 and 32 lanes use the LDS permute behind
// __shfl_*: their half-steps (D > 64) stream the largest volumes and are close to the
// vector issue rate, where the permute runs beside the vector unit (DPP there made the
// 1920x1080 D = 128 pair about 1 % slower overall).  Quad permutation codes: lane i of a
// quad reads lane sel_i, code = sel0 | sel1 << 2 | sel2 << 4 | sel3 << 6; row_shl:n = 0x100 + n, row_shr:n =
// 0x110 + n (within a 16-lane row: an 8-lane group's lanes that use the result read inside
// the group), row_half_mirror 0x141 (lane i reads 7 - i within each 8 lanes).
#define BPST_DPP(v, ctrl) __builtin_amdgcn_update_dpp((v), (v), (ctrl), 0xF, 0xF, false)

// value of lane ^ O of the group
template <int G, int O>
__device__ __forceinline__ int lanes_xor(int v)
{
    if constexpr (O == 1 && G <= 8) return BPST_DPP(v, 0xB1);             // 1,0,3,2
    else if constexpr (O == 2 && G <= 8) return BPST_DPP(v, 0x4E);        // 2,3,0,1
    else if constexpr (O == 4 && G <= 8) return BPST_DPP(BPST_DPP(v, 0x141), 0x1B);   // half mirror, quad reverse
    else return __shfl_xor(v, O, G);
}

// value of lane - O of the group (meaningful for lanes >= O)
template <int G, int O>
__device__ __forceinline__ int lanes_up(int v)
{
    if constexpr (G == 2) return BPST_DPP(v, 0xA0);                       // 0,0,2,2
    else if constexpr (G == 4 && O == 1) return BPST_DPP(v, 0x90);        // 0,0,1,2
    else if constexpr (G == 4 && O == 2) return BPST_DPP(v, 0x44);        // 0,1,0,1
    else if constexpr (G == 8) return BPST_DPP(v, 0x110 + O);             // row_shr:O
    else return __shfl_up(v, O, G);
}

// value of lane + O of the group (meaningful for lanes < G - O)
template <int G, int O>
__device__ __forceinline__ int lanes_down(int v)
{
    if constexpr (G == 2) return BPST_DPP(v, 0xF5);                       // 1,1,3,3
    else if constexpr (G == 4 && O == 1) return BPST_DPP(v, 0xF9);        // 1,2,3,3
    else if constexpr (G == 4 && O == 2) return BPST_DPP(v, 0xEE);        // 2,3,2,3
    else if constexpr (G == 8) return BPST_DPP(v, 0x100 + O);             // row_shl:O
    else return __shfl_down(v, O, G);
}
#undef BPST_DPP

template <int G, int O = 1>
__device__ __forceinline__ int group_min(int v)
{
    if constexpr (O < G) return group_min<G, 2 * O>(min(v, lanes_xor<G, O>(v)));
    else return v;
}

// Inclusive min-scan over the group, towards higher lanes: c(lane) = min over j <= lane of
// (c_j + step * (lane - j)).
template <int G, int O = 1>
__device__ __forceinline__ int scan_up(int c, int step, int lane)
{
    if constexpr (O < G) {
        const int t = lanes_up<G, O>(c);
        if (lane >= O) c = min(c, t + step * O);
        return scan_up<G, 2 * O>(c, step, lane);
    } else {
        return c;
    }
}

// The same towards lower lanes.
template <int G, int O = 1>
__device__ __forceinline__ int scan_down(int c, int step, int lane)
{
    if constexpr (O < G) {
        const int t = lanes_down<G, O>(c);
        if (lane + O < G) c = min(c, t + step * O);
        return scan_down<G, 2 * O>(c, step, lane);
    } else {
        return c;
    }
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
    if constexpr (G > 1) {
        const int c = scan_up<G>(last, 8 * lam, lane);
        cin = lanes_up<G, 1>(c);
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
    if constexpr (G > 1) {
        const int c = scan_down<G>(first, 8 * lam, lane);
        cb = lanes_down<G, 1>(c);
        if (lane == G - 1) cb = kScanId;
    }
    f[7] = min(f[7], cb + lam);
#pragma unroll
    for (int j = 6; j >= 0; --j) f[j] = min(f[j], f[j + 1] + lam);
#pragma unroll
    for (int j = 0; j < 8; ++j) out[j] = min(f[j] - hm, capv);
}

// 16-byte loads and stores of a half-step, with the nontemporal hint where the scale's
// volumes are far larger than the caches (they are streamed once per half-step, and the
// hint keeps them from evicting anything useful); plain where they stay cache-resident
// from one half-step to the next.
typedef int v4i_t __attribute__((ext_vector_type(4)));
template <bool STREAM>
__device__ __forceinline__ int4 ld16(const int16_t* p)
{
    if constexpr (STREAM) {
        const v4i_t v = __builtin_nontemporal_load(reinterpret_cast<const v4i_t*>(p));
        return make_int4(v.x, v.y, v.z, v.w);
    } else {
        return *reinterpret_cast<const int4*>(p);
    }
}
template <bool STREAM>
__device__ __forceinline__ void st16(int16_t* p, const int4 v)
{
    if constexpr (STREAM) {
        const v4i_t w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<v4i_t*>(p));
    } else {
        *reinterpret_cast<int4*>(p) = v;
    }
}

// ---- messages stored in 12 bits ----
// Where every message lies in [0, 4095] (capv <= 4095) and a pixel spans 16 or more lanes, a
// lane's 8 labels of a message are stored as 12-bit fields in 12 bytes (label j at bits
// 12 j .. 12 j + 11 of three little-endian words) instead of 16 bytes: a quarter fewer
// message bytes for the same values.  Element index e (a multiple of 8) of the 16-bit layout
// maps to byte 12 (e / 8), so every index computation stays as it is; loads unpack to the
// 16-bit register form the arithmetic uses, stores pack from it.
struct M12 {
    unsigned a, b, c;
};

__device__ __forceinline__ int4 unpack12(const M12 w)
{
    const unsigned l0 = w.a & 0xfffu, l1 = (w.a >> 12) & 0xfffu;
    const unsigned l2 = __builtin_amdgcn_alignbit(w.b, w.a, 24) & 0xfffu;
    const unsigned l3 = (w.b >> 4) & 0xfffu, l4 = (w.b >> 16) & 0xfffu;
    const unsigned l5 = __builtin_amdgcn_alignbit(w.c, w.b, 28) & 0xfffu;
    const unsigned l6 = (w.c >> 8) & 0xfffu, l7 = w.c >> 20;
    return make_int4((int)(l0 | (l1 << 16)), (int)(l2 | (l3 << 16)), (int)(l4 | (l5 << 16)), (int)(l6 | (l7 << 16)));
}

// (every label of v in [0, 4095])
__device__ __forceinline__ M12 pack12(const int4 v)
{
    const unsigned l0 = (unsigned)v.x & 0xffffu, l1 = (unsigned)v.x >> 16;
    const unsigned l2 = (unsigned)v.y & 0xffffu, l3 = (unsigned)v.y >> 16;
    const unsigned l4 = (unsigned)v.z & 0xffffu, l5 = (unsigned)v.z >> 16;
    const unsigned l6 = (unsigned)v.w & 0xffffu, l7 = (unsigned)v.w >> 16;
    M12 w;
    w.a = l0 | (l1 << 12) | (l2 << 24);
    w.b = (l2 >> 8) | (l3 << 4) | (l4 << 16) | (l5 << 28);
    w.c = (l5 >> 4) | (l6 << 8) | (l7 << 20);
    return w;
}

// A lane's 8 labels of a message volume at element index e (a multiple of 8), in either
// storage, as 8 16-bit values.
// (three words at a 4-byte-aligned address: one dwordx3 access)
typedef unsigned v3u_a4 __attribute__((ext_vector_type(3), aligned(4)));
template <bool STREAM, bool PACKED>
__device__ __forceinline__ int4 ldm(const int16_t* base, long long e)
{
    if constexpr (PACKED) {
        const v3u_a4* p = reinterpret_cast<const v3u_a4*>(reinterpret_cast<const char*>(base) + (e >> 3) * 12);
        const v3u_a4 v = STREAM ? __builtin_nontemporal_load(p) : *p;
        M12 w;
        w.a = v.x;
        w.b = v.y;
        w.c = v.z;
        return unpack12(w);
    } else {
        return ld16<STREAM>(base + e);
    }
}

template <bool STREAM, bool PACKED>
__device__ __forceinline__ void stm(int16_t* base, long long e, const int4 v)
{
    if constexpr (PACKED) {
        v3u_a4* p = reinterpret_cast<v3u_a4*>(reinterpret_cast<char*>(base) + (e >> 3) * 12);
        const M12 w = pack12(v);
        const v3u_a4 x = {w.a, w.b, w.c};
        if constexpr (STREAM)
            __builtin_nontemporal_store(x, p);
        else
            *p = x;
    } else {
        st16<STREAM>(base + e, v);
    }
}

// The 12-bit words of a lane's 8 labels as stored, label j of them, and a store of them.
template <bool STREAM>
__device__ __forceinline__ M12 ldm12(const int16_t* base, long long e)
{
    const v3u_a4* p = reinterpret_cast<const v3u_a4*>(reinterpret_cast<const char*>(base) + (e >> 3) * 12);
    const v3u_a4 v = STREAM ? __builtin_nontemporal_load(p) : *p;
    M12 w;
    w.a = v.x;
    w.b = v.y;
    w.c = v.z;
    return w;
}

__device__ __forceinline__ int lab12(const M12& w, int j)
{
    switch (j) {
    case 0: return (int)(w.a & 0xfffu);
    case 1: return (int)((w.a >> 12) & 0xfffu);
    case 2: return (int)(__builtin_amdgcn_alignbit(w.b, w.a, 24) & 0xfffu);
    case 3: return (int)((w.b >> 4) & 0xfffu);
    case 4: return (int)((w.b >> 16) & 0xfffu);
    case 5: return (int)(__builtin_amdgcn_alignbit(w.c, w.b, 28) & 0xfffu);
    case 6: return (int)((w.c >> 8) & 0xfffu);
    default: return (int)(w.c >> 20);
    }
}

template <bool STREAM>
__device__ __forceinline__ void stm12(int16_t* base, long long e, const M12 w)
{
    v3u_a4* p = reinterpret_cast<v3u_a4*>(reinterpret_cast<char*>(base) + (e >> 3) * 12);
    const v3u_a4 x = {w.a, w.b, w.c};
    if constexpr (STREAM)
        __builtin_nontemporal_store(x, p);
    else
        *p = x;
}

// Bits of the real labels (d0 + j < D) among a lane's 12-bit fields: a prefix of 12 n bits.
__device__ __forceinline__ M12 label_mask12(int d0, int D)
{
    const int n = D - d0 < 0 ? 0 : (D - d0 > 8 ? 8 : D - d0);
    auto ones = [](int bits) { return bits <= 0 ? 0u : (bits >= 32 ? 0xffffffffu : (1u << bits) - 1u); };
    M12 m;
    m.a = ones(12 * n);
    m.b = ones(12 * n - 32);
    m.c = ones(12 * n - 64);
    return m;
}

__device__ __forceinline__ bool same12(const M12& a, const M12& b, const M12& m)
{
    return (((a.a ^ b.a) & m.a) | ((a.b ^ b.b) & m.b) | ((a.c ^ b.c) & m.c)) == 0u;
}

// ---- two messages at once in packed 16-bit halves ----
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_pk(unsigned v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ unsigned pk_bits(u16x2 v) { return __builtin_bit_cast(unsigned, v); }
__device__ __forceinline__ u16x2 pk_min(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ u16x2 pk_adds(u16x2 a, u16x2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ u16x2 pk_splat(unsigned v) { return u16x2{(unsigned short)v, (unsigned short)v}; }

template <int G, int O = 1>
__device__ __forceinline__ u16x2 pk_scan_up(u16x2 c, unsigned step, int lane)
{
    if constexpr (O < G) {
        const u16x2 t = as_pk((unsigned)lanes_up<G, O>((int)pk_bits(c)));
        if (lane >= O) c = pk_min(c, pk_adds(t, pk_splat(min(step * O, 65535u))));
        return pk_scan_up<G, 2 * O>(c, step, lane);
    } else {
        return c;
    }
}

template <int G, int O = 1>
__device__ __forceinline__ u16x2 pk_scan_down(u16x2 c, unsigned step, int lane)
{
    if constexpr (O < G) {
        const u16x2 t = as_pk((unsigned)lanes_down<G, O>((int)pk_bits(c)));
        if (lane + O < G) c = pk_min(c, pk_adds(t, pk_splat(min(step * O, 65535u))));
        return pk_scan_down<G, 2 * O>(c, step, lane);
    } else {
        return c;
    }
}

// The messages a and b of one pixel (h inputs ha, hb) computed together: label j of a in
// the low half and of b in the high half of one register, so every min and add of the
// envelope passes serves both (v_pk_min_u16, v_pk_add_u16 with clamp).  The result is the
// same as transform() bit for bit: out = min(f - min h, C) with C = capv <= 32767, and the
// envelope is a min-plus convolution, so shifting h by its minimum first, clipping it at C
// and saturating every sum at 65535 (>= C) leave min(., C) unchanged; f <= C throughout.
// Outputs come in memory order (labels 2w, 2w+1 of one message per 32-bit word).
// PACKED: the results go to oa12, ob12 as 12-bit fields (outa, outb are left as they are).
template <int G, bool PACKED = false>
__device__ __forceinline__ void transform2(const int ha[8], const int hb[8], int lam, int capv, int lane, int4& outa,
                                           int4& outb, M12& oa12, M12& ob12)
{
    int ma = min(min(min(ha[0], ha[1]), min(ha[2], ha[3])), min(min(ha[4], ha[5]), min(ha[6], ha[7])));
    int mb = min(min(min(hb[0], hb[1]), min(hb[2], hb[3])), min(min(hb[4], hb[5]), min(hb[6], hb[7])));
    ma = group_min<G>(ma);
    mb = group_min<G>(mb);
    u16x2 x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        x[j] = as_pk((unsigned)min(ha[j] - ma, capv) | ((unsigned)min(hb[j] - mb, capv) << 16));
    const u16x2 L = pk_splat(min((unsigned)lam, 65535u));
    const unsigned step = 8u * (unsigned)lam;  // lam <= 65535: no overflow
    // forward
    u16x2 last = x[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) last = pk_min(x[j], pk_adds(last, L));
    u16x2 cin = pk_splat(0xffffu);  // no carry: 65535 + lam saturates and never wins
    if constexpr (G > 1) {
        const u16x2 c = pk_scan_up<G>(last, step, lane);
        cin = as_pk((unsigned)lanes_up<G, 1>((int)pk_bits(c)));
        if (lane == 0) cin = pk_splat(0xffffu);
    }
    u16x2 f[8];
    f[0] = pk_min(x[0], pk_adds(cin, L));
#pragma unroll
    for (int j = 1; j < 8; ++j) f[j] = pk_min(x[j], pk_adds(f[j - 1], L));
    // backward
    u16x2 first = f[7];
#pragma unroll
    for (int j = 6; j >= 0; --j) first = pk_min(f[j], pk_adds(first, L));
    u16x2 cb = pk_splat(0xffffu);
    if constexpr (G > 1) {
        const u16x2 c = pk_scan_down<G>(first, step, lane);
        cb = as_pk((unsigned)lanes_down<G, 1>((int)pk_bits(c)));
        if (lane == G - 1) cb = pk_splat(0xffffu);
    }
    f[7] = pk_min(f[7], pk_adds(cb, L));
#pragma unroll
    for (int j = 6; j >= 0; --j) f[j] = pk_min(f[j], pk_adds(f[j + 1], L));
    if constexpr (PACKED) {
        // straight into the 12-bit fields of each message (every value <= capv <= 4095): a
        // from the low halves, b from the high halves
        unsigned fa[8], fb[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            fa[j] = pk_bits(f[j]) & 0xffffu;
            fb[j] = pk_bits(f[j]) >> 16;
        }
        oa12.a = fa[0] | (fa[1] << 12) | (fa[2] << 24);
        oa12.b = (fa[2] >> 8) | (fa[3] << 4) | (fa[4] << 16) | (fa[5] << 28);
        oa12.c = (fa[5] >> 4) | (fa[6] << 8) | (fa[7] << 20);
        ob12.a = fb[0] | (fb[1] << 12) | (fb[2] << 24);
        ob12.b = (fb[2] >> 8) | (fb[3] << 4) | (fb[4] << 16) | (fb[5] << 28);
        ob12.c = (fb[5] >> 4) | (fb[6] << 8) | (fb[7] << 20);
    } else {
        // regroup: low halves of labels 2w, 2w+1 -> word w of a; high halves -> word w of b
        unsigned wa[4], wb[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            wa[w] = __builtin_amdgcn_perm(pk_bits(f[2 * w + 1]), pk_bits(f[2 * w]), 0x05040100u);
            wb[w] = __builtin_amdgcn_perm(pk_bits(f[2 * w + 1]), pk_bits(f[2 * w]), 0x07060302u);
        }
        outa = make_int4((int)wa[0], (int)wa[1], (int)wa[2], (int)wa[3]);
        outb = make_int4((int)wb[0], (int)wb[1], (int)wb[2], (int)wb[3]);
    }
}

template <int G>
__device__ __forceinline__ void transform2(const int ha[8], const int hb[8], int lam, int capv, int lane, int4& outa,
                                           int4& outb)
{
    M12 unused_a, unused_b;
    transform2<G, false>(ha, hb, lam, capv, lane, outa, outb, unused_a, unused_b);
}

// ---- the narrow path: whole message sums in packed 16-bit ----
//
// Every scale's internal cost is min-normalised per pixel (min over d = 0): the finest
// scale holds cost - min_d cost as u16 (0..65535), coarser scales the pyramid's values
// (0..32767).  Incoming messages are transform outputs in [0, C], C = capv.  Then the sums
// h_k = cost + (the three other incoming messages) can be formed with saturating 16-bit
// adds when C <= 16383, and every message is still exact: the minimum of h_k is at most
// 3C (take the label where the cost is 0), far below 65535, so it is never a saturated
// value; a label whose sum saturated has h - min h >= 65535 - 3C >= C, so it clips to C
// exactly as its true value would.  The message is then the envelope of
// x = min(h - min h, C), as in transform2.
//
// Lane mapping: a pixel keeps its G lanes.  With G = 1 the one lane computes both packed
// pairs (messages 0 and 1, messages 2 and 3) over its 8 labels.  With G >= 2 the pixel's
// lanes are split between the pairs: lanes [0, G/2) compute messages 0 and 1 and lanes
// [G/2, G) messages 2 and 3, each lane over 16 consecutive labels (two 16-byte vectors),
// label group g = lane % (G/2).  Each lane thus runs one envelope chain per pass over its
// labels, and a pixel of D <= 16 needs no lane exchange at all.

// Vectors per lane, pair and first label of a lane on the narrow path.
template <int G>
struct NarrowLane {
    static constexpr int NV = G == 1 ? 1 : 2;  // 16-byte vectors of labels per lane
    static constexpr int GL = G == 1 ? 1 : G / 2;  // lanes of one pair
    int q;   // the lane's pair (G >= 2): messages 2q, 2q + 1
    int g;   // label group inside the pair
    int d0;  // first label
    __device__ __forceinline__ explicit NarrowLane(int lane)
    {
        q = G == 1 ? 0 : lane / GL;
        g = G == 1 ? 0 : lane % GL;
        d0 = G == 1 ? 0 : 16 * g;
    }
};

// Minimum of n packed values as a tree (independent mins issue back to back; a linear
// chain of dependent packed ops costs a wait state each).
template <int N>
__device__ __forceinline__ u16x2 pk_min_tree(const u16x2* v)
{
    if constexpr (N == 1) return v[0];
    else return pk_min(pk_min_tree<N / 2>(v), pk_min_tree<N - N / 2>(v + N / 2));
}

__device__ __forceinline__ unsigned word_of(const int4 v, int u)
{
    return (unsigned)(u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w);
}

// Messages a and b (one packed pair) of one pixel over a lane's NV vectors of labels,
// GL lanes per pair: h_a = cost + m1 + m2 + mb, h_b = cost + m1 + m2 + ma, where ma, mb are
// the pair's own incoming messages and m1, m2 the other pair's.  Outputs in memory order.
template <int GL, int NV>
__device__ __forceinline__ void narrow_pair(const int4 (&c)[NV], const int4 (&ma)[NV], const int4 (&mb)[NV],
                                            const int4 (&m1)[NV], const int4 (&m2)[NV], int D, int d0, bool pad,
                                            unsigned lam, unsigned capv, int g, int4 (&outa)[NV], int4 (&outb)[NV])
{
    constexpr int NJ = 8 * NV;
    u16x2 x[NJ];  // label j of a in the low half, of b in the high half
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const u16x2 o = pk_adds(as_pk(word_of(c[v], u)), pk_adds(as_pk(word_of(m1[v], u)), as_pk(word_of(m2[v], u))));
            const unsigned ha = pk_bits(pk_adds(o, as_pk(word_of(mb[v], u))));
            const unsigned hb = pk_bits(pk_adds(o, as_pk(word_of(ma[v], u))));
            x[8 * v + 2 * u] = as_pk(__builtin_amdgcn_perm(hb, ha, 0x05040100u));
            x[8 * v + 2 * u + 1] = as_pk(__builtin_amdgcn_perm(hb, ha, 0x07060302u));
        }
    }
    if (pad) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) x[j] = as_pk(pk_bits(x[j]) | (d0 + j < D ? 0u : 0xffffffffu));
    }
    u16x2 mn = pk_min_tree<NJ>(x);
    if constexpr (GL > 1) {
        mn = pk_min(mn, as_pk((unsigned)lanes_xor<GL, 1>((int)pk_bits(mn))));
        if constexpr (GL > 2) mn = pk_min(mn, as_pk((unsigned)lanes_xor<GL, 2>((int)pk_bits(mn))));
        if constexpr (GL > 4) mn = pk_min(mn, as_pk((unsigned)lanes_xor<GL, 4>((int)pk_bits(mn))));
        if constexpr (GL > 8) mn = pk_min(mn, as_pk((unsigned)lanes_xor<GL, 8>((int)pk_bits(mn))));
    }
    const u16x2 C = pk_splat(capv), L = pk_splat(min(lam, 65535u));
#pragma unroll
    for (int j = 0; j < NJ; ++j) x[j] = pk_min(x[j] - mn, C);  // x >= mn: no wrap
    // forward pass, with the carry from the pair's lanes before this one
    if constexpr (GL > 1) {
        u16x2 last = x[0];
#pragma unroll
        for (int j = 1; j < NJ; ++j) last = pk_min(x[j], pk_adds(last, L));
        const u16x2 cs = pk_scan_up<GL>(last, (unsigned)NJ * lam, g);
        u16x2 cin = as_pk((unsigned)lanes_up<GL, 1>((int)pk_bits(cs)));
        if (g == 0) cin = pk_splat(0xffffu);  // no carry: 65535 + lam saturates and never wins
        x[0] = pk_min(x[0], pk_adds(cin, L));
    }
#pragma unroll
    for (int j = 1; j < NJ; ++j) x[j] = pk_min(x[j], pk_adds(x[j - 1], L));
    // backward pass
    if constexpr (GL > 1) {
        u16x2 first = x[NJ - 1];
#pragma unroll
        for (int j = NJ - 2; j >= 0; --j) first = pk_min(x[j], pk_adds(first, L));
        const u16x2 cs = pk_scan_down<GL>(first, (unsigned)NJ * lam, g);
        u16x2 cb = as_pk((unsigned)lanes_down<GL, 1>((int)pk_bits(cs)));
        if (g == GL - 1) cb = pk_splat(0xffffu);
        x[NJ - 1] = pk_min(x[NJ - 1], pk_adds(cb, L));
    }
#pragma unroll
    for (int j = NJ - 2; j >= 0; --j) x[j] = pk_min(x[j], pk_adds(x[j + 1], L));
    // back to memory order: word u of message a = low halves of labels 2u, 2u+1
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        unsigned wa[4], wb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 8 * v + 2 * u;
            wa[u] = __builtin_amdgcn_perm(pk_bits(x[j + 1]), pk_bits(x[j]), 0x05040100u);
            wb[u] = __builtin_amdgcn_perm(pk_bits(x[j + 1]), pk_bits(x[j]), 0x07060302u);
        }
        outa[v] = make_int4((int)wa[0], (int)wa[1], (int)wa[2], (int)wa[3]);
        outb[v] = make_int4((int)wb[0], (int)wb[1], (int)wb[2], (int)wb[3]);
    }
}

// The outgoing messages a lane computes on the narrow path.  c and m are the lane's NV
// vectors of the cost and of the incoming messages (zero where there is no neighbour), at
// labels [nl.d0, nl.d0 + 8 NV), the messages in the lane's role order: m[0], m[1] its own
// pair's (2q, 2q + 1), m[2], m[3] the other pair's.  out[e] is the message 2q + e it sends
// (with G = 1, q = 0 and all four), in memory order.
template <int G>
__device__ __forceinline__ void narrow_update(const NarrowLane<G>& nl, const int4 (&c)[NarrowLane<G>::NV],
                                              const int4 (&m)[4][NarrowLane<G>::NV], int D, bool pad, unsigned lam,
                                              unsigned capv, int4 (&out)[4][NarrowLane<G>::NV])
{
    constexpr int NV = NarrowLane<G>::NV, GL = NarrowLane<G>::GL;
    narrow_pair<GL, NV>(c, m[0], m[1], m[2], m[3], D, nl.d0, pad, lam, capv, nl.g, out[0], out[1]);
    if constexpr (G == 1) narrow_pair<1, NV>(c, m[2], m[3], m[0], m[1], D, nl.d0, pad, lam, capv, 0, out[2], out[3]);
}

// Message volume of role r for a lane that computes messages 2 and 3 (hi) or 0 and 1: its
// own pair first, then the other pair.
__device__ __forceinline__ int role_msg(bool hi, int r) { return hi ? (r + 2) & 3 : r; }

// Mask of the real labels (d < D) of this lane's four packed words.
__device__ __forceinline__ int4 label_mask(int d0, int D)
{
    unsigned w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        w[i] = (d0 + 2 * i < D ? 0xffffu : 0u) | (d0 + 2 * i + 1 < D ? 0xffff0000u : 0u);
    return make_int4((int)w[0], (int)w[1], (int)w[2], (int)w[3]);
}

// Packed words a and b agree on the real labels.
__device__ __forceinline__ bool same_labels(const int4 a, const int4 b, const int4 m)
{
    return (((a.x ^ b.x) & m.x) | ((a.y ^ b.y) & m.y) | ((a.z ^ b.z) & m.z) | ((a.w ^ b.w) & m.w)) == 0;
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

// Start a scale for the pixel with slot gi: copy its parent's messages (zero for a missing
// neighbour, on either scale, or when parent is null: the coarsest scale) and reset the
// skip state.
template <int G, bool PACKED = false>
__device__ __forceinline__ void init_pixel(const int16_t* __restrict__ parent, Level lp, long long pvol,
                                           int16_t* __restrict__ msgs, Level lv, long long vol, uint8_t* sa,
                                           uint8_t* sb, int mode, long long gi, int lane)
{
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
        if (parent && has[k] && phas[k]) v = ldm<false, PACKED>(parent, k * pvol + ps * (8 * G) + d0);
        stm<false, PACKED>(msgs, k * vol + gi * (8 * G) + d0, v);
    }
    if (lane == 0) {
        if (mode == 1) { sa[gi] = 1; sb[gi] = 0; }
        if (mode == 2) sa[gi] = 1;
    }
}

// The finest scale's internal cost of one pixel (lane's 8 labels of the caller's values v):
// cost - min_d cost over the real labels, as u16 (always 0..65535); padded labels hold 0.
// Messages and the winner are unchanged by a per-pixel shift of the cost, and with every
// scale min-normalised the narrow path's packed sums stay exact.
template <int G>
__device__ __forceinline__ int4 finest_internal(const int v[8], int d0, int D)
{
    int mn = kBig;
#pragma unroll
    for (int j = 0; j < 8; ++j) if (d0 + j < D) mn = min(mn, v[j]);
    mn = group_min<G>(mn);
    unsigned o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = d0 + j < D ? (unsigned)(v[j] - mn) : 0u;
    return pack8u(o);
}

// What a half-step body reports about its pixel, for the counters.
struct PixOut {
    bool act;     // the pixel was updated
    bool has[4];  // it has a neighbour on side k
};

// The whole cost pyramid in one launch.  A block is the set of pixels under one pixel
// (X, Y) of the coarsest scale: its lanes re-lay the block's finest costs into the internal
// layout and build every coarser scale of the block, handing each scale to the next in
// LDS.  Scale sizes halve with ceil, so the block's pixels at scale l are exactly
// [X s_l, (X+1) s_l) x [Y s_l, (Y+1) s_l) clipped to the scale, s_l = 2^(L-1-l).  A
// workgroup takes coarsest pixels c0, c0 + 1, ... (row-major), tree_blocks() of them, each
// with its own lanes and LDS slice; all blocks meet the same barriers.  A coarsest index
// past the last pixel has Y >= the coarsest height, so every pixel of its block is out of
// range on every scale and it only takes part in the barriers.
// Element of label j (0..7) of lane `lane` of block pixel p in the tree's LDS scale buffers.
// A lane's 8 labels are two 16-byte chunks, and chunk k of a pixel's G lanes lie side by
// side, so the lanes of a wave touch consecutive 16-byte chunks (no bank conflicts).
template <int G>
__device__ __forceinline__ int tree_at(int p, int lane, int j)
{
    return p * 8 * G + (j >> 2) * 4 * G + lane * 4 + (j & 3);
}

template <int G, bool VEC>
__device__ __forceinline__ void pyramid_tree_block(const int16_t* __restrict__ user, int16_t* const* cs,
                                                   const Level* lvs, int L, int D, int c0, int* lds,
                                                   bool write_finest = true)
{
    constexpr int Dp = 8 * G;
    const int s1 = 1 << (L - 2), s2 = s1 / 2;
    const int p1 = s1 * s1 * G;
    const int nt = p1 < (int)blockDim.x ? p1 : (int)blockDim.x;  // lanes per block
    const int sub = (int)threadIdx.x / nt, tid = (int)threadIdx.x % nt;
    const int Wc = lvs[L - 1].W;
    const int X = (c0 + sub) % Wc, Y = (c0 + sub) / Wc;
    int* cur = lds + sub * (s1 * s1 + s2 * s2) * Dp;  // scale l-1 of the block, [s_{l-1}^2][Dp]
    int* nxt = cur + s1 * s1 * Dp;                    // scale l
    // scale 1 from the caller's finest costs; also writes the internal finest layout, unless
    // the solve reads the caller's volume at the finest scale itself (write_finest false)
    {
        const Level l0 = lvs[0], l1 = lvs[1];
        const int tasks = s1 * s1 * G;
        for (int task = tid; task < tasks; task += nt) {
            const int p = task / G, lane = task & (G - 1), d0 = lane * 8;
            const int px = X * s1 + (p % s1), py = Y * s1 + (p / s1);
            const bool valid = px < l1.W && py < l1.H;
            int s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (valid) {
                // the four children's costs are all loaded (from the pixel itself where a child
                // lies past the image) before any is used or stored: one memory latency, not four
                int v[4][8];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int x = 2 * px + (k & 1), y = 2 * py + (k >> 1);
                    const bool in = x < l0.W && y < l0.H;
                    const int16_t* src = user + ((long long)(in ? y : 2 * py) * l0.W + (in ? x : 2 * px)) * D;
                    if (VEC) {
                        // a lane past the labels reads label 0's vector and drops it
                        unpack8(*reinterpret_cast<const int4*>(src + (d0 < D ? d0 : 0)), v[k]);
                        const int keep = d0 < D ? -1 : 0;
#pragma unroll
                        for (int j = 0; j < 8; ++j) v[k][j] &= keep;
                    } else {
                        src += d0;
#pragma unroll
                        for (int j = 0; j < 8; ++j) v[k][j] = (d0 + j < D) ? (int)src[j] : 0;
                    }
                }
                // then every result, then every store (arithmetic after a store waits for it)
                int4 fin[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int x = 2 * px + (k & 1), y = 2 * py + (k >> 1);
                    const int keep = x < l0.W && y < l0.H ? -1 : 0;
                    if (write_finest) fin[k] = finest_internal<G>(v[k], d0, D);
#pragma unroll
                    for (int j = 0; j < 8; ++j) s[j] += v[k][j] & keep;
                }
                if (write_finest) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int x = 2 * px + (k & 1), y = 2 * py + (k >> 1);
                        if (x < l0.W && y < l0.H)
                            *reinterpret_cast<int4*>(cs[0] + slot_of(x, y, l0.Wh) * Dp + d0) = fin[k];
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
            if (valid) {
                *reinterpret_cast<int4*>(cs[1] + slot_of(px, py, l1.Wh) * Dp + d0) = pack8(o);
#pragma unroll
                for (int j = 0; j < 8; ++j) cur[tree_at<G>(p, lane, j)] = o[j];
            }
        }
    }
    __syncthreads();
    for (int l = 2; l < L; ++l) {
        const Level lf = lvs[l - 1], lc = lvs[l];
        const int sl = 1 << (L - 1 - l), sf = 2 * sl;
        const int tasks = sl * sl * G;
        for (int task = tid; task < tasks; task += nt) {
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
                        const int child = (2 * qy + b) * sf + (2 * qx + c);
#pragma unroll
                        for (int j = 0; j < 8; ++j) s[j] += cur[tree_at<G>(child, lane, j)];
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
                *reinterpret_cast<int4*>(cs[l] + slot_of(px, py, lc.Wh) * Dp + d0) = pack8(o);
#pragma unroll
                for (int j = 0; j < 8; ++j) nxt[tree_at<G>(p, lane, j)] = o[j];
            }
        }
        __syncthreads();
        int* t = cur;
        cur = nxt;
        nxt = t;
    }
}

// Start a scale: copy each pixel's parent messages (zero for a missing neighbour or for

// new message to each of its neighbours.  Reads only slots of its own colour, writes only
// slots of the other colour, so the in-place update is race-free.
//   SRC == kSrcParent: first half-step of a scale; the incoming messages are read from the
//     parent's slots (the scale's own slots of this colour are never materialised);
//   SRC == kSrcZero: first half-step of the coarsest scale; incoming messages are zero.
// Skip mode 1 resets a pixel's state at its first update of the scale (t < 2).
// Handles pixel gi of the scale's colour-a.colour pixels with lane `lane` of its G lanes;
// returns whether it was updated and which neighbours it has (for the counters).
// STREAM: the scale's volumes are streamed (nontemporal loads and stores, see ld16).
// listed: the caller has already read the pixel's freeze state and passes only active
// pixels (or gi past the end), so the state is not read again.
// USER: the cost is the caller's finest volume [H][W][Dp] (signed values, D == Dp), read at
// (y W + x): messages and winners do not change under the per-pixel shift the internal finest
// layout applies, and the sums stay in int32.
// FULL_D: D == Dp, every label of every lane is a real one, so no label is masked (implied by
// USER).
template <int G, int MODE, int SRC, bool NARROW = false, bool STREAM = false, bool PACKED = false, bool USER = false,
          bool FULL_D = false>
__device__ __forceinline__ PixOut halfstep_pixel(const HalfstepArgs& a, int gi, int lane, bool listed = false)
{
    static_assert(!USER || (PACKED && !NARROW), "the caller's cost is read on the 12-bit path only");
    constexpr bool FULL = USER || FULL_D;
    constexpr int Dp = 8 * G;
    constexpr int NV = NARROW ? NarrowLane<G>::NV : 1;  // label vectors a lane reads per volume
    constexpr int GL = NARROW ? NarrowLane<G>::GL : G;  // lanes that share one message
    constexpr int NK = NARROW && G > 1 ? 2 : 4;         // messages a lane sends
    const NarrowLane<G> nl(lane);
    const int d0 = NARROW ? nl.d0 : lane * 8;
    const int glane = NARROW ? nl.g : lane;
    // incoming volumes in the lane's role order (identity unless the lane computes the
    // second pair on the narrow path)
    const bool hi = NARROW && G > 1 && nl.q != 0;
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
    if (!listed && (MODE == 2 || (MODE == 1 && a.t >= 2))) act = act && a.state_a[slot] != 0;
    bool hr[4];
    long long nbr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        hr[r] = hi ? has[(r + 2) & 3] : has[r];
        nbr[r] = hi ? nb[(r + 2) & 3] : nb[r];
    }
    const bool check = (MODE == 2) || (MODE == 1 && a.t >= 2);
    // The messages this lane sends: all four, or with the pairs split the two of its pair
    // (k = 2q + e).  The outgoing values this update may overwrite, and the pixel's count of
    // unchanged half-steps, are loaded first, before the incoming messages (nothing else
    // writes them during the half-step): placed after, the compiler would issue them only
    // once the incoming sums were formed, a second memory latency in the pixel's path.
    int sb = MODE == 1 && a.t >= 2 ? (int)a.state_b[act ? slot : 0] : 0;
    int4 op[NK][NV];
    M12 op12[NK];  // PACKED: the previous outgoing messages as stored (compared packed)
#pragma unroll
    for (int e = 0; e < NK; ++e) {
        op12[e] = M12{0u, 0u, 0u};
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            op[e][v] = make_int4(0, 0, 0, 0);
            if (check && act && hr[e]) {
                const long long eo = (role_msg(hi, e) ^ 1) * a.vol + nbr[e] * Dp + d0 + 8 * v;
                if constexpr (PACKED)
                    op12[e] = ldm12<STREAM>(a.msgs, eo);
                else
                    op[e][v] = ld16<STREAM>(a.msgs + eo);
            }
        }
    }
    // incoming messages stay packed (two int16 per register, values in [0, 32767])
    int4 c4[NV], mp[4][NV];
    M12 mp12[4];  // PACKED: the incoming messages as stored (labels taken straight from the fields)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        c4[v] = make_int4(0, 0, 0, 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) mp[k][v] = make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) mp12[k] = M12{0u, 0u, 0u};
    if (act) {
        const long long cslot = USER ? (long long)y * W + x : slot;
#pragma unroll
        for (int v = 0; v < NV; ++v) c4[v] = ld16<STREAM>(a.cost + cslot * Dp + d0 + 8 * v);
        if (SRC == kSrcOwn) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (hr[r])
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const long long em = role_msg(hi, r) * a.vol + slot * Dp + d0 + 8 * v;
                        if constexpr (PACKED)
                            mp12[r] = ldm12<STREAM>(a.msgs, em);
                        else
                            mp[r][v] = ld16<STREAM>(a.msgs + em);
                    }
        } else if (SRC == kSrcParent) {
            const int px = x >> 1, py = y >> 1;
            const bool phas[4] = {px > 0, px < a.plv.W - 1, py > 0, py < a.plv.H - 1};
            const long long ps = (long long)(2 * py + ((px + py) & 1)) * a.plv.Wh + (px >> 1);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (hr[r] && (hi ? phas[(r + 2) & 3] : phas[r]))
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const long long em = role_msg(hi, r) * a.pvol + ps * Dp + d0 + 8 * v;
                        if constexpr (PACKED)
                            mp12[r] = ldm12<STREAM>(a.pmsgs, em);
                        else
                            mp[r][v] = ld16<STREAM>(a.pmsgs + em);
                    }
        }
    }
    // label j of incoming message k, in either storage
    auto inc = [&](int k, int j) { return PACKED ? lab12(mp12[k], j) : msg_at(mp[k][0], j); };
    int4 out[4][NV];
    M12 out12[4];  // PACKED: the new outgoing messages as they are stored
    if constexpr (NARROW) {
        narrow_update<G>(nl, c4, mp, a.D, a.D < Dp, (unsigned)a.lambda, (unsigned)a.capv, out);
    } else {
        int Hs[8];
        if constexpr (USER)
            unpack8(c4[0], Hs);
        else
            unpack8u(c4[0], Hs);
#pragma unroll
        for (int j = 0; j < 8; ++j)
            Hs[j] = (FULL || d0 + j < a.D) ? Hs[j] + inc(0, j) + inc(1, j) + inc(2, j) + inc(3, j) : kBig;
#pragma unroll
        for (int k = 0; k < 4; k += 2) {
            int ha[8], hb[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                ha[j] = Hs[j] - inc(k, j);
                hb[j] = Hs[j] - inc(k + 1, j);
            }
            transform2<G, PACKED>(ha, hb, a.lambda, a.capv, lane, out[k][0], out[k + 1][0], out12[k], out12[k + 1]);
        }
        if (a.disp) {
            // the winner from the same sums: after plain BP's last half-step at the finest
            // scale the updated pixels' incoming messages are final (their neighbours, the
            // other colour, are not updated again), so Hs is their belief (as in wta_pixel)
            int key = 0x7fffffff;
#pragma unroll
            for (int j = 0; j < 8; ++j) if (FULL || d0 + j < a.D) key = min(key, Hs[j] * 256 + d0 + j);
            key = group_min<G>(key);
            if (act && lane == 0) a.disp[(long long)y * W + x] = (int16_t)(key & 255);
        }
    }
    // Every decision first, then every store: arithmetic placed after a store made the
    // compiler wait for the store to complete before it reused the store's registers.
    bool all_eq = true;
    bool stf[NK];
#pragma unroll
    for (int e = 0; e < NK; ++e) {
        bool store = act && hr[e];
        if (check) {
            bool same = true;
            if constexpr (PACKED) {
                same = same12(op12[e], out12[e], FULL ? M12{~0u, ~0u, ~0u} : label_mask12(d0, a.D));
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    same = same && same_labels(op[e][v], out[e][v], label_mask(d0 + 8 * v, a.D));
            }
            const int eq = group_min<GL>(same ? 1 : 0);  // the GL lanes of the message
            if (store && !eq) all_eq = false;
            if (eq) store = false;
        }
        stf[e] = store;
    }
    // the freeze state needs all four messages: combine the pixel's lanes
    if (NARROW && G > 1 && MODE == 1 && check) all_eq = group_min<G>(all_eq ? 1 : 0) != 0;
    int snew = 0;  // the pixel's new count of unchanged half-steps (freeze rule, t >= 2)
    if (MODE == 1 && a.t >= 2) {
        // (the empty asm keeps the compiler from forming sb + 1 right at the load, which
        // would wait for it before the other loads are issued)
        asm volatile("" : "+v"(sb));
        snew = all_eq ? sb + 1 : 0;
    }
#pragma unroll
    for (int e = 0; e < NK; ++e)
        if (stf[e]) {
            int16_t* dst = a.out ? a.out : a.msgs;
            const long long e0 = (role_msg(hi, e) ^ 1) * a.vol + nbr[e] * Dp + d0;
            if constexpr (PACKED) {
                stm12<STREAM>(dst, e0, out12[e]);
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) st16<STREAM>(dst + e0 + 8 * v, out[e][v]);
            }
            if (MODE == 2 && glane == 0) a.state_a[nbr[e]] = 1;
        }
    if (MODE == 2 && act && lane == 0) a.state_a[slot] = 0;  // own colour: no neighbour marks it now
    if (MODE == 1 && act && lane == 0) {
        if (a.t < 2) {
            a.state_a[slot] = 1;
            a.state_b[slot] = 0;
        } else {
            a.state_b[slot] = (uint8_t)snew;
            if (2 * snew >= a.K) a.state_a[slot] = 0;
        }
    }
    PixOut r;
    r.act = act;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.has[k] = has[k];
    return r;
}

// Winner-take-all of the pixel with slot gi (both colours), lane `lane` of its G lanes.
// USER: c0 is the caller's finest volume [H][W][8 G] (signed values), read at (y W + x).
template <int G, bool PACKED = false, bool USER = false>
__device__ __forceinline__ void wta_pixel(const int16_t* __restrict__ c0, const int16_t* __restrict__ msgs,
                                          long long vol, Level lv, int D, int16_t* __restrict__ disp, long long gi,
                                          int lane)
{
    constexpr int Dp = 8 * G;
    const bool in = gi < lv.slots();
    ColourPix p = any_pixel(in ? gi : 0, lv);
    const bool valid = in && p.valid;
    const int d0 = lane * 8;
    const bool has[4] = {p.x > 0, p.x < lv.W - 1, p.y > 0, p.y < lv.H - 1};
    // all five vectors are loaded before any is used, from the pixel's own slot (slot 0 for
    // a lane without a pixel), and masked after: a load under a branch that also sums would
    // be waited for inside the branch, one memory latency per volume
    const long long s = valid ? gi : 0;
    const long long cs = USER ? (valid ? (long long)p.y * lv.W + p.x : 0) : s;
    const int4 cv = *reinterpret_cast<const int4*>(c0 + cs * Dp + d0);
    int4 mv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) mv[k] = ldm<false, PACKED>(msgs, k * vol + s * Dp + d0);
    int b[8];
    if constexpr (USER)
        unpack8(cv, b);
    else
        unpack8u(cv, b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int keep = valid && has[k] ? -1 : 0;  // a side with no neighbour holds no message
        int v[8];
        unpack8u(make_int4(mv[k].x & keep, mv[k].y & keep, mv[k].z & keep, mv[k].w & keep), v);
#pragma unroll
        for (int j = 0; j < 8; ++j) b[j] += v[j];
    }
    // key = belief * 256 + d: the minimum key is the smallest d among the minimal beliefs
    int key = 0x7fffffff;
#pragma unroll
    for (int j = 0; j < 8; ++j) if (d0 + j < D) key = min(key, b[j] * 256 + d0 + j);
    key = group_min<G>(key);
    if (valid && lane == 0) disp[(long long)p.y * lv.W + p.x] = (int16_t)(key & 255);
}


}  // namespace
}  // namespace bpst
