/*
 * ORACLE — test infrastructure only (see bp_oracle.h).
 *
 * Every function follows a definition or the method's steps in the paper's order:
 *   - energy E(d) = E_D(d) + E_S(d)                    (paper, "Approach Description")
 *   - correlation volume by normalised cross-correlation (paper, Abstract and
 *     "Correlation volume computation")
 *   - message of a pixel recomputed from its own data term, its neighbours'
 *     previous messages and the jump cost                (paper, "Fast Converging BP")
 *   - only pixels that have not converged are updated    (paper, "Fast Converging BP")
 *   - hierarchy of scales, same process on each scale    (paper, "GPU Implementation")
 * Where the paper is silent the readings are: zero-mean NCC with clamp-to-edge
 * windows; cost = round-half-up(scale*(1-ncc)) clamped to [0, trunc], trunc for
 * x-d < 0; jump cost lambda*min(|d-d'|, T); coarse cost = children sum minus its
 * minimum, saturated to int16; checkerboard schedule (half-step t updates pixels of
 * colour (x+y)&1 == t&1, in place); children start from their parent's messages;
 * winner-take-all with the smallest d on ties.
 *
 * Plain loops, int64 for integers, IEEE double for the correlation value.  The
 * message is the O(D^2) minimum over all source labels (its definition).
 *
 * Loops over image rows may run on several host threads (OpenMP).  That never changes a
 * result: every output element of the correlation volume, the pyramid and the winner-
 * take-all is computed on its own, and within one checkerboard half-step the pixels of
 * the updated colour read only slots that the other colour wrote (each slot has one
 * writer), so the order in which they are visited does not matter (the schedule reading
 * above: colour (x+y)&1 == t&1 updates in place).  Integer counters are summed exactly.
 */
#include "bp_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ---- O1: luma (integer BT.601 weights 77/150/29 out of 256, round half up) ---- */
void oracle_luma(const uint8_t* rgb, int32_t width, int32_t height, uint8_t* luma)
{
    for (int64_t i = 0; i < (int64_t)width * height; ++i) {
        int r = rgb[3 * i], g = rgb[3 * i + 1], b = rgb[3 * i + 2];
        luma[i] = (uint8_t)((77 * r + 150 * g + 29 * b + 128) >> 8);
    }
}

/* ---- O2: normalised cross-correlation, by its definition with window means ---- */
double oracle_ncc_at(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t win,
                     int32_t x, int32_t y, int32_t d)
{
    if (x - d < 0) return -2.0; /* no right pixel: sentinel */
    const int r = win / 2, n = win * win;
    double mi = 0.0, mj = 0.0;
    for (int j = -r; j <= r; ++j) {
        int yy = clampi(y + j, 0, H - 1);
        for (int i = -r; i <= r; ++i) {
            mi += L[(size_t)yy * W + clampi(x + i, 0, W - 1)];
            mj += R[(size_t)yy * W + clampi(x - d + i, 0, W - 1)];
        }
    }
    mi /= n;
    mj /= n;
    double sij = 0.0, sii = 0.0, sjj = 0.0;
    for (int j = -r; j <= r; ++j) {
        int yy = clampi(y + j, 0, H - 1);
        for (int i = -r; i <= r; ++i) {
            double a = L[(size_t)yy * W + clampi(x + i, 0, W - 1)] - mi;
            double b = R[(size_t)yy * W + clampi(x - d + i, 0, W - 1)] - mj;
            sij += a * b;
            sii += a * a;
            sjj += b * b;
        }
    }
    if (sii == 0.0 || sjj == 0.0) return 0.0; /* flat window: correlation defined as 0 */
    return sij / sqrt(sii * sjj);
}

/*
 * Is B <= A * sqrt(P) exactly (P > 0)?  Used to decide the rounding of the cost
 * exactly when the double value sits next to a rounding boundary.
 */
static int le_times_sqrt(int64_t B, int64_t A, uint64_t P)
{
    typedef unsigned __int128 u128;
    u128 b2 = (u128)(B < 0 ? -B : B) * (u128)(B < 0 ? -B : B);
    u128 a2p = (u128)(uint64_t)(A < 0 ? -A : A) * (u128)(uint64_t)(A < 0 ? -A : A) * (u128)P;
    if (A >= 0) return B <= 0 ? 1 : (b2 <= a2p);
    return B >= 0 ? 0 : (b2 >= a2p);
}

/*
 * Quantised data cost: round-half-up of the real value scale*(1 - ncc), clamped to
 * [0, trunc]; trunc where x-d < 0.  The real value is never rounded through floating
 * point: with n*S_IJ - S_I*S_J = num and P = (n*S_II - S_I^2)(n*S_JJ - S_J^2), the
 * statement k <= scale*(1 - num/sqrt(P)) + 1/2 is 2*scale*num <= (2*scale - 2k + 1)*sqrt(P),
 * decided in 128-bit integers.
 */
int16_t oracle_cost_at(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t win,
                       int32_t x, int32_t y, int32_t d, int32_t scale, int32_t trunc)
{
    if (x - d < 0) return (int16_t)trunc;
    const int r = win / 2;
    const int64_t n = (int64_t)win * win;
    int64_t si = 0, sj = 0, sii = 0, sjj = 0, sij = 0;
    for (int j = -r; j <= r; ++j) {
        int yy = clampi(y + j, 0, H - 1);
        for (int i = -r; i <= r; ++i) {
            int64_t a = L[(size_t)yy * W + clampi(x + i, 0, W - 1)];
            int64_t b = R[(size_t)yy * W + clampi(x - d + i, 0, W - 1)];
            si += a; sj += b; sii += a * a; sjj += b * b; sij += a * b;
        }
    }
    int64_t num = n * sij - si * sj, vi = n * sii - si * si, vj = n * sjj - sj * sj;
    int64_t k;
    if (vi == 0 || vj == 0) {
        k = scale; /* ncc = 0 */
    } else {
        uint64_t P = (uint64_t)vi * (uint64_t)vj;
        double ncc = oracle_ncc_at(L, R, W, H, win, x, y, d);
        k = (int64_t)floor((double)scale * (1.0 - ncc) + 0.5);
        int64_t B = 2 * (int64_t)scale * num;
        while (!le_times_sqrt(B, 2 * (int64_t)scale - 2 * k + 1, P)) --k;
        while (le_times_sqrt(B, 2 * (int64_t)scale - 2 * (k + 1) + 1, P)) ++k;
    }
    if (k < 0) k = 0;
    if (k > trunc) k = trunc;
    return (int16_t)k;
}

void oracle_cost_volume(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t D,
                        int32_t win, int32_t scale, int32_t trunc, int16_t* cost, double* ncc)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int d = 0; d < D; ++d) {
                size_t o = ((size_t)y * W + x) * D + d;
                cost[o] = oracle_cost_at(L, R, W, H, win, x, y, d, scale, trunc);
                if (ncc) ncc[o] = oracle_ncc_at(L, R, W, H, win, x, y, d);
            }
}

/*
 * ---- O2 for colour views: the same correlation over the window's three channels ----
 * The views come from a regular RGB camera (paper, Abstract).  Reading: each channel is
 * taken about its own window mean and the three channels are pooled into one correlation,
 *   ncc = sum_c <I_c - mean I_c, J_c - mean J_c> / sqrt(sum_c |I_c - mean I_c|^2 * sum_c |J_c - mean J_c|^2),
 * 0 if either pooled variance is 0.  Images are interleaved RGB [H][W][3]; windows are
 * clamped to the image edge as for one channel.
 */
double oracle_ncc_rgb_at(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t win,
                         int32_t x, int32_t y, int32_t d)
{
    if (x - d < 0) return -2.0;
    const int r = win / 2, n = win * win;
    double sij = 0.0, sii = 0.0, sjj = 0.0;
    for (int c = 0; c < 3; ++c) {
        double mi = 0.0, mj = 0.0;
        for (int j = -r; j <= r; ++j) {
            int yy = clampi(y + j, 0, H - 1);
            for (int i = -r; i <= r; ++i) {
                mi += L[((size_t)yy * W + clampi(x + i, 0, W - 1)) * 3 + c];
                mj += R[((size_t)yy * W + clampi(x - d + i, 0, W - 1)) * 3 + c];
            }
        }
        mi /= n;
        mj /= n;
        for (int j = -r; j <= r; ++j) {
            int yy = clampi(y + j, 0, H - 1);
            for (int i = -r; i <= r; ++i) {
                double a = L[((size_t)yy * W + clampi(x + i, 0, W - 1)) * 3 + c] - mi;
                double b = R[((size_t)yy * W + clampi(x - d + i, 0, W - 1)) * 3 + c] - mj;
                sij += a * b;
                sii += a * a;
                sjj += b * b;
            }
        }
    }
    if (sii == 0.0 || sjj == 0.0) return 0.0;
    return sij / sqrt(sii * sjj);
}

/* Quantised colour data cost, decided exactly as for one channel: with
   num = sum_c (n S_IJc - S_Ic S_Jc) and P = sum_c (n S_IIc - S_Ic^2) * sum_c (n S_JJc - S_Jc^2). */
int16_t oracle_cost_rgb_at(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t win,
                           int32_t x, int32_t y, int32_t d, int32_t scale, int32_t trunc)
{
    if (x - d < 0) return (int16_t)trunc;
    const int r = win / 2;
    const int64_t n = (int64_t)win * win;
    int64_t num = 0, vi = 0, vj = 0;
    for (int c = 0; c < 3; ++c) {
        int64_t si = 0, sj = 0, sii = 0, sjj = 0, sij = 0;
        for (int j = -r; j <= r; ++j) {
            int yy = clampi(y + j, 0, H - 1);
            for (int i = -r; i <= r; ++i) {
                int64_t a = L[((size_t)yy * W + clampi(x + i, 0, W - 1)) * 3 + c];
                int64_t b = R[((size_t)yy * W + clampi(x - d + i, 0, W - 1)) * 3 + c];
                si += a; sj += b; sii += a * a; sjj += b * b; sij += a * b;
            }
        }
        num += n * sij - si * sj;
        vi += n * sii - si * si;
        vj += n * sjj - sj * sj;
    }
    int64_t k;
    if (vi == 0 || vj == 0) {
        k = scale;
    } else {
        uint64_t P = (uint64_t)vi * (uint64_t)vj;
        double ncc = oracle_ncc_rgb_at(L, R, W, H, win, x, y, d);
        k = (int64_t)floor((double)scale * (1.0 - ncc) + 0.5);
        int64_t B = 2 * (int64_t)scale * num;
        while (!le_times_sqrt(B, 2 * (int64_t)scale - 2 * k + 1, P)) --k;
        while (le_times_sqrt(B, 2 * (int64_t)scale - 2 * (k + 1) + 1, P)) ++k;
    }
    if (k < 0) k = 0;
    if (k > trunc) k = trunc;
    return (int16_t)k;
}

void oracle_cost_volume_rgb(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t D,
                            int32_t win, int32_t scale, int32_t trunc, int16_t* cost, double* ncc)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int d = 0; d < D; ++d) {
                size_t o = ((size_t)y * W + x) * D + d;
                cost[o] = oracle_cost_rgb_at(L, R, W, H, win, x, y, d, scale, trunc);
                if (ncc) ncc[o] = oracle_ncc_rgb_at(L, R, W, H, win, x, y, d);
            }
}

/* ---- O3: next coarser scale: sum the (up to 4) children, subtract the minimum, saturate ---- */
void oracle_pyramid_level(const int16_t* c, int32_t W, int32_t H, int32_t D, int16_t* out)
{
    const int W2 = (W + 1) / 2, H2 = (H + 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int Y = 0; Y < H2; ++Y) {
        int64_t* s = (int64_t*)malloc(sizeof(int64_t) * (size_t)D);
        for (int X = 0; X < W2; ++X) {
            for (int d = 0; d < D; ++d) s[d] = 0;
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    int x = 2 * X + a, y = 2 * Y + b;
                    if (x >= W || y >= H) continue;
                    for (int d = 0; d < D; ++d) s[d] += c[((size_t)y * W + x) * D + d];
                }
            int64_t mn = s[0];
            for (int d = 1; d < D; ++d) if (s[d] < mn) mn = s[d];
            for (int d = 0; d < D; ++d) {
                int64_t v = s[d] - mn;
                out[((size_t)Y * W2 + X) * D + d] = (int16_t)(v > 32767 ? 32767 : v);
            }
        }
        free(s);
    }
}

/*
 * ---- O5 (one message): min-sum message with truncated-linear jump cost ----
 * out(d) = min_{d'} [ h(d') + lambda*min(|d-d'|, T) ]  -  min_{d''} (same),
 * saturated to int16.  Direct O(D^2) definition.
 */
void oracle_message(const int32_t* h, int32_t D, int32_t lambda, int32_t T, int16_t* out)
{
    int64_t* f = (int64_t*)malloc(sizeof(int64_t) * (size_t)D);
    int64_t fmin = INT64_MAX;
    for (int d = 0; d < D; ++d) {
        int64_t best = INT64_MAX;
        for (int e = 0; e < D; ++e) {
            int64_t dist = d > e ? d - e : e - d;
            if (dist > T) dist = T;
            int64_t v = (int64_t)h[e] + (int64_t)lambda * dist;
            if (v < best) best = v;
        }
        f[d] = best;
        if (best < fmin) fmin = best;
    }
    for (int d = 0; d < D; ++d) {
        int64_t v = f[d] - fmin;
        out[d] = (int16_t)(v > 32767 ? 32767 : v);
    }
    free(f);
}

/* ---- grid helpers ---- */
enum { FROM_LEFT = 0, FROM_RIGHT = 1, FROM_UP = 2, FROM_DOWN = 3 };

/* Neighbour of (x,y) on side k (the side the slot-k message comes from); 0 if none. */
static int neighbour(int k, int x, int y, int W, int H, int* qx, int* qy)
{
    static const int dx[4] = {-1, 1, 0, 0}, dy[4] = {0, 0, -1, 1};
    *qx = x + dx[k];
    *qy = y + dy[k];
    return *qx >= 0 && *qx < W && *qy >= 0 && *qy < H;
}
static int opposite(int k) { return k ^ 1; }

typedef struct {
    int W, H, D, lambda, T;
    const int16_t* cost;  /* [H][W][D] */
    int16_t* m;           /* [4][H][W][D] */
} grid;

static int16_t* slot(const grid* g, int k, int x, int y)
{
    return g->m + (((size_t)k * g->H + y) * g->W + x) * g->D;
}

/*
 * Recompute every outgoing message of pixel (x,y) from its data term and its incoming
 * messages, writing each into the receiving neighbour's slot.  changed_out/eq flags
 * report, per direction, whether the new message differs from what the slot held.
 * Returns the number of messages sent.
 */
static int update_pixel(grid* g, int x, int y, int32_t* H, int32_t* h, int16_t* m, int* all_equal,
                        uint8_t* dirty /* nullable */)
{
    const int D = g->D;
    const int16_t* c = g->cost + ((size_t)y * g->W + x) * D;
    int qx, qy, sent = 0;
    for (int d = 0; d < D; ++d) H[d] = c[d];
    for (int k = 0; k < 4; ++k)
        if (neighbour(k, x, y, g->W, g->H, &qx, &qy)) {
            const int16_t* in = slot(g, k, x, y);
            for (int d = 0; d < D; ++d) H[d] += in[d];
        }
    *all_equal = 1;
    for (int k = 0; k < 4; ++k) {
        if (!neighbour(k, x, y, g->W, g->H, &qx, &qy)) continue;
        const int16_t* back = slot(g, k, x, y); /* what q sent to p: excluded */
        for (int d = 0; d < D; ++d) h[d] = H[d] - back[d];
        oracle_message(h, D, g->lambda, g->T, m);
        int16_t* dst = slot(g, opposite(k), qx, qy);
        int same = memcmp(dst, m, sizeof(int16_t) * (size_t)D) == 0;
        if (!same) {
            *all_equal = 0;
            if (dirty) {
                /* q may be flagged by senders in other rows, on other threads */
#pragma omp atomic write
                dirty[(size_t)qy * g->W + qx] = 1;
            }
        }
        memcpy(dst, m, sizeof(int16_t) * (size_t)D);
        ++sent;
    }
    return sent;
}

/* ---- O7: winner-take-all on the beliefs, smallest d on ties ---- */
void oracle_wta(const int16_t* cost, const int16_t* msgs, int32_t W, int32_t H, int32_t D, int16_t* disp)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t best = INT64_MAX;
            int bd = 0;
            for (int d = 0; d < D; ++d) {
                int64_t b = cost[((size_t)y * W + x) * D + d];
                int qx, qy;
                for (int k = 0; k < 4; ++k)
                    if (neighbour(k, x, y, W, H, &qx, &qy))
                        b += msgs[(((size_t)k * H + y) * W + x) * D + d];
                if (b < best) { best = b; bd = d; }
            }
            disp[(size_t)y * W + x] = (int16_t)bd;
        }
}

/* Host threads the row loops may use (OpenMP), and a way to set their number. */
int32_t oracle_threads(void) { return (int32_t)omp_get_max_threads(); }
void oracle_set_threads(int32_t n) { if (n >= 1) omp_set_num_threads(n); }

/* Left-right consistency, the plain definition: the left pixel (x, y) with disparity d
   matches the right pixel (x - d, y); it is kept when that pixel's own disparity (right
   view as reference) is within tol of d. */
void oracle_lr_check(const int16_t* dl, const int16_t* dr, int32_t W, int32_t H, int32_t D, int32_t tol,
                     int16_t* out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int d = dl[(size_t)y * W + x];
            int keep = 0;
            if (d >= 0 && d < D && x - d >= 0) {
                const int e = dr[(size_t)y * W + (x - d)];
                keep = abs(e - d) <= tol;
            }
            out[(size_t)y * W + x] = (int16_t)(keep ? d : -1);
        }
}

/* ---- O8: E = sum_p C(p, d_p) + lambda * sum_{4-edges} min(|d_p - d_q|, T) ---- */
int64_t oracle_bp_energy(const int16_t* cost, const int16_t* disp, int32_t W, int32_t H, int32_t D,
                         int32_t lambda, int32_t T)
{
    int64_t e = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int dp = disp[(size_t)y * W + x];
            if (dp < 0 || dp >= D) return INT64_MIN;
            e += cost[((size_t)y * W + x) * D + dp];
        }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int dp = disp[(size_t)y * W + x];
            if (x + 1 < W) {
                int t = abs(dp - disp[(size_t)y * W + x + 1]);
                e += (int64_t)lambda * (t < T ? t : T);
            }
            if (y + 1 < H) {
                int t = abs(dp - disp[(size_t)(y + 1) * W + x]);
                e += (int64_t)lambda * (t < T ? t : T);
            }
        }
    return e;
}

static int valid_common(int W, int H, int D, int lambda, int T)
{
    return W >= 1 && H >= 1 && D >= 1 && D <= 256 && lambda >= 0 && lambda <= 65535 && T >= 0;
}

/* ---- checkerboard half-steps on one scale, no skipping (used by the schedule pin) ---- */
int32_t oracle_bp_flat_checkerboard(const int16_t* cost, int32_t W, int32_t H, int32_t D, int32_t lambda,
                                    int32_t T, int32_t halfsteps, const int16_t* init, int16_t* out)
{
    if (!valid_common(W, H, D, lambda, T) || halfsteps < 0) return -1;
    size_t nm = (size_t)4 * W * H * D;
    memcpy(out, init, nm * sizeof(int16_t));
    grid g = {W, H, D, lambda, T, cost, out};
    for (int t = 0; t < halfsteps; ++t) {
#pragma omp parallel
        {
            int32_t* Hb = (int32_t*)malloc(sizeof(int32_t) * (size_t)D);
            int32_t* hb = (int32_t*)malloc(sizeof(int32_t) * (size_t)D);
            int16_t* mb = (int16_t*)malloc(sizeof(int16_t) * (size_t)D);
#pragma omp for schedule(dynamic, 1)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    int eq;
                    if (((x + y) & 1) == (t & 1)) update_pixel(&g, x, y, Hb, hb, mb, &eq, NULL);
                }
            free(Hb); free(hb); free(mb);
        }
    }
    return 0;
}

/* ---- Jacobi iterations: every pixel sends from the previous iteration's messages ---- */
int32_t oracle_bp_flat_jacobi(const int16_t* cost, int32_t W, int32_t H, int32_t D, int32_t lambda,
                              int32_t T, int32_t iterations, const int16_t* init, int16_t* out)
{
    if (!valid_common(W, H, D, lambda, T) || iterations < 0) return -1;
    size_t nm = (size_t)4 * W * H * D;
    int16_t* prev = (int16_t*)malloc(nm * sizeof(int16_t));
    memcpy(out, init, nm * sizeof(int16_t));
    for (int it = 0; it < iterations; ++it) {
        memcpy(prev, out, nm * sizeof(int16_t));
        grid src = {W, H, D, lambda, T, cost, prev};
#pragma omp parallel
        {
        int32_t* Hb = (int32_t*)malloc(sizeof(int32_t) * (size_t)D);
        int32_t* hb = (int32_t*)malloc(sizeof(int32_t) * (size_t)D);
        int16_t* mb = (int16_t*)malloc(sizeof(int16_t) * (size_t)D);
#pragma omp for schedule(dynamic, 1)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int qx, qy;
                const int16_t* c = cost + ((size_t)y * W + x) * D;
                for (int d = 0; d < D; ++d) Hb[d] = c[d];
                for (int k = 0; k < 4; ++k)
                    if (neighbour(k, x, y, W, H, &qx, &qy)) {
                        const int16_t* in = slot(&src, k, x, y);
                        for (int d = 0; d < D; ++d) Hb[d] += in[d];
                    }
                for (int k = 0; k < 4; ++k) {
                    if (!neighbour(k, x, y, W, H, &qx, &qy)) continue;
                    const int16_t* back = slot(&src, k, x, y);
                    for (int d = 0; d < D; ++d) hb[d] = Hb[d] - back[d];
                    oracle_message(hb, D, lambda, T, mb);
                    memcpy(out + (((size_t)opposite(k) * H + qy) * W + qx) * D, mb, sizeof(int16_t) * (size_t)D);
                }
            }
        free(Hb); free(hb); free(mb);
        }
    }
    free(prev);
    return 0;
}

/*
 * ---- the hierarchical solve (O3-O7) ----
 * Scales l = 0 (finest) .. L-1 (coarsest), W_{l+1} = ceil(W_l/2).  The coarsest scale
 * starts from zero messages (or from warm_msgs at scale L-2, skipping L-1); every finer
 * scale starts from its parent's messages in the same direction (zero where the pixel
 * has no neighbour on that side).  On each scale, half-step t updates the pixels of
 * colour (x+y)&1 == t&1.  Skip mode 1: a pixel whose update at half-step t >= 2 leaves
 * every outgoing message unchanged counts one stable update; after K/2 consecutive
 * stable updates it is frozen for the rest of the scale.  Skip mode 2: a pixel is
 * recomputed only if one of its incoming messages changed since its last update.
 */
int32_t oracle_bp_solve(const int16_t* cost, int32_t W, int32_t H, const oracle_params* p,
                        int16_t* disp, int16_t* final_msgs, oracle_stats* st)
{
    const int D = p->num_disp, L = p->num_scales;
    if (!valid_common(W, H, D, p->lambda, p->trunc) || L < 1 || L > 8 || p->skip_mode < 0 ||
        p->skip_mode > 2)
        return -1;
    if (p->skip_mode == 1 && (p->converge_iters < 2 || p->converge_iters > 64 || (p->converge_iters & 1))) return -1;
    if (p->warm_msgs && L < 2) return -1;
    for (int l = 0; l < L; ++l) if (p->iters[l] < 0 || p->iters[l] > 1024) return -1;

    int Ws[8], Hs[8];
    Ws[0] = W; Hs[0] = H;
    for (int l = 1; l < L; ++l) { Ws[l] = (Ws[l - 1] + 1) / 2; Hs[l] = (Hs[l - 1] + 1) / 2; }
    int16_t* C[8];
    C[0] = (int16_t*)cost;
    for (int l = 1; l < L; ++l) {
        C[l] = (int16_t*)malloc(sizeof(int16_t) * (size_t)Ws[l] * Hs[l] * D);
        oracle_pyramid_level(C[l - 1], Ws[l - 1], Hs[l - 1], D, C[l]);
    }
    if (st) memset(st, 0, sizeof(*st));

    int start = p->warm_msgs ? L - 2 : L - 1;
    int16_t* prev = NULL; /* messages of scale l+1 */
    for (int l = start; l >= 0; --l) {
        const int w = Ws[l], h = Hs[l];
        size_t npx = (size_t)w * h;
        int16_t* m = (int16_t*)calloc((size_t)4 * npx * D, sizeof(int16_t));
        grid g = {w, h, D, p->lambda, p->trunc, C[l], m};
        /* O4: initial messages */
        for (int k = 0; k < 4; ++k)
            for (int y = 0; y < h; ++y)
                for (int x = 0; x < w; ++x) {
                    int qx, qy;
                    if (!neighbour(k, x, y, w, h, &qx, &qy)) continue;
                    const int16_t* srcp = NULL;
                    if (l == start && p->warm_msgs)
                        srcp = p->warm_msgs + (((size_t)k * h + y) * w + x) * D;
                    else if (l < start)
                        srcp = prev + (((size_t)k * Hs[l + 1] + (y >> 1)) * Ws[l + 1] + (x >> 1)) * D;
                    if (srcp) memcpy(slot(&g, k, x, y), srcp, sizeof(int16_t) * (size_t)D);
                }
        free(prev);
        prev = NULL;
        uint8_t* active = (uint8_t*)malloc(npx);
        uint8_t* stable = (uint8_t*)calloc(npx, 1);
        uint8_t* dirty = (uint8_t*)malloc(npx);
        memset(active, 1, npx);
        memset(dirty, 1, npx);
        for (int t = 0; t < p->iters[l]; ++t) {
            int64_t count = 0, msgs_sent = 0;
#pragma omp parallel reduction(+ : count, msgs_sent)
            {
            int32_t* Hb = (int32_t*)malloc(sizeof(int32_t) * (size_t)D);
            int32_t* hb = (int32_t*)malloc(sizeof(int32_t) * (size_t)D);
            int16_t* mb = (int16_t*)malloc(sizeof(int16_t) * (size_t)D);
#pragma omp for schedule(dynamic, 1)
            for (int y = 0; y < h; ++y)
                for (int x = 0; x < w; ++x) {
                    if (((x + y) & 1) != (t & 1)) continue;
                    size_t i = (size_t)y * w + x;
                    if (p->skip_mode == 1 && !active[i]) continue;
                    if (p->skip_mode == 2) {
                        uint8_t was_dirty;
#pragma omp atomic read
                        was_dirty = dirty[i];
                        if (!was_dirty) continue;
#pragma omp atomic write
                        dirty[i] = 0;
                    }
                    int eq;
                    int sent = update_pixel(&g, x, y, Hb, hb, mb, &eq, p->skip_mode == 2 ? dirty : NULL);
                    if (p->skip_mode == 1 && t >= 2) {
                        stable[i] = eq ? (uint8_t)(stable[i] + 1) : 0;
                        if (2 * (int)stable[i] >= p->converge_iters) active[i] = 0;
                    }
                    ++count;
                    msgs_sent += sent;
                }
            free(Hb); free(hb); free(mb);
            }
            if (st) {
                st->pixel_updates += count;
                st->msg_updates += msgs_sent;
                if (t < 64) st->active[l][t] = (int32_t)count;
            }
        }
        if (st) st->n_halfsteps[l] = p->iters[l];
        free(active); free(stable); free(dirty);
        prev = m;
    }
    /* prev now holds the finest scale's messages */
    oracle_wta(cost, prev, W, H, D, disp);
    if (final_msgs) memcpy(final_msgs, prev, sizeof(int16_t) * (size_t)4 * W * H * D);
    free(prev);
    for (int l = 1; l < L; ++l) free(C[l]);
    return 0;
}

/*
 * ---- sampled checks at full size ----
 * The message pixel (x,y) sends to its neighbour on side k, recomputed from a given
 * message state (the O5 update of one pixel, read-only).  Returns 0, or -1 if there is
 * no neighbour on that side.
 */
int32_t oracle_message_at(const int16_t* cost, const int16_t* msgs, int32_t W, int32_t H, int32_t D,
                          int32_t lambda, int32_t T, int32_t x, int32_t y, int32_t k, int16_t* out)
{
    int qx, qy;
    if (!neighbour(k, x, y, W, H, &qx, &qy)) return -1;
    int32_t* h = (int32_t*)malloc(sizeof(int32_t) * (size_t)D);
    const int16_t* c = cost + ((size_t)y * W + x) * D;
    for (int d = 0; d < D; ++d) h[d] = c[d];
    for (int j = 0; j < 4; ++j)
        if (neighbour(j, x, y, W, H, &qx, &qy) && j != k)
            for (int d = 0; d < D; ++d) h[d] += msgs[(((size_t)j * H + y) * W + x) * D + d];
    oracle_message(h, D, lambda, T, out);
    free(h);
    return 0;
}

/* Winner-take-all of one pixel (O7). */
int32_t oracle_wta_at(const int16_t* cost, const int16_t* msgs, int32_t W, int32_t H, int32_t D, int32_t x,
                      int32_t y)
{
    int64_t best = INT64_MAX;
    int bd = 0, qx, qy;
    for (int d = 0; d < D; ++d) {
        int64_t b = cost[((size_t)y * W + x) * D + d];
        for (int k = 0; k < 4; ++k)
            if (neighbour(k, x, y, W, H, &qx, &qy)) b += msgs[(((size_t)k * H + y) * W + x) * D + d];
        if (b < best) { best = b; bd = d; }
    }
    return bd;
}

/*
 * ---- learned warm start: the small CNN that predicts initial messages ----
 * Not in the paper: a coarse-scale message initialiser (a learned replacement for the
 * coarsest scale of the hierarchy).  Readings: input at scale s = L-2 is the two views
 * box-averaged over 2^s x 2^s blocks and scaled to [0, 1], plus the coarsest-scale cost
 * (scale s+1) repeated over its 2x2 children and scaled by 1/1024, all rounded to bf16;
 * the network is 3x3 convolutions with zero padding; its output y is turned into
 * messages by round(y * lambda*T) clamped to [0, lambda*T], minus the minimum over d.
 */

/* bf16 (round to nearest even) of a float, and back. */
uint16_t oracle_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

float oracle_bf16_value(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/* Input of the CNN at scale s: [Hs][Ws][cin_p] bf16, channels 0 = left, 1 = right, 2.. = cost. */
void oracle_warm_input(const uint8_t* L, const uint8_t* R, int32_t W, int32_t H, int32_t s,
                       const int16_t* coarse, int32_t D, int32_t cin_p, uint16_t* out)
{
    int Ws = W, Hs = H;
    for (int i = 0; i < s; ++i) { Ws = (Ws + 1) / 2; Hs = (Hs + 1) / 2; }
    const int Wc = (Ws + 1) / 2;
    const int B = 1 << s;
    for (int Y = 0; Y < Hs; ++Y)
        for (int X = 0; X < Ws; ++X) {
            long sl = 0, sr = 0, cnt = 0;
            for (int y = Y * B; y < (Y + 1) * B && y < H; ++y)
                for (int x = X * B; x < (X + 1) * B && x < W; ++x) {
                    sl += L[(size_t)y * W + x];
                    sr += R[(size_t)y * W + x];
                    ++cnt;
                }
            uint16_t* o = out + ((size_t)Y * Ws + X) * cin_p;
            o[0] = oracle_bf16((float)sl / ((float)cnt * 255.0f));
            o[1] = oracle_bf16((float)sr / ((float)cnt * 255.0f));
            const int16_t* c = coarse + ((size_t)(Y >> 1) * Wc + (X >> 1)) * D;
            for (int d = 0; d < D; ++d) o[2 + d] = oracle_bf16((float)c[d] / 1024.0f);
            for (int ch = 2 + D; ch < cin_p; ++ch) o[ch] = 0;
        }
}

/* z[y][x][co] = b[co] + sum_{dy,dx,ci} in[y+dy-1][x+dx-1][ci] * w[co][3dy+dx][ci], zero padding. */
void oracle_conv3x3(const double* in, int32_t H, int32_t W, int32_t Cin, const double* w, const double* b,
                    int32_t Cout, double* z)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int co = 0; co < Cout; ++co) {
                double acc = b ? b[co] : 0.0;
                for (int dy = 0; dy < 3; ++dy)
                    for (int dx = 0; dx < 3; ++dx) {
                        int yy = y + dy - 1, xx = x + dx - 1;
                        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                        const double* iv = in + ((size_t)yy * W + xx) * Cin;
                        const double* wv = w + ((size_t)co * 9 + dy * 3 + dx) * Cin;
                        for (int ci = 0; ci < Cin; ++ci) acc += iv[ci] * wv[ci];
                    }
                z[((size_t)y * W + x) * Cout + co] = acc;
            }
}

/* Gradients of the same convolution given dz = dLoss/dz: din (nullable), dw, db. */
void oracle_conv3x3_backward(const double* in, int32_t H, int32_t W, int32_t Cin, const double* w, int32_t Cout,
                             const double* dz, double* din, double* dw, double* db)
{
    if (din) memset(din, 0, sizeof(double) * (size_t)H * W * Cin);
    memset(dw, 0, sizeof(double) * (size_t)Cout * 9 * Cin);
    memset(db, 0, sizeof(double) * (size_t)Cout);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int co = 0; co < Cout; ++co) {
                const double g = dz[((size_t)y * W + x) * Cout + co];
                db[co] += g;
                for (int dy = 0; dy < 3; ++dy)
                    for (int dx = 0; dx < 3; ++dx) {
                        int yy = y + dy - 1, xx = x + dx - 1;
                        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                        const double* iv = in + ((size_t)yy * W + xx) * Cin;
                        const double* wv = w + ((size_t)co * 9 + dy * 3 + dx) * Cin;
                        double* dwv = dw + ((size_t)co * 9 + dy * 3 + dx) * Cin;
                        double* div = din ? din + ((size_t)yy * W + xx) * Cin : NULL;
                        for (int ci = 0; ci < Cin; ++ci) {
                            dwv[ci] += g * iv[ci];
                            if (div) div[ci] += g * wv[ci];
                        }
                    }
            }
}

/* Messages from the CNN output y [Hs][Ws][4D] (channel k*D + d): round(y*lamT) clamped to
   [0, lamT], minus its minimum over d; zero where the pixel has no neighbour on side k. */
void oracle_warm_messages(const float* y, int32_t Ws, int32_t Hs, int32_t D, int32_t lamT, int16_t* out)
{
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)D);
    for (int k = 0; k < 4; ++k)
        for (int Y = 0; Y < Hs; ++Y)
            for (int X = 0; X < Ws; ++X) {
                int qx, qy;
                int16_t* o = out + (((size_t)k * Hs + Y) * Ws + X) * D;
                if (!neighbour(k, X, Y, Ws, Hs, &qx, &qy)) {
                    for (int d = 0; d < D; ++d) o[d] = 0;
                    continue;
                }
                int32_t mn = INT32_MAX;
                for (int d = 0; d < D; ++d) {
                    float p = y[((size_t)Y * Ws + X) * 4 * D + k * D + d] * (float)lamT;
                    float r = nearbyintf(p);
                    int32_t v = r < 0.0f ? 0 : (r > (float)lamT ? lamT : (int32_t)r);
                    q[d] = v;
                    if (v < mn) mn = v;
                }
                for (int d = 0; d < D; ++d) o[d] = (int16_t)(q[d] - mn);
            }
    free(q);
}

/* Mean L1 distance between y*lamT and the label messages over the slots that have a
   neighbour; dy (nullable) = its gradient with respect to y. */
double oracle_warm_l1(const float* y, const int16_t* label, int32_t Ws, int32_t Hs, int32_t D, int32_t lamT,
                      double* dy)
{
    long n = 0;
    double s = 0.0;
    for (int k = 0; k < 4; ++k)
        for (int Y = 0; Y < Hs; ++Y)
            for (int X = 0; X < Ws; ++X) {
                int qx, qy;
                if (!neighbour(k, X, Y, Ws, Hs, &qx, &qy)) continue;
                n += D;
                for (int d = 0; d < D; ++d) {
                    double r = (double)y[((size_t)Y * Ws + X) * 4 * D + k * D + d] * lamT -
                               label[(((size_t)k * Hs + Y) * Ws + X) * D + d];
                    s += fabs(r);
                }
            }
    if (dy) {
        for (size_t i = 0; i < (size_t)Hs * Ws * 4 * D; ++i) dy[i] = 0.0;
        for (int k = 0; k < 4; ++k)
            for (int Y = 0; Y < Hs; ++Y)
                for (int X = 0; X < Ws; ++X) {
                    int qx, qy;
                    if (!neighbour(k, X, Y, Ws, Hs, &qx, &qy)) continue;
                    for (int d = 0; d < D; ++d) {
                        size_t i = ((size_t)Y * Ws + X) * 4 * D + k * D + d;
                        double r = (double)y[i] * lamT - label[(((size_t)k * Hs + Y) * Ws + X) * D + d];
                        dy[i] = (r > 0 ? 1.0 : (r < 0 ? -1.0 : 0.0)) * lamT / (double)n;
                    }
                }
    }
    return n ? s / (double)n : 0.0;
}

/* One Adam step (bias-corrected), step counted from 1. */
void oracle_adam(double* w, double* m, double* v, const double* g, int64_t n, int32_t step, double lr, double b1,
                 double b2, double eps)
{
    const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
