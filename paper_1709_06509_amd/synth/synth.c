/*
 * Seeded synthetic stereo pairs.
 *
 * This module only makes test and benchmark inputs: a textured left view, a right
 * view obtained by warping the left view through a piecewise-planar disparity map,
 * the ground-truth disparity and an occlusion mask.  It holds none of the stereo
 * method's arithmetic (no correlation, no cost, no message passing) and is shared
 * by the CPU checker and by the GPU library's tests and benchmark alike.
 *
 * Recipe (every draw comes from a counter-based hash of the seed, so a pair is a
 * pure function of its spec):
 *   texture   I = clamp(round(128 + 80*fbm(x,y) + U(-10,10)), 0, 255), where fbm
 *             is 4 octaves of 2-D gradient noise, base period 32 px, persistence 0.5;
 *   planes    Voronoi cells, each d = a(x-cx) + b(y-cy) + c, rounded and clamped to
 *             [0, D-1]; optional fronto-parallel background cell at small d;
 *   slabs     optional thin vertical foreground bars (8-24 px wide) at large d;
 *   warp      right(x - d, y) = left(x, y), z-buffered so the larger d wins;
 *             holes get fresh texture; the right view gets N(0, 2^2) noise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t width, height, num_disp;
    int32_t planes_min, planes_max; /* number of slanted planes, drawn in [min,max] */
    int32_t background;             /* 1: one extra fronto-parallel cell at small d */
    int32_t slabs;                  /* number of thin foreground slabs              */
    int32_t rgb;                    /* 1: interleaved RGB output (3 bytes per px)   */
    int32_t pad_;
    uint64_t seed;
} synth_spec;

static uint64_t mix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* Counter-based hash of (seed, stream, a, b). */
static uint64_t hash4(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b)
{
    uint64_t h = mix64(seed ^ mix64(stream + 0x632BE59BD9B4E019ull));
    h = mix64(h ^ (a * 0xD6E8FEB86659FD93ull));
    return mix64(h ^ (b * 0xA0761D6478BD642Full));
}

static double u01(uint64_t h) { return (double)(h >> 11) * (1.0 / 9007199254740992.0); }

enum { ST_TEX = 1, ST_TEXC = 2, ST_UNI = 3, ST_HOLE = 4, ST_NOISE = 5, ST_PARAM = 6 };

static double fade(double t) { return t * t * t * (t * (t * 6.0 - 15.0) + 10.0); }

static double lattice_dot(uint64_t seed, uint64_t stream, int64_t ix, int64_t iy, double fx, double fy)
{
    static const double gx[8] = {1.0, 0.70710678118654752, 0.0, -0.70710678118654752,
                                 -1.0, -0.70710678118654752, 0.0, 0.70710678118654752};
    static const double gy[8] = {0.0, 0.70710678118654752, 1.0, 0.70710678118654752,
                                 0.0, -0.70710678118654752, -1.0, -0.70710678118654752};
    unsigned g = (unsigned)(hash4(seed, stream, (uint64_t)ix, (uint64_t)iy) & 7u);
    return gx[g] * fx + gy[g] * fy;
}

static double gradient_noise(uint64_t seed, uint64_t stream, double x, double y)
{
    double fx0 = floor(x), fy0 = floor(y);
    int64_t ix = (int64_t)fx0, iy = (int64_t)fy0;
    double fx = x - fx0, fy = y - fy0;
    double n00 = lattice_dot(seed, stream, ix, iy, fx, fy);
    double n10 = lattice_dot(seed, stream, ix + 1, iy, fx - 1.0, fy);
    double n01 = lattice_dot(seed, stream, ix, iy + 1, fx, fy - 1.0);
    double n11 = lattice_dot(seed, stream, ix + 1, iy + 1, fx - 1.0, fy - 1.0);
    double u = fade(fx), v = fade(fy);
    double a = n00 + u * (n10 - n00);
    double b = n01 + u * (n11 - n01);
    return a + v * (b - a);
}

/* 4 octaves, base period 32 px, persistence 0.5, rescaled to roughly [-1, 1]. */
static double fbm(uint64_t seed, uint64_t stream, double x, double y)
{
    double s = 0.0, amp = 1.0, freq = 1.0 / 32.0, norm = 0.0;
    for (int o = 0; o < 4; ++o) {
        s += amp * gradient_noise(seed, stream * 16u + (uint64_t)o, x * freq, y * freq);
        norm += amp;
        amp *= 0.5;
        freq *= 2.0;
    }
    return 1.4 * s / norm;
}

static uint8_t to_u8(double v)
{
    double r = floor(v + 0.5);
    if (r < 0.0) r = 0.0;
    if (r > 255.0) r = 255.0;
    return (uint8_t)r;
}

/* Texture value of channel ch at (x, y); tex_stream selects an independent texture. */
static uint8_t texture(uint64_t seed, uint64_t tex_stream, int ch, int nch, int x, int y)
{
    double base = fbm(seed, ST_TEX + 64u * tex_stream, (double)x, (double)y);
    double v;
    if (nch == 1) {
        v = 128.0 + 80.0 * base;
    } else {
        double own = fbm(seed, ST_TEXC + 64u * tex_stream + 8u * (uint64_t)ch, (double)x, (double)y);
        v = 128.0 + 80.0 * (0.8 * base + 0.35 * own);
    }
    double un = u01(hash4(seed, ST_UNI + 64u * tex_stream + 8u * (uint64_t)ch, (uint64_t)x, (uint64_t)y));
    return to_u8(v + (20.0 * un - 10.0));
}

typedef struct {
    uint64_t seed, ctr;
} seq_rng;

static double seq_u01(seq_rng* r) { return u01(hash4(r->seed, ST_PARAM, r->ctr++, 0)); }
static int seq_int(seq_rng* r, int lo, int hi) /* inclusive */
{
    int v = lo + (int)floor(seq_u01(r) * (double)(hi - lo + 1));
    return v > hi ? hi : v;
}

typedef struct {
    double cx, cy, a, b, c;
} plane;

/* Ground-truth disparity of the spec (integer levels in [0, D-1]). */
static void make_disparity(const synth_spec* s, int16_t* gt)
{
    const int W = s->width, H = s->height, D = s->num_disp;
    seq_rng r = {s->seed, 0};
    int np = seq_int(&r, s->planes_min, s->planes_max);
    int nc = np + (s->background ? 1 : 0);
    plane* P = (plane*)malloc(sizeof(plane) * (size_t)(nc > 0 ? nc : 1));
    double slope = 0.25 * (double)D / (double)(W > H ? W : H);
    double dlo = s->background ? 0.25 * (double)(D - 1) : 0.0;
    for (int i = 0; i < nc; ++i) {
        P[i].cx = seq_u01(&r) * W;
        P[i].cy = seq_u01(&r) * H;
        if (s->background && i == 0) {
            int bmax = D / 8 > 1 ? D / 8 : 1;
            P[i].a = P[i].b = 0.0;
            P[i].c = (double)seq_int(&r, D > 1 ? 1 : 0, D > 1 ? bmax : 0);
        } else {
            P[i].a = (2.0 * seq_u01(&r) - 1.0) * slope;
            P[i].b = (2.0 * seq_u01(&r) - 1.0) * slope;
            P[i].c = dlo + seq_u01(&r) * ((double)(D - 1) - dlo);
        }
    }
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int best = 0;
            double bd = 1e300;
            for (int i = 0; i < nc; ++i) {
                double dx = x - P[i].cx, dy = y - P[i].cy, q = dx * dx + dy * dy;
                if (q < bd) { bd = q; best = i; }
            }
            double d = P[best].a * (x - P[best].cx) + P[best].b * (y - P[best].cy) + P[best].c;
            double rd = floor(d + 0.5);
            if (rd < 0.0) rd = 0.0;
            if (rd > D - 1) rd = D - 1;
            gt[(size_t)y * W + x] = (int16_t)rd;
        }
    }
    for (int k = 0; k < s->slabs; ++k) {
        int w = seq_int(&r, 8, 24);
        int x0 = seq_int(&r, 0, W > w ? W - w : 0);
        int h = seq_int(&r, H / 3, H);
        int y0 = seq_int(&r, 0, H - h);
        int lo = (int)floor(0.85 * (D - 1));
        int d = seq_int(&r, lo, D - 1);
        for (int y = y0; y < y0 + h && y < H; ++y)
            for (int x = x0; x < x0 + w && x < W; ++x) gt[(size_t)y * W + x] = (int16_t)d;
    }
    free(P);
}

/*
 * Fill one pair.  left/right: H*W*(rgb?3:1) bytes, row-major, channels interleaved.
 * gt: H*W int16 disparity of the left view.  occ: H*W bytes, 1 where the left pixel
 * has no visible match in the right view.  Returns 0, or -1 on a bad spec.
 */
int synth_pair(const synth_spec* s, uint8_t* left, uint8_t* right, int16_t* gt, uint8_t* occ)
{
    if (!s || s->width < 1 || s->height < 1 || s->num_disp < 1 || s->num_disp > 4096 ||
        s->planes_min < 0 || s->planes_max < s->planes_min || (s->planes_max + s->background) < 1 ||
        s->slabs < 0)
        return -1;
    const int W = s->width, H = s->height, D = s->num_disp, C = s->rgb ? 3 : 1;
    make_disparity(s, gt);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c)
                left[((size_t)y * W + x) * C + c] = texture(s->seed, 0, c, C, x, y);
    int* src = (int*)malloc(sizeof(int) * (size_t)W);
    int* zb = (int*)malloc(sizeof(int) * (size_t)W);
    (void)D;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) { src[x] = -1; zb[x] = -1; }
        for (int x = 0; x < W; ++x) {
            int d = gt[(size_t)y * W + x], xr = x - d;
            if (xr >= 0 && d > zb[xr]) { zb[xr] = d; src[xr] = x; }
        }
        for (int x = 0; x < W; ++x) {
            int d = gt[(size_t)y * W + x], xr = x - d;
            occ[(size_t)y * W + x] = (uint8_t)((xr < 0 || src[xr] != x) ? 1 : 0);
        }
        for (int xr = 0; xr < W; ++xr) {
            for (int c = 0; c < C; ++c) {
                double v;
                if (src[xr] >= 0) v = (double)left[((size_t)y * W + src[xr]) * C + c];
                else v = (double)texture(s->seed, 1, c, C, xr, y);
                uint64_t h1 = hash4(s->seed, ST_NOISE + 8u * (uint64_t)c, (uint64_t)xr, (uint64_t)y);
                uint64_t h2 = hash4(s->seed, ST_NOISE + 8u * (uint64_t)c + 4u, (uint64_t)xr, (uint64_t)y);
                double u1 = (double)((h1 >> 11) + 1) * (1.0 / 9007199254740993.0);
                double u2 = u01(h2);
                double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
                right[((size_t)y * W + xr) * C + c] = to_u8(v + 2.0 * g);
            }
        }
    }
    free(src);
    free(zb);
    return 0;
}

/*
 * Shape of pair i of an uneven batch: W in {160,176,...,640}, H in {128,144,...,480},
 * D in {16,32,64}, planes in [4,20], each drawn uniformly from the pair's seed.
 */
void synth_batch_shape(uint64_t seed, int32_t* width, int32_t* height, int32_t* num_disp, int32_t* planes)
{
    seq_rng r = {seed ^ 0x5bd1e9955bd1e995ull, 1000};
    *width = 160 + 16 * seq_int(&r, 0, (640 - 160) / 16);
    *height = 128 + 16 * seq_int(&r, 0, (480 - 128) / 16);
    static const int ds[3] = {16, 32, 64};
    *num_disp = ds[seq_int(&r, 0, 2)];
    *planes = seq_int(&r, 4, 20);
}
