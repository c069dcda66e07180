/*
 * bpstereo — dense stereo correspondence on MI355X (gfx950): a normalised-cross-
 * correlation volume followed by hierarchical, fast-converging min-sum loopy belief
 * propagation on the 4-connected pixel grid.
 *
 * Method: "A LBP Based Correspondence Identification Scheme for Multi-view Sensing
 * Network" (arXiv:1709.06509).  The labelling d minimises E(d) = E_D(d) + E_S(d)
 * (section "Approach Description"); E_D comes from the correlation volume (Abstract;
 * "Correlation volume computation"); E_S is the jump cost between 4-neighbours, here
 * truncated linear lambda*min(|d_p - d_q|, T); messages are recomputed from a pixel's
 * data term, its neighbours' previous messages and the jump cost, and only pixels
 * that have not converged keep being updated ("Fast Converging BP"); the solve runs
 * coarse to fine over a hierarchy of scales with the same process on every scale
 * ("GPU Implementation").
 *
 * Conventions for every entry point:
 *  - Pointers marked [device] are HIP device memory; [host] are host memory.  The
 *    caller owns all memory; the library never frees or keeps caller pointers.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it
 *    asynchronously; the call returns once every launch is enqueued.
 *  - Return 0 on success, or a negative BP_E_* code; the message of the last error on
 *    the calling thread is bp_last_error().  Arguments are validated before anything is
 *    launched: an invalid call enqueues nothing.  Errors raised later on the device
 *    (none are expected from valid arguments) surface at the next synchronisation.
 *  - Layouts: images uint8 [H][W] row-major, contiguous; cost volume int16
 *    [H][W][D] (D fastest); messages int16 [4][H][W][D] with direction
 *    k = 0 from-left, 1 from-right, 2 from-up, 3 from-down (slot k of pixel p holds the
 *    message p received from its neighbour on side k; 0 where there is no neighbour).
 */
#ifndef BPSTEREO_H
#define BPSTEREO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BP_OK 0
#define BP_E_INVAL (-1)       /* an argument is out of range or inconsistent     */
#define BP_E_NOMEM (-2)       /* a host-side allocation failed                    */
#define BP_E_HIP (-3)         /* a HIP runtime call failed                        */
#define BP_E_UNSUPPORTED (-4) /* valid but not supported by the library          */
#define BP_E_WORKSPACE (-5)   /* the workspace is missing or too small            */

/* Opaque per-caller state: kernel timing events.  Not thread-safe; use one per stream. */
typedef struct bp_context bp_context;

/* Solver parameters, passed [host]. */
typedef struct {
    int32_t num_disp;        /* D, 1..256 disparity levels                                   */
    int32_t num_scales;      /* L, 1..8 scales; scale l+1 halves scale l (ceil)             */
    int32_t iters[8];        /* half-steps per scale, [0] = finest, each 0..1024           */
    int32_t lambda;          /* smoothness weight, 0..65535                                 */
    int32_t trunc;           /* T, truncation of |d_p - d_q| in levels, >= 0                */
    int32_t skip_mode;       /* 0 plain; 1 freeze converged pixels; 2 exact dirty-skip      */
    int32_t converge_iters;  /* K for skip_mode 1, in half-steps: even, 2..64               */
    const int16_t* warm_msgs; /* [device] nullable: [4][H_s][W_s][D] initial messages at
                                 scale s = L-2 (needs L >= 2); the solve then skips scale
                                 L-1 and starts at s.  Values 0..32767 (messages are never
                                 negative).  Slots without a neighbour are ignored.       */
} bp_params;

/* Counters of one solve, returned [host]. */
typedef struct {
    int64_t msg_updates;    /* directed messages recomputed, all scales                  */
    int64_t pixel_updates;  /* pixel updates (each recomputes all its outgoing messages) */
    int32_t n_halfsteps[8]; /* half-steps run per scale                                  */
    int32_t active[8][64];  /* pixels recomputed in half-step t of scale l (t < 64)      */
} bp_stats;

/* Device time of the message-update launches since the last bp_context_take_timing. */
typedef struct {
    double halfstep_ms;         /* summed device time of the half-step kernels          */
    int64_t halfstep_launches;  /* number of half-step launches the events bracket       */
    int64_t halfstep_pixel_updates_max; /* pixels those launches could update (all active) */
    double scale_ms[8];         /* the same time split by scale (0 = finest)              */
    int64_t scale_launches[8];  /* and the launches of each scale                          */
} bp_timing;

int32_t bp_context_create(bp_context** out);
int32_t bp_context_destroy(bp_context* ctx);

/*
 * Timing of the message-update launches, with HIP events on the stream the launches go to.
 * on = 1: every later bp_hierarchical_solve on this context records an event pair around
 * each half-step launch (and the batched solve around each half-step phase); on = 2: one
 * event pair around each scale's run of consecutive half-step launches (the average launch
 * time then includes the short gaps between them, and the events perturb the run far less);
 * on = 0: off.
 */
int32_t bp_context_set_timing(bp_context* ctx, int32_t on);
/* Synchronises on the recorded events, returns their sums in *out [host] and clears them. */
int32_t bp_context_take_timing(bp_context* ctx, bp_timing* out);

/*
 * Several consecutive half-steps of a scale in one launch, from LDS: a workgroup loads an
 * interior tile plus a halo as wide as the number of half-steps, runs them, and writes back
 * the interior, which is then bit-identical to one launch per half-step.  It saves launch
 * latency on small scales.  mode 0: never; 1: wherever a tile fits (D <= 64, no counters,
 * skip modes 0 and 1); 2 (default, also without a context): on scales whose cost and
 * messages take at most 48 MB.  Results never depend on the mode.
 */
int32_t bp_context_set_fused(bp_context* ctx, int32_t mode);
/*
 * When `on` is non-zero, bp_hierarchical_solve on this context records its launch
 * sequence into a HIP graph the first time it sees a given set of arguments (shape,
 * parameters and every pointer) and replays that graph on later identical calls.  Applies
 * only to calls on a non-NULL stream that is not already being captured, without stats
 * and with timing off; other calls, or a capture that fails, launch eagerly with the same
 * result.  Up to 32 graphs are kept per context (oldest dropped first).
 */
int32_t bp_context_set_graphs(bp_context* ctx, int32_t on);
/* counts[0..2] [host] = graphs captured, graph replays, eager fallbacks after a failed capture. */
int32_t bp_context_graph_counts(bp_context* ctx, int64_t* counts);

/*
 * Luma of an interleaved RGB image: Y = (77 R + 150 G + 29 B + 128) >> 8 (integer
 * BT.601 weights).  rgb [device] uint8 [H][W][3]; luma [device] uint8 [H][W].
 * The method takes one channel per view (Abstract: views of a regular RGB camera).
 */
int32_t stereo_luma(const uint8_t* rgb, int32_t width, int32_t height, uint8_t* luma, void* stream);

/*
 * Correlation volume (Abstract; "Correlation volume computation").  For every pixel
 * (x, y) of the left view and disparity d in [0, D): zero-mean normalised cross-
 * correlation of the window x window patch around left(x, y) with the patch around
 * right(x - d, y), windows clamped to the image edge.  A patch without variance has
 * correlation 0.  The data cost is round-half-up(cost_scale * (1 - ncc)) clamped to
 * [0, cost_trunc], decided exactly (no floating-point rounding on the way); where
 * x - d < 0 the cost is cost_trunc and the reported ncc is -2.
 *   left, right   [device] uint8 [H][W]
 *   width, height 1..16384 each
 *   num_disp      D, 1..256;  window odd, 1..13;  cost_scale 1..4096;  cost_trunc 0..32767
 *   cost          [device] int16 [H][W][D] output
 *   ncc_or_null   [device] float [H][W][D] output, or NULL
 */
int32_t stereo_cost_volume(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                           int32_t num_disp, int32_t window, int32_t cost_scale, int32_t cost_trunc,
                           int16_t* cost, float* ncc_or_null, void* stream);

/*
 * Correlation volume of colour views (Abstract: views from a regular RGB camera).  As
 * stereo_cost_volume, with each channel taken about its own window mean and the three
 * channels pooled into one correlation:
 *   ncc = sum_c <I_c - mean I_c, J_c - mean J_c> / sqrt(sum_c |I_c - mean I_c|^2 sum_c |J_c - mean J_c|^2),
 * 0 when either pooled variance is 0.  Grey views (R = G = B) give exactly the costs of
 * stereo_cost_volume on one channel; a common gain with per-channel offsets leaves it unchanged.
 *   left_rgb, right_rgb [device] uint8 [H][W][3], interleaved
 *   window odd, 1..9 (the pooled integer sums then fit 32 bits); other arguments as
 *   stereo_cost_volume
 */
int32_t stereo_cost_volume_rgb(const uint8_t* left_rgb, const uint8_t* right_rgb, int32_t width, int32_t height,
                               int32_t num_disp, int32_t window, int32_t cost_scale, int32_t cost_trunc,
                               int16_t* cost, float* ncc_or_null, void* stream);

/* Bytes of device workspace bp_hierarchical_solve needs for this shape; 0 if invalid. */
size_t bp_workspace_bytes(int32_t width, int32_t height, const bp_params* params);

/*
 * Bits per label in which the solve keeps its messages in the workspace: 12 where a pixel's
 * labels span 16 or more lanes (num_disp > 64), every message lies in [0, 4095]
 * (min(lambda * min(trunc, num_disp), 32767) <= 4095) and no warm_msgs are given; else 16;
 * 0 if the arguments are invalid.  Results do not depend on it (the values are the same);
 * the half-steps move 14 * D bytes per pixel update instead of 18 * D.
 */
int32_t bp_message_bits(int32_t width, int32_t height, const bp_params* params);

/*
 * Hierarchical min-sum BP ("Fast Converging BP"; "GPU Implementation").
 *  - Scale l+1 data cost: sum of the (up to 4) children's costs minus its minimum over d,
 *    saturated to 32767.  Scale sizes: W_{l+1} = ceil(W_l / 2).
 *  - The coarsest scale starts from zero messages; each finer scale starts from its
 *    parent's messages in the same direction.
 *  - Half-step t of a scale updates the pixels with (x + y) & 1 == t & 1: each computes
 *    H = C + sum of incoming messages and, for each neighbour q, the message
 *    m(d) = min_d' [H(d') - M_q(d') + lambda*min(|d - d'|, T)] minus its minimum,
 *    saturated to int16, stored in q's slot.
 *  - skip_mode 1: after a pixel's update at half-step t >= 2 leaves every outgoing message
 *    unchanged K/2 times in a row, it is no longer updated on that scale.
 *    skip_mode 2: a pixel is recomputed only if an incoming message changed since its
 *    last update (same result as plain).
 *  - Output disparity = argmin_d of C + sum of incoming messages at the finest scale,
 *    smallest d on ties.
 *   cost           [device] int16 [H][W][D], any values
 *   workspace      [device] at least bp_workspace_bytes(...) bytes, 256-byte aligned;
 *                  its content on entry does not matter; one solve at a time per workspace
 *   disparity      [device] int16 [H][W] output
 *   final_msgs_or_null [device] int16 [4][H][W][D] output: finest-scale messages, or NULL
 *   stats_or_null  [host] if non-NULL the call synchronises the stream and fills it
 */
int32_t bp_hierarchical_solve(bp_context* ctx, const int16_t* cost, int32_t width, int32_t height,
                              const bp_params* params, void* workspace, size_t workspace_bytes,
                              int16_t* disparity, int16_t* final_msgs_or_null, bp_stats* stats_or_null,
                              void* stream);

/*
 * Allocation-free variant of bp_hierarchical_solve, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, semantics and results as bp_hierarchical_solve, except that
 * the workspace is the library's own static device scratch of bp_noalloc_scratch_bytes()
 * bytes (32 MiB; each GPU the library runs on holds one until the process ends).  The call
 * allocates no device memory and creates no runtime object: the context's graph and timing
 * modes are ignored (a caller may capture the call itself).  Shapes whose workspace
 * (bp_workspace_bytes) exceeds the scratch return BP_E_WORKSPACE; the 384x288, D = 16,
 * 4-scale solve needs about 22 MiB.  Every call on one GPU uses that GPU's one scratch, so
 * calls that overlap on one GPU (other streams, other threads) race and must be serialised
 * by the caller; the scratch keeps the last call's contents, which the next call does not
 * depend on.
 */
int32_t bp_hierarchical_solve_noalloc(bp_context* ctx, const int16_t* cost, int32_t width, int32_t height,
                                      const bp_params* params, int16_t* disparity, int16_t* final_msgs_or_null,
                                      bp_stats* stats_or_null, void* stream);
/* Bytes of the static device scratch bp_hierarchical_solve_noalloc uses. */
size_t bp_noalloc_scratch_bytes(void);

/*
 * Left-right consistency of two disparity maps (occlusion and mismatch detection): the
 * left pixel (x, y) with disparity d matches the right pixel (x - d, y), and keeps d when
 * the right map's disparity there (the right view as reference, matching right column u
 * with left column u + d) is within tol of it.  A right map comes from the same calls on
 * both views mirrored left to right and swapped, with the result mirrored back.
 *   disp_left, disp_right [device] int16 [H][W]
 *   out        [device] int16 [H][W] output: d where kept, -1 where x - d < 0, d lies
 *              outside 0..num_disp-1, or the maps disagree by more than tol
 */
int32_t bp_lr_check(const int16_t* disp_left, const int16_t* disp_right, int32_t width, int32_t height,
                    int32_t num_disp, int32_t tol, int16_t* out, void* stream);

/* Bytes of device workspace bp_jacobi_iterations needs (0 if the sizes are invalid). */
size_t bp_jacobi_workspace_bytes(int32_t width, int32_t height, int32_t num_disp);

/*
 * Flat min-sum BP on one scale with the Jacobi schedule ("GPU Implementation": the
 * messages of an iteration are computed from the previous iteration's, held in a second
 * set of four volumes; the paper keeps eight textures per scale for this).  Iteration i
 * computes, for every pixel p and neighbour q, the message of "Fast Converging BP" from
 * C(p) and p's incoming messages of iteration i - 1 (the same rule as a checkerboard
 * half-step, applied to both colours at once).  Iteration i's messages from the pixels
 * of colour c equal half-step i - 1 of a checkerboard run started from the same messages
 * when i - 1 has colour c, which makes this schedule a cross-check of the solve's.
 *   cost               [device] int16 [H][W][D], any values
 *   iterations         0..65536
 *   init_msgs_or_null  [device] int16 [4][H][W][D], values 0..32767, the messages at
 *                      iteration 0 in the layout of final_msgs (slot k of a pixel holds
 *                      the message from its neighbour on side k: 0 left, 1 right, 2 up,
 *                      3 down); slots without a neighbour are ignored; NULL: zeros
 *   msgs_out           [device] int16 [4][H][W][D] output, the same layout; slots without
 *                      a neighbour are written as zero
 *   workspace          [device] at least bp_jacobi_workspace_bytes(...) bytes, 256-byte
 *                      aligned; its content on entry does not matter
 */
int32_t bp_jacobi_iterations(const int16_t* cost, int32_t width, int32_t height, int32_t num_disp,
                             int32_t lambda, int32_t trunc, int32_t iterations,
                             const int16_t* init_msgs_or_null, int16_t* msgs_out, void* workspace,
                             size_t workspace_bytes, void* stream);

/* Bytes of device workspace bp_energy needs (a fixed small amount). */
size_t bp_energy_workspace_bytes(int32_t width, int32_t height);

/*
 * Energy E(d) = E_D(d) + E_S(d) ("Approach Description"):
 * sum_p cost(p, d_p) + lambda * sum over 4-neighbour pairs of min(|d_p - d_q|, trunc).
 *   cost       [device] int16 [H][W][D];  disparity [device] int16 [H][W]
 *   energy     [device] int64, 1 element, output; INT64_MIN if any disparity lies
 *              outside [0, D) (those pixels are never read out of bounds)
 *   workspace  [device] at least bp_energy_workspace_bytes(...) bytes
 */
int32_t bp_energy(const int16_t* cost, const int16_t* disparity, int32_t width, int32_t height,
                  int32_t num_disp, int32_t lambda, int32_t trunc, int64_t* energy, void* workspace,
                  size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * Batched solve: the whole method (correlation volume, hierarchy, half-steps, winner-take-
 * all) for many independent pairs of different sizes and disparity ranges.  It enqueues
 * one launch for every pair's correlation volume, then walks the same phase sequence as
 * bp_hierarchical_solve (pyramid; per scale, coarsest first, its start and its half-steps;
 * winner-take-all) for all pairs together: by default one launch per phase, each covering
 * that phase of every pair; optionally (bp_autotune_batched, bp_context_set_batch_schedule)
 * one persistent launch with a grid-wide barrier between phases.  Each pair's cost volume
 * and disparity are bit-identical to stereo_cost_volume + bp_hierarchical_solve on that
 * pair alone, whatever the schedule.
 * ------------------------------------------------------------------------------------- */
typedef struct {
    const uint8_t* left;   /* [device] uint8 [H][W] */
    const uint8_t* right;  /* [device] uint8 [H][W] */
    int16_t* cost;         /* [device] int16 [H][W][D] output: the pair's correlation volume */
    int16_t* disparity;    /* [device] int16 [H][W] output */
    int32_t width, height, num_disp, pad_;  /* width/height 1..16384, num_disp 1..256 */
} bp_pair_desc;

typedef struct {
    int32_t window, cost_scale, cost_trunc;  /* as stereo_cost_volume */
    int32_t num_scales;                      /* 2..8, the same for every pair */
    int32_t iters[8];                        /* as bp_params */
    int32_t lambda, trunc, skip_mode, converge_iters;
} bp_batch_params;

/*
 * Bytes of device workspace for this batch (pairs [host], n >= 1); 0 if the batch is
 * invalid or unsupported (a pair whose finest 2^(L-1) x 2^(L-1) block of costs does not
 * fit the 64 KB LDS of one workgroup: D * (4^(L-2) + 4^(L-3)) * 32 bytes must be <= 64 KB).
 */
size_t bp_batch_workspace_bytes(const bp_pair_desc* pairs, int32_t n, const bp_batch_params* params);

/*
 * Bits per label in which a batched solve keeps every pair's messages: 12 where every
 * message lies in [0, 4095] (lambda * trunc <= 4095), whatever num_disp; else 16; 0 if the
 * batch is invalid (as bp_batch_workspace_bytes).  Results do not depend on it.
 */
int32_t bp_batch_message_bits(const bp_pair_desc* pairs, int32_t n, const bp_batch_params* params);

/*
 * Solve a batch.  ctx is required: it owns the pinned staging buffer the per-batch tables
 * are uploaded from (a stream-ordered copy into the workspace at every call), the tuned
 * launch shape (bp_autotune_batched) and, when graphs are enabled, the captured graph of
 * the launches.  workspace [device], 256-byte aligned, at least bp_batch_workspace_bytes.
 * Asynchronous; a persistent-launch failure (a grid barrier that timed out because not all
 * workgroups could be resident) is reported by bp_batch_status.
 */
int32_t bp_solve_batched(bp_context* ctx, const bp_pair_desc* pairs, int32_t n, const bp_batch_params* params,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Synchronises `stream` and stores 0 in *status [host] if the last batched solve on this
   workspace completed, 1 if its persistent launch gave up at a grid barrier. */
int32_t bp_batch_status(const void* workspace, void* stream, int32_t* status);

/* Launch shapes tried by the autotuner, with their measured time. */
typedef struct {
    int32_t n_candidates;
    int32_t schedule[16];      /* 0: one persistent launch; 1: one launch per phase (no grid barrier);
                                  2: as 1, with packed 16-bit message sums in the half-steps of
                                  scales that fit the caches (offered when lambda * trunc <= 16383;
                                  the same as 1 where messages are kept in 12 bits;
                                  results are identical) */
    int32_t blocks_per_cu[16]; /* persistent launch: resident workgroups per compute unit */
    int32_t order[16];         /* 0: tiles dealt round-robin; 1: one contiguous eighth per XCD */
    float ms[16];              /* device time of the candidate's solve */
    int32_t best;              /* index of the fastest */
} bp_batch_tuning;

/*
 * Autotune the batched solve: times every candidate schedule on the real batch with HIP
 * events (the one-launch-per-phase schedule, and the persistent launch at each number of
 * workgroups per compute unit and tile order), keeps the fastest in ctx for later
 * bp_solve_batched calls with the same pair shapes and parameters, and reports the table in
 * *out [host].  Synchronises the stream.  Results do not depend on the schedule.
 * Without tuning (or a forced shape) a batch runs one launch per phase (schedule 2, which
 * runs as schedule 1 when lambda * trunc > 16383).
 */
int32_t bp_autotune_batched(bp_context* ctx, const bp_pair_desc* pairs, int32_t n, const bp_batch_params* params,
                            void* workspace, size_t workspace_bytes, void* stream, bp_batch_tuning* out);

/* Force the schedule of later batched solves on ctx (overrides tuning): schedule 0 with
   blocks_per_cu >= 1 (capped at the resident maximum) and order 0/1, or schedule 1 or 2
   (2 runs as 1 when lambda * trunc > 16383); schedule -1 returns to the tuned or default
   choice. */
int32_t bp_context_set_batch_schedule(bp_context* ctx, int32_t schedule, int32_t blocks_per_cu, int32_t order);

/* ---------------------------------------------------------------------------------------
 * Learned warm start.  A small CNN predicts the initial messages of scale s = L-2; the
 * solve then skips scale L-1 and starts at s from them (bp_params.warm_msgs).  The plain,
 * zero-initialised hierarchy stays the fallback and judge.  This is not from the paper: it
 * replaces the coarsest scale of its hierarchy ("GPU Implementation") by a learned guess.
 *
 * Network (D disparity levels): six 3x3 convolutions with zero padding, stride 1:
 * (2 + D) -> 32, ReLU; four times 32 -> 32, ReLU; 32 -> 4D, linear.  Weights and activations
 * are bf16 (round to nearest even), accumulation fp32 on MFMA, biases fp32.
 * Tensors are NHWC: [H][W][C_p] with C_p the channel count padded (layer inputs to a multiple
 * of 16, layer outputs to a multiple of 32); padded channels hold 0.
 * Parameters: one fp32 vector, per layer the weights [Cout_p][9][Cin_p] (tap 3*dy + dx,
 * dy/dx in 0..2 for offsets -1..1) followed by the bias [Cout_p]; the bf16 copy used by the
 * kernels has the same layout.
 * ------------------------------------------------------------------------------------- */

/* Length of the parameter vector for D = num_disp (1..256), or -1. */
int64_t bp_cnn_param_count(int32_t num_disp);
/* Layer 0..5: dims[0..4] [host] = cin, cin_p, cout, cout_p, relu; offsets[0..1] [host] =
   offsets of its weights and bias in the parameter vector. */
int32_t bp_cnn_layer(int32_t num_disp, int32_t layer, int32_t* dims, int64_t* offsets);
/* Bytes of the workspace bp_cnn_forward/bp_cnn_backward use at scale size Ws x Hs (<= 4096 each). */
size_t bp_cnn_workspace_bytes(int32_t Ws, int32_t Hs, int32_t num_disp);

/*
 * One 3x3 convolution: out[p][co] = b[co] + sum_{tap, ci} in[p + tap offset][ci] * w[co][tap][ci]
 * (zero outside the image); then ReLU if relu, or multiplied by (mask[p][co] > 0) if mask is
 * non-NULL; written as bf16 (out_bf16) and/or fp32 before rounding (out_f32), both [P][cout_p]
 * with 0 in channels >= cout.  in [device] bf16 [H][W][cin_p] (cin_p % 16 == 0); w [device] bf16
 * [cout_p][9][cin_p] (cout_p % 32 == 0); bias [device] fp32 [cout_p] or NULL; mask [device] bf16
 * [P][cout_p] or NULL.  in and w are read 16 bytes at a time: both 16-byte aligned
 * (BP_E_INVAL otherwise).
 */
int32_t bp_conv3x3_forward(const uint16_t* in, int32_t H, int32_t W, int32_t cin_p, const uint16_t* weights,
                           const float* bias, int32_t cout, int32_t cout_p, int32_t relu, const uint16_t* mask,
                           uint16_t* out_bf16, float* out_f32, void* stream);
/*
 * Gradient of a 3x3 convolution with respect to its input: for the output gradient g [device]
 * bf16 [P][cout_p] and the layer's weights [cout_p][9][cin_p], computes
 * d[p][ci] = sum_{tap, co} g[p - tap offset][co] * w[co][tap][ci], multiplied by (mask[p][ci] > 0)
 * when mask (the layer input after its ReLU) is non-NULL.  flip_scratch [device] bf16,
 * cin_p * 9 * cout_p elements.  cin_p and cout_p multiples of 32; g and flip_scratch
 * 16-byte aligned.
 */
int32_t bp_conv3x3_data_grad(const uint16_t* g, int32_t H, int32_t W, int32_t cout_p, const uint16_t* weights,
                             int32_t cin, int32_t cin_p, const uint16_t* mask, uint16_t* flip_scratch,
                             uint16_t* out_bf16, float* out_f32, void* stream);
size_t bp_conv3x3_wgrad_workspace_bytes(int32_t H, int32_t W, int32_t cin_p, int32_t cout_p);
/*
 * Gradient of a 3x3 convolution with respect to its weights and bias:
 * dw[co][tap][ci] = sum_p g[p][co] * in[p + tap offset][ci], db[co] = sum_p g[p][co]; fp32,
 * summed in a fixed order (deterministic).  dw [device] fp32 [cout_p][9][cin_p]; db [cout_p].
 */
int32_t bp_conv3x3_weight_grad(const uint16_t* in, const uint16_t* g, int32_t H, int32_t W, int32_t cin_p,
                               int32_t cout_p, void* workspace, size_t workspace_bytes, float* dw, float* db,
                               void* stream);

/*
 * Forward pass: input [device] bf16 [Hs][Ws][cin_p of layer 0]; params [device] fp32 (biases
 * are read from it); weights_bf16 [device]; y [device] fp32 [Hs][Ws][cout_p of layer 5], the
 * last layer's output.  The workspace keeps every layer's activation for bp_cnn_backward.
 * input, weights_bf16 and workspace 16-byte aligned (BP_E_INVAL otherwise).
 */
int32_t bp_cnn_forward(const uint16_t* input, int32_t Ws, int32_t Hs, int32_t num_disp, const float* params,
                       const uint16_t* weights_bf16, void* workspace, size_t workspace_bytes, float* y, void* stream);
/*
 * Backward pass after bp_cnn_forward on the same input and workspace.  Loss = mean over the
 * slots that have a neighbour of |y * lam_t - label| (label [device] int16 [4][Hs][Ws][D],
 * the target messages); its gradient flows back through the network in bf16 with fp32
 * accumulation.  grads [device] fp32, the parameter layout (overwritten); loss [device] fp32.
 * workspace 16-byte aligned.
 */
int32_t bp_cnn_backward(const uint16_t* input, int32_t Ws, int32_t Hs, int32_t num_disp, const uint16_t* weights_bf16,
                        void* workspace, size_t workspace_bytes, const float* y, const int16_t* label, int32_t lam_t,
                        float* grads, float* loss, void* stream);
/* One Adam step (bias-corrected, step >= 1) on fp32 params with moments m, v [device]; also
   refreshes the bf16 copy. */
int32_t bp_adam_step(float* params, float* m, float* v, const float* grads, uint16_t* weights_bf16, int64_t n,
                     int32_t step, float lr, float beta1, float beta2, float eps, void* stream);
/* bf16 copy of the fp32 parameters (round to nearest even). */
int32_t bp_cnn_to_bf16(const float* params, int64_t n, uint16_t* weights_bf16, void* stream);

/*
 * Network input at scale s = L-2 for a pair: channel 0/1 = left/right view averaged over
 * each 2^s x 2^s block / 255, channels 2..D+1 = the coarsest scale's cost of the pixel's
 * parent / 1024, bf16.  cost [device] int16 [H][W][D] (finest); params as for the solve
 * (num_scales >= 2); workspace: a solve workspace (bp_workspace_bytes), whose cost pyramid
 * this call fills.  input [device] bf16 [Hs][Ws][cin_p of layer 0].
 */
int32_t bp_warmstart_input(const uint8_t* left, const uint8_t* right, const int16_t* cost, int32_t width,
                           int32_t height, const bp_params* params, void* workspace, size_t workspace_bytes,
                           uint16_t* input, void* stream);
/*
 * Initial messages from the network output y [device] fp32 [Hs][Ws][cout_p of layer 5]
 * (channel k*D + d): with c = min(lambda * min(trunc, D), 32767), round-to-nearest-even(y * c)
 * clamped to [0, c], minus its minimum over d; zero where the pixel has no neighbour on side k.
 * msgs [device] int16 [4][Hs][Ws][D], ready for bp_params.warm_msgs.
 */
int32_t bp_warmstart_messages(const float* y, int32_t Ws, int32_t Hs, int32_t num_disp, int32_t lambda, int32_t trunc,
                              int16_t* msgs, void* stream);

/*
 * The warm-started solve in one call: bp_warmstart_input, bp_cnn_forward,
 * bp_warmstart_messages and bp_hierarchical_solve with those messages, with bit-identical
 * disparities, messages and counters.  The network runs as ONE launch between the cost pyramid
 * and the first half-step (every layer's activations stay in LDS over a shrinking tile) and
 * writes the start of scale L-2 straight into the solve's workspace.
 *   left, right  [device] uint8 [H][W], the views the cost volume was built from
 *   params       as for bp_hierarchical_solve, warm_msgs NULL; iters[L-1] is not used (scale
 *                L-1 is skipped); num_scales >= 2; num_disp a multiple of 16 in 16..64
 *                (BP_E_UNSUPPORTED otherwise: the layer-level calls above take any D)
 *   cnn_params   [device] fp32 parameter vector (biases are read from it)
 *   cnn_weights  [device] bf16 copy of it (bp_cnn_to_bf16), 16-byte aligned
 *   workspace, disparity, final_msgs_or_null, stats_or_null as for bp_hierarchical_solve
 * Asynchronous unless stats are requested; always eager (the context's graph mode is not used).
 */
int32_t bp_warmstart_solve(bp_context* ctx, const uint8_t* left, const uint8_t* right, const int16_t* cost,
                           int32_t width, int32_t height, const bp_params* params, const float* cnn_params,
                           const uint16_t* cnn_weights, void* workspace, size_t workspace_bytes, int16_t* disparity,
                           int16_t* final_msgs_or_null, bp_stats* stats_or_null, void* stream);

/* Scale `level` (0..num_scales-1) of the solve's cost pyramid, in the caller's layout
   out [device] int16 [H_level][W_level][D]; workspace: a solve workspace. */
int32_t bp_pyramid_level(const int16_t* cost, int32_t width, int32_t height, const bp_params* params, int32_t level,
                         void* workspace, size_t workspace_bytes, int16_t* out, void* stream);

/* Message of the last failed call on this thread ("" if none); valid until the next call. */
const char* bp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
