/*
 * ORACLE — test infrastructure only.
 *
 * A plain, slow, CPU implementation of the stereo method of "A LBP Based
 * Correspondence Identification Scheme for Multi-view Sensing Network"
 * (arXiv:1709.06509): a normalised-cross-correlation volume followed by
 * hierarchical, fast-converging min-sum loopy belief propagation on the
 * 4-connected pixel grid, minimising E(d) = E_D(d) + E_S(d).
 *
 * It exists to check the GPU library.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * Layouts: images uint8 [H][W] row-major; cost int16 [H][W][D] (D fastest);
 * messages int16 [4][H][W][D], direction k = 0 from-left, 1 from-right, 2 from-up,
 * 3 from-down (the message stored at pixel p in slot k is the one p received from
 * its neighbour on that side).
 */
#ifndef BP_ORACLE_H
#define BP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t num_disp;        /* D */
    int32_t num_scales;      /* L */
    int32_t iters[8];        /* half-steps per scale, [0] = finest, 0..1024 */
    int32_t lambda;          /* smoothness weight */
    int32_t trunc;           /* truncation T, in disparity levels */
    int32_t skip_mode;       /* 0 plain, 1 freeze converged pixels, 2 exact dirty-skip */
    int32_t converge_iters;  /* K, in half-steps (even, >= 2) */
    const int16_t* warm_msgs; /* nullable: [4][H_s][W_s][D] at s = L-2 */
} oracle_params;

typedef struct {
    int64_t msg_updates;     /* directed messages recomputed */
    int64_t pixel_updates;   /* pixels recomputed */
    int32_t n_halfsteps[8];
    int32_t active[8][64];   /* pixels recomputed in each half-step of each scale */
} oracle_stats;

void oracle_luma(const uint8_t* rgb, int32_t width, int32_t height, uint8_t* luma);

double oracle_ncc_at(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                     int32_t window, int32_t x, int32_t y, int32_t d);
int16_t oracle_cost_at(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                       int32_t window, int32_t x, int32_t y, int32_t d, int32_t cost_scale,
                       int32_t cost_trunc);
void oracle_cost_volume(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                        int32_t num_disp, int32_t window, int32_t cost_scale, int32_t cost_trunc,
                        int16_t* cost, double* ncc_or_null);

/* Colour views (interleaved RGB [H][W][3]): each channel about its own window mean, the
   three channels pooled into one correlation; cost quantised as for one channel. */
double oracle_ncc_rgb_at(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                         int32_t window, int32_t x, int32_t y, int32_t d);
int16_t oracle_cost_rgb_at(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                           int32_t window, int32_t x, int32_t y, int32_t d, int32_t cost_scale,
                           int32_t cost_trunc);
void oracle_cost_volume_rgb(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                            int32_t num_disp, int32_t window, int32_t cost_scale, int32_t cost_trunc,
                            int16_t* cost, double* ncc_or_null);

void oracle_pyramid_level(const int16_t* cost, int32_t width, int32_t height, int32_t num_disp,
                          int16_t* out);

void oracle_message(const int32_t* h, int32_t num_disp, int32_t lambda, int32_t trunc, int16_t* out);

int32_t oracle_bp_solve(const int16_t* cost, int32_t width, int32_t height, const oracle_params* p,
                        int16_t* disparity, int16_t* final_msgs_or_null, oracle_stats* stats_or_null);

int32_t oracle_bp_flat_checkerboard(const int16_t* cost, int32_t width, int32_t height, int32_t num_disp,
                                    int32_t lambda, int32_t trunc, int32_t halfsteps,
                                    const int16_t* init_msgs, int16_t* out_msgs);
int32_t oracle_bp_flat_jacobi(const int16_t* cost, int32_t width, int32_t height, int32_t num_disp,
                              int32_t lambda, int32_t trunc, int32_t iterations,
                              const int16_t* init_msgs, int16_t* out_msgs);

void oracle_wta(const int16_t* cost, const int16_t* msgs, int32_t width, int32_t height,
                int32_t num_disp, int16_t* disparity);

int32_t oracle_message_at(const int16_t* cost, const int16_t* msgs, int32_t width, int32_t height,
                          int32_t num_disp, int32_t lambda, int32_t trunc, int32_t x, int32_t y, int32_t k,
                          int16_t* out);
int32_t oracle_wta_at(const int16_t* cost, const int16_t* msgs, int32_t width, int32_t height, int32_t num_disp,
                      int32_t x, int32_t y);

/* learned warm start (test infrastructure for the CNN kernels) */
uint16_t oracle_bf16(float f);
float oracle_bf16_value(uint16_t b);
void oracle_warm_input(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height, int32_t s,
                       const int16_t* coarse, int32_t num_disp, int32_t cin_p, uint16_t* out);
void oracle_conv3x3(const double* in, int32_t H, int32_t W, int32_t Cin, const double* w, const double* b,
                    int32_t Cout, double* z);
void oracle_conv3x3_backward(const double* in, int32_t H, int32_t W, int32_t Cin, const double* w, int32_t Cout,
                             const double* dz, double* din, double* dw, double* db);
void oracle_warm_messages(const float* y, int32_t Ws, int32_t Hs, int32_t D, int32_t lamT, int16_t* out);
double oracle_warm_l1(const float* y, const int16_t* label, int32_t Ws, int32_t Hs, int32_t D, int32_t lamT,
                      double* dy);
void oracle_adam(double* w, double* m, double* v, const double* g, int64_t n, int32_t step, double lr, double b1,
                 double b2, double eps);

/* Left-right consistency: out = disp_left where the right view's disparity at the matched
   column x - d agrees within tol (and d is in 0..D-1 with x - d >= 0), else -1. */
void oracle_lr_check(const int16_t* disp_left, const int16_t* disp_right, int32_t width, int32_t height,
                     int32_t num_disp, int32_t tol, int16_t* out);

/* Host threads that the row loops may use (OpenMP); set their number (n >= 1). */
int32_t oracle_threads(void);
void oracle_set_threads(int32_t n);

int64_t oracle_bp_energy(const int16_t* cost, const int16_t* disparity, int32_t width, int32_t height,
                         int32_t num_disp, int32_t lambda, int32_t trunc);

#ifdef __cplusplus
}
#endif
#endif
