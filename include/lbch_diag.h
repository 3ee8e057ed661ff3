/*
 * lbch_diag.h — measurement helper of liblbch (not part of the method).
 *
 * A plain streaming copy, used to measure the practical HBM copy bandwidth
 * next to the step kernel and to calibrate the FETCH_SIZE / WRITE_SIZE
 * hardware counters against a kernel that moves a known number of bytes.
 */
#ifndef LBCH_DIAG_H
#define LBCH_DIAG_H

#include <stdint.h>

#include "lbch.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Copies `bytes` bytes from src to dst (both device pointers, 16-byte
 * aligned, non-overlapping; bytes a multiple of 16 and > 0) with one kernel
 * of 16-byte loads and stores, enqueued on hip_stream (NULL = null stream).
 * Does not synchronise.  Bad arguments -> LBCH_E_INVALID. */
lbch_status lbch_diag_copy(const void* src, void* dst, int64_t bytes, void* hip_stream);

/* Single-operator checks of the surrogate's matrix-core kernels (used by the
 * tests; FP32 host-side values are rounded to BF16 on the device first).
 * All pointers are device pointers, channels-last; H, W multiples of 16,
 * Ci, Co multiples of 32.  Allocate their own scratch; synchronise. */

/* y[N][H][W][Co] = act(bias + conv3(x[N][H][W][Ci], w[Co][Ci][3][3])), periodic;
 * act = ReLU if relu != 0; bias nullable.  y is the kernel's BF16 output widened. */
lbch_status lbsg_diag_conv3(const float* x, const float* w, const float* bias, float* y, int32_t n, int32_t h,
                            int32_t wd, int32_t ci, int32_t co, int32_t relu);

/* The network's first convolution with its K packed (ci <= 8 real input
 * channels: 12 taps x 8 channels instead of 9 taps x 32): y as
 * lbsg_diag_conv3 with ReLU for x[N][H][W][ci] (phi NULL), or, with x NULL,
 * for the input whose channel 0 is phi[N][H][W] and whose channels 1..ci-1
 * are the constants cond[0..ci-2] (host array); both forms give the same
 * bits for the same input. */
lbch_status lbsg_diag_conv3_first(const float* x, const float* phi, const float* cond, const float* w, const float* bias,
                                  float* y, int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co);

/* As lbsg_diag_conv3 on the channel concatenation [nearest 2x upsampling of
 * u[N][H/2][W/2][Cu], sk[N][H][W][Cs]] (Ci = Cu + Cs), read by the kernel
 * from its two sources (the decoder's first convolution).  Cu, Cs multiples
 * of 32; w is [Co][Cu + Cs][3][3]. */
lbch_status lbsg_diag_conv3_upcat(const float* u, const float* sk, const float* w, const float* bias, float* y,
                                  int32_t n, int32_t h, int32_t wd, int32_t cu, int32_t cs, int32_t co, int32_t relu);

/* The encoder's second convolution: y as lbsg_diag_conv3 with ReLU, and
 * yp[N][H/2][W/2][Co] its 2x2 average (BF16), formed in the same kernel. */
lbch_status lbsg_diag_conv3_pool(const float* x, const float* w, const float* bias, float* y, float* yp, int32_t n,
                                 int32_t h, int32_t wd, int32_t ci, int32_t co);

/* The decoder's last convolution with the 1x1 head in its epilogue:
 * out[p] = xin[p * cin] + scale (hb[0] + sum_c hw[c] y[p][c]), y the BF16
 * ReLU activations of conv3(x, w) + bias (not stored); Co = 32 or 64. */
lbch_status lbsg_diag_conv3_head(const float* x, const float* w, const float* bias, const float* hw, const float* hb,
                                 const float* xin, int32_t cin, float scale, float* out, int32_t n, int32_t h,
                                 int32_t wd, int32_t ci, int32_t co);

/* dx[N][H][W][Ci] = data gradient of conv3 for dy[N][H][W][Co] (flipped,
 * transposed weights through the forward kernel). */
lbch_status lbsg_diag_conv3_dgrad(const float* dy, const float* w, float* dx, int32_t n, int32_t h, int32_t wd,
                                  int32_t ci, int32_t co);

/* dw[Co][Ci][3][3] = sum over pixels of dy[p][co] x[p + tap][ci] (FP32). */
lbch_status lbsg_diag_conv3_wgrad(const float* x, const float* dy, float* dw, int32_t n, int32_t h, int32_t wd,
                                  int32_t ci, int32_t co);

/* dw as lbsg_diag_conv3_wgrad for the input [nearest 2x upsampling of
 * u[N][H/2][W/2][Cu], sk[N][H][W][Cs]] (the decoder's first convolution),
 * read by the kernel from its two sources; dw is [Co][Cu + Cs][3][3]. */
lbch_status lbsg_diag_conv3_wgrad_upcat(const float* u, const float* sk, const float* dy, float* dw, int32_t n,
                                        int32_t h, int32_t wd, int32_t cu, int32_t cs, int32_t co);

/* The data gradient of the decoder's first convolution (input [nearest 2x
 * upsampling of u (Cu channels), sk (Cs channels)], weights w[Co][Cu + Cs][3][3])
 * for dy[N][H][W][Co], passed straight through the adjoints of the upsampling
 * and the concatenation in the convolution's epilogue:
 * du[N][H/2][W/2][Cu] = bf16(((a + b) + c) + d) over the BF16 data gradient's
 * 2x2 blocks (a, b the upper row), ds[N][H][W][Cs] its remaining channels;
 * mask_u / mask_s (nullable, laid out as du / ds) zero them where <= 0. */
lbch_status lbsg_diag_conv3_dgrad_upadj(const float* dy, const float* w, const float* mask_u, const float* mask_s,
                                        float* du, float* ds, int32_t n, int32_t h, int32_t wd, int32_t cu,
                                        int32_t cs, int32_t co);

/* The data gradient of an encoder level's first convolution (input: the 2x2
 * average of a 2H x 2W tensor, weights w[Co][Ci][3][3]) for dy[N][H][W][Co],
 * passed through the pooling's adjoint in the convolution's epilogue and
 * accumulated in place: dx2[N][2H][2W][Ci] = bf16(0.25 dx + bf16(dx2)) at the
 * four children of each pixel, dx the BF16 data gradient; mask (nullable,
 * laid out as dx2) zeroes the result where <= 0. */
lbch_status lbsg_diag_conv3_dgrad_pooladj(const float* dy, const float* w, const float* mask, float* dx2, int32_t n,
                                          int32_t h, int32_t wd, int32_t ci, int32_t co);

/* db[Co] = sum over pixels of dy[p][co] (FP32), as the weight-gradient kernel
 * forms it beside dw (split partials, fixed-order reduction). */
lbch_status lbsg_diag_conv3_bgrad(const float* x, const float* dy, float* db, int32_t n, int32_t h, int32_t wd,
                                  int32_t ci, int32_t co);

#ifdef __cplusplus
}
#endif

#endif /* LBCH_DIAG_H */
