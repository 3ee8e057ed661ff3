/*
 * lbsg.h — the learned surrogate that jumps the order parameter phi forward
 * (a periodic U-Net of 3x3 convolutions).  BF16 weights and activations,
 * FP32 accumulation on the MI355X matrix cores, FP32 master weights and Adam.
 *
 * Network (levels L, channels C_0..C_{L-1}, in_ch input planes):
 *   encoder  e_0 = B(x),  e_l = B(avgpool2(e_{l-1}))
 *   decoder  d_{L-1} = e_{L-1},  d_l = B(concat(up2(d_{l+1}), e_l))
 *   B(z)     = relu(conv3(relu(conv3(z)+b))+b); conv3 pads periodically
 *   output   phi_pred = x[..., 0] + s (conv1(d_0) + b)  (residual on phi, fixed scale s)
 * Parameters, flat FP32 in this layer order: enc0a, enc0b, ..., enc{L-1}b,
 * dec{L-2}a, dec{L-2}b, ..., dec0a, dec0b, head; each layer W[co][ci][k][k]
 * followed by b[co].
 *
 * Shapes: tensors are channels-last [B][H][W][C] FP32 on the device; H and W
 * multiples of 16 * 2^(L-1).  Conventions as in lbch.h (status codes,
 * lbch_last_error, stream ordering, caller-owned device pointers).
 */
#ifndef LBSG_H
#define LBSG_H

#include <stdint.h>

#include "lbch.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBSG_MAX_LEVELS 6

typedef struct lbsg_arch {
    int32_t levels;                  /* 2 .. LBSG_MAX_LEVELS */
    int32_t chans[LBSG_MAX_LEVELS];  /* each a multiple of 32, <= 512 */
    int32_t in_ch;                   /* 1 .. 32 input planes (phi first) */
    float out_scale;                 /* s > 0 (0 is read as 1): the size of the residual the head is scaled to */
} lbsg_arch;

typedef struct lbsg_net lbsg_net;

/* Allocates parameters (initialised He-normal from `seed`) and activation
 * buffers for up to max_batch images of max_h x max_w; with train != 0 also
 * gradient, Adam and backward buffers.  max_h and max_w are multiples of
 * 16 * 2^(levels - 1) and max_batch x max_h x max_w is below 2^31 pixels (the
 * kernels index pixels in 32 bits); otherwise LBCH_E_INVALID before any device
 * work. */
lbch_status lbsg_create(const lbsg_arch* arch, int32_t max_batch, int32_t max_h, int32_t max_w, int32_t train,
                        uint64_t seed, void* hip_stream, lbsg_net** out);
lbch_status lbsg_destroy(lbsg_net* net);

lbch_status lbsg_param_count(const lbsg_net* net, int64_t* count);
/* Host FP32 copies of the flat parameters (layout above); set re-packs the BF16 weights. */
lbch_status lbsg_get_params(lbsg_net* net, float* host, int64_t count);
lbch_status lbsg_set_params(lbsg_net* net, const float* host, int64_t count);

/* Forward: x_dev [B][H][W][in_ch] FP32 -> phi_dev [B][H][W] FP32.  Stream-ordered. */
lbch_status lbsg_forward(lbsg_net* net, const float* x_dev, int32_t batch, int32_t h, int32_t w, float* phi_dev);

/* Backward of the last forward: dphi_dev [B][H][W] = dLoss/dphi_pred; writes the
 * FP32 parameter gradients (flat layout) to grads_dev.  Needs train != 0. */
lbch_status lbsg_backward(lbsg_net* net, const float* dphi_dev, float* grads_dev);

/* One optimisation step: forward, masked mean squared error against
 * target_dev [B][H][W] over the interior (margin pixels excluded on every
 * side), backward, Adam (lr, betas 0.9/0.999, eps 1e-8, no weight decay).
 * loss_out (host, nullable) receives the loss (synchronises when given). */
lbch_status lbsg_train_step(lbsg_net* net, const float* x_dev, const float* target_dev, int32_t batch, int32_t h,
                            int32_t w, int32_t margin, float lr, double* loss_out);

/* Inference on one field for the hybrid: phi_dev [h][w] FP32 plus cond[ncond]
 * constant conditioning values (planes 1..ncond; ncond = in_ch - 1) ->
 * phi_out_dev [h][w].  Stream-ordered. */
lbch_status lbsg_predict(lbsg_net* net, const float* phi_dev, const float* cond, int32_t ncond, int32_t h, int32_t w,
                         float* phi_out_dev);

/* Training samples cut from a periodic field_dev [h][w] (FP32, device):
 * crop q (q < k) of side `crop` starts at row yx[2q], column yx[2q+1]
 * (host array, wrapped periodically).  x_dev (nullable) receives
 * [k][crop][crop][1 + ncond]: phi then the sample's conditioning values
 * cond[q*ncond .. q*ncond + ncond - 1] (host array); y_dev (nullable)
 * receives [k][crop][crop] phi.  Stream-ordered (host arrays are copied
 * before return). */
lbch_status lbsg_gather(const float* field_dev, int32_t h, int32_t w, const int32_t* yx, int32_t k, int32_t crop,
                        const float* cond, int32_t ncond, float* x_dev, float* y_dev, void* hip_stream);

/* As lbsg_gather, for callers that cannot allocate device memory (a training
 * loop that must not call hipMalloc, code that runs under a memory budget or
 * beside graph capture): the crop origins and conditioning values are staged in
 * a fixed device array of the library (2,162,688 bytes per device, held until
 * the process ends) instead of a per-call allocation, so at most
 * LBSG_GATHER_NOALLOC_MAX_CROPS crops per call (more -> LBCH_E_INVALID).  Calls
 * nothing that allocates.  Every call on a device shares that array: calls that
 * overlap on one device (other threads or streams) race; a call has finished
 * with it when it returns (it synchronises hip_stream).  Other arguments, errors
 * and results as lbsg_gather, bit for bit. */
#define LBSG_GATHER_NOALLOC_MAX_CROPS 16384
lbch_status lbsg_gather_noalloc(const float* field_dev, int32_t h, int32_t w, const int32_t* yx, int32_t k,
                                int32_t crop, const float* cond, int32_t ncond, float* x_dev, float* y_dev,
                                void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBSG_H */
