// Internal declarations of the surrogate (lbsg) kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbsg {

// Segments of the one-launch weight packing (pack_all): per segment the
// FP32 master W[co][ci][3][3], its BF16 output, and the layout: flip 0 ->
// out[co][tap][cip] (zero padded ci), flip 1 -> out[ci][8 - tap][co],
// flip 2 -> out[co][12][8] (the K-packed first layer, ci <= 8).
constexpr int kPackMaxSeg = 64;
struct PackAll {
    int nseg;
    long long end[kPackMaxSeg];   // cumulative element counts
    const float* W[kPackMaxSeg];
    __bf16* out[kPackMaxSeg];
    int co[kPackMaxSeg], ci[kPackMaxSeg], cip[kPackMaxSeg], flip[kPackMaxSeg];
};
hipError_t pack_all(const PackAll& t, hipStream_t s);

hipError_t conv3_fwd(const __bf16* X, const __bf16* Wt, const float* bias, __bf16* Y, int N, int H, int Wd, int Ci,
                     int Co, bool relu, hipStream_t s);
// conv3_fwd of the channel concatenation [nearest 2x upsampling of U (Cu
// channels, H/2 x Wd/2), Sk (Cs channels, H x Wd)] without forming it.
hipError_t conv3_fwd_upcat(const __bf16* U, const __bf16* Sk, const __bf16* Wt, const float* bias, __bf16* Y, int N,
                           int H, int Wd, int Cu, int Cs, int Co, bool relu, hipStream_t s);
// conv3_fwd without bias or activation whose BF16 result is masked:
// Y = Mask > 0 ? y : 0 (Mask laid out as Y): the ReLU backward of the result.
// data gradient of a convolution whose input was [up2(U) (Cu channels), S (Cs
// channels)]: dU (H/2 x Wd/2 x Cu) receives the upsampling's adjoint (2x2
// sums) and dS (H x Wd x Cs) the skip channels, each ReLU-masked by its
// nullable mask (same layout); the full data gradient is never stored
hipError_t conv3_fwd_upadj(const __bf16* X, const __bf16* Wt, __bf16* dU, __bf16* dS, const __bf16* mask_u,
                           const __bf16* mask_s, int N, int H, int Wd, int Ci, int Cu, int Cs, hipStream_t s);
// data gradient of a convolution whose input was the 2x2 average of a
// 2H x 2Wd tensor, passed through the pooling's adjoint and accumulated into
// dX2 (2H x 2Wd x Co): dX2 = bf16(0.25 dx + dX2) per child, ReLU-masked by
// mask (nullable, same layout); the level's own data gradient is never stored
hipError_t conv3_fwd_pooladj(const __bf16* X, const __bf16* Wt, __bf16* dX2, const __bf16* mask, int N, int H, int Wd,
                            int Ci, int Co, hipStream_t s);
hipError_t conv3_fwd_masked(const __bf16* X, const __bf16* Wt, const __bf16* Mask, __bf16* Y, int N, int H, int Wd,
                            int Ci, int Co, hipStream_t s);
// ReLU conv3_fwd writing Y and, to Yp (N x H/2 x Wd/2 x Co), its 2x2
// average (the encoder's second convolution and the pooling after it).
hipError_t conv3_fwd_relu_pool(const __bf16* X, const __bf16* Wt, const float* bias, __bf16* Y, __bf16* Yp, int N, int H,
                               int Wd, int Ci, int Co, hipStream_t s);
// ReLU conv3_fwd (Co = 32 or 64, one workgroup per 16 x 16 pixel tile) with
// the 1x1 head in its epilogue: out[p] = xin[p * cin] + scale (hb[0] + sum_c
// hw[c] y[p][c]) over the BF16 activations y, which go to Y unless it is NULL.
hipError_t conv3_fwd_relu_head(const __bf16* X, const __bf16* Wt, const float* bias, __bf16* Y, int N, int H, int Wd,
                               int Ci, int Co, const float* hw, const float* hb, const float* xin, int cin, float* out,
                               float scale, hipStream_t s);
// The first convolution (ci <= 8 real channels) with K = 12 taps x 8
// channels: input the packed X (channel stride Cs) or, X null, phi[N][H][W]
// FP32 with the constant values cond[0..ncond) as channels 1..ncond; Wk
// [Co][12][8] (pack flip 2); bias, ReLU.  Both input forms give the same bits.
hipError_t conv3_first(const __bf16* X, int Cs, const float* phi, const float* cond, int ncond, const __bf16* Wk,
                       const float* bias, __bf16* Y, int N, int H, int Wd, int Co, hipStream_t s);
// Inference: the first encoder block at 32 channels in one launch, a =
// relu(conv3_first(phi, cond) + b1) kept in LDS, E = relu(conv3(a) + b2) and
// P (N x H/2 x Wd/2 x 32) its 2x2 average; W1k as conv3_first, W2 [32][9][32].
// Bitwise the same E and P as conv3_first followed by conv3_fwd_relu_pool.
hipError_t conv3_pair0(const float* phi, const float* cond, int ncond, const __bf16* W1k, const float* b1,
                       const __bf16* W2, const float* b2, __bf16* E, __bf16* P, int N, int H, int Wd, hipStream_t s);
// Weight-gradient split partials; bpart (nullable, S x Co floats) receives the
// bias gradient's split partials, reduced beside the weights by wgrad_reduce.
hipError_t conv3_dw(const __bf16* X, const __bf16* dY, float* part, int S, int N, int H, int Wd, int Ci, int Co,
                    hipStream_t s, float* bpart = nullptr);
// conv3_dw of the channel concatenation [nearest 2x upsampling of U (Cu
// channels, H/2 x Wd/2), Sk (Cs channels, H x Wd)] without forming it.
hipError_t conv3_dw_upcat(const __bf16* U, const __bf16* Sk, const __bf16* dY, float* part, int S, int N, int H, int Wd,
                          int Cu, int Cs, int Co, hipStream_t s, float* bpart = nullptr);
// bpart / db (both or neither): the bias gradient's split partials [S][Co]
// are reduced into db[Co] in the same launch
hipError_t wgrad_reduce(const float* part, float* dW, int S, int Co, int Ci, int ci_real, hipStream_t s,
                        const float* bpart = nullptr, float* db = nullptr);
hipError_t colsum_bf16(const __bf16* G, long long P, int C, int S, float* part, float* out, hipStream_t s);
hipError_t gather(const float* field, int H, int W, const int* yx, int k, int crop, const float* cond, int ncond,
                  float* x, float* y, hipStream_t s);
hipError_t widen(const __bf16* a, float* b, long long n, hipStream_t s);
hipError_t pack_w(const float* W, __bf16* Wt, int Co, int Ci, int Cip, hipStream_t s);
hipError_t pack_wflip(const float* W, __bf16* Wf, int Co, int Ci, hipStream_t s);
hipError_t pack_input(const float* x, __bf16* out, long long P, int cin, int cpad, hipStream_t s);
hipError_t pack_phi_cond(const float* phi, const float* cond, int ncond, __bf16* out, float* xin, long long P, int cpad,
                         hipStream_t s);
hipError_t head_fwd(const __bf16* d, const float* w, const float* b, const float* xin, int cin, float* out,
                    long long P, int C, float scale, hipStream_t s);
// mask_dd: dd is ReLU-masked by d (the head's input is a post-ReLU activation)
hipError_t head_bwd(const float* g, const __bf16* d, const float* w, __bf16* dd, long long P, int C, int S, float scale,
                    float* part, float* grad_wb, hipStream_t s, bool mask_dd = false);
hipError_t mse(const float* pred, const float* target, float* g, int N, int H, int Wd, int margin, double* part,
               double* out, hipStream_t s);
hipError_t adam(float* w, const float* g, float* m, float* v, long long n, float lr, float b1, float b2, float eps,
                float wd, float c1, float c2, hipStream_t s);

}  // namespace lbsg
