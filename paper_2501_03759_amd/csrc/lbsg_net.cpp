// The surrogate network (include/lbsg.h): parameter storage, activation
// buffers and the order of kernel launches for forward, backward, Adam.
#include "../../include/lbch_diag.h"
#include "../../include/lbsg.h"
#include "lbch_internal.h"
#include "lbsg_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <vector>

using lbch::fail;

#define HIP_TRY(expr)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(LBCH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace {

struct Layer {
    int ci_real, ci_pad, co, k;
    long long offW, offB;
    __bf16* wt = nullptr;     // [co][9][ci_pad]
    __bf16* wf = nullptr;     // [ci_pad][9][co] flipped (data gradient), not for the first layer
    __bf16* wk = nullptr;     // [co][12][8] K-packed (the first layer with at most 8 input channels)
};

struct Level {
    // forward activations (bf16, channels-last)
    __bf16 *z = nullptr, *a = nullptr, *e = nullptr;      // encoder block input, mid, output
    __bf16 *da = nullptr, *d = nullptr;                   // decoder block mid, output
    // gradients
    __bf16 *ga = nullptr, *ge = nullptr, *gda = nullptr, *gd = nullptr;
};

int round32(int c) { return (c + 31) / 32 * 32; }

}  // namespace

struct lbsg_net {
    lbsg_arch arch{};
    int max_b = 0, max_h = 0, max_w = 0;
    bool train = false;
    hipStream_t stream = nullptr;
    std::vector<Layer> layers;
    std::vector<Level> lv;
    long long nparam = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float* wpart = nullptr;          // weight-gradient split partials
    long long wpart_elems = 0;
    float* cpart = nullptr;          // column-sum partials
    long long cpart_elems = 0;
    float* out = nullptr;            // fp32 prediction [B][H][W]
    float* gout = nullptr;           // fp32 dLoss/dprediction
    float* xin1 = nullptr;           // fp32 phi (one channel) for lbsg_predict
    float* cond = nullptr;           // conditioning values (device)
    double* dpart = nullptr;
    double* dloss = nullptr;
    int adam_t = 0;
    float scale = 1.f;               // residual scale of the head
    // shape of the last forward
    int cur_b = 0, cur_h = 0, cur_w = 0;
    std::vector<void*> allocs;       // every device allocation of the net
};

namespace {

struct Alloc {
    std::vector<void*> ptrs;
    hipError_t err = hipSuccess;
    template <typename T>
    T* get(size_t count) {
        if (err != hipSuccess) return nullptr;
        void* p = nullptr;
        err = hipMalloc(&p, count * sizeof(T) > 0 ? count * sizeof(T) : 16);
        if (err != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return (T*)p;
    }
};

}  // namespace

namespace {

lbch_status ok() { return LBCH_OK; }

void release(lbsg_net* n) {
    for (void* p : n->allocs)
        if (p) (void)hipFree(p);
    n->allocs.clear();
}

// BF16 copies of every 3x3 layer's weights (and the flipped copies used by the
// data gradient) from the FP32 masters, in one launch
lbch_status repack(lbsg_net* n) {
    lbsg::PackAll t{};
    long long end = 0;
    auto add = [&](const Layer& L, __bf16* out, int flip) {
        const int sg = t.nseg++;
        end += flip == 2 ? (long long)L.co * 96 : flip ? (long long)L.ci_real * 9 * L.co : (long long)L.co * 9 * L.ci_pad;
        t.end[sg] = end;
        t.W[sg] = n->w + L.offW;
        t.out[sg] = out;
        t.co[sg] = L.co;
        t.ci[sg] = L.ci_real;
        t.cip[sg] = L.ci_pad;
        t.flip[sg] = flip;
    };
    for (const Layer& L : n->layers) {
        if (L.k != 3) continue;
        if (t.nseg + 3 > lbsg::kPackMaxSeg) return fail(LBCH_E_INVALID, "too many layers to pack");
        add(L, L.wt, 0);
        if (L.wf) add(L, L.wf, 1);
        if (L.wk) add(L, L.wk, 2);
    }
    HIP_TRY(lbsg::pack_all(t, n->stream));
    return ok();
}

// workgroups of one weight-gradient launch (splits x channel blocks).  More
// splits feed the kernel better but grow the FP32 partials that the split
// reduction reads; measured per training step of 16 x 256^2 (weight-gradient
// kernels + reduction): 256 -> 1.45 ms, 512 -> 1.00 ms, 1024 -> 1.10 ms
constexpr int kWgradBlocks = 512;

// gradient of one conv layer with input z: g = dLoss/d(pre-ReLU output),
// i.e. the gradient of the post-ReLU output already masked by it (every
// producer of such a gradient applies the mask).  dz (nullable) receives the
// data gradient, masked by dz_mask > 0 when given (the previous layer's
// activation).  z_up (nullable): the layer's input is [nearest 2x upsampling
// of z_up (cu channels), z].
lbch_status conv_back(lbsg_net* n, const Layer& L, const __bf16* z, const __bf16* g, __bf16* dz, int B, int H, int W,
                      const __bf16* dz_mask = nullptr, const __bf16* z_up = nullptr, int cu = 0) {
    const long long P = (long long)B * H * W;
    const int ntiles = B * (H / 16) * (W / 16);
    const int other = (L.co % 64 == 0 ? L.co / 64 : L.co / 32) * (L.ci_pad / 16);
    int S = kWgradBlocks / (other > 0 ? other : 1);
    if (S < 1) S = 1;
    if (S > ntiles) S = ntiles;
    while ((long long)S * L.co * 9 * L.ci_pad > n->wpart_elems && S > 1) S /= 2;
    // the bias gradient's split partials come from the weight-gradient kernel when they fit
    const bool fused_bias = (long long)S * L.co <= n->cpart_elems;
    float* bpart = fused_bias ? n->cpart : nullptr;
    if (z_up)
        HIP_TRY(lbsg::conv3_dw_upcat(z_up, z, g, n->wpart, S, B, H, W, cu, L.ci_pad - cu, L.co, n->stream, bpart));
    else
        HIP_TRY(lbsg::conv3_dw(z, g, n->wpart, S, B, H, W, L.ci_pad, L.co, n->stream, bpart));
    HIP_TRY(lbsg::wgrad_reduce(n->wpart, n->g + L.offW, S, L.co, L.ci_pad, L.ci_real, n->stream, bpart,
                               fused_bias ? n->g + L.offB : nullptr));
    if (!fused_bias) HIP_TRY(lbsg::colsum_bf16(g, P, L.co, 256, n->cpart, n->g + L.offB, n->stream));
    if (dz) {
        if (dz_mask)
            HIP_TRY(lbsg::conv3_fwd_masked(g, L.wf, dz_mask, dz, B, H, W, L.co, L.ci_pad, n->stream));
        else
            HIP_TRY(lbsg::conv3_fwd(g, L.wf, nullptr, dz, B, H, W, L.co, L.ci_pad, false, n->stream));
    }
    return ok();
}

lbch_status check_shape(const lbsg_net* n, int B, int H, int W) {
    const int unit = 16 << (n->arch.levels - 1);
    if (B < 1 || B > n->max_b || H < unit || W < unit || H > n->max_h || W > n->max_w || H % unit || W % unit)
        return fail(LBCH_E_INVALID, "batch %d of %dx%d: need 1..%d images, sides multiples of %d up to %dx%d", B, H, W,
                    n->max_b, unit, n->max_h, n->max_w);
    return ok();
}

// everything after the packed input (z_0) is in place; with phi (not null) the
// first convolution reads phi and the conditioning values n->cond (in_ch - 1
// of them) directly instead (z_0 is then not formed)
lbch_status forward_body(lbsg_net* n, int B, int H, int W, const float* xres, int cres, const float* phi = nullptr) {
    const int Lv = n->arch.levels;
    const int* C = n->arch.chans;
    int li = 0;
    for (int l = 0; l < Lv; ++l) {
        const int h = H >> l, w = W >> l;
        Level& lv = n->lv[l];
        const Layer& La = n->layers[li++];
        const Layer& Lb = n->layers[li++];
        if (l == 0 && phi && La.wk && La.co == 32 && Lv > 1) {
            // inference: the whole first block in one launch, its intermediate kept on chip
            HIP_TRY(lbsg::conv3_pair0(phi, n->cond, n->arch.in_ch - 1, La.wk, n->w + La.offB, Lb.wt, n->w + Lb.offB,
                                      lv.e, n->lv[1].z, B, h, w, n->stream));
            continue;
        }
        if (La.wk)   // the first layer, its at most 8 input channels packed into K
            HIP_TRY(lbsg::conv3_first(phi ? nullptr : lv.z, 32, phi, n->cond, n->arch.in_ch - 1, La.wk,
                                      n->w + La.offB, lv.a, B, h, w, La.co, n->stream));
        else
            HIP_TRY(lbsg::conv3_fwd(lv.z, La.wt, n->w + La.offB, lv.a, B, h, w, La.ci_pad, La.co, true, n->stream));
        if (l + 1 < Lv)   // the next level's input, pooled in the epilogue
            HIP_TRY(lbsg::conv3_fwd_relu_pool(lv.a, Lb.wt, n->w + Lb.offB, lv.e, n->lv[l + 1].z, B, h, w, Lb.ci_pad,
                                              Lb.co, n->stream));
        else
            HIP_TRY(lbsg::conv3_fwd(lv.a, Lb.wt, n->w + Lb.offB, lv.e, B, h, w, Lb.ci_pad, Lb.co, true, n->stream));
    }
    const __bf16* d = n->lv[Lv - 1].e;
    for (int l = Lv - 2; l >= 0; --l) {
        const int h = H >> l, w = W >> l;
        Level& lv = n->lv[l];
        const Layer& La = n->layers[li++];
        const Layer& Lb = n->layers[li++];
        // the upsampled-and-concatenated input is read from its two sources
        HIP_TRY(lbsg::conv3_fwd_upcat(d, lv.e, La.wt, n->w + La.offB, lv.da, B, h, w, C[l + 1], C[l], La.co, true,
                                      n->stream));
        const Layer& Lh = n->layers[li];
        if (l == 0 && (Lb.co == 32 || Lb.co == 64)) {
            // the head in the last convolution's epilogue; the activations are kept only for training
            HIP_TRY(lbsg::conv3_fwd_relu_head(lv.da, Lb.wt, n->w + Lb.offB, n->train ? lv.d : nullptr, B, h, w,
                                              Lb.ci_pad, Lb.co, n->w + Lh.offW, n->w + Lh.offB, xres, cres, n->out,
                                              n->scale, n->stream));
            d = nullptr;
        } else {
            HIP_TRY(lbsg::conv3_fwd(lv.da, Lb.wt, n->w + Lb.offB, lv.d, B, h, w, Lb.ci_pad, Lb.co, true, n->stream));
            d = lv.d;
        }
    }
    const Layer& Lh = n->layers[li];
    if (d)
        HIP_TRY(lbsg::head_fwd(d, n->w + Lh.offW, n->w + Lh.offB, xres, cres, n->out, (long long)B * H * W, C[0],
                               n->scale, n->stream));
    n->cur_b = B;
    n->cur_h = H;
    n->cur_w = W;
    return ok();
}

lbch_status backward_body(lbsg_net* n, const float* gphi) {
    const int Lv = n->arch.levels;
    const int* C = n->arch.chans;
    const int B = n->cur_b, H = n->cur_h, W = n->cur_w;
    const long long P0 = (long long)B * H * W;
    const Layer& Lh = n->layers.back();
    // every gradient below leaves its producer already ReLU-masked by the
    // activation it is the gradient of (head: d0; up / skip: d or e; pool: e)
    HIP_TRY(lbsg::head_bwd(gphi, n->lv[0].d, n->w + Lh.offW, n->lv[0].gd, P0, C[0], 256, n->scale, n->cpart,
                           n->g + Lh.offW, n->stream, true));
    // decoder layers sit after the 2*Lv encoder layers, dec{Lv-2} first
    auto dec_layer = [&](int l, int ab) -> const Layer& { return n->layers[2 * Lv + 2 * (Lv - 2 - l) + ab]; };
    const __bf16* gcur = n->lv[0].gd;
    for (int l = 0; l <= Lv - 2; ++l) {
        const int h = H >> l, w = W >> l;
        Level& lv = n->lv[l];
        lbch_status st = conv_back(n, dec_layer(l, 1), lv.da, gcur, lv.gda, B, h, w, lv.da);
        if (st != LBCH_OK) return st;
        // the weight gradient reads the concatenated input from its two sources
        const __bf16* up = (l == Lv - 2) ? n->lv[Lv - 1].e : n->lv[l + 1].d;
        const Layer& L0 = dec_layer(l, 0);
        if (L0.ci_pad != C[l + 1] + C[l]) return fail(LBCH_E_STATE, "decoder layer %d: unexpected input width", l);
        st = conv_back(n, L0, lv.e, lv.gda, nullptr, B, h, w, nullptr, up, C[l + 1]);
        if (st != LBCH_OK) return st;
        // its data gradient goes straight through the adjoints of the upsampling
        // (into the lower level's gradient) and of the concatenation (into the
        // skip's), each ReLU-masked by the activation it is the gradient of
        __bf16* du = (l + 1 < Lv - 1) ? n->lv[l + 1].gd : n->lv[Lv - 1].ge;
        const __bf16* du_mask = (l + 1 < Lv - 1) ? n->lv[l + 1].d : n->lv[Lv - 1].e;
        HIP_TRY(lbsg::conv3_fwd_upadj(lv.gda, L0.wf, du, lv.ge, du_mask, lv.e, B, h, w, L0.co, C[l + 1], C[l],
                                      n->stream));
        gcur = du;
    }
    for (int l = Lv - 1; l >= 0; --l) {
        const int h = H >> l, w = W >> l;
        Level& lv = n->lv[l];
        lbch_status st = conv_back(n, n->layers[2 * l + 1], lv.a, lv.ge, lv.ga, B, h, w, lv.a);
        if (st != LBCH_OK) return st;
        const Layer& La = n->layers[2 * l];
        if (l > 0 && La.ci_pad != C[l - 1]) return fail(LBCH_E_STATE, "encoder layer %d: unexpected input width", l);
        st = conv_back(n, La, lv.z, lv.ga, nullptr, B, h, w);
        if (st != LBCH_OK) return st;
        // the data gradient of a level's first layer goes straight through the
        // pooling's adjoint into the finer level's output gradient (which
        // already holds the skip's part), ReLU-masked by that output
        if (l > 0)
            HIP_TRY(lbsg::conv3_fwd_pooladj(lv.ga, La.wf, n->lv[l - 1].ge, n->lv[l - 1].e, B, h, w, La.co, La.ci_pad,
                                            n->stream));
    }
    return ok();
}

}  // namespace

extern "C" lbch_status lbsg_create(const lbsg_arch* arch, int32_t max_batch, int32_t max_h, int32_t max_w,
                                   int32_t train, uint64_t seed, void* hip_stream, lbsg_net** out) {
    if (!arch || !out) return fail(LBCH_E_INVALID, "NULL argument");
    const int Lv = arch->levels;
    if (Lv < 2 || Lv > LBSG_MAX_LEVELS) return fail(LBCH_E_INVALID, "levels %d outside 2..%d", Lv, LBSG_MAX_LEVELS);
    for (int l = 0; l < Lv; ++l)
        if (arch->chans[l] < 32 || arch->chans[l] % 32 || arch->chans[l] > 512)
            return fail(LBCH_E_INVALID, "chans[%d] = %d must be a multiple of 32 in 32..512", l, arch->chans[l]);
    if (arch->in_ch < 1 || arch->in_ch > 32) return fail(LBCH_E_INVALID, "in_ch %d outside 1..32", arch->in_ch);
    if (!(arch->out_scale >= 0) || !std::isfinite(arch->out_scale))
        return fail(LBCH_E_INVALID, "out_scale must be >= 0 (0 = 1)");
    const int unit = 16 << (Lv - 1);
    if (max_batch < 1 || max_h < unit || max_w < unit || max_h % unit || max_w % unit)
        return fail(LBCH_E_INVALID, "max sizes must be positive multiples of %d", unit);
    // the convolution kernels index pixels in 32 bits
    if ((long long)max_batch * max_h * max_w >= (1LL << 31))
        return fail(LBCH_E_INVALID, "max_batch x max_h x max_w = %lld pixels, at most 2^31 - 1",
                    (long long)max_batch * max_h * max_w);
    lbsg_net* n = new (std::nothrow) lbsg_net();
    if (!n) return fail(LBCH_E_OOM, "host allocation failed");
    n->arch = *arch;
    n->scale = arch->out_scale > 0 ? arch->out_scale : 1.f;
    n->max_b = max_batch;
    n->max_h = max_h;
    n->max_w = max_w;
    n->train = train != 0;
    n->stream = (hipStream_t)hip_stream;
    const int* C = arch->chans;
    // layer table (same order as the flat parameter layout)
    auto add = [&](int ci, int co, int k) {
        Layer L;
        L.ci_real = ci;
        L.ci_pad = k == 3 ? round32(ci) : ci;
        L.co = co;
        L.k = k;
        L.offW = n->nparam;
        n->nparam += (long long)co * ci * k * k;
        L.offB = n->nparam;
        n->nparam += co;
        n->layers.push_back(L);
    };
    int prev = arch->in_ch;
    for (int l = 0; l < Lv; ++l) {
        add(prev, C[l], 3);
        add(C[l], C[l], 3);
        prev = C[l];
    }
    for (int l = Lv - 2; l >= 0; --l) {
        add(C[l + 1] + C[l], C[l], 3);
        add(C[l], C[l], 3);
    }
    add(C[0], 1, 1);

    Alloc A;
    n->w = A.get<float>(n->nparam);
    const long long P0 = (long long)max_batch * max_h * max_w;
    n->lv.resize(Lv);
    for (int l = 0; l < Lv; ++l) {
        const long long P = P0 >> (2 * l);
        Level& lv = n->lv[l];
        const int cz = l == 0 ? 32 : C[l - 1];
        lv.z = A.get<__bf16>(P * cz);
        lv.a = A.get<__bf16>(P * C[l]);
        lv.e = A.get<__bf16>(P * C[l]);
        if (l < Lv - 1) {
            lv.da = A.get<__bf16>(P * C[l]);
            lv.d = A.get<__bf16>(P * C[l]);
        }
        if (n->train) {
            lv.ga = A.get<__bf16>(P * C[l]);
            lv.ge = A.get<__bf16>(P * C[l]);
            if (l < Lv - 1) {
                lv.gda = A.get<__bf16>(P * C[l]);
                lv.gd = A.get<__bf16>(P * C[l]);
            }
        }
    }
    for (Layer& L : n->layers) {
        if (L.k != 3) continue;
        L.wt = A.get<__bf16>((size_t)L.co * 9 * L.ci_pad);
        if (n->train && &L != &n->layers[0]) L.wf = A.get<__bf16>((size_t)L.co * 9 * L.ci_pad);
    }
    if (arch->in_ch <= 8) n->layers[0].wk = A.get<__bf16>((size_t)n->layers[0].co * 96);
    n->out = A.get<float>(P0);
    n->xin1 = A.get<float>(P0);
    n->cond = A.get<float>(32);
    n->cpart_elems = 256 * 513;
    n->cpart = A.get<float>(n->cpart_elems);
    if (n->train) {
        n->g = A.get<float>(n->nparam);
        n->m = A.get<float>(n->nparam);
        n->v = A.get<float>(n->nparam);
        n->gout = A.get<float>(P0);
        long long wp = 0;
        for (const Layer& L : n->layers)
            if (L.k == 3)
                wp = std::max(wp, (long long)kWgradBlocks * L.co * 9 * L.ci_pad /
                                      std::max(1, (L.co % 64 == 0 ? L.co / 64 : L.co / 32) * (L.ci_pad / 16)));
        n->wpart_elems = wp;
        n->wpart = A.get<float>(wp);
        n->dpart = A.get<double>(256);
        n->dloss = A.get<double>(1);
    }
    if (A.err != hipSuccess) {
        for (void* p : A.ptrs) (void)hipFree(p);
        delete n;
        (void)hipGetLastError();
        return fail(A.err == hipErrorOutOfMemory ? LBCH_E_OOM : LBCH_E_DEVICE, "surrogate allocation failed: %s",
                    hipGetErrorString(A.err));
    }
    n->allocs = A.ptrs;
    // He-normal initialisation on the host (deterministic from seed)
    std::vector<float> host(n->nparam);
    std::mt19937_64 rng(seed);
    for (const Layer& L : n->layers) {
        std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (float)(L.ci_real * L.k * L.k)));
        for (long long i = 0; i < (long long)L.co * L.ci_real * L.k * L.k; ++i) host[L.offW + i] = nd(rng);
        for (int c = 0; c < L.co; ++c) host[L.offB + c] = 0.f;
    }
    // the head starts at zero: the untrained net is the identity map on phi
    for (int c = 0; c < C[0] + 1; ++c) host[n->layers.back().offW + c] = 0.f;
    lbch_status st = lbsg_set_params(n, host.data(), n->nparam);
    if (st != LBCH_OK) {
        lbsg_destroy(n);
        return st;
    }
    if (n->train) {
        HIP_TRY(hipMemset(n->m, 0, n->nparam * sizeof(float)));
        HIP_TRY(hipMemset(n->v, 0, n->nparam * sizeof(float)));
        HIP_TRY(hipMemset(n->g, 0, n->nparam * sizeof(float)));
    }
    *out = n;
    return ok();
}

extern "C" lbch_status lbsg_destroy(lbsg_net* n) {
    if (!n) return ok();
    (void)hipStreamSynchronize(n->stream);
    release(n);
    delete n;
    return ok();
}

extern "C" lbch_status lbsg_param_count(const lbsg_net* n, int64_t* count) {
    if (!n || !count) return fail(LBCH_E_INVALID, "NULL argument");
    *count = n->nparam;
    return ok();
}

extern "C" lbch_status lbsg_get_params(lbsg_net* n, float* host, int64_t count) {
    if (!n || !host) return fail(LBCH_E_INVALID, "NULL argument");
    if (count != n->nparam) return fail(LBCH_E_INVALID, "count %lld != %lld parameters", (long long)count, n->nparam);
    HIP_TRY(hipStreamSynchronize(n->stream));
    HIP_TRY(hipMemcpy(host, n->w, count * sizeof(float), hipMemcpyDeviceToHost));
    return ok();
}

extern "C" lbch_status lbsg_set_params(lbsg_net* n, const float* host, int64_t count) {
    if (!n || !host) return fail(LBCH_E_INVALID, "NULL argument");
    if (count != n->nparam) return fail(LBCH_E_INVALID, "count %lld != %lld parameters", (long long)count, n->nparam);
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(host[i])) return fail(LBCH_E_INVALID, "parameter %lld is not finite", (long long)i);
    HIP_TRY(hipStreamSynchronize(n->stream));
    HIP_TRY(hipMemcpy(n->w, host, count * sizeof(float), hipMemcpyHostToDevice));
    lbch_status st = repack(n);
    if (st != LBCH_OK) return st;
    HIP_TRY(hipStreamSynchronize(n->stream));
    n->adam_t = 0;
    return ok();
}

extern "C" lbch_status lbsg_forward(lbsg_net* n, const float* x, int32_t B, int32_t H, int32_t W, float* phi_out) {
    if (!n || !x || !phi_out) return fail(LBCH_E_INVALID, "NULL argument");
    lbch_status st = check_shape(n, B, H, W);
    if (st != LBCH_OK) return st;
    const long long P0 = (long long)B * H * W;
    HIP_TRY(lbsg::pack_input(x, n->lv[0].z, P0, n->arch.in_ch, 32, n->stream));
    st = forward_body(n, B, H, W, x, n->arch.in_ch);
    if (st != LBCH_OK) return st;
    HIP_TRY(hipMemcpyAsync(phi_out, n->out, P0 * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    return ok();
}

extern "C" lbch_status lbsg_backward(lbsg_net* n, const float* dphi, float* grads) {
    if (!n || !dphi) return fail(LBCH_E_INVALID, "NULL argument");
    if (!n->train) return fail(LBCH_E_STATE, "network was created without training buffers");
    if (n->cur_b == 0) return fail(LBCH_E_STATE, "backward before forward");
    lbch_status st = backward_body(n, dphi);
    if (st != LBCH_OK) return st;
    if (grads) HIP_TRY(hipMemcpyAsync(grads, n->g, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    return ok();
}

extern "C" lbch_status lbsg_train_step(lbsg_net* n, const float* x, const float* target, int32_t B, int32_t H,
                                       int32_t W, int32_t margin, float lr, double* loss_out) {
    if (!n || !x || !target) return fail(LBCH_E_INVALID, "NULL argument");
    if (!n->train) return fail(LBCH_E_STATE, "network was created without training buffers");
    lbch_status st = check_shape(n, B, H, W);
    if (st != LBCH_OK) return st;
    if (margin < 0 || 2 * margin >= H || 2 * margin >= W) return fail(LBCH_E_INVALID, "margin %d too large", margin);
    if (!(lr > 0) || !std::isfinite(lr)) return fail(LBCH_E_INVALID, "lr must be positive");
    const long long P0 = (long long)B * H * W;
    HIP_TRY(lbsg::pack_input(x, n->lv[0].z, P0, n->arch.in_ch, 32, n->stream));
    st = forward_body(n, B, H, W, x, n->arch.in_ch);
    if (st != LBCH_OK) return st;
    HIP_TRY(lbsg::mse(n->out, target, n->gout, B, H, W, margin, n->dpart, n->dloss, n->stream));
    st = backward_body(n, n->gout);
    if (st != LBCH_OK) return st;
    n->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)n->adam_t), c2 = 1.f - std::pow(b2, (float)n->adam_t);
    HIP_TRY(lbsg::adam(n->w, n->g, n->m, n->v, n->nparam, lr, b1, b2, 1e-8f, 0.f, c1, c2, n->stream));
    st = repack(n);
    if (st != LBCH_OK) return st;
    if (loss_out) {
        HIP_TRY(hipMemcpyAsync(loss_out, n->dloss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
        HIP_TRY(hipStreamSynchronize(n->stream));
    }
    return ok();
}

extern "C" lbch_status lbsg_predict(lbsg_net* n, const float* phi, const float* cond, int32_t ncond, int32_t H,
                                    int32_t W, float* phi_out) {
    if (!n || !phi || !phi_out || (ncond > 0 && !cond)) return fail(LBCH_E_INVALID, "NULL argument");
    if (ncond != n->arch.in_ch - 1) return fail(LBCH_E_INVALID, "ncond %d != in_ch - 1 = %d", ncond, n->arch.in_ch - 1);
    lbch_status st = check_shape(n, 1, H, W);
    if (st != LBCH_OK) return st;
    if (ncond > 0) HIP_TRY(hipMemcpyAsync(n->cond, cond, ncond * sizeof(float), hipMemcpyHostToDevice, n->stream));
    const long long P0 = (long long)H * W;
    if (!n->train && n->layers[0].wk) {
        // inference only: the first convolution reads phi itself (no packed copy; a
        // training net keeps the packed input, which its backward pass reads)
        st = forward_body(n, 1, H, W, phi, 1, phi);
    } else {
        HIP_TRY(lbsg::pack_phi_cond(phi, n->cond, ncond, n->lv[0].z, n->xin1, P0, 32, n->stream));
        st = forward_body(n, 1, H, W, n->xin1, 1);
    }
    if (st != LBCH_OK) return st;
    HIP_TRY(hipMemcpyAsync(phi_out, n->out, P0 * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));     // cond is a host array the copy reads
    return ok();
}

// ------------------------------------------------------- operator checks
namespace {

struct Scratch {
    std::vector<void*> p;
    ~Scratch() {
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    T* get(size_t n) {
        void* q = nullptr;
        if (hipMalloc(&q, n * sizeof(T) + 16) != hipSuccess) return nullptr;
        p.push_back(q);
        return (T*)q;
    }
};

lbch_status diag_shape(int n, int h, int wd, int ci, int co) {
    if (n < 1 || h < 16 || wd < 16 || h % 16 || wd % 16 || ci < 32 || co < 32 || ci % 32 || co % 32)
        return fail(LBCH_E_INVALID, "operator check needs H, W multiples of 16 and Ci, Co multiples of 32");
    return LBCH_OK;
}

}  // namespace

extern "C" lbch_status lbsg_diag_conv3(const float* x, const float* w, const float* bias, float* y, int32_t n,
                                       int32_t h, int32_t wd, int32_t ci, int32_t co, int32_t relu) {
    if (!x || !w || !y) return fail(LBCH_E_INVALID, "NULL argument");
    lbch_status st = diag_shape(n, h, wd, ci, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    __bf16* xb = S.get<__bf16>(P * ci);
    __bf16* wt = S.get<__bf16>((size_t)co * 9 * ci);
    __bf16* yb = S.get<__bf16>(P * co);
    if (!xb || !wt || !yb) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(x, xb, P, ci, ci, nullptr));
    HIP_TRY(lbsg::pack_w(w, wt, co, ci, ci, nullptr));
    HIP_TRY(lbsg::conv3_fwd(xb, wt, bias, yb, n, h, wd, ci, co, relu != 0, nullptr));
    HIP_TRY(lbsg::widen(yb, y, P * co, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_first(const float* x, const float* phi, const float* cond, const float* w,
                                             const float* bias, float* y, int32_t n, int32_t h, int32_t wd, int32_t ci,
                                             int32_t co) {
    if ((x == nullptr) == (phi == nullptr) || !w || !y || (phi && ci > 1 && !cond))
        return fail(LBCH_E_INVALID, "exactly one of x and phi, and w, y (and cond with phi) are needed");
    if (ci < 1 || ci > 8) return fail(LBCH_E_INVALID, "ci = %d not in 1..8", ci);
    lbch_status st = diag_shape(n, h, wd, 32, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    __bf16* xb = x ? S.get<__bf16>(P * 32) : nullptr;
    __bf16* wk = S.get<__bf16>((size_t)co * 96);
    __bf16* yb = S.get<__bf16>(P * co);
    float* cd = S.get<float>(8);
    if ((x && !xb) || !wk || !yb || !cd) return fail(LBCH_E_OOM, "scratch allocation failed");
    if (x) HIP_TRY(lbsg::pack_input(x, xb, P, ci, 32, nullptr));
    if (phi && ci > 1) HIP_TRY(hipMemcpy(cd, cond, (ci - 1) * sizeof(float), hipMemcpyHostToDevice));
    lbsg::PackAll t{};
    t.nseg = 1;
    t.end[0] = (long long)co * 96;
    t.W[0] = w;
    t.out[0] = wk;
    t.co[0] = co;
    t.ci[0] = ci;
    t.cip[0] = 8;
    t.flip[0] = 2;
    HIP_TRY(lbsg::pack_all(t, nullptr));
    HIP_TRY(lbsg::conv3_first(xb, 32, phi, cd, ci - 1, wk, bias, yb, n, h, wd, co, nullptr));
    HIP_TRY(lbsg::widen(yb, y, P * co, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_upcat(const float* u, const float* sk, const float* w, const float* bias,
                                             float* y, int32_t n, int32_t h, int32_t wd, int32_t cu, int32_t cs,
                                             int32_t co, int32_t relu) {
    if (!u || !sk || !w || !y) return fail(LBCH_E_INVALID, "NULL argument");
    if (cu < 32 || cu % 32) return fail(LBCH_E_INVALID, "cu = %d must be a positive multiple of 32", cu);
    lbch_status st = diag_shape(n, h, wd, cs, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    const int ci = cu + cs;
    __bf16* ub = S.get<__bf16>(P / 4 * cu);
    __bf16* sb = S.get<__bf16>(P * cs);
    __bf16* wt = S.get<__bf16>((size_t)co * 9 * ci);
    __bf16* yb = S.get<__bf16>(P * co);
    if (!ub || !sb || !wt || !yb) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(u, ub, P / 4, cu, cu, nullptr));
    HIP_TRY(lbsg::pack_input(sk, sb, P, cs, cs, nullptr));
    HIP_TRY(lbsg::pack_w(w, wt, co, ci, ci, nullptr));
    HIP_TRY(lbsg::conv3_fwd_upcat(ub, sb, wt, bias, yb, n, h, wd, cu, cs, co, relu != 0, nullptr));
    HIP_TRY(lbsg::widen(yb, y, P * co, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_pool(const float* x, const float* w, const float* bias, float* y, float* yp,
                                            int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co) {
    if (!x || !w || !y || !yp) return fail(LBCH_E_INVALID, "NULL argument");
    lbch_status st = diag_shape(n, h, wd, ci, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    __bf16* xb = S.get<__bf16>(P * ci);
    __bf16* wt = S.get<__bf16>((size_t)co * 9 * ci);
    __bf16* yb = S.get<__bf16>(P * co);
    __bf16* pb = S.get<__bf16>(P / 4 * co);
    if (!xb || !wt || !yb || !pb) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(x, xb, P, ci, ci, nullptr));
    HIP_TRY(lbsg::pack_w(w, wt, co, ci, ci, nullptr));
    HIP_TRY(lbsg::conv3_fwd_relu_pool(xb, wt, bias, yb, pb, n, h, wd, ci, co, nullptr));
    HIP_TRY(lbsg::widen(yb, y, P * co, nullptr));
    HIP_TRY(lbsg::widen(pb, yp, P / 4 * co, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_head(const float* x, const float* w, const float* bias, const float* hw,
                                            const float* hb, const float* xin, int32_t cin, float scale, float* out,
                                            int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co) {
    if (!x || !w || !hw || !hb || !xin || !out) return fail(LBCH_E_INVALID, "NULL argument");
    if (co != 32 && co != 64) return fail(LBCH_E_INVALID, "co = %d: the fused head needs 32 or 64 channels", co);
    if (cin < 1) return fail(LBCH_E_INVALID, "cin = %d must be >= 1", cin);
    lbch_status st = diag_shape(n, h, wd, ci, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    __bf16* xb = S.get<__bf16>(P * ci);
    __bf16* wt = S.get<__bf16>((size_t)co * 9 * ci);
    if (!xb || !wt) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(x, xb, P, ci, ci, nullptr));
    HIP_TRY(lbsg::pack_w(w, wt, co, ci, ci, nullptr));
    HIP_TRY(lbsg::conv3_fwd_relu_head(xb, wt, bias, nullptr, n, h, wd, ci, co, hw, hb, xin, cin, out, scale, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_dgrad(const float* dy, const float* w, float* dx, int32_t n, int32_t h,
                                             int32_t wd, int32_t ci, int32_t co) {
    if (!dy || !w || !dx) return fail(LBCH_E_INVALID, "NULL argument");
    lbch_status st = diag_shape(n, h, wd, ci, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    __bf16* gb = S.get<__bf16>(P * co);
    __bf16* wf = S.get<__bf16>((size_t)co * 9 * ci);
    __bf16* xb = S.get<__bf16>(P * ci);
    if (!gb || !wf || !xb) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(dy, gb, P, co, co, nullptr));
    HIP_TRY(lbsg::pack_wflip(w, wf, co, ci, nullptr));
    HIP_TRY(lbsg::conv3_fwd(gb, wf, nullptr, xb, n, h, wd, co, ci, false, nullptr));
    HIP_TRY(lbsg::widen(xb, dx, P * ci, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_wgrad_upcat(const float* u, const float* sk, const float* dy, float* dw,
                                                   int32_t n, int32_t h, int32_t wd, int32_t cu, int32_t cs,
                                                   int32_t co) {
    if (!u || !sk || !dy || !dw) return fail(LBCH_E_INVALID, "NULL argument");
    if (cu < 32 || cu % 32) return fail(LBCH_E_INVALID, "cu = %d must be a positive multiple of 32", cu);
    lbch_status st = diag_shape(n, h, wd, cs, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    const int ci = cu + cs;
    const int ntiles = n * (h / 16) * (wd / 16);
    const int splits = ntiles < 7 ? ntiles : 7;
    __bf16* ub = S.get<__bf16>(P / 4 * cu);
    __bf16* sb = S.get<__bf16>(P * cs);
    __bf16* gb = S.get<__bf16>(P * co);
    float* part = S.get<float>((size_t)splits * co * 9 * ci);
    if (!ub || !sb || !gb || !part) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(u, ub, P / 4, cu, cu, nullptr));
    HIP_TRY(lbsg::pack_input(sk, sb, P, cs, cs, nullptr));
    HIP_TRY(lbsg::pack_input(dy, gb, P, co, co, nullptr));
    HIP_TRY(lbsg::conv3_dw_upcat(ub, sb, gb, part, splits, n, h, wd, cu, cs, co, nullptr));
    HIP_TRY(lbsg::wgrad_reduce(part, dw, splits, co, ci, ci, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_dgrad_upadj(const float* dy, const float* w, const float* mask_u,
                                                   const float* mask_s, float* du, float* ds, int32_t n, int32_t h,
                                                   int32_t wd, int32_t cu, int32_t cs, int32_t co) {
    if (!dy || !w || !du || !ds) return fail(LBCH_E_INVALID, "NULL argument");
    if (cu < 32 || cu % 32) return fail(LBCH_E_INVALID, "cu = %d must be a positive multiple of 32", cu);
    lbch_status st = diag_shape(n, h, wd, cs, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    const int ci = cu + cs;
    __bf16* gb = S.get<__bf16>(P * co);
    __bf16* wf = S.get<__bf16>((size_t)co * 9 * ci);
    __bf16* dub = S.get<__bf16>(P / 4 * cu);
    __bf16* dsb = S.get<__bf16>(P * cs);
    __bf16* mub = mask_u ? S.get<__bf16>(P / 4 * cu) : nullptr;
    __bf16* msb = mask_s ? S.get<__bf16>(P * cs) : nullptr;
    if (!gb || !wf || !dub || !dsb || (mask_u && !mub) || (mask_s && !msb))
        return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(dy, gb, P, co, co, nullptr));
    HIP_TRY(lbsg::pack_wflip(w, wf, co, ci, nullptr));
    if (mask_u) HIP_TRY(lbsg::pack_input(mask_u, mub, P / 4, cu, cu, nullptr));
    if (mask_s) HIP_TRY(lbsg::pack_input(mask_s, msb, P, cs, cs, nullptr));
    HIP_TRY(lbsg::conv3_fwd_upadj(gb, wf, dub, dsb, mub, msb, n, h, wd, co, cu, cs, nullptr));
    HIP_TRY(lbsg::widen(dub, du, P / 4 * cu, nullptr));
    HIP_TRY(lbsg::widen(dsb, ds, P * cs, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_dgrad_pooladj(const float* dy, const float* w, const float* mask, float* dx2,
                                                     int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co) {
    if (!dy || !w || !dx2) return fail(LBCH_E_INVALID, "NULL argument");
    lbch_status st = diag_shape(n, h, wd, ci, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    __bf16* gb = S.get<__bf16>(P * co);
    __bf16* wf = S.get<__bf16>((size_t)co * 9 * ci);
    __bf16* db = S.get<__bf16>(4 * P * ci);
    __bf16* mb = mask ? S.get<__bf16>(4 * P * ci) : nullptr;
    if (!gb || !wf || !db || (mask && !mb)) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(dy, gb, P, co, co, nullptr));
    HIP_TRY(lbsg::pack_wflip(w, wf, co, ci, nullptr));
    HIP_TRY(lbsg::pack_input(dx2, db, 4 * P, ci, ci, nullptr));
    if (mask) HIP_TRY(lbsg::pack_input(mask, mb, 4 * P, ci, ci, nullptr));
    HIP_TRY(lbsg::conv3_fwd_pooladj(gb, wf, db, mb, n, h, wd, co, ci, nullptr));
    HIP_TRY(lbsg::widen(db, dx2, 4 * P * ci, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_bgrad(const float* x, const float* dy, float* db, int32_t n, int32_t h,
                                             int32_t wd, int32_t ci, int32_t co) {
    if (!x || !dy || !db) return fail(LBCH_E_INVALID, "NULL argument");
    lbch_status st = diag_shape(n, h, wd, ci, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    const int ntiles = n * (h / 16) * (wd / 16);
    const int splits = ntiles < 7 ? ntiles : 7;      // several splits, uneven tile counts per split
    __bf16* xb = S.get<__bf16>(P * ci);
    __bf16* gb = S.get<__bf16>(P * co);
    float* part = S.get<float>((size_t)splits * co * 9 * ci);
    float* bpart = S.get<float>((size_t)splits * co);
    float* dw = S.get<float>((size_t)co * 9 * ci);
    if (!xb || !gb || !part || !bpart || !dw) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(x, xb, P, ci, ci, nullptr));
    HIP_TRY(lbsg::pack_input(dy, gb, P, co, co, nullptr));
    HIP_TRY(lbsg::conv3_dw(xb, gb, part, splits, n, h, wd, ci, co, nullptr, bpart));
    HIP_TRY(lbsg::wgrad_reduce(part, dw, splits, co, ci, ci, nullptr, bpart, db));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

extern "C" lbch_status lbsg_diag_conv3_wgrad(const float* x, const float* dy, float* dw, int32_t n, int32_t h,
                                             int32_t wd, int32_t ci, int32_t co) {
    if (!x || !dy || !dw) return fail(LBCH_E_INVALID, "NULL argument");
    lbch_status st = diag_shape(n, h, wd, ci, co);
    if (st != LBCH_OK) return st;
    Scratch S;
    const long long P = (long long)n * h * wd;
    const int ntiles = n * (h / 16) * (wd / 16);
    const int splits = ntiles < 7 ? ntiles : 7;      // several splits, uneven tile counts per split
    __bf16* xb = S.get<__bf16>(P * ci);
    __bf16* gb = S.get<__bf16>(P * co);
    float* part = S.get<float>((size_t)splits * co * 9 * ci);
    if (!xb || !gb || !part) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(lbsg::pack_input(x, xb, P, ci, ci, nullptr));
    HIP_TRY(lbsg::pack_input(dy, gb, P, co, co, nullptr));
    HIP_TRY(lbsg::conv3_dw(xb, gb, part, splits, n, h, wd, ci, co, nullptr));
    HIP_TRY(lbsg::wgrad_reduce(part, dw, splits, co, ci, ci, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return LBCH_OK;
}

// ------------------------------------------------ allocation-free crop gather
// The crop origins (two int32 per crop) followed by the crops' conditioning
// values (up to 31 floats per crop), in device memory that lives as long as
// the library.  Each device holds its own copy of the array; host code uses
// only the address hipGetSymbolAddress returns for the current device.
namespace {
constexpr size_t kGatherYxBytes = (size_t)LBSG_GATHER_NOALLOC_MAX_CROPS * 2 * sizeof(int32_t);
constexpr size_t kGatherScratchBytes = kGatherYxBytes + (size_t)LBSG_GATHER_NOALLOC_MAX_CROPS * 31 * sizeof(float);
static_assert(kGatherYxBytes % 256 == 0, "the conditioning values start on a 256-byte boundary");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kGatherScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// this device's address of `scratch`, looked up once per device (with it current)
lbch_status gather_scratch(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBCH_E_UNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBCH_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return LBCH_OK;
}
}  // namespace

extern "C" lbch_status lbsg_gather_noalloc(const float* field, int32_t h, int32_t w, const int32_t* yx, int32_t k,
                                           int32_t crop, const float* cond, int32_t ncond, float* x, float* y,
                                           void* hip_stream) {
    if (!field || !yx || (!x && !y) || (ncond > 0 && !cond)) return fail(LBCH_E_INVALID, "NULL argument");
    if (h < 1 || w < 1 || k < 1 || crop < 1 || ncond < 0 || ncond > 31) return fail(LBCH_E_INVALID, "bad sizes");
    if (k > LBSG_GATHER_NOALLOC_MAX_CROPS)
        return fail(LBCH_E_INVALID, "%d crops exceed the allocation-free gather's limit of %d per call", k,
                    LBSG_GATHER_NOALLOC_MAX_CROPS);
    void* base = nullptr;
    lbch_status st = gather_scratch(&base);
    if (st != LBCH_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    int* dyx = (int*)base;
    float* dc = (float*)((char*)base + kGatherYxBytes);
    HIP_TRY(hipMemcpyAsync(dyx, yx, 2 * (size_t)k * sizeof(int), hipMemcpyHostToDevice, s));
    if (ncond > 0) HIP_TRY(hipMemcpyAsync(dc, cond, (size_t)k * ncond * sizeof(float), hipMemcpyHostToDevice, s));
    HIP_TRY(lbsg::gather(field, h, w, dyx, k, crop, dc, ncond, x, y, s));
    // the next call reuses the scratch: this one's kernel has read it on return
    HIP_TRY(hipStreamSynchronize(s));
    return LBCH_OK;
}

extern "C" lbch_status lbsg_gather(const float* field, int32_t h, int32_t w, const int32_t* yx, int32_t k, int32_t crop,
                                   const float* cond, int32_t ncond, float* x, float* y, void* hip_stream) {
    if (!field || !yx || (!x && !y) || (ncond > 0 && !cond)) return fail(LBCH_E_INVALID, "NULL argument");
    if (h < 1 || w < 1 || k < 1 || crop < 1 || ncond < 0 || ncond > 31) return fail(LBCH_E_INVALID, "bad sizes");
    hipStream_t s = (hipStream_t)hip_stream;
    Scratch S;
    int* dyx = S.get<int>(2 * (size_t)k);
    float* dc = S.get<float>((size_t)k * (ncond > 0 ? ncond : 1));
    if (!dyx || !dc) return fail(LBCH_E_OOM, "scratch allocation failed");
    HIP_TRY(hipMemcpyAsync(dyx, yx, 2 * (size_t)k * sizeof(int), hipMemcpyHostToDevice, s));
    if (ncond > 0) HIP_TRY(hipMemcpyAsync(dc, cond, (size_t)k * ncond * sizeof(float), hipMemcpyHostToDevice, s));
    HIP_TRY(lbsg::gather(field, h, w, dyx, k, crop, dc, ncond, x, y, s));
    HIP_TRY(hipStreamSynchronize(s));     // scratch is freed on return
    return LBCH_OK;
}
