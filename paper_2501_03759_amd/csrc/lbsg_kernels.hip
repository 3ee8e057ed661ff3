// Kernels of the convolutional surrogate (periodic U-Net) for gfx950:
// BF16 activations and weights, FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16), NHWC layout with channels padded to 32.
#include "lbsg_internal.h"

#include <algorithm>
#include <type_traits>

namespace lbsg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

// LDS layout of the forward convolution's tiles: one 64-byte row per pixel
// (or weight row) holding its 32-channel chunk as four 16-byte parts, part k
// of row p stored in slot k ^ ((p >> 1) & 3).  Measured on gfx950 (rocprofv3
// SQ_LDS_BANK_CONFLICT), this keeps both the 16-byte staging writes (four
// lanes per row) and the MFMA fragment reads (16 consecutive rows, one part
// per lane group) free of bank conflicts; an 80-byte padded row conflicts
// two-way on both.
__device__ __forceinline__ int lds_part(int p, int k) { return p * 32 + ((k ^ ((p >> 1) & 3)) << 3); }

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ f32x4 mfma16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// v from lane (lane ^ 1): DPP quad permutation [1, 0, 3, 2]
__device__ __forceinline__ float lane_xor1(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
}

// Scheduling pattern for NL LDS reads among MF matrix-core instructions: one
// read, then two (or one, when reads outnumber half the MFMAs) MFMAs, repeated.
template <int NL, int MF>
__device__ __forceinline__ void interleave_ds_mfma() {
    if constexpr (NL > 0 && MF > 0) {
        constexpr int m = MF >= 2 * NL ? 2 : 1;
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read
        __builtin_amdgcn_sched_group_barrier(0x008, m, 0);   // MFMA
        interleave_ds_mfma<NL - 1, MF - m>();
    } else if constexpr (NL > 0) {
        __builtin_amdgcn_sched_group_barrier(0x100, NL, 0);
    } else if constexpr (MF > 0) {
        __builtin_amdgcn_sched_group_barrier(0x008, MF, 0);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// 3x3 periodic convolution as an implicit GEMM on the matrix cores.
//   Y[n,y,x,co] = act(bias[co] + sum_{tap,ci} W[co][tap][ci] X[n, y+dy, x+dx, ci])
// GEMM view per workgroup: M = TC output channels, N = a 16x16 pixel tile,
// K = 9 taps x Ci.  The A operand (weights, 8 consecutive ci per lane) and
// the B operand (pixels, 8 consecutive ci per lane) are both read from LDS.
// Per 32-channel chunk the workgroup stages the pixel tile with its periodic
// 1-pixel halo and the weights of all nine taps (two barriers per chunk);
// the global loads of the next chunk are issued into registers before the
// matrix-core work on the current one, so they overlap it.  Each wave owns 4
// pixel rows x TC channels (4 x TC/16 MFMA tiles); the result fragment of a
// lane is 4 consecutive output channels of one pixel (one 8-byte store).
// UPCAT: the input is the channel concatenation of X (half resolution, Cu
// channels, nearest-neighbour upsampled) and X2 (full resolution, Ci - Cu
// channels), read from the two sources; both counts are multiples of 32, so
// every chunk comes from one of them.
// HEAD (Co = TC, one workgroup per pixel tile): the 1x1 output head is applied
// in the epilogue, out[p] = xin[p][0] + scale (b + sum_c w_c y[p][c]) over the
// BF16-rounded activations; Y (nullable) still receives them.
// POOL: Y as usual, and Yp (H/2 x Wd/2) receives its 2x2 average of the BF16
// outputs, bf16(0.25 ((a + b) + (c + d))) in FP32 with a, b the upper and c, d
// the lower row of the block: the rows belong to one wave (rows r, r + 1),
// the columns to lanes l16 and l16 ^ 1.
// Mask (nullable, same layout as Y): Y = Mask > 0 ? y : 0 elementwise, the
// ReLU backward applied to the BF16 result (for data gradients whose next
// consumer masks them by the previous layer's activation).
// UPADJ (data gradient of a convolution whose input was [nearest 2x upsampling
// of U (Cu channels), S (Co - Cu channels)]): the output is never formed;
// channels below Cu go through the upsampling's adjoint, Yp (H/2 x Wd/2 x Cu)
// = bf16(((a + b) + c) + d) over the BF16 outputs of each 2x2 block (a, b the
// upper row), channels from Cu on are stored in Y (H x Wd x (Co - Cu)); Mask2
// (layout of Yp) and Mask (layout of Y), both nullable, ReLU-mask the two
// results.  Cu is a multiple of TC, so each workgroup feeds one of them.
// POOLADJ (data gradient of a convolution whose input was the 2x2 average of
// a 2H x 2Wd tensor): the output is never formed; each of its pixels goes
// through the pooling's adjoint into Y (2H x 2Wd x Co), which is accumulated:
// Y[child] = bf16(0.25 y + Y[child]) for the four children, then ReLU-masked
// by Mask (nullable, layout of Y).  Each child belongs to one lane.
// ---------------------------------------------------------------------------
struct HeadArgs {
    const float* w;      // [Co] head weights
    const float* b;      // [1] head bias
    const float* xin;    // [P][cin] FP32 input; channel 0 is the residual base
    int cin;
    float* out;          // [P]
    float scale;
};

template <int TC, bool RELU, bool UPCAT, bool HEAD = false, bool POOL = false, bool UPADJ = false,
          bool POOLADJ = false>
__global__ __launch_bounds__(256, TC == 32 ? 3 : 2) void conv3_fwd_k(const __bf16* __restrict__ X, const __bf16* __restrict__ X2, int Cu,
                                                   const __bf16* __restrict__ Wt, const float* __restrict__ bias,
                                                   __bf16* __restrict__ Y, int H, int Wd, int Ci, int Co,
                                                   const HeadArgs hd = HeadArgs{}, __bf16* __restrict__ Yp = nullptr,
                                                   const __bf16* __restrict__ Mask = nullptr,
                                                   const __bf16* __restrict__ Mask2 = nullptr) {
    constexpr int NXQ = 18 * 18 * 4;              // 16-byte chunks of the pixel tile
    constexpr int NWQ = 9 * TC * 4;               // 16-byte chunks of the weights
    constexpr int RX = (NXQ + 255) / 256, RW = (NWQ + 255) / 256;
    __shared__ __align__(16) __bf16 sx[18 * 18 * 32];
    __shared__ __align__(16) __bf16 sw[9 * TC * 32];
    constexpr int CB = TC / 16;
    const int tiles_x = Wd / 16, tiles_y = H / 16;
    int b = blockIdx.x;
    const int tx0 = (b % tiles_x) * 16;
    b /= tiles_x;
    const int ty0 = (b % tiles_y) * 16;
    const int n = b / tiles_y;
    const int co0 = blockIdx.y * TC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, kb = lane >> 4;
    f32x4 acc[4][CB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    // per-thread source offsets (chunk-independent parts); indices past the
    // end are clamped to the last chunk (loaded, never stored).  Pixel indices
    // are 32-bit (the launchers require N H W < 2^31), widened by one multiply;
    // weight offsets are 32-bit.
    long long xoff[RX];
    long long xoff2[UPCAT ? RX : 1];
    unsigned woff[RW];
#pragma unroll
    for (int i = 0; i < RX; ++i) {
        const int q = min((int)threadIdx.x + i * 256, NXQ - 1);
        const int px = q >> 2;
        const unsigned part8 = (unsigned)(q & 3) * 8u;
        const int py = px / 18, pxx = px - py * 18;
        const int y = wrap(ty0 - 1 + py, H), x = wrap(tx0 - 1 + pxx, Wd);
        if constexpr (UPCAT) {
            const unsigned pu = (unsigned)(n * (H / 2) + (y >> 1)) * (unsigned)(Wd / 2) + (unsigned)(x >> 1);
            const unsigned ps = (unsigned)(n * H + y) * (unsigned)Wd + (unsigned)x;
            xoff[i] = (long long)((unsigned long long)pu * (unsigned)Cu + part8);
            xoff2[i] = (long long)((unsigned long long)ps * (unsigned)(Ci - Cu) + part8);
        } else {
            const unsigned ps = (unsigned)(n * H + y) * (unsigned)Wd + (unsigned)x;
            xoff[i] = (long long)((unsigned long long)ps * (unsigned)Ci + part8);
        }
    }
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int q = min((int)threadIdx.x + i * 256, NWQ - 1);
        const int row = q >> 2, part = q & 3;
        const int tap = row / TC, co = row - tap * TC;
        woff[i] = ((unsigned)(co0 + co) * 9u + (unsigned)tap) * (unsigned)Ci + (unsigned)part * 8u;
    }
    // LDS element offsets.  Staging: chunk q = threadIdx.x + 256 i goes to
    // lds_part(q / 4, q % 4); its swizzle term ((q / 4) >> 1) & 3 does not
    // depend on i, so the offsets are ls + 2048 i.  A reads: row tap TC + 16 c
    // + l16 has the swizzle term of row l16.  B reads: row P0 + l16 with
    // P0 = 72 wave + 18 j + kx has the swizzle term ((r + l16) >> 1) & 3,
    // r = P0 mod 8 = (18 j + kx) mod 8, so eight lane bases serve every (j, kx).
    const int ls = lds_part((int)threadIdx.x >> 2, (int)threadIdx.x & 3);
    const int la = lds_part(l16, kb);
    int lbb[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) lbb[r] = (wave * 72 + l16) * 32 + ((kb ^ (((r + l16) >> 1) & 3)) << 3);
    // staged chunks are held as plain 32-bit words (moved, never computed on)
    u32x4 rx[RX], rw[RW];
    // pixel-tile chunk starting at input channel cc
    auto load_x = [&](int cc) {
        if constexpr (UPCAT) {
            if (cc >= Cu) {
#pragma unroll
                for (int i = 0; i < RX; ++i) rx[i] = *reinterpret_cast<const u32x4*>(X2 + xoff2[i] + (cc - Cu));
                return;
            }
        }
#pragma unroll
        for (int i = 0; i < RX; ++i) rx[i] = *reinterpret_cast<const u32x4*>(X + xoff[i] + cc);
    };
    load_x(0);
#pragma unroll
    for (int i = 0; i < RW; ++i) rw[i] = *reinterpret_cast<const u32x4*>(Wt + woff[i]);

    for (int cc = 0; cc < Ci; cc += 32) {
        __syncthreads();                          // every wave is done with the previous chunk
#pragma unroll
        for (int i = 0; i < RX; ++i) {
            const int q = (int)threadIdx.x + i * 256;
            if (q < NXQ) *reinterpret_cast<u32x4*>(sx + ls + 2048 * i) = rx[i];
        }
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int q = (int)threadIdx.x + i * 256;
            if (q < NWQ) *reinterpret_cast<u32x4*>(sw + ls + 2048 * i) = rw[i];
        }
        __syncthreads();
        if (cc + 32 < Ci) {                       // next chunk in flight during the MFMAs
            load_x(cc + 32);
#pragma unroll
            for (int i = 0; i < RW; ++i) rw[i] = *reinterpret_cast<const u32x4*>(Wt + (woff[i] + (unsigned)(cc + 32)));
        }
        // Taps in kx-major order t = 3 kx + ky.  B rows wave * 4 + j (j = 0..5) at
        // column l16 + kx live in bq[kx & 1][j] (tap (kx, ky) uses rows ky..ky+3);
        // the A fragments of tap t in aq[t % 3].  The operands of tap t + 2 are
        // read from LDS while the MFMAs of tap t run (two B buffers suffice: the
        // tap column changes every three taps, so a two-tap lead never writes
        // rows that tap t or t + 1 reads).
        bf16x8 bq[2][6], aq[3][CB];
        auto ld_b = [&](int kx, int j, bf16x8& v) {
            v = *reinterpret_cast<const bf16x8*>(sx + lbb[(18 * j + kx) & 7] + (18 * j + kx) * 32);
        };
        auto ld_a = [&](int kx, int ky, bf16x8 (&a)[CB]) {
#pragma unroll
            for (int c = 0; c < CB; ++c)
                a[c] = *reinterpret_cast<const bf16x8*>(sw + la + ((ky * 3 + kx) * TC + c * 16) * 32);
        };
#pragma unroll
        for (int j = 0; j < 4; ++j) ld_b(0, j, bq[0][j]);
        ld_a(0, 0, aq[0]);
        ld_b(0, 4, bq[0][4]);
        ld_a(0, 1, aq[1]);
        auto tap = [&](auto tc) {
            constexpr int t = decltype(tc)::value, kx = t / 3, ky = t % 3;
            constexpr int t2 = t + 2, kx2 = t2 / 3, ky2 = t2 % 3;
            constexpr int nl = t2 < 9 ? (ky2 == 0 ? 4 : 1) + CB : 0;
            if constexpr (t2 < 9) {
                ld_a(kx2, ky2, aq[t2 % 3]);
                if constexpr (ky2 == 0) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) ld_b(kx2, j, bq[kx2 & 1][j]);
                } else {
                    ld_b(kx2, ky2 + 3, bq[kx2 & 1][ky2 + 3]);
                }
            }
#pragma unroll
            for (int c = 0; c < CB; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r][c] = mfma16(aq[t % 3][c], bq[kx & 1][ky + r], acc[r][c]);
            interleave_ds_mfma<nl, 4 * CB>();
        };
        tap(std::integral_constant<int, 0>{});
        tap(std::integral_constant<int, 1>{});
        tap(std::integral_constant<int, 2>{});
        tap(std::integral_constant<int, 3>{});
        tap(std::integral_constant<int, 4>{});
        tap(std::integral_constant<int, 5>{});
        tap(std::integral_constant<int, 6>{});
        tap(std::integral_constant<int, 7>{});
        tap(std::integral_constant<int, 8>{});
    }
    // per-lane constants of the epilogue, loaded once: bias (and head weights) of the
    // lane's 4 x CB channels, the head's residual base of its four pixels
    float bv[CB][4], hv[HEAD ? CB : 1][4], xr[4], hb0 = 0.f;
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[c][j] = 0.f;
    if (bias) {
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[c][j] = bias[co0 + c * 16 + kb * 4 + j];
    }
    if constexpr (HEAD) {
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) hv[c][j] = hd.w[co0 + c * 16 + kb * 4 + j];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            xr[r] = hd.xin[(size_t)((unsigned)(n * H + ty0 + wave * 4 + r) * (unsigned)Wd + (unsigned)(tx0 + l16)) *
                           (unsigned)hd.cin];
        hb0 = hd.b[0];
    }
    // byte addresses of lanes lane ^ 16 and lane ^ 32 (the head's channel-group sum)
    const int bp16 = (lane ^ 16) << 2, bp32 = (lane ^ 32) << 2;
    bf16x4 prev[POOL || UPADJ ? CB : 1];   // row r - 1 of the 2x2 block (POOL, UPADJ)
    // the mask of the lane's outputs, loaded at once (data-gradient use)
    constexpr bool MASKABLE = !RELU && !HEAD && !POOL && !UPADJ && !POOLADJ;
    bf16x4 mk[MASKABLE || UPADJ ? 4 : 1][MASKABLE || UPADJ ? CB : 1];
    const bool up_part = UPADJ && co0 < Cu;   // workgroup-uniform
    if constexpr (UPADJ) {
        const int cs = Co - Cu;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int y = ty0 + wave * 4 + r, x = tx0 + l16;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                if (up_part) {
                    // the pooled position of rows r - 1, r (r odd)
                    if ((r & 1) && Mask2)
                        mk[r][c] = *reinterpret_cast<const bf16x4*>(
                            Mask2 + (((size_t)n * (H / 2) + y / 2) * (Wd / 2) + x / 2) * Cu + co0 + c * 16 + kb * 4);
                } else if (Mask) {
                    mk[r][c] = *reinterpret_cast<const bf16x4*>(
                        Mask + (((size_t)n * H + y) * Wd + x) * cs + (co0 - Cu) + c * 16 + kb * 4);
                }
            }
        }
    }
    if constexpr (MASKABLE) {
        if (Mask) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    mk[r][c] = *reinterpret_cast<const bf16x4*>(
                        Mask + (size_t)((unsigned)(n * H + ty0 + wave * 4 + r) * (unsigned)Wd + (unsigned)(tx0 + l16)) *
                                   Co + co0 + c * 16 + kb * 4);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int y = ty0 + wave * 4 + r, x = tx0 + l16;
        const size_t pix = (unsigned)(n * H + y) * (unsigned)Wd + (unsigned)x;   // N H W < 2^31
        float part = 0.f;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int co = co0 + c * 16 + kb * 4;
            bf16x4 o;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float v = acc[r][c][j] + bv[c][j];
                if (RELU) v = v > 0.f ? v : 0.f;
                o[j] = (__bf16)v;
                if constexpr (HEAD) part += hv[c][j] * (float)o[j];
            }
            if constexpr (MASKABLE) {
                if (Mask) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) o[j] = (float)mk[r][c][j] > 0.f ? o[j] : (__bf16)0.f;
                }
            }
            if constexpr (POOLADJ) {
#pragma unroll
                for (int ab = 0; ab < 4; ++ab) {
                    const size_t off =
                        (((size_t)n * 2 * H + 2 * y + (ab >> 1)) * (2 * (size_t)Wd) + 2 * x + (ab & 1)) * Co + co;
                    const bf16x4 old = *reinterpret_cast<const bf16x4*>(Y + off);
                    bf16x4 q;
#pragma unroll
                    for (int j = 0; j < 4; ++j) q[j] = (__bf16)(0.25f * (float)o[j] + (float)old[j]);
                    if (Mask) {
                        const bf16x4 m = *reinterpret_cast<const bf16x4*>(Mask + off);
#pragma unroll
                        for (int j = 0; j < 4; ++j) q[j] = (float)m[j] > 0.f ? q[j] : (__bf16)0.f;
                    }
                    *reinterpret_cast<bf16x4*>(Y + off) = q;
                }
                continue;
            }
            if constexpr (UPADJ) {
                if (up_part) {
                    if ((r & 1) == 0) {
                        prev[c] = o;
                    } else {
                        // even lanes: ((a + b) + c) + d, a and b the upper row
                        bf16x4 q;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float a = (float)prev[c][j], lo = (float)o[j];
                            q[j] = (__bf16)(((a + lane_xor1(a)) + lo) + lane_xor1(lo));
                            if (Mask2) q[j] = (float)mk[r][c][j] > 0.f ? q[j] : (__bf16)0.f;
                        }
                        if ((l16 & 1) == 0)
                            *reinterpret_cast<bf16x4*>(Yp + (((size_t)n * (H / 2) + y / 2) * (Wd / 2) + x / 2) * Cu +
                                                       co) = q;
                    }
                } else {
                    if (Mask) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) o[j] = (float)mk[r][c][j] > 0.f ? o[j] : (__bf16)0.f;
                    }
                    *reinterpret_cast<bf16x4*>(Y + (((size_t)n * H + y) * Wd + x) * (Co - Cu) + (co - Cu)) = o;
                }
                continue;
            }
            if (!HEAD || Y) *reinterpret_cast<bf16x4*>(Y + pix * Co + co) = o;
            if constexpr (POOL) {
                if ((r & 1) == 0) {
                    prev[c] = o;
                } else {
                    // even lanes: ((a + b) + (c + d)) with a, b the upper row, c, d this one
                    bf16x4 q;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float up = (float)prev[c][j], lo = (float)o[j];
                        q[j] = (__bf16)(0.25f * ((up + lane_xor1(up)) + (lo + lane_xor1(lo))));
                    }
                    if ((l16 & 1) == 0)
                        *reinterpret_cast<bf16x4*>(Yp + (((size_t)n * (H / 2) + y / 2) * (Wd / 2) + x / 2) * Co + co) = q;
                }
            }
        }
        if constexpr (HEAD) {
            // lanes l16, l16 + 16, l16 + 32, l16 + 48 hold the four channel groups of one pixel
            part += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(bp16, __builtin_bit_cast(int, part)));
            part += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(bp32, __builtin_bit_cast(int, part)));
            if (kb == 0) hd.out[pix] = xr[r] + hd.scale * (hb0 + part);
        }
    }
}

// ---------------------------------------------------------------------------
// The network's first convolution (at most 8 real input channels) with its K
// packed.  The generic kernel pads the input to 32 channels and runs 9 taps x
// 32 channels, of which at most 9 x 8 carry data; here K = 12 taps x 8
// channels (taps 9..11 zero): three matrix-core K-steps instead of nine.  In
// K-step s, lane group kb holds tap t = 4 s + kb (t = 3 ky + kx) and its 8
// channels.  Wk is [Co][12][8] BF16 (zero past the real channels and taps).
// The input is either the packed tensor X (channel stride Cs, its first 8
// channels read) or, with X null, phi[N][H][W] (FP32) and the constant
// conditioning values cond[0..ncond) (device), rounded to BF16 as the packing
// rounds them: both forms give the same bits.  32 output channels per
// workgroup over a 16-column, TH-row pixel tile (the weights are staged once
// for it; each wave takes TH / 4 rows, four at a time); bias and ReLU in the
// epilogue; the result fragment of a lane is as in conv3_fwd_k.
// ---------------------------------------------------------------------------
template <int TH>
__global__ __launch_bounds__(256, 2) void conv3_first_k(const __bf16* __restrict__ X, int Cs,
                                                       const float* __restrict__ phi, const float* __restrict__ cond,
                                                       int ncond, const __bf16* __restrict__ Wk,
                                                       const float* __restrict__ bias, __bf16* __restrict__ Y, int H,
                                                       int Wd, int Co) {
    constexpr int CB = 2, RPW = TH / 4;
    __shared__ __align__(16) __bf16 sx[(TH + 2) * 18 * 8];
    __shared__ __align__(16) __bf16 sw[32 * 12 * 8];
    const int tiles_x = Wd / 16, tiles_y = H / TH;
    int b = blockIdx.x;
    const int tx0 = (b % tiles_x) * 16;
    b /= tiles_x;
    const int ty0 = (b % tiles_y) * TH;
    const int n = b / tiles_y;
    const int co0 = blockIdx.y * 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, kb = lane >> 4;
    for (int q = threadIdx.x; q < (TH + 2) * 18; q += 256) {
        const int py = q / 18, px = q - py * 18;
        const int y = wrap(ty0 - 1 + py, H), x = wrap(tx0 - 1 + px, Wd);
        const size_t p = ((size_t)n * H + y) * Wd + x;
        bf16x8 v;
        if (X) {
            v = *reinterpret_cast<const bf16x8*>(X + p * Cs);
        } else {
            v[0] = (__bf16)phi[p];
#pragma unroll
            for (int c = 1; c < 8; ++c) v[c] = (__bf16)(c <= ncond ? cond[c - 1] : 0.f);
        }
        *reinterpret_cast<bf16x8*>(sx + q * 8) = v;
    }
    for (int q = threadIdx.x; q < 32 * 12; q += 256)
        *reinterpret_cast<bf16x8*>(sw + q * 8) = *reinterpret_cast<const bf16x8*>(Wk + ((size_t)co0 * 12 + q) * 8);
    __syncthreads();
    // the lane's A fragments of the three K-steps, and its bias values
    bf16x8 a[3][CB];
    float bv[CB][4];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int c = 0; c < CB; ++c)
            a[s][c] = *reinterpret_cast<const bf16x8*>(sw + ((c * 16 + l16) * 12 + 4 * s + kb) * 8);
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[c][j] = bias ? bias[co0 + c * 16 + kb * 4 + j] : 0.f;
    for (int g = 0; g < RPW / 4; ++g) {
        const int r0 = wave * RPW + g * 4;    // first of the four rows (tile coordinates)
        f32x4 acc[4][CB];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < CB; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int t = 4 * s + kb;
            const int ky = t / 3, kx = t - 3 * (t / 3);
            bf16x8 bq[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (t < 9) {
                    bq[r] = *reinterpret_cast<const bf16x8*>(sx + ((r0 + r + ky) * 18 + l16 + kx) * 8);
                } else {
#pragma unroll
                    for (int c = 0; c < 8; ++c) bq[r][c] = (__bf16)0.f;
                }
            }
#pragma unroll
            for (int c = 0; c < CB; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r][c] = mfma16(a[s][c], bq[r], acc[r][c]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int y = ty0 + r0 + r, x = tx0 + l16;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                bf16x4 o;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float v = acc[r][c][j] + bv[c][j];
                    o[j] = (__bf16)(v > 0.f ? v : 0.f);
                }
                *reinterpret_cast<bf16x4*>(Y + (((size_t)n * H + y) * Wd + x) * Co + co0 + c * 16 + kb * 4) = o;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The first encoder block at 32 channels, fused for inference:
//   a = relu(conv3_first(phi, cond) + b1)   (the K-packed first convolution)
//   E = relu(conv3(a) + b2), P = its 2x2 average
// with a kept in LDS.  A workgroup stages both layers' weights once and then
// takes NT 16 x 16 output tiles stacked in y, one after the other: per tile, a
// is formed over the tile and its 1-pixel halo (18 x 18: each row as two
// 16-pixel segments, columns 0..15 and 2..17, the second storing only 16 and
// 17) from a 20 x 20 tile of phi (loaded into registers while the previous
// tile's second convolution runs), then the second convolution runs on it as
// conv3_fwd_k does on its staged input (taps in the same order, one 32-channel
// chunk) with the pooling epilogue.  Every value is formed with the same
// operations in the same order as the two separate launches, so E and P are
// bitwise theirs; the block's intermediate a never reaches HBM.
// W1k: [32][12][8] (pack flip 2), W2: [32][9][32] (the generic packed layout).
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(256, 3) void conv3_pair0_k(const float* __restrict__ phi, const float* __restrict__ cond,
                                                       int ncond, const __bf16* __restrict__ W1k,
                                                       const float* __restrict__ b1, const __bf16* __restrict__ W2,
                                                       const float* __restrict__ b2, __bf16* __restrict__ E,
                                                       __bf16* __restrict__ P, int H, int Wd) {
    constexpr int CB = 2;
    constexpr int NPQ = (20 * 20 + 255) / 256;   // phi values per thread and tile
    __shared__ __align__(16) __bf16 sphi[20 * 20 * 8];
    __shared__ __align__(16) __bf16 sa[18 * 18 * 32];
    __shared__ __align__(16) __bf16 sw1[32 * 12 * 8];
    __shared__ __align__(16) __bf16 sw2[9 * 32 * 32];
    const int tiles_x = Wd / 16, groups_y = H / (16 * NT);
    int b = blockIdx.x;
    const int tx0 = (b % tiles_x) * 16;
    b /= tiles_x;
    const int gy0 = (b % groups_y) * 16 * NT;
    const int n = b / groups_y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, kb = lane >> 4;
    float pv[NPQ];
    auto load_phi = [&](int ty0) {
#pragma unroll
        for (int i = 0; i < NPQ; ++i) {
            const int q = (int)threadIdx.x + i * 256;
            if (q < 20 * 20) {
                const int py = q / 20, px = q - py * 20;
                const int y = wrap(ty0 - 2 + py, H), x = wrap(tx0 - 2 + px, Wd);
                pv[i] = phi[(unsigned)(n * H + y) * (unsigned)Wd + (unsigned)x];   // N H W < 2^31
            }
        }
    };
    load_phi(gy0);
    for (int q = threadIdx.x; q < 32 * 12; q += 256)
        *reinterpret_cast<bf16x8*>(sw1 + q * 8) = *reinterpret_cast<const bf16x8*>(W1k + (size_t)q * 8);
    // second convolution's weights as conv3_fwd_k stages them: row tap * 32 + co
    for (int q = threadIdx.x; q < 9 * 32 * 4; q += 256) {
        const int row = q >> 2, part = q & 3;
        const int tap = row / 32, co = row - tap * 32;
        *reinterpret_cast<bf16x8*>(sw2 + lds_part(row, part)) =
            *reinterpret_cast<const bf16x8*>(W2 + ((size_t)co * 9 + tap) * 32 + part * 8);
    }
    // the first layer's input vector of a pixel: bf16(phi), the conditioning values, zeros
    bf16x8 cv;
    cv[0] = (__bf16)0.f;
#pragma unroll
    for (int c = 1; c < 8; ++c) cv[c] = (__bf16)(c <= ncond ? cond[c - 1] : 0.f);
    __syncthreads();
    bf16x8 a1[3][CB];
    float bv1[CB][4], bv[CB][4];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int c = 0; c < CB; ++c)
            a1[s][c] = *reinterpret_cast<const bf16x8*>(sw1 + ((c * 16 + l16) * 12 + 4 * s + kb) * 8);
    const int la = lds_part(l16, kb);   // A row tap * 32 + 16 c + l16 has the swizzle term of row l16
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            bv1[c][j] = b1 ? b1[c * 16 + kb * 4 + j] : 0.f;
            bv[c][j] = b2 ? b2[c * 16 + kb * 4 + j] : 0.f;
        }
    // Stage 1 work of a wave: halo rows r = wave / 2 + 2 i (i = 0..8), column
    // segment c0 = 2 (wave & 1) of width 16 (the two segments of a row overlap
    // in columns 2..15; the second stores only columns 16, 17).  Its sphi reads
    // (tap t = 4 s + kb of the packed K) sit at fixed offsets from the lane's
    // base; its sa row p = (wave / 2 + 2 i) 18 + c0 + l16 has the swizzle term
    // ((p0 >> 1) + 2 i) & 3 with p0 the row at i = 0, so two lane bases serve
    // the nine rows.  Stage 2 reads rows P0 + l16, P0 = 72 wave + 18 j + kx,
    // whose swizzle term is fixed by (18 j + kx) mod 8: eight lane bases.
    const int c0 = (wave & 1) * 2, r0 = wave >> 1;
    int sp[3];
    bool tz[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int t = 4 * s + kb, ky = t / 3, kx = t - 3 * (t / 3);
        tz[s] = t >= 9;
        sp[s] = ((r0 + (t < 9 ? ky : 0)) * 20 + c0 + l16 + (t < 9 ? kx : 0)) * 8;
    }
    const int col = c0 + l16;
    const bool st1 = c0 == 0 || col >= 16;
    int sab[CB][2];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p0 = r0 * 18 + col, part = 2 * c + (kb >> 1);
            sab[c][h] = p0 * 32 + ((part ^ (((p0 >> 1) + 2 * h) & 3)) << 3) + (kb & 1) * 4;
        }
    int lbb[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) lbb[r] = (wave * 72 + l16) * 32 + ((kb ^ (((r + l16) >> 1) & 3)) << 3);
    for (int it = 0; it < NT; ++it) {
        const int ty0 = gy0 + 16 * it;
        if (it > 0) __syncthreads();              // every wave is done with the previous tile's sphi, sa
#pragma unroll
        for (int i = 0; i < NPQ; ++i) {
            const int q = (int)threadIdx.x + i * 256;
            if (q < 20 * 20) {
                bf16x8 v = cv;
                v[0] = (__bf16)pv[i];
                *reinterpret_cast<bf16x8*>(sphi + q * 8) = v;
            }
        }
        __syncthreads();
        if (it + 1 < NT) load_phi(ty0 + 16);   // the next tile's phi in flight during this one
        // ---- stage 1: a over the 18 x 18 halo tile (36 row segments, 9 per wave) ----
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            f32x4 acc[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                bf16x8 bq = *reinterpret_cast<const bf16x8*>(sphi + sp[s] + i * 2 * 20 * 8);
                if (s == 2 && tz[2]) {   // taps 9..11 exist only in K-step 2
#pragma unroll
                    for (int c = 0; c < 8; ++c) bq[c] = (__bf16)0.f;
                }
#pragma unroll
                for (int c = 0; c < CB; ++c) acc[c] = mfma16(a1[s][c], bq, acc[c]);
            }
            if (st1) {
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    bf16x4 o;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float v = acc[c][j] + bv1[c][j];
                        o[j] = (__bf16)(v > 0.f ? v : 0.f);
                    }
                    // channels c * 16 + 4 kb .. + 3: 16-byte part 2 c + kb / 2, half kb & 1
                    *reinterpret_cast<bf16x4*>(sa + sab[c][i & 1] + i * 36 * 32) = o;
                }
            }
        }
        __syncthreads();
        // ---- stage 2: the second convolution over the output tile, taps t = 3 kx + ky ----
        f32x4 acc[4][CB];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < CB; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            bf16x8 bq[6];   // rows wave * 4 + j at column l16 + kx; tap (kx, ky) uses rows ky..ky+3
#pragma unroll
            for (int j = 0; j < 6; ++j)
                bq[j] = *reinterpret_cast<const bf16x8*>(sa + lbb[(18 * j + kx) & 7] + (18 * j + kx) * 32);
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
                bf16x8 aq[CB];
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    aq[c] = *reinterpret_cast<const bf16x8*>(sw2 + la + ((ky * 3 + kx) * 32 + c * 16) * 32);
#pragma unroll
                for (int c = 0; c < CB; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r][c] = mfma16(aq[c], bq[ky + r], acc[r][c]);
            }
        }
        bf16x4 prev[CB];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int y = ty0 + wave * 4 + r, x = tx0 + l16;
            const size_t pix = (unsigned)(n * H + y) * (unsigned)Wd + (unsigned)x;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int co = c * 16 + kb * 4;
                bf16x4 o;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float v = acc[r][c][j] + bv[c][j];
                    v = v > 0.f ? v : 0.f;
                    o[j] = (__bf16)v;
                }
                *reinterpret_cast<bf16x4*>(E + pix * 32 + co) = o;
                if ((r & 1) == 0) {
                    prev[c] = o;
                } else {
                    // even lanes: ((a + b) + (c + d)) with a, b the upper row, c, d this one
                    bf16x4 q;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float up = (float)prev[c][j], lo = (float)o[j];
                        q[j] = (__bf16)(0.25f * ((up + lane_xor1(up)) + (lo + lane_xor1(lo))));
                    }
                    if ((l16 & 1) == 0)
                        *reinterpret_cast<bf16x4*>(
                            P + (size_t)((unsigned)(n * (H / 2) + y / 2) * (unsigned)(Wd / 2) + (unsigned)(x / 2)) * 32 +
                            co) = q;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient of the 3x3 convolution on the matrix cores:
//   P[s][co][tap][ci] = sum over the pixels of split s of dY[p][co] X[p + tap][ci]
// GEMM per tap: M = co, N = ci, K = pixels.  Per 16x16 pixel tile the
// workgroup copies, channels-last as in HBM, the tile's dY (TCO channels) and
// the X halo (18 x 18 pixels, 16 channels of the ci block) into LDS with
// 16-byte stores.  The operands need 8 pixels of one channel per lane;
// gfx950's transposing LDS read (ds_read_b64_tr_b16) delivers them: in a group
// of 16 lanes, lane m reads 4 channels (4 (m & 3) ..) of pixel pb + m/4, and
// lane i receives channel i of pixels pb .. pb + 3.  Two such reads (four
// pixels of a row, then the same four of the next row) give one operand.  The A operand (dY) of a K step serves all nine taps.  The next
// tile's global loads are in flight during the MFMAs.  Wave w owns output
// channels 16w..16w+15 and all 9 taps of a 16-channel ci block.  Splits are
// reduced by wgrad_reduce_k (fixed order: deterministic).  With bpart, the
// workgroups of the first ci block also form the bias gradient's split
// partials bpart[s][co] = sum over the split's pixels of dY[p][co]: each thread
// always stages the same 8 channels and sums them in tile order, then a fixed
// order over the threads of a channel (reduced over splits by wgrad_reduce_k).
// UPCAT: X is the channel concatenation [nearest 2x upsampling of X (Cu
// channels, H/2 x Wd/2), X2 (Ci - Cu channels)], read from its two sources;
// a 16-channel ci block lies in one of them (Cu is a multiple of 32).
// ---------------------------------------------------------------------------
typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x4 lds_read_tr(const __bf16* p) {
    const s16x4 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4*)p);
    return __builtin_bit_cast(bf16x4, v);
}

__device__ __forceinline__ bf16x8 cat8(const bf16x4& a, const bf16x4& b) {
    return bf16x8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
}

template <int TCO, bool UPCAT>
__global__ __launch_bounds__(TCO * 4) void conv3_dw_k(const __bf16* __restrict__ X, const __bf16* __restrict__ dY,
                                                      float* __restrict__ part, int N, int H, int Wd, int Ci, int Co,
                                                      int S, float* __restrict__ bpart,
                                                      const __bf16* __restrict__ X2, int Cu) {
    constexpr int NT = TCO * 4;          // 64 threads (one wave) per 16 output channels
    // LDS strides (bf16) of one dY pixel and one X halo pixel, chosen by
    // measurement (SQ_LDS_BANK_CONFLICT per LDS-active cycle): with the K steps
    // over row spans, 80 / 16 leave the 64-channel kernel without conflicts
    // (72: 0.12) and 32 / 16 the 32-channel one at 0.11 (48: 0.21); the time
    // differs by about 1 % between these (before the row spans: 0.43)
    constexpr int SP = TCO == 64 ? 80 : 32;
    constexpr int SXP = 16;
    constexpr int NYQ = 256 * TCO / 8, NYI = NYQ / NT;           // dY 16-byte chunks (NYI = 8 per thread)
    constexpr int NXQ = 18 * 18 * 2, NXI = (NXQ + NT - 1) / NT;  // X halo chunks, the last item guarded
    __shared__ __align__(16) __bf16 sdy[256 * SP];
    __shared__ __align__(16) __bf16 sx[18 * 18 * SXP];
    const int s = blockIdx.x;
    const int co0 = blockIdx.y * TCO;
    const int ci0 = blockIdx.z * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, kb = lane >> 4;
    const int tiles_x = Wd / 16, tiles_y = H / 16, ntiles = N * tiles_x * tiles_y;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ry[NYI], rx[NXI];
    const bool bsum = bpart != nullptr && blockIdx.z == 0;
    float csum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // channels co0 + 8 (tid % (TCO / 8)) + e
    // dY chunk q = threadIdx.x + NT i is pixel q / (TCO / 8) of the tile (row
    // dyr + 2 i, column dyc) and channels 8 (q % (TCO / 8)): a lane-constant
    // offset from the tile's first pixel plus i rows of two.  Pixel indices
    // are 32-bit (the launcher requires N H W < 2^31).
    const int dyr = (int)threadIdx.x / (16 * TCO / 8), dyc = ((int)threadIdx.x / (TCO / 8)) & 15;
    const unsigned dych = co0 + ((int)threadIdx.x % (TCO / 8)) * 8;
    auto load_tile = [&](int tile) {
        int b = tile;
        const int tx0 = (b % tiles_x) * 16;
        b /= tiles_x;
        const int ty0 = (b % tiles_y) * 16;
        const int n = b / tiles_y;
        const __bf16* py0 = dY + (size_t)((unsigned)(n * H + ty0 + dyr) * (unsigned)Wd + (unsigned)(tx0 + dyc)) * Co + dych;
#pragma unroll
        for (int i = 0; i < NYI; ++i)
            ry[i] = *reinterpret_cast<const bf16x8*>(py0 + (size_t)i * 2 * Wd * Co);
#pragma unroll
        for (int i = 0; i < NXI; ++i) {
            const int q = (int)threadIdx.x + i * NT;
            if (q < NXQ) {
                const int hp = q >> 1, ch = q & 1;
                const int y = wrap(ty0 - 1 + hp / 18, H), x = wrap(tx0 - 1 + hp % 18, Wd);
                const __bf16* src;
                if constexpr (UPCAT) {
                    src = ci0 < Cu ? X + (size_t)((unsigned)(n * (H / 2) + (y >> 1)) * (unsigned)(Wd / 2) +
                                                  (unsigned)(x >> 1)) * Cu + ci0 + ch * 8
                                   : X2 + (size_t)((unsigned)(n * H + y) * (unsigned)Wd + (unsigned)x) * (Ci - Cu) +
                                         (ci0 - Cu) + ch * 8;
                } else {
                    src = X + (size_t)((unsigned)(n * H + y) * (unsigned)Wd + (unsigned)x) * Ci + ci0 + ch * 8;
                }
                rx[i] = *reinterpret_cast<const bf16x8*>(src);
            }
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int i = 0; i < NYI; ++i) {
            const int q = (int)threadIdx.x + i * NT;
            *reinterpret_cast<bf16x8*>(sdy + (q / (TCO / 8)) * SP + (q % (TCO / 8)) * 8) = ry[i];
        }
        if (bsum) {
#pragma unroll
            for (int i = 0; i < NYI; ++i)
#pragma unroll
                for (int e = 0; e < 8; ++e) csum[e] += (float)ry[i][e];
        }
#pragma unroll
        for (int i = 0; i < NXI; ++i) {
            const int q = (int)threadIdx.x + i * NT;
            if (q < NXQ) *reinterpret_cast<bf16x8*>(sx + (q >> 1) * SXP + (q & 1) * 8) = rx[i];
        }
    };
    // lane m = l16 of its group reads channels 4 (m & 3) .. of pixel (group base) + m / 4
    const int mp = l16 >> 2, mc = (l16 & 3) * 4;
    if (s < ntiles) load_tile(s);
    for (int tile = s; tile < ntiles; tile += S) {
        __syncthreads();                          // every wave is done with the previous tile
        store_tile();
        __syncthreads();
        if (tile + S < ntiles) load_tile(tile + S);
#pragma unroll
        for (int py = 0; py < 16; py += 2) {
            // a K step is the 32 pixels of tile rows py and py + 1; lane group kb takes
            // columns 4 kb .. 4 kb + 3 of both rows, so that each transposing read of a
            // wave covers 16 consecutive pixels of one row (one contiguous span of the
            // halo tile: free of bank conflicts)
            const __bf16* pa = sdy + (py * 16 + kb * 4 + mp) * SP + wave * 16 + mc;
            const bf16x8 a = cat8(lds_read_tr(pa), lds_read_tr(pa + 16 * SP));
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3 - 1, dx = tap % 3 - 1;
                const __bf16* pb = sx + ((py + 1 + dy) * 18 + kb * 4 + 1 + dx + mp) * SXP + mc;
                const bf16x8 bb = cat8(lds_read_tr(pb), lds_read_tr(pb + 18 * SXP));
                acc[tap] = mfma16(a, bb, acc[tap]);
            }
        }
    }
    // lane holds ci = ci0 + l16, co = co0 + 16*wave + 4*kb + j
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = co0 + wave * 16 + kb * 4 + j;
            part[(((size_t)s * Co + co) * 9 + tap) * Ci + ci0 + l16] = acc[tap][j];
        }
    if (bsum) {
        // the 32 threads tid = g + k TCO / 8 (k = 0..31) hold channels 8 g .. 8 g + 7
        __syncthreads();                          // every wave is done reading sdy
        float* red = reinterpret_cast<float*>(sdy);   // NT x 8 floats <= the dY tile's bytes
#pragma unroll
        for (int e = 0; e < 8; ++e) red[threadIdx.x * 8 + e] = csum[e];
        __syncthreads();
        if ((int)threadIdx.x < TCO) {
            const int g = threadIdx.x >> 3, e = threadIdx.x & 7;
            float v = 0.f;
            for (int k = 0; k < NT / (TCO / 8); ++k) v += red[(g + k * (TCO / 8)) * 8 + e];
            bpart[(size_t)s * Co + co0 + threadIdx.x] = v;
        }
    }
}

// dW[co][ci][ky][kx] (FP32 parameter layout, only the first ci_real input
// channels) = sum_s P[s][co][tap][ci].
// dW[co][ci][tap] = sum_s part[s][co][tap][ci] (ci < ci_real).  A block owns 32
// consecutive partial entries e = (co * 9 + tap) * Ci + ci; its 8 lanes of 32
// threads take every 8th split, then a fixed-order tree adds the lanes
// (deterministic).  With bpart, the blocks past the weights reduce the bias
// gradient's split partials the same way, 32 columns per block:
// db[co] = sum_s bpart[s][co] (one launch for both).
__global__ __launch_bounds__(256) void wgrad_reduce_k(const float* __restrict__ part, float* __restrict__ dW, int S,
                                                      int Co, int Ci, int ci_real, const float* __restrict__ bpart,
                                                      float* __restrict__ db) {
    __shared__ float sh[8][32];
    const long long E = (long long)Co * 9 * Ci;
    const int el = threadIdx.x & 31, sl = threadIdx.x >> 5;
    const long long wblocks = (E + 31) / 32;
    if ((long long)blockIdx.x >= wblocks) {      // a bias block (uniform over the block)
        const int c = (int)(blockIdx.x - wblocks) * 32 + el;
        float acc = 0.f;
        if (c < Co)
            for (int s = sl; s < S; s += 8) acc += bpart[(size_t)s * Co + c];
        sh[sl][el] = acc;
        __syncthreads();
        if (sl == 0 && c < Co)
            db[c] = ((sh[0][el] + sh[1][el]) + (sh[2][el] + sh[3][el])) +
                    ((sh[4][el] + sh[5][el]) + (sh[6][el] + sh[7][el]));
        return;
    }
    const long long e = (long long)blockIdx.x * 32 + el;
    float acc = 0.f;
    if (e < E)
        for (int s = sl; s < S; s += 8) acc += part[(size_t)s * E + e];
    sh[sl][el] = acc;
    __syncthreads();
    if (sl == 0 && e < E) {
        const float v = ((sh[0][el] + sh[1][el]) + (sh[2][el] + sh[3][el])) +
                        ((sh[4][el] + sh[5][el]) + (sh[6][el] + sh[7][el]));
        const int ci = (int)(e % Ci);
        const long long r = e / Ci;
        const int tap = (int)(r % 9);
        const int co = (int)(r / 9);
        if (ci < ci_real) dW[((size_t)co * ci_real + ci) * 9 + tap] = v;
    }
}

// Column sums over pixels (bias gradients): part[s][c] = sum_{p in split s} G[p][c]
// Column sums of a row-major [P][C] BF16 matrix, optionally weighted per row
// (part[s][c] = scale sum_{p in block s} wt[p] G[p][c], and with a weight also
// part[s][C] = scale sum wt[p]).  Block s owns a contiguous range of rows;
// thread t reads 16-byte chunk t % Q (Q = C / 8) of rows t / Q, t / Q + R, ...
// (R = 256 / Q), so a wave reads whole rows; the R row-lanes of a chunk are
// then summed through LDS.  C must be a multiple of 8, at most 512.
template <bool WEIGHTED>
__global__ __launch_bounds__(256) void colsum_part_k(const __bf16* __restrict__ G, const float* __restrict__ wt,
                                                     long long P, int C, float scale, float* __restrict__ part) {
    __shared__ float sh[256 * 8];
    __shared__ float shw[256];
    const int Q = C / 8, R = 256 / Q;
    const int t = threadIdx.x, q = t % Q, r0 = t / Q;
    const long long rows = (P + gridDim.x - 1) / gridDim.x;
    const long long p0 = blockIdx.x * rows, p1 = p0 + rows < P ? p0 + rows : P;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float accw = 0.f;
    if (r0 < R) {
        for (long long p = p0 + r0; p < p1; p += R) {
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(G + p * C + q * 8);
            const float w = WEIGHTED ? wt[p] : 1.f;
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] += w * (float)v[i];
            if (WEIGHTED) accw += w;
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) sh[t * 8 + i] = acc[i];
    shw[t] = (q == 0 && r0 < R) ? accw : 0.f;
    __syncthreads();
    // element c of a chunk-row lives at sh[(r * Q + c / 8) * 8 + c % 8] = sh[r * C + c]
    for (int c = t; c < C; c += 256) {
        float sum = 0.f;
        for (int r = 0; r < R; ++r) sum += sh[r * C + c];
        part[(size_t)blockIdx.x * (C + (WEIGHTED ? 1 : 0)) + c] = scale * sum;
    }
    if (WEIGHTED && t == 0) {
        float sum = 0.f;
        for (int k = 0; k < 256; ++k) sum += shw[k];
        part[(size_t)blockIdx.x * (C + 1) + C] = scale * sum;
    }
}

// out[c] = sum_s part[s][c] for c < C: a block owns 4 columns; 64 lanes per
// column take every 64th split, then a fixed-order tree (deterministic).
__global__ __launch_bounds__(256) void colsum_reduce_k(const float* __restrict__ part, int S, int C,
                                                       float* __restrict__ out) {
    __shared__ float sh[4][64];
    const int cl = threadIdx.x & 3, sl = threadIdx.x >> 2;
    const int c = blockIdx.x * 4 + cl;
    float acc = 0.f;
    if (c < C)
        for (int s = sl; s < S; s += 64) acc += part[(size_t)s * C + c];
    sh[cl][sl] = acc;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (sl < w) sh[cl][sl] += sh[cl][sl + w];
        __syncthreads();
    }
    if (sl == 0 && c < C) out[c] = sh[cl][0];
}

// ----------------------------------------------------------- weight packing
// master W[co][ci][3][3] (FP32) -> Wt[co][tap][cip] (BF16, zero padded ci)
__global__ void pack_w_k(const float* __restrict__ W, __bf16* __restrict__ Wt, int Co, int Ci, int Cip) {
    const long long total = (long long)Co * 9 * Cip;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int ci = (int)(i % Cip);
        const int tap = (int)((i / Cip) % 9);
        const int co = (int)(i / (9LL * Cip));
        Wt[i] = (__bf16)(ci < Ci ? W[((size_t)co * Ci + ci) * 9 + tap] : 0.f);
    }
}

// master W[co][ci][3][3] -> Wf[ci][tap'][co] = W[co][ci][8 - tap'] (the flipped,
// transposed kernel that turns the data gradient into a forward convolution)
__global__ void pack_wflip_k(const float* __restrict__ W, __bf16* __restrict__ Wf, int Co, int Ci) {
    const long long total = (long long)Ci * 9 * Co;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int co = (int)(i % Co);
        const int tp = (int)((i / Co) % 9);
        const int ci = (int)(i / (9LL * Co));
        Wf[i] = (__bf16)W[((size_t)co * Ci + ci) * 9 + (8 - tp)];
    }
}

// Every layer's packing in one launch: grid row s (blockIdx.y) writes out[s]
// either as pack_w_k (flip 0) or as pack_wflip_k (flip 1) from W[s]; end[]
// holds the cumulative element counts.
__global__ void pack_all_k(const PackAll t) {
    const int sg = blockIdx.y;
    const long long n = t.end[sg] - (sg ? t.end[sg - 1] : 0);
    for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n;
         j += (long long)gridDim.x * blockDim.x) {
        const int Co = t.co[sg], Ci = t.ci[sg];
        if (t.flip[sg] == 2) {
            // first layer, K packed: out[co][t][c], 12 taps x 8 channels, zero past the real ones
            const int c = (int)(j % 8), tp = (int)((j / 8) % 12), co = (int)(j / 96);
            t.out[sg][j] = (__bf16)(tp < 9 && c < Ci ? t.W[sg][((size_t)co * Ci + c) * 9 + tp] : 0.f);
        } else if (!t.flip[sg]) {
            const int Cip = t.cip[sg];
            const int ci = (int)(j % Cip), tap = (int)((j / Cip) % 9), co = (int)(j / (9LL * Cip));
            t.out[sg][j] = (__bf16)(ci < Ci ? t.W[sg][((size_t)co * Ci + ci) * 9 + tap] : 0.f);
        } else {
            const int co = (int)(j % Co), tp = (int)((j / Co) % 9), ci = (int)(j / (9LL * Co));
            t.out[sg][j] = (__bf16)t.W[sg][((size_t)co * Ci + ci) * 9 + (8 - tp)];
        }
    }
}

// ------------------------------------------------------------- elementwise
// Every activation tensor is [pixels][C] BF16 with C a multiple of 8: these
// kernels move 8 channels (16 bytes) per thread and index by chunk.

// fp32 [P][cin] -> bf16 [P][cpad] (zero padded channels)
__global__ void pack_input_k(const float* __restrict__ x, __bf16* __restrict__ out, long long P, int cin, int cpad) {
    const int Q = cpad / 8;
    const long long n = P * Q;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long p = i / Q;
        const int c0 = (int)(i - p * Q) * 8;
        bf16x8 v;
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (__bf16)(c0 + k < cin ? x[p * cin + c0 + k] : 0.f);
        *reinterpret_cast<bf16x8*>(out + p * cpad + c0) = v;
    }
}

// Surrogate input for a single field: channel 0 = phi (fp32), channels
// 1..ncond = constant conditioning values, rest zero.  Also writes the fp32
// copy of phi used by the residual head (xin with one channel).
__global__ void pack_phi_cond_k(const float* __restrict__ phi, const float* __restrict__ cond, int ncond,
                                __bf16* __restrict__ out, float* __restrict__ xin, long long P, int cpad) {
    const int Q = cpad / 8;
    const long long n = P * Q;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long p = i / Q;
        const int c0 = (int)(i - p * Q) * 8;
        bf16x8 v;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = c0 + k;
            float f = 0.f;
            if (c == 0) {
                f = phi[p];
                xin[p] = f;
            } else if (c <= ncond) {
                f = cond[c - 1];
            }
            v[k] = (__bf16)f;
        }
        *reinterpret_cast<bf16x8*>(out + p * cpad + c0) = v;
    }
}

// ReLU backward folded into a gradient's producer: v where the stored
// post-activation m is positive, else 0 (no-op for a null mask)
__device__ __forceinline__ bf16x8 relu_mask8(const bf16x8 v, const __bf16* __restrict__ mask, long long off) {
    if (!mask) return v;
    const bf16x8 m = *reinterpret_cast<const bf16x8*>(mask + off);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (float)m[k] > 0.f ? v[k] : (__bf16)0.f;
    return o;
}

// head: out[p] = phi[p] + scale (b + sum_c w[c] d[p][c])   (phi = input channel 0, fp32)
__global__ void head_fwd_k(const __bf16* __restrict__ d, const float* __restrict__ w, const float* __restrict__ b,
                           const float* __restrict__ xin, int cin, float* __restrict__ out, long long P, int C,
                           float scale) {
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
        float acc = b[0];
        for (int c0 = 0; c0 < C; c0 += 8) {
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(d + p * C + c0);
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += w[c0 + k] * (float)v[k];
        }
        out[p] = xin[p * cin] + scale * acc;
    }
}

// data gradient of the 1x1 head: dd[p][c] = scale g[p] w[c] (8 channels per thread)
__global__ void head_dd_k(const float* __restrict__ g, const float* __restrict__ w, __bf16* __restrict__ dd,
                          long long P, int C, float scale, const __bf16* __restrict__ mask) {
    const int Q = C / 8;
    const long long n = P * Q;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long p = i / Q;
        const int q = (int)(i - p * Q);
        const float gs = scale * g[p];
        bf16x8 v;
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (__bf16)(gs * w[q * 8 + k]);
        *reinterpret_cast<bf16x8*>(dd + p * C + q * 8) = relu_mask8(v, mask, p * C + q * 8);
    }
}

// masked MSE: g = 2 (pred - target) / count inside the interior, 0 outside;
// part[block] = partial sum of squared differences (float64)
__global__ void mse_k(const float* __restrict__ pred, const float* __restrict__ target, float* __restrict__ g, int N,
                      int H, int Wd, int margin, double inv_count, double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    const long long total = (long long)N * H * Wd;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % Wd);
        const int y = (int)((i / Wd) % H);
        const bool in = y >= margin && y < H - margin && x >= margin && x < Wd - margin;
        const double diff = (double)pred[i] - (double)target[i];
        g[i] = in ? (float)(2.0 * diff * inv_count) : 0.f;
        if (in) acc += diff * diff;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void sum_k(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// Adam (bias-corrected) on the FP32 master parameters.
__global__ void adam_k(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long long n, float lr, float b1, float b2, float eps, float wd, float c1, float c2) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i] + wd * w[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Training samples from a periodic field: crop q of side `crop` starts at
// (yx[2q], yx[2q+1]) and wraps.  x (nullable): [k][crop][crop][1 + ncond]
// with phi first and the constant conditioning values of the sample
// (cond[q * ncond + j]) after it; y (nullable): [k][crop][crop] phi only.
__global__ void gather_k(const float* __restrict__ field, int H, int W, const int* __restrict__ yx, int k, int crop,
                         const float* __restrict__ cond, int ncond, float* __restrict__ x, float* __restrict__ y) {
    const long long total = (long long)k * crop * crop;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int q = (int)(i / ((long long)crop * crop));
        const int r = (int)((i / crop) % crop), c = (int)(i % crop);
        int yy = (yx[2 * q] + r) % H, xx = (yx[2 * q + 1] + c) % W;
        if (yy < 0) yy += H;
        if (xx < 0) xx += W;
        const float v = field[(long long)yy * W + xx];
        if (y) y[i] = v;
        if (x) {
            float* o = x + i * (1 + ncond);
            o[0] = v;
            for (int j = 0; j < ncond; ++j) o[1 + j] = cond[q * ncond + j];
        }
    }
}

__global__ void widen_k(const __bf16* __restrict__ a, float* __restrict__ b, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// ----------------------------------------------------------------- launchers
namespace {
// the convolution kernels form pixel indices in 32 bits
bool pix_over(int N, int H, int Wd) { return (long long)N * H * Wd >= (1LL << 31); }

int grid_for(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}
}  // namespace

namespace {
template <bool UPCAT>
hipError_t conv3_fwd_any(const __bf16* X, const __bf16* X2, int Cu, const __bf16* Wt, const float* bias, __bf16* Y,
                         int N, int H, int Wd, int Ci, int Co, bool relu, hipStream_t s) {
    const int tiles = N * (H / 16) * (Wd / 16);
    // 64 output channels per workgroup unless that leaves fewer than two
    // workgroups per CU of a 256-CU part (the deep, small levels)
    if (Co % 64 == 0 && (long long)tiles * (Co / 64) >= 512) {
        dim3 grid(tiles, Co / 64);
        if (relu) conv3_fwd_k<64, true, UPCAT><<<grid, 256, 0, s>>>(X, X2, Cu, Wt, bias, Y, H, Wd, Ci, Co);
        else conv3_fwd_k<64, false, UPCAT><<<grid, 256, 0, s>>>(X, X2, Cu, Wt, bias, Y, H, Wd, Ci, Co);
    } else {
        dim3 grid(tiles, Co / 32);
        if (relu) conv3_fwd_k<32, true, UPCAT><<<grid, 256, 0, s>>>(X, X2, Cu, Wt, bias, Y, H, Wd, Ci, Co);
        else conv3_fwd_k<32, false, UPCAT><<<grid, 256, 0, s>>>(X, X2, Cu, Wt, bias, Y, H, Wd, Ci, Co);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t conv3_fwd(const __bf16* X, const __bf16* Wt, const float* bias, __bf16* Y, int N, int H, int Wd, int Ci,
                     int Co, bool relu, hipStream_t s) {
    if (pix_over(N, H, Wd)) return hipErrorInvalidValue;
    if (H % 16 || Wd % 16 || Ci % 32 || Co % 32) return hipErrorInvalidValue;
    return conv3_fwd_any<false>(X, nullptr, 0, Wt, bias, Y, N, H, Wd, Ci, Co, relu, s);
}

hipError_t conv3_fwd_masked(const __bf16* X, const __bf16* Wt, const __bf16* Mask, __bf16* Y, int N, int H, int Wd,
                            int Ci, int Co, hipStream_t s) {
    if (pix_over(N, H, Wd)) return hipErrorInvalidValue;
    if (H % 16 || Wd % 16 || Ci % 32 || Co % 32 || !Mask) return hipErrorInvalidValue;
    const int tiles = N * (H / 16) * (Wd / 16);
    if (Co % 64 == 0 && (long long)tiles * (Co / 64) >= 512)
        conv3_fwd_k<64, false, false><<<dim3(tiles, Co / 64), 256, 0, s>>>(X, nullptr, 0, Wt, nullptr, Y, H, Wd, Ci, Co,
                                                                           HeadArgs{}, nullptr, Mask);
    else
        conv3_fwd_k<32, false, false><<<dim3(tiles, Co / 32), 256, 0, s>>>(X, nullptr, 0, Wt, nullptr, Y, H, Wd, Ci, Co,
                                                                           HeadArgs{}, nullptr, Mask);
    return hipGetLastError();
}

hipError_t conv3_fwd_upadj(const __bf16* X, const __bf16* Wt, __bf16* dU, __bf16* dS, const __bf16* mask_u,
                           const __bf16* mask_s, int N, int H, int Wd, int Ci, int Cu, int Cs, hipStream_t s) {
    if (pix_over(N, H, Wd)) return hipErrorInvalidValue;
    if (H % 16 || Wd % 16 || Ci % 32 || Cu < 32 || Cu % 32 || Cs < 32 || Cs % 32 || !dU || !dS)
        return hipErrorInvalidValue;
    const int tiles = N * (H / 16) * (Wd / 16);
    const int Co = Cu + Cs;
    if (Cu % 64 == 0 && Cs % 64 == 0 && (long long)tiles * (Co / 64) >= 512)
        conv3_fwd_k<64, false, false, false, false, true><<<dim3(tiles, Co / 64), 256, 0, s>>>(
            X, nullptr, Cu, Wt, nullptr, dS, H, Wd, Ci, Co, HeadArgs{}, dU, mask_s, mask_u);
    else
        conv3_fwd_k<32, false, false, false, false, true><<<dim3(tiles, Co / 32), 256, 0, s>>>(
            X, nullptr, Cu, Wt, nullptr, dS, H, Wd, Ci, Co, HeadArgs{}, dU, mask_s, mask_u);
    return hipGetLastError();
}

hipError_t conv3_fwd_pooladj(const __bf16* X, const __bf16* Wt, __bf16* dX2, const __bf16* mask, int N, int H, int Wd,
                            int Ci, int Co, hipStream_t s) {
    if (pix_over(N, H, Wd)) return hipErrorInvalidValue;
    if (H % 16 || Wd % 16 || Ci % 32 || Co % 32 || !dX2) return hipErrorInvalidValue;
    const int tiles = N * (H / 16) * (Wd / 16);
    if (Co % 64 == 0 && (long long)tiles * (Co / 64) >= 512)
        conv3_fwd_k<64, false, false, false, false, false, true><<<dim3(tiles, Co / 64), 256, 0, s>>>(
            X, nullptr, 0, Wt, nullptr, dX2, H, Wd, Ci, Co, HeadArgs{}, nullptr, mask);
    else
        conv3_fwd_k<32, false, false, false, false, false, true><<<dim3(tiles, Co / 32), 256, 0, s>>>(
            X, nullptr, 0, Wt, nullptr, dX2, H, Wd, Ci, Co, HeadArgs{}, nullptr, mask);
    return hipGetLastError();
}

hipError_t conv3_fwd_upcat(const __bf16* U, const __bf16* Sk, const __bf16* Wt, const float* bias, __bf16* Y, int N,
                           int H, int Wd, int Cu, int Cs, int Co, bool relu, hipStream_t s) {
    if (pix_over(N, H, Wd)) return hipErrorInvalidValue;
    if (H % 16 || Wd % 16 || Cu < 32 || Cu % 32 || Cs < 32 || Cs % 32 || Co % 32) return hipErrorInvalidValue;
    return conv3_fwd_any<true>(U, Sk, Cu, Wt, bias, Y, N, H, Wd, Cu + Cs, Co, relu, s);
}

hipError_t conv3_fwd_relu_pool(const __bf16* X, const __bf16* Wt, const float* bias, __bf16* Y, __bf16* Yp, int N, int H,
                               int Wd, int Ci, int Co, hipStream_t s) {
    if (pix_over(N, H, Wd)) return hipErrorInvalidValue;
    if (H % 16 || Wd % 16 || Ci % 32 || Co % 32 || !Y || !Yp) return hipErrorInvalidValue;
    const int tiles = N * (H / 16) * (Wd / 16);
    if (Co % 64 == 0 && (long long)tiles * (Co / 64) >= 512) {
        conv3_fwd_k<64, true, false, false, true><<<dim3(tiles, Co / 64), 256, 0, s>>>(X, nullptr, 0, Wt, bias, Y, H,
                                                                                      Wd, Ci, Co, HeadArgs{}, Yp);
    } else {
        conv3_fwd_k<32, true, false, false, true><<<dim3(tiles, Co / 32), 256, 0, s>>>(X, nullptr, 0, Wt, bias, Y, H,
                                                                                      Wd, Ci, Co, HeadArgs{}, Yp);
    }
    return hipGetLastError();
}

hipError_t conv3_first(const __bf16* X, int Cs, const float* phi, const float* cond, int ncond, const __bf16* Wk,
                       const float* bias, __bf16* Y, int N, int H, int Wd, int Co, hipStream_t s) {
    if (H % 16 || Wd % 16 || Co % 32 || ncond < 0 || ncond > 7 || (X ? (Cs < 8 || Cs % 8) : (!phi || (ncond && !cond))))
        return hipErrorInvalidValue;
    // 64-row tiles where H allows (the weights staged once per 1024 pixels), else 16
    if (H % 64 == 0)
        conv3_first_k<64><<<dim3(N * (H / 64) * (Wd / 16), Co / 32), 256, 0, s>>>(X, Cs, phi, cond, ncond, Wk, bias,
                                                                               Y, H, Wd, Co);
    else
        conv3_first_k<16><<<dim3(N * (H / 16) * (Wd / 16), Co / 32), 256, 0, s>>>(X, Cs, phi, cond, ncond, Wk, bias,
                                                                               Y, H, Wd, Co);
    return hipGetLastError();
}

hipError_t conv3_pair0(const float* phi, const float* cond, int ncond, const __bf16* W1k, const float* b1,
                       const __bf16* W2, const float* b2, __bf16* E, __bf16* P, int N, int H, int Wd, hipStream_t s) {
    if (pix_over(N, H, Wd) || H % 16 || Wd % 16 || ncond < 0 || ncond > 7 || !phi || (ncond && !cond) || !E || !P)
        return hipErrorInvalidValue;
    // four tiles per workgroup where H allows (the weights staged once per 1024 pixels)
    if (H % 64 == 0)
        conv3_pair0_k<4><<<dim3(N * (H / 64) * (Wd / 16)), 256, 0, s>>>(phi, cond, ncond, W1k, b1, W2, b2, E, P, H, Wd);
    else
        conv3_pair0_k<1><<<dim3(N * (H / 16) * (Wd / 16)), 256, 0, s>>>(phi, cond, ncond, W1k, b1, W2, b2, E, P, H, Wd);
    return hipGetLastError();
}

hipError_t conv3_fwd_relu_head(const __bf16* X, const __bf16* Wt, const float* bias, __bf16* Y, int N, int H, int Wd,
                               int Ci, int Co, const float* hw, const float* hb, const float* xin, int cin, float* out,
                               float scale, hipStream_t s) {
    if (pix_over(N, H, Wd)) return hipErrorInvalidValue;
    if (H % 16 || Wd % 16 || Ci % 32 || (Co != 32 && Co != 64) || !hw || !hb || !xin || !out || cin < 1)
        return hipErrorInvalidValue;
    const HeadArgs hd{hw, hb, xin, cin, out, scale};
    const dim3 grid(N * (H / 16) * (Wd / 16), 1);
    if (Co == 64)
        conv3_fwd_k<64, true, false, true><<<grid, 256, 0, s>>>(X, nullptr, 0, Wt, bias, Y, H, Wd, Ci, Co, hd);
    else
        conv3_fwd_k<32, true, false, true><<<grid, 256, 0, s>>>(X, nullptr, 0, Wt, bias, Y, H, Wd, Ci, Co, hd);
    return hipGetLastError();
}

namespace {
template <bool UPCAT>
hipError_t conv3_dw_any(const __bf16* X, const __bf16* X2, int Cu, const __bf16* dY, float* part, int S, int N, int H,
                        int Wd, int Ci, int Co, hipStream_t s, float* bpart) {
    if (pix_over(N, H, Wd) || H % 16 || Wd % 16 || Ci % 16 || Co % 32 || S < 1 || S > N * (H / 16) * (Wd / 16))
        return hipErrorInvalidValue;
    if (Co % 64 == 0) {
        dim3 grid(S, Co / 64, Ci / 16);
        conv3_dw_k<64, UPCAT><<<grid, 256, 0, s>>>(X, dY, part, N, H, Wd, Ci, Co, S, bpart, X2, Cu);
    } else {
        dim3 grid(S, Co / 32, Ci / 16);
        conv3_dw_k<32, UPCAT><<<grid, 128, 0, s>>>(X, dY, part, N, H, Wd, Ci, Co, S, bpart, X2, Cu);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t conv3_dw(const __bf16* X, const __bf16* dY, float* part, int S, int N, int H, int Wd, int Ci, int Co,
                    hipStream_t s, float* bpart) {
    return conv3_dw_any<false>(X, nullptr, 0, dY, part, S, N, H, Wd, Ci, Co, s, bpart);
}

hipError_t conv3_dw_upcat(const __bf16* U, const __bf16* Sk, const __bf16* dY, float* part, int S, int N, int H, int Wd,
                          int Cu, int Cs, int Co, hipStream_t s, float* bpart) {
    if (Cu < 32 || Cu % 32 || Cs < 16 || Cs % 16) return hipErrorInvalidValue;
    return conv3_dw_any<true>(U, Sk, Cu, dY, part, S, N, H, Wd, Cu + Cs, Co, s, bpart);
}

hipError_t wgrad_reduce(const float* part, float* dW, int S, int Co, int Ci, int ci_real, hipStream_t s,
                        const float* bpart, float* db) {
    if ((bpart == nullptr) != (db == nullptr)) return hipErrorInvalidValue;
    const long long wblocks = ((long long)Co * 9 * Ci + 31) / 32;
    const long long bblocks = bpart ? (Co + 31) / 32 : 0;
    wgrad_reduce_k<<<(int)(wblocks + bblocks), 256, 0, s>>>(part, dW, S, Co, Ci, ci_real, bpart, db);
    return hipGetLastError();
}

hipError_t colsum_bf16(const __bf16* G, long long P, int C, int S, float* part, float* out, hipStream_t s) {
    if (C % 8 != 0 || C > 512) return hipErrorInvalidValue;
    colsum_part_k<false><<<S, 256, 0, s>>>(G, nullptr, P, C, 1.f, part);
    colsum_reduce_k<<<(C + 3) / 4, 256, 0, s>>>(part, S, C, out);
    return hipGetLastError();
}

hipError_t gather(const float* field, int H, int W, const int* yx, int k, int crop, const float* cond, int ncond,
                  float* x, float* y, hipStream_t s) {
    gather_k<<<grid_for((long long)k * crop * crop), 256, 0, s>>>(field, H, W, yx, k, crop, cond, ncond, x, y);
    return hipGetLastError();
}

hipError_t widen(const __bf16* a, float* b, long long n, hipStream_t s) {
    widen_k<<<grid_for(n), 256, 0, s>>>(a, b, n);
    return hipGetLastError();
}

hipError_t pack_w(const float* W, __bf16* Wt, int Co, int Ci, int Cip, hipStream_t s) {
    pack_w_k<<<grid_for((long long)Co * 9 * Cip), 256, 0, s>>>(W, Wt, Co, Ci, Cip);
    return hipGetLastError();
}

hipError_t pack_all(const PackAll& t, hipStream_t s) {
    if (t.nseg < 1 || t.nseg > kPackMaxSeg) return hipErrorInvalidValue;
    long long largest = 0;
    for (int i = 0; i < t.nseg; ++i) largest = std::max(largest, t.end[i] - (i ? t.end[i - 1] : 0));
    pack_all_k<<<dim3(std::min(grid_for(largest), 1024), t.nseg), 256, 0, s>>>(t);
    return hipGetLastError();
}

hipError_t pack_wflip(const float* W, __bf16* Wf, int Co, int Ci, hipStream_t s) {
    pack_wflip_k<<<grid_for((long long)Co * 9 * Ci), 256, 0, s>>>(W, Wf, Co, Ci);
    return hipGetLastError();
}

hipError_t pack_input(const float* x, __bf16* out, long long P, int cin, int cpad, hipStream_t s) {
    if (cpad % 8 != 0) return hipErrorInvalidValue;
    pack_input_k<<<grid_for(P * cpad / 8), 256, 0, s>>>(x, out, P, cin, cpad);
    return hipGetLastError();
}

hipError_t pack_phi_cond(const float* phi, const float* cond, int ncond, __bf16* out, float* xin, long long P, int cpad,
                         hipStream_t s) {
    if (cpad % 8 != 0) return hipErrorInvalidValue;
    pack_phi_cond_k<<<grid_for(P * cpad / 8), 256, 0, s>>>(phi, cond, ncond, out, xin, P, cpad);
    return hipGetLastError();
}

hipError_t head_fwd(const __bf16* d, const float* w, const float* b, const float* xin, int cin, float* out,
                    long long P, int C, float scale, hipStream_t s) {
    if (C % 8 != 0) return hipErrorInvalidValue;
    head_fwd_k<<<grid_for(P), 256, 0, s>>>(d, w, b, xin, cin, out, P, C, scale);
    return hipGetLastError();
}

hipError_t head_bwd(const float* g, const __bf16* d, const float* w, __bf16* dd, long long P, int C, int S, float scale,
                    float* part, float* grad_wb, hipStream_t s, bool mask_dd) {
    if (C % 8 != 0 || C > 512) return hipErrorInvalidValue;
    head_dd_k<<<grid_for(P * (C / 8)), 256, 0, s>>>(g, w, dd, P, C, scale, mask_dd ? d : nullptr);
    colsum_part_k<true><<<S, 256, 0, s>>>(d, g, P, C, scale, part);
    colsum_reduce_k<<<(C + 4) / 4, 256, 0, s>>>(part, S, C + 1, grad_wb);
    return hipGetLastError();
}

hipError_t mse(const float* pred, const float* target, float* g, int N, int H, int Wd, int margin, double* part,
               double* out, hipStream_t s) {
    const long long inner = (long long)N * (H - 2 * margin) * (Wd - 2 * margin);
    if (inner <= 0) return hipErrorInvalidValue;
    mse_k<<<256, 256, 0, s>>>(pred, target, g, N, H, Wd, margin, 1.0 / (double)inner, part);
    sum_k<<<1, 256, 0, s>>>(part, 256, out);
    return hipGetLastError();
}

hipError_t adam(float* w, const float* g, float* m, float* v, long long n, float lr, float b1, float b2, float eps,
                float wd, float c1, float c2, hipStream_t s) {
    adam_k<<<grid_for(n), 256, 0, s>>>(w, g, m, v, n, lr, b1, b2, eps, wd, c1, c2);
    return hipGetLastError();
}

}  // namespace lbsg
