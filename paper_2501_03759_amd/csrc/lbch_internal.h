// Internal declarations shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbch.h"

namespace lbch {

// Geometry of one periodic grid as stored in HBM: 9 population planes
// (structure of arrays), each ny rows of `pitch` elements (pitch >= nx).
struct Grid {
    int nx, ny, pitch;
    int pad_;
    long long plane;      // elements between consecutive population planes
};

// Decomposition of the fused step: strips of W = NT - 8 * depth columns,
// chunks of `hc` rows; tiles are strip-fastest; blocks are dealt to the 8
// XCDs in contiguous tile ranges of `per_xcd`.  depth = time steps per
// launch (1 or 2).
struct Tiling {
    int nt, W, strips, hc, chunks, ntiles, per_xcd, nblocks;
    int staged;           // FP32 row loader through LDS (used when nx % 4 == 0)
    int depth;
};

// Per-step constants in the working precision T (lattice units folded in).
template <typename T>
struct StepCoef {
    T g3, g12;            // gradient eq 26a: (1/3)/dx, (1/12)/dx
    T l23, l16, l103;     // Laplacian eq 26b: (2/3)/dx^2, (1/6)/dx^2, (10/3)/dx^2
    T kappa, beta4, eps, alpha, floor2;
    T rot_c, rot_s;       // cos(m theta0), sin(m theta0)
    T alpha_m;            // alpha * m
    T cs1, cs2, cs3, cs4, cs5, cs6, cs7, cs8;   // s_k / |row k of M|^2
    T cf3, cf4, cf5, cf6;                       // dt (1 - s_k/2) (c/3) / |row k|^2
    T u3, u5, v4, v6;     // unit free rates: (1 - s_j)/6 and dt (c/3) / (2 * 12)
    int m, reg, qform;
    int unit;             // every free rate (k != 0, 3, 5) equals 1
};

// Reduction constants (always float64).
struct RedCoef {
    double g3, g12, l23, l16, l103;
    double kappa, beta, eps, alpha, floor2, rot_c, rot_s, area;
    int m, reg;
};

enum { REG_NONE = 0, REG_LINEAR = 1, REG_WILLMORE = 2 };

// Launchers (lbch_kernels.hip).  All are stream-ordered and return the
// launch status.
hipError_t launch_step(int precision, const void* fin, void* fout, const Grid& g, const Tiling& t,
                       const void* coef, hipStream_t s);
// One two-step launch storing f_{n+2} + ext (f_{n+2} - f_n) (fin holds f_n);
// t must be a two-step tiling.
hipError_t launch_step2_extrap(int precision, const void* fin, void* fout, const Grid& g, const Tiling& t,
                               const void* coef, double ext, hipStream_t s);
hipError_t launch_init(int precision, const void* phi0, int phi_dtype, void* fout, const Grid& g,
                       const void* coef, unsigned* bad_count, hipStream_t s);
// phi of the current state (float64 math) -> optional dense output + partial sums
hipError_t launch_moments(int precision, const void* fin, const Grid& g, void* phi_out, int out_dtype,
                          double* partials, int nparts, hipStream_t s);
hipError_t launch_energy(const double* phi, const Grid& g, const RedCoef& c, double* partials,
                         int nparts, hipStream_t s);
hipError_t launch_finalize(const double* partials, int nparts, int nvals, const int* kinds,
                           double* out, hipStream_t s);
hipError_t launch_gather(int precision, const void* fin, const Grid& g, void* dense, hipStream_t s);
hipError_t launch_scatter(int precision, const void* dense, const Grid& g, void* fout, hipStream_t s);
hipError_t launch_fill_zero(double* p, long long n, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s);
hipError_t launch_copy16(const void* src, void* dst, long long n16, hipStream_t s);

// Ensemble (lbch_batch): one descriptor per member; the members' populations
// live at `base` elements into two shared buffers.
template <typename T>
struct BatchMember {
    Grid g;
    long long base;
    StepCoef<T> c;
    int strips, hc, chunks, tile_begin;
};

// depth: time steps per launch (1 or 2); members' strips are nt - 8 * depth columns wide
hipError_t launch_batch_step(int precision, int depth, int nt, bool unit_all, const void* fin, void* fout,
                             const void* members, const int* tile_member, int total_tiles, int nblocks,
                             unsigned long long* ctr, hipStream_t s);
// resident workgroups per CU of the batch kernel (for sizing its persistent grid)
int batch_blocks_per_cu(int precision, int depth, int nt, bool unit_all);
// resident workgroups per CU of the step kernel of the given depth and shape
int step_blocks_per_cu(int precision, int depth, int nt, bool unit, bool staged);

// Host helpers shared by the C-ABI files (lbch_api.cpp).
lbch_status fail(lbch_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
template <typename T>
void fill_coef(const lbch_params* p, StepCoef<T>& c);
void fill_red(const lbch_params* p, RedCoef& r);
// slots: resident workgroups on the device; cus: its compute units (0 = unknown)
Tiling make_tiling(int nx, int ny, int nt, int hc, int depth = 1, int esize = 4, int slots = 0, int cus = 0);

constexpr int kRedBlocks = 1024;   // partial-sum blocks of every reduction
constexpr int kRedThreads = 256;

// Workgroup reduction of NV float64 values per lane (kind: 0 = sum, 1 = min,
// 2 = max) for blocks of kRedThreads lanes, stored by lane 0 to out[0..NV).
// Each wavefront reduces its 64 lanes by lane exchange (butterfly over 32, 16,
// ..., 1 lanes; every lane ends with the same value), then lane 0 combines the
// wavefronts' results in wavefront order: one LDS exchange and one barrier, a
// fixed order, so the result is deterministic.
template <int NV>
__device__ __forceinline__ void block_reduce_waves(double (&v)[NV], const int (&kind)[NV], double* out) {
    constexpr int kWaves = kRedThreads / 64;
    __shared__ double sh[NV][kWaves];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double b = __shfl_xor(v[q], off, 64);
            v[q] = kind[q] == 0 ? v[q] + b : (kind[q] == 1 ? fmin(v[q], b) : fmax(v[q], b));
        }
    }
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) sh[q][wave] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double a = sh[q][0];
            for (int w = 1; w < kWaves; ++w) {
                const double b = sh[q][w];
                a = kind[q] == 0 ? a + b : (kind[q] == 1 ? fmin(a, b) : fmax(a, b));
            }
            out[q] = a;
        }
    }
}

// Hybrid-schedule helpers (lbch_kernels.hip)
hipError_t launch_sum_f32(const float* x, long long n, double* partials, double* out, hipStream_t s);
hipError_t launch_add_f32(float* x, long long n, const double* num, const double* den_minus, double inv_n,
                          hipStream_t s);
hipError_t launch_copy_window(int precision, const void* src, const Grid& sg, int y0, int x0, void* dst,
                              const Grid& dg, hipStream_t s);
hipError_t launch_extrap_f32(const float* base, const float* a, const float* b, float k, long long n, float* out,
                             hipStream_t s);
// cur += k (cur - prev) over `elems` elements (a multiple of 16 bytes) of population storage
hipError_t launch_extrap_pop(int precision, void* cur, const void* prev, double k, long long elems, hipStream_t s);
hipError_t launch_window_err(const float* win, int side, const float* big, int ny, int nx, int y0, int x0, int margin,
                             int interior, double* partials, double* out2, hipStream_t s);

// ---- three-dimensional lattice (D3Q15, eq 21; lbch3_kernels.hip) ----
// 15 population planes of nz slabs of ny rows of `pitch` elements.
struct Grid3 {
    int nx, ny, nz, pitch;
    long long slab;       // elements between consecutive z slabs (pitch * ny)
    long long plane;      // elements between consecutive population planes
};

// Workgroups of tx x ty lanes store x-y tiles of (tx - 6) x (ty - 6) nodes,
// each swept over `hz` consecutive slabs; tiles are x-fastest, then y, then
// z chunk, and are dealt to the 8 XCDs in contiguous ranges of `per_xcd`.
// Built shapes: 32 x 16 (both precisions) and 32 x 32 (FP32).
struct Tiling3 {
    int tx, ty, tiles_x, tiles_y, hz, zchunks, ntiles, per_xcd, nblocks;
};

// Per-step constants of the D3Q15 step in the working precision.
template <typename T>
struct StepCoef3 {
    T gf, gd;             // gradient eq 26a: face (1/3)/dx, body diagonal (1/24)/dx
    T lf, ld, lc;         // Laplacian eq 26b: (2/3)/dx^2, (1/12)/dx^2, (14/3)/dx^2
    T kappa, beta4, eps, alpha, alpha16, floor2;
    T u;                  // (s_q - s_j) / 10
    T v;                  // dt c / 6
    T hd;                 // (1 - s_q / 2) dt c
    T w0, wf, wd;         // eq 21b weights
    T se1, sq1;           // 1 - s_e, 1 - s_q (even rows, odd non-flux rows)
    int reg, qform;
    int gen;              // s_e != 1 or s_q != 1: the collision reads every population
};

template <typename T>
void fill_coef3(const lbch_params* p, StepCoef3<T>& c);
Tiling3 make_tiling3(int nx, int ny, int nz, int hz, int slots, int tx, int ty);
bool tile3_shape(int precision, int block_threads, int* tx, int* ty);
int step3_blocks_per_cu(int precision, int tx, int ty, bool gen);
hipError_t launch_step3(int precision, const void* fin, void* fout, const Grid3& g, const Tiling3& t,
                        const void* coef, hipStream_t s);
hipError_t launch_init3(int precision, const void* phi0, int phi_dtype, void* fout, const Grid3& g, const void* coef,
                        unsigned* bad, hipStream_t s);
hipError_t launch_moments3(int precision, const void* fin, const Grid3& g, void* phi_out, int out_dtype,
                           double* partials, int nparts, hipStream_t s);
hipError_t launch_energy3(const double* phi, const Grid3& g, const StepCoef3<double>& c, double* partials,
                          int nparts, hipStream_t s);
hipError_t launch_gather3(int precision, const void* fin, const Grid3& g, void* dense, hipStream_t s);
hipError_t launch_scatter3(int precision, const void* dense, const Grid3& g, void* fout, hipStream_t s);

}  // namespace lbch

// The simulation handle (opaque in the C ABI).
struct lbch_sim {
    lbch_params p{};
    int precision = 0;
    size_t esize = 8;
    lbch::Grid g{};
    lbch::Tiling t{};                // tiling of the active depth
    lbch::Tiling t1{};               // depth-1 tiling (odd remainders of lbch_step)
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    hipStream_t stream = nullptr;
    int64_t step = 0;
    bool initialized = false;
    double* phi64 = nullptr;         // nx*ny float64 scratch for reductions
    double* partials = nullptr;      // kRedBlocks * 4
    double* result = nullptr;        // 8 doubles (device)
    unsigned* bad = nullptr;         // non-finite counter of init_device
    lbch::StepCoef<double> cd{};
    lbch::StepCoef<float> cf{};
    lbch::RedCoef rc{};
    int user_nt = 0, user_hc = 0, user_loader = 0;
    int cus = 256;                   // compute units of the device
    // D3Q15 (lattice == LBCH_D3Q15): the 2D fields above other than the
    // buffers, stream and counters are unused
    bool d3 = false;
    lbch::Grid3 g3{};
    lbch::Tiling3 t3{};
    lbch::StepCoef3<double> c3d{};
    lbch::StepCoef3<float> c3f{};
    long long nodes = 0;             // nx * ny * nz
    int nq = 9;                      // populations per node
    // workspace of lbch_hybrid_advance: allocated by its first call, kept until
    // lbch_destroy (a third population buffer for the snapshot, FP32 fields of
    // phi, the jumped phi and phi one step on, sums, and the shadow-window
    // ensemble of hyb_windows windows of side hyb_side with their phi output)
    void* hyb_snap = nullptr;
    float* hyb_phi[3] = {nullptr, nullptr, nullptr};
    double* hyb_dsum = nullptr;
    double* hyb_part = nullptr;
    float* hyb_wphi = nullptr;
    struct lbch_batch* hyb_win = nullptr;
    int hyb_windows = 0, hyb_side = 0;
};

// Ensemble helper used by the hybrid schedule: member `member` of batch b
// takes the populations of the window of sim s whose corner is (y0, x0)
// (wrapped periodically), in the internal pull layout of both.
struct lbch_batch;
lbch_status lbch_batch_load_window(lbch_batch* b, int member, const lbch_sim* s, int y0, int x0);

