// HIP kernels of the D2Q9 MRT lattice Boltzmann scheme for the anisotropic
// Cahn-Hilliard equation (arXiv 2501.03759, Sections 2-3), written for
// gfx950 (CDNA4: 64-wide wavefronts, 160 KB LDS per CU, 8 XCDs).
//
// The hot kernel is step_fused: one launch per time step reads the
// post-collision populations of the previous step once (pull streaming),
// evaluates every stencil of the step on chip and writes the new
// post-collision populations once.  Nothing else touches HBM per step.
#include "lbch_internal.h"

#include <math.h>

namespace lbch {

namespace {

// Barrier that waits for LDS traffic only (not for outstanding global loads),
// so that the prefetch of the next row stays in flight across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <typename T> __device__ __forceinline__ T rsqrt_t(T x);
template <> __device__ __forceinline__ float rsqrt_t<float>(float x) { return rsqrtf(x); }
template <> __device__ __forceinline__ double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

// gamma(n) and gamma'(theta) for n = p/|p| (eqs 2, 6 generalised to
// 1 + alpha cos(m(theta - theta0))): Re/Im of (n_x + i n_y)^m e^{-i m theta0}.
template <typename T>
__device__ __forceinline__ void anisotropy(T px, T py, T g2, int m, T alpha, T alpha_m, T rot_c,
                                           T rot_s, T floor2, T& gamma, T& gp) {
    gamma = T(1);
    gp = T(0);
    if (g2 > floor2) {
        const T inv = rsqrt_t<T>(g2);
        const T ux = px * inv, uy = py * inv;
        // z2 = n^2
        const T z2r = ux * ux - uy * uy, z2i = T(2) * ux * uy;
        T zr, zi;
        if (m == 4) {
            zr = z2r * z2r - z2i * z2i;
            zi = T(2) * z2r * z2i;
        } else if (m == 6) {
            const T z4r = z2r * z2r - z2i * z2i, z4i = T(2) * z2r * z2i;
            zr = z4r * z2r - z4i * z2i;
            zi = z4r * z2i + z4i * z2r;
        } else {
            zr = T(1);
            zi = T(0);
            for (int k = 0; k < m; ++k) {
                const T a = zr * ux - zi * uy;
                zi = zr * uy + zi * ux;
                zr = a;
            }
        }
        const T cr = zr * rot_c + zi * rot_s;
        const T ci = zi * rot_c - zr * rot_s;
        gamma = T(1) + alpha * cr;
        gp = -alpha_m * ci;
    }
}

// MRT collision in moment space (eqs 17, 23, 25) for one node with the
// closed forms m_eq = (phi, -4phi + 2mu_a, 4phi - 3mu_a, 0, ...) (eq 18) and
// F_m = (c/3) (0, 0, 0, -gx, gx, -gy, gy, 0, 0) (eq 19); the inverse
// transform is M^T diag(1/|row k|^2).
template <typename T>
__device__ __forceinline__ void collide(const T (&f)[9], T mua, T gx, T gy, const StepCoef<T>& c,
                                        T (&o)[9]) {
    const T a = (f[1] + f[2]) + (f[3] + f[4]);
    const T b = (f[5] + f[6]) + (f[7] + f[8]);
    const T phi = f[0] + a + b;
    const T m1 = T(2) * b - a - T(4) * f[0];
    const T m2 = b - T(2) * a + T(4) * f[0];
    const T d13 = f[1] - f[3], d24 = f[2] - f[4];
    const T ex = (f[5] - f[7]) + (f[8] - f[6]);    // f5 - f6 - f7 + f8
    const T ey = (f[5] - f[7]) + (f[6] - f[8]);    // f5 + f6 - f7 - f8
    const T m3 = d13 + ex;
    const T m4 = ex - T(2) * d13;
    const T m5 = d24 + ey;
    const T m6 = ey - T(2) * d24;
    const T m7 = (f[1] + f[3]) - (f[2] + f[4]);
    const T m8 = (f[5] + f[7]) - (f[6] + f[8]);
    const T d1 = c.cs1 * (m1 - (T(2) * mua - T(4) * phi));
    const T d2 = c.cs2 * (m2 - (T(4) * phi - T(3) * mua));
    const T d3 = c.cs3 * m3 + c.cf3 * gx;
    const T d4 = c.cs4 * m4 - c.cf4 * gx;
    const T d5 = c.cs5 * m5 + c.cf5 * gy;
    const T d6 = c.cs6 * m6 - c.cf6 * gy;
    const T d7 = c.cs7 * m7;
    const T d8 = c.cs8 * m8;
    const T ax = d1 + T(2) * d2;            // axis-direction common part
    const T dg = T(2) * d1 + d2;            // diagonal common part
    o[0] = f[0] + T(4) * (d1 - d2);
    o[1] = f[1] + ax - d3 + T(2) * d4 - d7;
    o[2] = f[2] + ax - d5 + T(2) * d6 + d7;
    o[3] = f[3] + ax + d3 - T(2) * d4 - d7;
    o[4] = f[4] + ax + d5 - T(2) * d6 + d7;
    const T p34 = d3 + d4, p56 = d5 + d6;
    o[5] = f[5] - (dg + p34 + p56 + d8);
    o[6] = f[6] - (dg - p34 + p56 - d8);
    o[7] = f[7] - (dg - p34 - p56 + d8);
    o[8] = f[8] - (dg + p34 - p56 - d8);
}

}  // namespace

// ---------------------------------------------------------------------------
// Fused step.  Workgroup = strip of W = NT - 6 output columns x hc output rows.
// Lane t owns column x0 - 3 + t (wrapped) for the whole sweep.  Each loop
// iteration j brings in one new row r = y0 - 3 + j and runs four stages
// that lag behind it:
//   A(row r)   : pull f_i(x, r) = f*_i(x - c_i, r - c_iy), phi = sum f_i (eq 22)
//   B(row r-1) : grad phi, lap phi (eq 26), gamma, Q (eq 15), w (eq 9), mu_alpha (eq 16)
//   C(row r-2) : div Q, lap w -> mu_beta (eqs 13, 16)
//   D(row r-3) : grad mu_beta, source (eq 19), collision (eq 17), store
// Stage outputs live in 3-row LDS rings; the populations of a row stay in
// registers from A until D three iterations later.  The next row's loads
// are issued before the stencil stages so their latency overlaps compute.
// ---------------------------------------------------------------------------
template <typename T, int NT>
__global__ __launch_bounds__(NT) void step_fused(const T* __restrict__ fin, T* __restrict__ fout,
                                                 const Grid g, const Tiling tl, const StepCoef<T> c) {
    __shared__ T s_phi[3][NT];
    __shared__ T s_qx[3][NT];
    __shared__ T s_qy[3][NT];
    __shared__ T s_w[3][NT];
    __shared__ T s_mb[3][NT];

    const int bid = blockIdx.x;
    const int tile = (bid & 7) * tl.per_xcd + (bid >> 3);
    if (tile >= tl.ntiles) return;
    const int strip = tile % tl.strips;
    const int chunk = tile / tl.strips;
    const int nx = g.nx, ny = g.ny, pitch = g.pitch;
    const int x0 = strip * tl.W;
    const int wlen = min(tl.W, nx - x0);
    const int y0 = chunk * tl.hc;
    const int niter = min(tl.hc, ny - y0) + 6;
    const int t = threadIdx.x;

    int xc = (x0 - 3 + t) % nx;
    if (xc < 0) xc += nx;
    const int cm = (xc == 0) ? nx - 1 : xc - 1;
    const int cp = (xc == nx - 1) ? 0 : xc + 1;

    const T* __restrict__ P0 = fin;
    const T* __restrict__ P1 = fin + g.plane;
    const T* __restrict__ P2 = fin + 2 * g.plane;
    const T* __restrict__ P3 = fin + 3 * g.plane;
    const T* __restrict__ P4 = fin + 4 * g.plane;
    const T* __restrict__ P5 = fin + 5 * g.plane;
    const T* __restrict__ P6 = fin + 6 * g.plane;
    const T* __restrict__ P7 = fin + 7 * g.plane;
    const T* __restrict__ P8 = fin + 8 * g.plane;

    int rA = (y0 - 3) % ny;   // row of the next stage-A load (wrapped)
    if (rA < 0) rA += ny;

    T fr[5][9];               // register ring of pulled populations
    T mua[5];                 // mu_alpha ring (B -> D, two iterations)
    T tloc[5];                // local part of mu_beta (B -> C, one iteration)

    auto load_row = [&](int r, T (&f)[9]) {
        const int rm = (r == 0) ? ny - 1 : r - 1;
        const int rp = (r == ny - 1) ? 0 : r + 1;
        const int o0 = r * pitch, om = rm * pitch, op = rp * pitch;
        f[0] = P0[o0 + xc];
        f[1] = P1[o0 + cm];
        f[2] = P2[om + xc];
        f[3] = P3[o0 + cp];
        f[4] = P4[op + xc];
        f[5] = P5[om + cm];
        f[6] = P6[om + cp];
        f[7] = P7[op + cp];
        f[8] = P8[op + cm];
    };

    load_row(rA, fr[0]);

    for (int jb = 0; jb < niter; jb += 5) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int j = jb + k;
            if (j < niter) {
                const int sN = j % 3, sC = (j + 2) % 3, sS = (j + 1) % 3;
                // ---- A: phi of row r (same summation order as collide()) ----
                {
                    const T(&f)[9] = fr[k];
                    const T a = (f[1] + f[2]) + (f[3] + f[4]);
                    const T b = (f[5] + f[6]) + (f[7] + f[8]);
                    s_phi[sN][t] = f[0] + a + b;
                }
                if (j + 1 < niter) {
                    rA = (rA == ny - 1) ? 0 : rA + 1;
                    load_row(rA, fr[(k + 1) % 5]);
                }
                lds_barrier();
                // ---- B: row r-1 ----
                if (j >= 2 && t >= 1 && t < NT - 1) {
                    const T pC = s_phi[sC][t], pE = s_phi[sC][t + 1], pW = s_phi[sC][t - 1];
                    const T pN = s_phi[sN][t], pNE = s_phi[sN][t + 1], pNW = s_phi[sN][t - 1];
                    const T pS = s_phi[sS][t], pSE = s_phi[sS][t + 1], pSW = s_phi[sS][t - 1];
                    const T px = c.g3 * (pE - pW) + c.g12 * ((pNE - pSW) + (pSE - pNW));
                    const T py = c.g3 * (pN - pS) + c.g12 * ((pNE - pSW) + (pNW - pSE));
                    const T lap = c.l23 * ((pE + pW) + (pN + pS)) + c.l16 * ((pNE + pSW) + (pNW + pSE)) -
                                  c.l103 * pC;
                    const T fb = c.beta4 * pC * (pC * pC - T(1));
                    const T g2 = px * px + py * py;
                    T gamma, gp;
                    anisotropy<T>(px, py, g2, c.m, c.alpha, c.alpha_m, c.rot_c, c.rot_s, c.floor2, gamma, gp);
                    T qx, qy;
                    if (c.qform == 0) {
                        qx = c.kappa * (gamma * px - gp * py);
                        qy = c.kappa * (gamma * py + gp * px);
                    } else {
                        qx = gamma * c.kappa * px - gp * py;
                        qy = gamma * c.kappa * py + gp * px;
                    }
                    T w, tl0 = (gamma - T(1)) * fb + c.kappa * lap;
                    if (c.reg == REG_WILLMORE) {
                        w = lap - fb;
                        const T fpr = c.beta4 * (T(3) * pC * pC - T(1));
                        tl0 -= c.eps * fpr * w;
                    } else if (c.reg == REG_LINEAR) {
                        w = lap;
                    } else {
                        w = T(0);
                    }
                    s_qx[sN][t] = qx;
                    s_qy[sN][t] = qy;
                    s_w[sN][t] = w;
                    tloc[k] = tl0;
                    mua[k] = fb - c.kappa * lap;
                }
                lds_barrier();
                // ---- C: row r-2 ----
                if (j >= 4 && t >= 2 && t < NT - 2) {
                    const T divq =
                        c.g3 * (s_qx[sC][t + 1] - s_qx[sC][t - 1]) +
                        c.g12 * ((s_qx[sN][t + 1] - s_qx[sS][t - 1]) + (s_qx[sS][t + 1] - s_qx[sN][t - 1])) +
                        c.g3 * (s_qy[sN][t] - s_qy[sS][t]) +
                        c.g12 * ((s_qy[sN][t + 1] - s_qy[sS][t - 1]) + (s_qy[sN][t - 1] - s_qy[sS][t + 1]));
                    T mb = tloc[(k + 4) % 5] - divq;
                    if (c.reg != REG_NONE) {
                        const T lw = c.l23 * ((s_w[sC][t + 1] + s_w[sC][t - 1]) + (s_w[sN][t] + s_w[sS][t])) +
                                     c.l16 * ((s_w[sN][t + 1] + s_w[sS][t - 1]) + (s_w[sN][t - 1] + s_w[sS][t + 1])) -
                                     c.l103 * s_w[sC][t];
                        mb += c.eps * lw;
                    }
                    s_mb[sN][t] = mb;
                }
                lds_barrier();
                // ---- D: row r-3 ----
                if (j >= 6 && t >= 3 && t < 3 + wlen) {
                    const T gx = c.g3 * (s_mb[sC][t + 1] - s_mb[sC][t - 1]) +
                                 c.g12 * ((s_mb[sN][t + 1] - s_mb[sS][t - 1]) + (s_mb[sS][t + 1] - s_mb[sN][t - 1]));
                    const T gy = c.g3 * (s_mb[sN][t] - s_mb[sS][t]) +
                                 c.g12 * ((s_mb[sN][t + 1] - s_mb[sS][t - 1]) + (s_mb[sN][t - 1] - s_mb[sS][t + 1]));
                    T o[9];
                    collide<T>(fr[(k + 2) % 5], mua[(k + 3) % 5], gx, gy, c, o);
                    const int rd = y0 - 6 + j;
                    const long long base = (long long)rd * pitch + xc;
                    T* __restrict__ q = fout + base;
#pragma unroll
                    for (int i = 0; i < 9; ++i) q[i * g.plane] = o[i];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Initialisation at equilibrium (eq 18 with mu_alpha of eq 16 at phi0), stored
// in the post-collision layout consumed by the pull of step_fused: population
// i at node x is written where the next step will pull it from, x - c_i.
// ---------------------------------------------------------------------------
template <typename T, typename P>
__global__ __launch_bounds__(256) void init_eq(const P* __restrict__ phi0, T* __restrict__ fout, const Grid g,
                                               const StepCoef<T> c, unsigned* bad) {
    const long long n = (long long)g.nx * g.ny;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(idx / g.nx), x = (int)(idx % g.nx);
        const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
        auto at = [&](int yy, int xx) { return (T)phi0[(long long)yy * g.nx + xx]; };
        const T pC = at(y, x);
        if (!isfinite((double)pC)) atomicAdd(bad, 1u);
        const T lap = c.l23 * ((at(y, xp) + at(y, xm)) + (at(yp, x) + at(ym, x))) +
                      c.l16 * ((at(yp, xp) + at(ym, xm)) + (at(yp, xm) + at(ym, xp))) - c.l103 * pC;
        const T fb = c.beta4 * pC * (pC * pC - T(1));
        const T mu = fb - c.kappa * lap;
        const T w1 = T(1) / T(9), w5 = T(1) / T(36);
        const T val[9] = {pC + (T(4) / T(9) - T(1)) * mu, w1 * mu, w1 * mu, w1 * mu, w1 * mu,
                          w5 * mu, w5 * mu, w5 * mu, w5 * mu};
        const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int xs = x - ex[i], ys = y - ey[i];
            xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            fout[i * g.plane + (long long)ys * g.pitch + xs] = val[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Reductions (float64 partials in a fixed order: deterministic).
// ---------------------------------------------------------------------------
namespace {

template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], const int (&kind)[NV], double* out) {
    // kind: 0 = sum, 1 = min, 2 = max
    __shared__ double sh[NV][kRedThreads];
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const double a = sh[q][threadIdx.x], b = sh[q][threadIdx.x + s];
                sh[q][threadIdx.x] = kind[q] == 0 ? a + b : (kind[q] == 1 ? fmin(a, b) : fmax(a, b));
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q] = sh[q][0];
    }
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kRedThreads) void moments_k(const T* __restrict__ fin, const Grid g, void* phi_out,
                                                         int out_dtype, double* partials) {
    double v[4] = {0.0, INFINITY, -INFINITY, 0.0};
    const int kind[4] = {0, 1, 2, 0};
    const long long n = (long long)g.nx * g.ny;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(idx / g.nx), x = (int)(idx % g.nx);
        const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
        auto F = [&](int i, int yy, int xx) { return (double)fin[i * g.plane + (long long)yy * g.pitch + xx]; };
        const double a = (F(1, y, xm) + F(2, ym, x)) + (F(3, y, xp) + F(4, yp, x));
        const double b = (F(5, ym, xm) + F(6, ym, xp)) + (F(7, yp, xp) + F(8, yp, xm));
        const double phi = F(0, y, x) + a + b;
        if (phi_out) {
            if (out_dtype == 0) ((double*)phi_out)[idx] = phi;
            else ((float*)phi_out)[idx] = (float)phi;
        }
        if (isfinite(phi)) {
            v[0] += phi;
            v[1] = fmin(v[1], phi);
            v[2] = fmax(v[2], phi);
        } else {
            v[3] += 1.0;
        }
    }
    block_reduce_store<4>(v, kind, partials + 4 * blockIdx.x);
}

__global__ __launch_bounds__(kRedThreads) void energy_k(const double* __restrict__ phi, const Grid g,
                                                        const RedCoef c, double* partials) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int kind[4] = {0, 0, 0, 0};
    const long long n = (long long)g.nx * g.ny;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(idx / g.nx), x = (int)(idx % g.nx);
        const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
        auto P = [&](int yy, int xx) { return phi[(long long)yy * g.nx + xx]; };
        const double pC = P(y, x), pE = P(y, xp), pW = P(y, xm), pN = P(yp, x), pS = P(ym, x);
        const double pNE = P(yp, xp), pNW = P(yp, xm), pSE = P(ym, xp), pSW = P(ym, xm);
        const double px = c.g3 * (pE - pW) + c.g12 * ((pNE - pSW) + (pSE - pNW));
        const double py = c.g3 * (pN - pS) + c.g12 * ((pNE - pSW) + (pNW - pSE));
        const double lap = c.l23 * ((pE + pW) + (pN + pS)) + c.l16 * ((pNE + pSW) + (pNW + pSE)) - c.l103 * pC;
        const double g2 = px * px + py * py;
        double gamma, gp;
        anisotropy<double>(px, py, g2, c.m, c.alpha, c.alpha * c.m, c.rot_c, c.rot_s, c.floor2, gamma, gp);
        const double q = pC * pC - 1.0;
        const double Fb = c.beta * q * q;
        const double fb = 4.0 * c.beta * pC * q;
        double G = 0.0;
        if (c.reg == REG_WILLMORE) G = (lap - fb) * (lap - fb);
        else if (c.reg == REG_LINEAR) G = lap * lap;
        const double tg = gamma * 0.5 * c.kappa * g2, tb = gamma * Fb, tr = 0.5 * c.eps * G;
        if (isfinite(tg + tb + tr)) {
            v[0] += tg;
            v[1] += tb;
            v[2] += tr;
        } else {
            v[3] += 1.0;
        }
    }
    block_reduce_store<4>(v, kind, partials + 4 * blockIdx.x);
}

// Combines nparts partial records of nvals values; kinds[q]: 0 sum, 1 min, 2 max.
__global__ __launch_bounds__(kRedThreads) void finalize_k(const double* __restrict__ partials, int nparts, int nvals,
                                                          int k0, int k1, int k2, int k3, double* out) {
    double v[4];
    const int kind[4] = {k0, k1, k2, k3};
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = kind[q] == 0 ? 0.0 : (kind[q] == 1 ? INFINITY : -INFINITY);
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= nvals) break;
            const double b = partials[(long long)i * nvals + q];
            v[q] = kind[q] == 0 ? v[q] + b : (kind[q] == 1 ? fmin(v[q], b) : fmax(v[q], b));
        }
    }
    block_reduce_store<4>(v, kind, out);
}

// Canonical pre-collision populations f_i(x) = f*_i(x - c_i) <-> internal layout.
template <typename T>
__global__ __launch_bounds__(256) void gather_k(const T* __restrict__ fin, const Grid g, T* __restrict__ dense) {
    const long long n = (long long)g.nx * g.ny;
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(idx / g.nx), x = (int)(idx % g.nx);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int xs = x - ex[i], ys = y - ey[i];
            xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            dense[i * n + idx] = fin[i * g.plane + (long long)ys * g.pitch + xs];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void scatter_k(const T* __restrict__ dense, const Grid g, T* __restrict__ fout) {
    const long long n = (long long)g.nx * g.ny;
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(idx / g.nx), x = (int)(idx % g.nx);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int xs = x - ex[i], ys = y - ey[i];
            xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            fout[i * g.plane + (long long)ys * g.pitch + xs] = dense[i * n + idx];
        }
    }
}

__global__ void fill_zero_k(double* p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// ----------------------------------------------------------------- launchers
namespace {
int elementwise_blocks(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}
}  // namespace

template <typename T>
static hipError_t launch_step_t(const T* fin, T* fout, const Grid& g, const Tiling& t, const StepCoef<T>& c,
                                hipStream_t s) {
    dim3 grid(t.nblocks);
    switch (t.nt) {
        case 64: step_fused<T, 64><<<grid, 64, 0, s>>>(fin, fout, g, t, c); break;
        case 128: step_fused<T, 128><<<grid, 128, 0, s>>>(fin, fout, g, t, c); break;
        case 256: step_fused<T, 256><<<grid, 256, 0, s>>>(fin, fout, g, t, c); break;
        case 512: step_fused<T, 512><<<grid, 512, 0, s>>>(fin, fout, g, t, c); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step(int precision, const void* fin, void* fout, const Grid& g, const Tiling& t, const void* coef,
                       hipStream_t s) {
    if (precision == 0)
        return launch_step_t<double>((const double*)fin, (double*)fout, g, t, *(const StepCoef<double>*)coef, s);
    return launch_step_t<float>((const float*)fin, (float*)fout, g, t, *(const StepCoef<float>*)coef, s);
}

hipError_t launch_init(int precision, const void* phi0, int phi_dtype, void* fout, const Grid& g, const void* coef,
                       unsigned* bad, hipStream_t s) {
    const int nb = elementwise_blocks((long long)g.nx * g.ny);
    if (precision == 0) {
        const auto& c = *(const StepCoef<double>*)coef;
        if (phi_dtype == 0) init_eq<double, double><<<nb, 256, 0, s>>>((const double*)phi0, (double*)fout, g, c, bad);
        else init_eq<double, float><<<nb, 256, 0, s>>>((const float*)phi0, (double*)fout, g, c, bad);
    } else {
        const auto& c = *(const StepCoef<float>*)coef;
        if (phi_dtype == 0) init_eq<float, double><<<nb, 256, 0, s>>>((const double*)phi0, (float*)fout, g, c, bad);
        else init_eq<float, float><<<nb, 256, 0, s>>>((const float*)phi0, (float*)fout, g, c, bad);
    }
    return hipGetLastError();
}

hipError_t launch_moments(int precision, const void* fin, const Grid& g, void* phi_out, int out_dtype,
                          double* partials, int nparts, hipStream_t s) {
    if (precision == 0)
        moments_k<double><<<nparts, kRedThreads, 0, s>>>((const double*)fin, g, phi_out, out_dtype, partials);
    else
        moments_k<float><<<nparts, kRedThreads, 0, s>>>((const float*)fin, g, phi_out, out_dtype, partials);
    return hipGetLastError();
}

hipError_t launch_energy(const double* phi, const Grid& g, const RedCoef& c, double* partials, int nparts,
                         hipStream_t s) {
    energy_k<<<nparts, kRedThreads, 0, s>>>(phi, g, c, partials);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nparts, int nvals, const int* kinds, double* out,
                           hipStream_t s) {
    finalize_k<<<1, kRedThreads, 0, s>>>(partials, nparts, nvals, kinds[0], kinds[1], kinds[2], kinds[3], out);
    return hipGetLastError();
}

hipError_t launch_gather(int precision, const void* fin, const Grid& g, void* dense, hipStream_t s) {
    const int nb = elementwise_blocks((long long)g.nx * g.ny);
    if (precision == 0) gather_k<double><<<nb, 256, 0, s>>>((const double*)fin, g, (double*)dense);
    else gather_k<float><<<nb, 256, 0, s>>>((const float*)fin, g, (float*)dense);
    return hipGetLastError();
}

hipError_t launch_scatter(int precision, const void* dense, const Grid& g, void* fout, hipStream_t s) {
    const int nb = elementwise_blocks((long long)g.nx * g.ny);
    if (precision == 0) scatter_k<double><<<nb, 256, 0, s>>>((const double*)dense, g, (double*)fout);
    else scatter_k<float><<<nb, 256, 0, s>>>((const float*)dense, g, (float*)fout);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, long long n, hipStream_t s) {
    fill_zero_k<<<elementwise_blocks(n), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace lbch
