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

// Collision when every free rate (k != 0, 3, 5) is 1: those moments relax to
// m_eq + dt F/2, so f* = M^-1 m* needs only phi, j_x = m_3, j_y = m_5 of f:
// m* = (phi, 2mu_a - 4phi, 4phi - 3mu_a, (1-s_j) j_x - dt(1-s_j/2)(c/3)gx,
//       dt(c/3)gx/2, (1-s_j) j_y - dt(1-s_j/2)(c/3)gy, dt(c/3)gy/2, 0, 0).
template <typename T>
__device__ __forceinline__ void collide_unit(T phi, T jx, T jy, T mua, T gx, T gy, const StepCoef<T>& c,
                                             T (&o)[9]) {
    const T e0 = phi * T(1.0 / 9.0);
    const T e1 = (T(2) * mua - T(4) * phi) * T(1.0 / 36.0);
    const T e2 = (T(4) * phi - T(3) * mua) * T(1.0 / 36.0);
    const T e3 = c.u3 * jx - c.cf3 * gx;
    const T e4 = c.v4 * gx;
    const T e5 = c.u5 * jy - c.cf5 * gy;
    const T e6 = c.v6 * gy;
    const T ax = e0 - e1 - T(2) * e2;        // axis directions
    const T dg = e0 + T(2) * e1 + e2;        // diagonal directions
    const T p34 = e3 + e4, p56 = e5 + e6;
    o[0] = e0 + T(4) * (e2 - e1);
    o[1] = ax + e3 - T(2) * e4;
    o[2] = ax + e5 - T(2) * e6;
    o[3] = ax - e3 + T(2) * e4;
    o[4] = ax - e5 + T(2) * e6;
    o[5] = dg + p34 + p56;
    o[6] = dg - p34 + p56;
    o[7] = dg - p34 - p56;
    o[8] = dg + p34 - p56;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fused step.  Workgroup = strip of W = NT - 8 output columns x hc output rows.
// Lane t owns column x0 - 3 + t (wrapped) for the whole sweep.  Each loop
// iteration j brings in one new row r = y0 - 3 + j and runs four stages
// that lag behind it:
//   A(row r)   : pull f_i(x, r) = f*_i(x - c_i, r - c_iy), phi = sum f_i (eq 22)
//   B(row r-1) : grad phi, lap phi (eq 26), gamma, Q (eq 15), w (eq 9), mu_alpha (eq 16)
//   C(row r-2) : div Q, lap w -> mu_beta (eqs 13, 16)
//   D(row r-3) : grad mu_beta, source (eq 19), collision (eq 17), store
// Stage outputs live in 3-row LDS rings; what D needs of a row's populations
// stays in registers from A until D three iterations later (all nine
// populations in general; only phi, j_x, j_y when every free relaxation
// rate is 1, because those moments then relax fully to m_eq + F/2 and the
// collision needs no other moment of f).  Rows are loaded PF iterations
// ahead, so their latency overlaps the stencil stages of the current row.
// The loop is unrolled by U so that every register ring index is static.
// ---------------------------------------------------------------------------
#ifndef LBCH_PF
#define LBCH_PF 1
#endif

// Native 16-byte vectors (not HIP_vector_type: arrays of those are not split
// into registers and end up in scratch memory).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = f32x4; };
template <> struct Vec16<double> { using type = f64x2; };

// Row loader.  Direct form: each lane pulls its nine populations with one
// 4- or 8-byte load per plane (shifted by the pull, so unaligned to the row).
// Staged form: the lanes of the workgroup fetch the nine plane-rows the strip
// needs as aligned 16-byte chunks (full cache lines, one wide load per chunk),
// park them in LDS and each lane then reads its shifted values from there.
template <typename T, int NT, bool STAGED>
struct RowLoader;

template <typename T, int NT>
struct RowLoader<T, NT, false> {
    using Buf = T[9];
    const T* P[9];
    int xc, cm, cp, nx, ny, pitch;
    // lane0: column of lane 0 (the strip's first column minus its halo)
    __device__ __forceinline__ void setup(const T* fin, const Grid& g, int lane0, T* /*s_f*/) {
        nx = g.nx;
        ny = g.ny;
        pitch = g.pitch;
#pragma unroll
        for (int i = 0; i < 9; ++i) P[i] = fin + i * g.plane;
        xc = (lane0 + (int)threadIdx.x) % nx;
        if (xc < 0) xc += nx;
        cm = (xc == 0) ? nx - 1 : xc - 1;
        cp = (xc == nx - 1) ? 0 : xc + 1;
    }
    __device__ __forceinline__ void issue(int r, Buf& f) const {
        const int rm = (r == 0) ? ny - 1 : r - 1;
        const int rp = (r == ny - 1) ? 0 : r + 1;
        const int o0 = r * pitch, om = rm * pitch, op = rp * pitch;
        f[0] = P[0][o0 + xc];
        f[1] = P[1][o0 + cm];
        f[2] = P[2][om + xc];
        f[3] = P[3][o0 + cp];
        f[4] = P[4][op + xc];
        f[5] = P[5][om + cm];
        f[6] = P[6][om + cp];
        f[7] = P[7][op + cp];
        f[8] = P[8][op + cm];
    }
    // no LDS staging: the lane's values are the loaded ones
    __device__ __forceinline__ void park(const Buf&, T*) const {}
    __device__ __forceinline__ void fetch(const Buf& b, const T*, T (&f)[9]) const {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = b[i];
    }
    static constexpr bool kNeedsBarrier = false;
};

template <typename T, int NT>
struct RowLoader<T, NT, true> {
    using V = typename Vec16<T>::type;
    static constexpr int VEC = 16 / sizeof(T);
    static constexpr int SPAN = NT + 4;             // staged columns lane0-1 .. lane0+NT+2
    static constexpr int CPR = SPAN / VEC;          // chunks per plane-row
    static constexpr int NCH = 9 * CPR;
    static constexpr int M = (NCH + NT - 1) / NT;   // chunks per lane
    using Buf = V[M];
    const T* fin;
    int off[M];            // element offset of the chunk: plane + first column (wrapped)
    int dy[M];             // row offset of the plane's pull: -1, 0, +1
    unsigned live;         // bit m: chunk m exists
    int nx, ny, pitch;
    // lane0: column of lane 0; staged column 0 is lane0 - 1, which must be a
    // multiple of VEC
    __device__ __forceinline__ void setup(const T* f, const Grid& g, int lane0, T* /*s_f*/) {
        fin = f;
        nx = g.nx;
        ny = g.ny;
        pitch = g.pitch;
        live = 0u;
        // requires nx % VEC == 0 (checked by the launcher): a chunk that starts
        // on a VEC boundary then never straddles the periodic seam, so even the
        // wrapped chunks of the first and last strips are single aligned loads
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int ch = (int)threadIdx.x + m * NT;
            const int i = ch / CPR;
            const int q = ch - i * CPR;
            const int ii = i < 9 ? i : 0;
            // c_iy of eq 20a: the pull of plane i reads row r - c_iy
            dy[m] = (ii == 2 || ii == 5 || ii == 6) ? -1 : ((ii == 4 || ii == 7 || ii == 8) ? 1 : 0);
            int cw = (lane0 - 1 + q * VEC) % nx;
            if (cw < 0) cw += nx;
            off[m] = ii * (int)g.plane + cw;
            if (ch < NCH) live |= 1u << m;
        }
    }
    __device__ __forceinline__ void issue(int r, Buf& b) const {
        const int rm = (r == 0) ? ny - 1 : r - 1;
        const int rp = (r == ny - 1) ? 0 : r + 1;
        const int o0 = r * pitch, om = rm * pitch, op = rp * pitch;
        // unconditional (lanes past the last chunk re-read a valid chunk of
        // plane 0 and discard it): no branch around the loads, so they stay
        // in flight until park()
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int o = off[m] + (dy[m] < 0 ? om : (dy[m] > 0 ? op : o0));
            b[m] = *reinterpret_cast<const V*>(fin + o);
        }
    }
    __device__ __forceinline__ void park(const Buf& b, T* s_f) const {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (live & (1u << m)) {
                const int ch = (int)threadIdx.x + m * NT;
                *reinterpret_cast<V*>(s_f + ch * VEC) = b[m];
            }
        }
    }
    __device__ __forceinline__ void fetch(const Buf&, const T* s_f, T (&f)[9]) const {
        const int t = threadIdx.x;
        // staged index of the lane's column is t + 1; the pull of direction i reads column x - c_ix
        f[0] = s_f[0 * SPAN + t + 1];
        f[1] = s_f[1 * SPAN + t];
        f[2] = s_f[2 * SPAN + t + 1];
        f[3] = s_f[3 * SPAN + t + 2];
        f[4] = s_f[4 * SPAN + t + 1];
        f[5] = s_f[5 * SPAN + t];
        f[6] = s_f[6 * SPAN + t + 2];
        f[7] = s_f[7 * SPAN + t + 2];
        f[8] = s_f[8 * SPAN + t];
    }
    static constexpr bool kNeedsBarrier = true;
};

template <typename T, int NT, bool STAGED>
struct StageLds {
    static constexpr int kF = STAGED ? 9 * (NT + 4) : 1;
};

// ---- stage bodies shared by the one-step and the two-step sweeps ----------
// Rings hold three consecutive rows: slot sN = newest (row r+1 of the stage's
// centre row r), sC = row r, sS = row r - 1.

// Stage B at one lane: grad phi and lap phi (eq 26), gamma and gamma' (eq 6
// generalised), Q (eq 15, derived or printed form), w (eq 9 / eq 8); writes
// Q and w to their rings and returns the pointwise part of mu_beta (eq 16
// without div Q and lap w) and mu_alpha (eq 16).
template <typename T, int NT>
__device__ __forceinline__ void stage_b(const StepCoef<T>& c, T (*s_phi)[NT], T (*s_qx)[NT], T (*s_qy)[NT],
                                        T (*s_w)[NT], int sN, int sC, int sS, int t, T& tl, T& mua) {
    const T pC = s_phi[sC][t], pE = s_phi[sC][t + 1], pW = s_phi[sC][t - 1];
    const T pN = s_phi[sN][t], pNE = s_phi[sN][t + 1], pNW = s_phi[sN][t - 1];
    const T pS = s_phi[sS][t], pSE = s_phi[sS][t + 1], pSW = s_phi[sS][t - 1];
    const T px = c.g3 * (pE - pW) + c.g12 * ((pNE - pSW) + (pSE - pNW));
    const T py = c.g3 * (pN - pS) + c.g12 * ((pNE - pSW) + (pNW - pSE));
    const T lap = c.l23 * ((pE + pW) + (pN + pS)) + c.l16 * ((pNE + pSW) + (pNW + pSE)) - c.l103 * pC;
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
    tl = tl0;
    mua = fb - c.kappa * lap;
}

// Stage C at one lane: div Q (eq 26a per component) and lap w (eq 26b)
// complete mu_beta (eqs 13, 16).
template <typename T, int NT>
__device__ __forceinline__ T stage_c(const StepCoef<T>& c, T (*s_qx)[NT], T (*s_qy)[NT], T (*s_w)[NT], int sN,
                                     int sC, int sS, int t, T tl) {
    const T divq = c.g3 * (s_qx[sC][t + 1] - s_qx[sC][t - 1]) +
                   c.g12 * ((s_qx[sN][t + 1] - s_qx[sS][t - 1]) + (s_qx[sS][t + 1] - s_qx[sN][t - 1])) +
                   c.g3 * (s_qy[sN][t] - s_qy[sS][t]) +
                   c.g12 * ((s_qy[sN][t + 1] - s_qy[sS][t - 1]) + (s_qy[sN][t - 1] - s_qy[sS][t + 1]));
    T mb = tl - divq;
    if (c.reg != REG_NONE) {
        const T lw = c.l23 * ((s_w[sC][t + 1] + s_w[sC][t - 1]) + (s_w[sN][t] + s_w[sS][t])) +
                     c.l16 * ((s_w[sN][t + 1] + s_w[sS][t - 1]) + (s_w[sN][t - 1] + s_w[sS][t + 1])) -
                     c.l103 * s_w[sC][t];
        mb += c.eps * lw;
    }
    return mb;
}

// Stage D at one lane: grad mu_beta (eq 26a), then the collision (eqs 17-19,
// 23, 25) of the node's pulled populations (all nine, or phi, j_x, j_y).
template <typename T, int NT, bool UNIT>
__device__ __forceinline__ void stage_d(const StepCoef<T>& c, T (*s_mb)[NT], int sN, int sC, int sS, int t,
                                        const T (&pop)[9], const T (&red)[3], T mu_a, T (&o)[9]) {
    const T gx = c.g3 * (s_mb[sC][t + 1] - s_mb[sC][t - 1]) +
                 c.g12 * ((s_mb[sN][t + 1] - s_mb[sS][t - 1]) + (s_mb[sS][t + 1] - s_mb[sN][t - 1]));
    const T gy = c.g3 * (s_mb[sN][t] - s_mb[sS][t]) +
                 c.g12 * ((s_mb[sN][t + 1] - s_mb[sS][t - 1]) + (s_mb[sN][t - 1] - s_mb[sS][t + 1]));
    if (UNIT) collide_unit<T>(red[0], red[1], red[2], mu_a, gx, gy, c, o);
    else collide<T>(pop, mu_a, gx, gy, c, o);
}

// Stage A after the pull: phi = sum f_i (eq 22) in the summation order the
// collision uses, and what stage D keeps of the node.
template <typename T, bool UNIT>
__device__ __forceinline__ T stage_a(const T (&f)[9], T (&pop)[9], T (&red)[3]) {
    const T a = (f[1] + f[2]) + (f[3] + f[4]);
    const T b = (f[5] + f[6]) + (f[7] + f[8]);
    const T phi = f[0] + a + b;
    if (UNIT) {
        red[0] = phi;
        red[1] = (f[1] - f[3]) + ((f[5] - f[7]) + (f[8] - f[6]));   // j_x = m_3
        red[2] = (f[2] - f[4]) + ((f[5] - f[7]) + (f[6] - f[8]));   // j_y = m_5
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) pop[i] = f[i];
    }
    return phi;
}

template <typename T, int NT, bool UNIT, bool STAGED>
__device__ __forceinline__ void sweep_strip(const T* __restrict__ fin, T* __restrict__ fout, const Grid& g,
                                            const int x0, const int wlen, const int y0, const int hlen,
                                            const StepCoef<T>& c, T (*s_phi)[NT], T (*s_qx)[NT], T (*s_qy)[NT],
                                            T (*s_w)[NT], T (*s_mb)[NT], T* s_f) {
    constexpr int U = 4;
    constexpr int PF = LBCH_PF;
    static_assert(PF >= 1 && PF <= 2, "prefetch distance");
    using Loader = RowLoader<T, NT, STAGED>;
    const int nx = g.nx, ny = g.ny, pitch = g.pitch;
    const int niter = hlen + 6;
    const int t = threadIdx.x;

    Loader ld;
    ld.setup(fin, g, x0 - 3, s_f);
    int xc = (x0 - 3 + t) % nx;      // the lane's column (wrapped)
    if (xc < 0) xc += nx;

    int rA = (y0 - 3) % ny;          // row of the next load (wrapped)
    if (rA < 0) rA += ny;

    typename Loader::Buf buf[U];     // rows in flight
    T pop[U][9];                     // general path: pulled populations kept until D
    T red[U][3];                     // unit-rate path: phi, j_x, j_y kept until D
    T mua[U];                        // mu_alpha (B -> D, two iterations)
    T tloc[U];                       // local part of mu_beta (B -> C, one iteration)

#pragma unroll
    for (int q = 0; q < PF; ++q) {
        if (q < niter) {
            ld.issue(rA, buf[q]);
            rA = (rA == ny - 1) ? 0 : rA + 1;
        }
    }

    for (int jb = 0; jb < niter; jb += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int j = jb + k;
            if (j < niter) {
                const int sN = j % 3, sC = (j + 2) % 3, sS = (j + 1) % 3;
                // ---- A: populations of row r, phi ----
                if (Loader::kNeedsBarrier) {
                    ld.park(buf[k], s_f);
                    lds_barrier();
                }
                {
                    T f[9];
                    ld.fetch(buf[k], s_f, f);
                    s_phi[sN][t] = stage_a<T, UNIT>(f, pop[k], red[k]);
                }
                // unconditional: past the last row of the sweep this fetches a
                // (wrapped, valid) row that is never used; a branch here would
                // force the loads to complete before the join
                ld.issue(rA, buf[(k + PF) % U]);
                rA = (rA == ny - 1) ? 0 : rA + 1;
                lds_barrier();
                // ---- B: row r-1 ----
                if (j >= 2 && t >= 1 && t < NT - 1)
                    stage_b<T, NT>(c, s_phi, s_qx, s_qy, s_w, sN, sC, sS, t, tloc[k], mua[k]);
                lds_barrier();
                // ---- C: row r-2 ----
                if (j >= 4 && t >= 2 && t < NT - 2)
                    s_mb[sN][t] = stage_c<T, NT>(c, s_qx, s_qy, s_w, sN, sC, sS, t, tloc[(k + U - 1) % U]);
                lds_barrier();
                // ---- D: row r-3 ----
                if (j >= 6 && t >= 3 && t < 3 + wlen) {
                    T o[9];
                    stage_d<T, NT, UNIT>(c, s_mb, sN, sC, sS, t, pop[(k + U - 3) % U], red[(k + U - 3) % U],
                                         mua[(k + U - 2) % U], o);
                    const int rd = y0 - 6 + j;
                    T* __restrict__ q = fout + ((long long)rd * pitch + xc);
#pragma unroll
                    for (int i = 0; i < 9; ++i) q[i * g.plane] = o[i];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Two time steps per sweep (temporal blocking).  Lane t owns column
// x0 - 7 + t; a strip yields W = NT - 16 columns of the second step.  Each
// iteration j loads row a = y0 - 7 + j and runs the eight stages of the two
// steps in two phases with one barrier between them; every stage reads only
// rows that an earlier phase has finished, so a stage trails its producer by
// the rows that needs (offsets below a):
//   phase 1: A1 (a), C1 (a-3), A2 (a-6), C2 (a-9)
//   phase 2: B1 (a-1), D1 (a-4), B2 (a-7), D2 (a-10, stored)
// A1..D1 are the first step as in sweep_strip, except that D1 keeps its
// post-collision row d on chip: planes 0, 2, 4 (whose pull stays in the
// lane's column) in registers, 1/3, 5/6 and 7/8 in LDS rings of 2, 3 and 1
// rows (A2 pulls them 2, 3 and 1 iterations after D1 wrote them).  A2..D2
// are the second step; D2 stores.  Every population is read from and written
// to HBM once per two updates.  With the staged row loader one more barrier
// separates parking a row in LDS from reading it: three barriers per row.
// Every ring slot is indexed by the iteration that wrote it (LDS rings: j mod
// 3, register rings: j mod 6); the loop is unrolled six times so that all of
// them are static.  Valid lanes shrink by one per stage: A1 all, B1
// [1, NT-1), C1 [2, NT-2), D1 [3, NT-3), A2 [4, NT-4), B2 [5, NT-5),
// C2 [6, NT-6), D2 [7, NT-7).
// ---------------------------------------------------------------------------
template <typename T, int NT>
struct Pass2Lds {
    T phi[3][NT], qx[3][NT], qy[3][NT], w[3][NT], mb[3][NT];
};

constexpr int mod3(int v) { return ((v % 3) + 3) % 3; }
constexpr int mod6(int v) { return ((v % 6) + 6) % 6; }

// EXTRAP: the stored state is f_{n+2} + ext (f_{n+2} - f_n) elementwise, f_n
// being this launch's input at the same element (a projective step of the
// populations fused into the store).
template <typename T, int NT, bool UNIT, bool STAGED, bool EXTRAP = false>
__device__ __forceinline__ void sweep_strip2(const T* __restrict__ fin, T* __restrict__ fout, const Grid& g,
                                             const int x0, const int wlen, const int y0, const int hlen,
                                             const StepCoef<T>& c, Pass2Lds<T, NT>& L1, Pass2Lds<T, NT>& L2,
                                             T (*s_13)[2][NT], T (*s_56)[2][NT], T (*s_78)[NT], T* s_f,
                                             const T ext = T(0)) {
    constexpr int U = 6;
    using Loader = RowLoader<T, NT, STAGED>;
    const int nx = g.nx, ny = g.ny, pitch = g.pitch;
    const int niter = hlen + 17;
    const int t = threadIdx.x;

    Loader ld;
    ld.setup(fin, g, x0 - 7, s_f);
    int xc = (x0 - 7 + t) % nx;
    if (xc < 0) xc += nx;
    int rA = (y0 - 7) % ny;
    if (rA < 0) rA += ny;

    typename Loader::Buf buf[2];
    T pop1[U][9], red1[U][3], mua1[U], tl1[U];
    T pop2[U][9], red2[U][3], mua2[U], tl2[U];
    T o0r[U], o2r[U], o4r[U];          // D1 planes 0, 2, 4 of the lane (A2 pulls them 2, 3, 1 iterations later)
#pragma unroll
    for (int k = 0; k < U; ++k) o0r[k] = o2r[k] = o4r[k] = T(0);

    ld.issue(rA, buf[0]);
    rA = (rA == ny - 1) ? 0 : rA + 1;

    for (int jb = 0; jb < niter; jb += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int j = jb + k;
            if (j < niter) {
                // slots written by iterations j, j-1, j-2, j-3 (LDS rings of three rows)
                const int s0 = mod3(k), s1 = mod3(k - 1), s2 = mod3(k - 2);
                if (Loader::kNeedsBarrier) {
                    ld.park(buf[k & 1], s_f);
                    lds_barrier();
                }
                // ======== phase 1 ========
                // ---- A1: row a ----
                {
                    T f[9];
                    ld.fetch(buf[k & 1], s_f, f);
                    L1.phi[s0][t] = stage_a<T, UNIT>(f, pop1[k], red1[k]);
                }
                // unconditional: past the last row of the sweep this fetches a
                // (wrapped, valid) row that is never used
                ld.issue(rA, buf[(k + 1) & 1]);
                rA = (rA == ny - 1) ? 0 : rA + 1;
                // ---- C1: row a-3 (its q, w rows come from B1 of iterations j-1 .. j-3) ----
                if (j >= 5 && t >= 2 && t < NT - 2)
                    L1.mb[s0][t] = stage_c<T, NT>(c, L1.qx, L1.qy, L1.w, s1, s2, s0, t, tl1[mod6(k - 2)]);
                // ---- A2: row a-6, pulled from D1's rows of iterations j-1 .. j-3 ----
                if (j >= 10 && t >= 4 && t < NT - 4) {
                    T f[9];
                    const int p13 = (k + U - 2) & 1, p56 = mod3(k - 3);
                    f[0] = o0r[mod6(k - 2)];
                    f[1] = s_13[p13][0][t - 1];
                    f[2] = o2r[mod6(k - 3)];
                    f[3] = s_13[p13][1][t + 1];
                    f[4] = o4r[mod6(k - 1)];
                    f[5] = s_56[p56][0][t - 1];
                    f[6] = s_56[p56][1][t + 1];
                    f[7] = s_78[0][t + 1];
                    f[8] = s_78[1][t - 1];
                    L2.phi[s0][t] = stage_a<T, UNIT>(f, pop2[k], red2[k]);
                }
                // ---- C2: row a-9 ----
                if (j >= 15 && t >= 6 && t < NT - 6)
                    L2.mb[s0][t] = stage_c<T, NT>(c, L2.qx, L2.qy, L2.w, s1, s2, s0, t, tl2[mod6(k - 2)]);
                lds_barrier();
                // ======== phase 2 ========
                // ---- B1: row a-1 ----
                if (j >= 2 && t >= 1 && t < NT - 1)
                    stage_b<T, NT>(c, L1.phi, L1.qx, L1.qy, L1.w, s0, s1, s2, t, tl1[k], mua1[k]);
                // ---- D1: row d = a-4, kept on chip ----
                if (j >= 7 && t >= 3 && t < NT - 3) {
                    T o[9];
                    stage_d<T, NT, UNIT>(c, L1.mb, s0, s1, s2, t, pop1[mod6(k - 4)], red1[mod6(k - 4)],
                                         mua1[mod6(k - 3)], o);
                    o0r[k] = o[0];
                    o2r[k] = o[2];
                    o4r[k] = o[4];
                    s_13[k & 1][0][t] = o[1];
                    s_13[k & 1][1][t] = o[3];
                    s_56[s0][0][t] = o[5];
                    s_56[s0][1][t] = o[6];
                    s_78[0][t] = o[7];
                    s_78[1][t] = o[8];
                }
                // ---- B2: row a-7 ----
                if (j >= 12 && t >= 5 && t < NT - 5)
                    stage_b<T, NT>(c, L2.phi, L2.qx, L2.qy, L2.w, s0, s1, s2, t, tl2[k], mua2[k]);
                // ---- D2: row a-10, stored ----
                if (j >= 17 && t >= 7 && t < 7 + wlen) {
                    T o[9];
                    stage_d<T, NT, UNIT>(c, L2.mb, s0, s1, s2, t, pop2[mod6(k - 4)], red2[mod6(k - 4)],
                                         mua2[mod6(k - 3)], o);
                    const int rd = y0 - 17 + j;
                    T* __restrict__ q = fout + ((long long)rd * pitch + xc);
                    if constexpr (EXTRAP) {
                        const T* __restrict__ pv = fin + ((long long)rd * pitch + xc);
                        T prev[9];
#pragma unroll
                        for (int i = 0; i < 9; ++i) prev[i] = pv[i * g.plane];
#pragma unroll
                        for (int i = 0; i < 9; ++i) q[i * g.plane] = o[i] + ext * (o[i] - prev[i]);
                    } else {
#pragma unroll
                        for (int i = 0; i < 9; ++i) q[i * g.plane] = o[i];
                    }
                }
                lds_barrier();
            }
        }
    }
}

template <typename T, int NT, bool UNIT, bool STAGED>
__global__ __launch_bounds__(NT) void step_fused(const T* __restrict__ fin, T* __restrict__ fout,
                                                 const Grid g, const Tiling tl, const StepCoef<T> c) {
    __shared__ T s_phi[3][NT];
    __shared__ T s_qx[3][NT];
    __shared__ T s_qy[3][NT];
    __shared__ T s_w[3][NT];
    __shared__ T s_mb[3][NT];
    __shared__ __align__(16) T s_f[StageLds<T, NT, STAGED>::kF];
    const int bid = blockIdx.x;
    const int tile = (bid & 7) * tl.per_xcd + (bid >> 3);
    if (tile >= tl.ntiles) return;
    const int strip = tile % tl.strips;
    const int chunk = tile / tl.strips;
    const int x0 = strip * tl.W;
    const int y0 = chunk * tl.hc;
    sweep_strip<T, NT, UNIT, STAGED>(fin, fout, g, x0, min(tl.W, g.nx - x0), y0, min(tl.hc, g.ny - y0), c, s_phi,
                                     s_qx, s_qy, s_w, s_mb, s_f);
}

// Waves per SIMD the two-step sweep is compiled for (the launch bound's second
// argument): the LDS of one CU holds three FP32 workgroups of 256 lanes or six
// of 128, twelve waves, and with unit free rates the register budget is held
// to that (three waves per SIMD, 168 VGPRs).  The general-rate collision keeps all nine
// populations of five rows per step in registers (about 190 VGPRs, two waves);
// FP64 rings and 512-lane workgroups are limited by LDS.
template <typename T, int NT, bool UNIT>
constexpr int kStep2Waves = (UNIT && sizeof(T) == 4 && NT <= 256) ? 3 : 1;

// Two steps per launch: fin holds the state at step n, fout receives step n + 2.
template <typename T, int NT, bool UNIT, bool STAGED>
__global__ __launch_bounds__(NT, (kStep2Waves<T, NT, UNIT>)) void step2_fused(const T* __restrict__ fin, T* __restrict__ fout,
                                                  const Grid g, const Tiling tl, const StepCoef<T> c) {
    __shared__ Pass2Lds<T, NT> L1;
    __shared__ Pass2Lds<T, NT> L2;
    __shared__ T s_13[2][2][NT];
    __shared__ T s_56[3][2][NT];
    __shared__ T s_78[2][NT];
    __shared__ __align__(16) T s_f[StageLds<T, NT, STAGED>::kF];
    const int bid = blockIdx.x;
    const int tile = (bid & 7) * tl.per_xcd + (bid >> 3);
    if (tile >= tl.ntiles) return;
    const int strip = tile % tl.strips;
    const int chunk = tile / tl.strips;
    const int x0 = strip * tl.W;
    const int y0 = chunk * tl.hc;
    sweep_strip2<T, NT, UNIT, STAGED>(fin, fout, g, x0, min(tl.W, g.nx - x0), y0, min(tl.hc, g.ny - y0), c, L1, L2,
                                      s_13, s_56, s_78, s_f);
}

// Two steps per launch with the projective extrapolation of the populations
// in the store: fout = f_{n+2} + ext (f_{n+2} - f_n), fin holding f_n.
template <typename T, int NT, bool UNIT, bool STAGED>
__global__ __launch_bounds__(NT, (kStep2Waves<T, NT, UNIT>)) void step2_extrap(const T* __restrict__ fin, T* __restrict__ fout,
                                                   const Grid g, const Tiling tl, const StepCoef<T> c, const T ext) {
    __shared__ Pass2Lds<T, NT> L1;
    __shared__ Pass2Lds<T, NT> L2;
    __shared__ T s_13[2][2][NT];
    __shared__ T s_56[3][2][NT];
    __shared__ T s_78[2][NT];
    __shared__ __align__(16) T s_f[StageLds<T, NT, STAGED>::kF];
    const int bid = blockIdx.x;
    const int tile = (bid & 7) * tl.per_xcd + (bid >> 3);
    if (tile >= tl.ntiles) return;
    const int strip = tile % tl.strips;
    const int chunk = tile / tl.strips;
    const int x0 = strip * tl.W;
    const int y0 = chunk * tl.hc;
    sweep_strip2<T, NT, UNIT, STAGED, true>(fin, fout, g, x0, min(tl.W, g.nx - x0), y0, min(tl.hc, g.ny - y0), c,
                                            L1, L2, s_13, s_56, s_78, s_f, ext);
}

// ---------------------------------------------------------------------------
// Ensemble step: every strip-tile of every member of a batch, one persistent
// launch.  Workgroups take tiles from a work queue: a 64-bit counter that
// only ever grows; in one launch the counter passes through exactly
// total_tiles + gridDim.x values (each workgroup's last take is the one past
// the end), so taking `counter mod (total_tiles + gridDim.x)` needs no reset
// between launches and works unchanged inside a captured graph.  Every
// workgroup leaves the loop after its first take past the end.
// ---------------------------------------------------------------------------
template <typename T, int NT, int DEPTH>
struct BatchLds;
template <typename T, int NT>
struct BatchLds<T, NT, 1> {
    T phi[3][NT], qx[3][NT], qy[3][NT], w[3][NT], mb[3][NT];
};
template <typename T, int NT>
struct BatchLds<T, NT, 2> {
    Pass2Lds<T, NT> L1, L2;
    T s13[2][2][NT], s56[3][2][NT], s78[2][NT];
};

// DEPTH time steps per launch (1 or 2); members' tiles are strips of
// NT - 8 * DEPTH columns.
template <typename T, int NT, bool UNIT_ALL, int DEPTH>
__global__ __launch_bounds__(NT) void batch_step(const T* __restrict__ fin, T* __restrict__ fout,
                                                 const BatchMember<T>* __restrict__ members,
                                                 const int* __restrict__ tile_member, const int total_tiles,
                                                 unsigned long long* __restrict__ counter) {
    __shared__ BatchLds<T, NT, DEPTH> sh;
    __shared__ int s_tile;
    const unsigned long long period = (unsigned long long)total_tiles + gridDim.x;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)(atomicAdd(counter, 1ull) % period);
        __syncthreads();
        const int tile = s_tile;
        __syncthreads();
        if (tile >= total_tiles) break;
        const BatchMember<T>& d = members[tile_member[tile]];
        const Grid g = d.g;
        const StepCoef<T> c = d.c;
        const int local = tile - d.tile_begin;
        const int strip = local % d.strips;
        const int chunk = local / d.strips;
        constexpr int W = NT - 8 * DEPTH;
        const int x0 = strip * W;
        const int y0 = chunk * d.hc;
        const T* mfin = fin + d.base;
        T* mfout = fout + d.base;
        const int wl = min(W, g.nx - x0), hl = min(d.hc, g.ny - y0);
        if constexpr (DEPTH == 1) {
            if (UNIT_ALL || c.unit)
                sweep_strip<T, NT, true, false>(mfin, mfout, g, x0, wl, y0, hl, c, sh.phi, sh.qx, sh.qy, sh.w, sh.mb,
                                                nullptr);
            else
                sweep_strip<T, NT, false, false>(mfin, mfout, g, x0, wl, y0, hl, c, sh.phi, sh.qx, sh.qy, sh.w, sh.mb,
                                                 nullptr);
        } else {
            if (UNIT_ALL || c.unit)
                sweep_strip2<T, NT, true, false>(mfin, mfout, g, x0, wl, y0, hl, c, sh.L1, sh.L2, sh.s13, sh.s56,
                                                 sh.s78, nullptr);
            else
                sweep_strip2<T, NT, false, false>(mfin, mfout, g, x0, wl, y0, hl, c, sh.L1, sh.L2, sh.s13, sh.s56,
                                                  sh.s78, nullptr);
        }
        __syncthreads();
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
// Reductions: float64 partials per workgroup (block_reduce_waves), combined by
// finalize_k, in a fixed order: deterministic.
// ---------------------------------------------------------------------------
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
    block_reduce_waves<4>(v, kind, partials + 4 * blockIdx.x);
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
    block_reduce_waves<4>(v, kind, partials + 4 * blockIdx.x);
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
    block_reduce_waves<4>(v, kind, out);
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

__global__ void zero_u64_k(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void zero_u32_k(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
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

template <typename T, bool UNIT, bool STAGED>
static hipError_t launch_step_v(const T* fin, T* fout, const Grid& g, const Tiling& t, const StepCoef<T>& c,
                                hipStream_t s) {
    dim3 grid(t.nblocks);
    if (t.depth == 2) {
        switch (t.nt) {
            case 128: step2_fused<T, 128, UNIT, STAGED><<<grid, 128, 0, s>>>(fin, fout, g, t, c); break;
            case 256: step2_fused<T, 256, UNIT, STAGED><<<grid, 256, 0, s>>>(fin, fout, g, t, c); break;
            case 512:
                // the float64 rings of 512 lanes exceed the LDS of one workgroup
                if constexpr (sizeof(T) == 4) {
                    step2_fused<T, 512, UNIT, STAGED><<<grid, 512, 0, s>>>(fin, fout, g, t, c);
                    break;
                } else {
                    return hipErrorInvalidValue;
                }
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (t.depth != 1) return hipErrorInvalidValue;
    switch (t.nt) {
        case 64: step_fused<T, 64, UNIT, STAGED><<<grid, 64, 0, s>>>(fin, fout, g, t, c); break;
        case 128: step_fused<T, 128, UNIT, STAGED><<<grid, 128, 0, s>>>(fin, fout, g, t, c); break;
        case 256: step_fused<T, 256, UNIT, STAGED><<<grid, 256, 0, s>>>(fin, fout, g, t, c); break;
        case 512: step_fused<T, 512, UNIT, STAGED><<<grid, 512, 0, s>>>(fin, fout, g, t, c); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// FP32 grids whose width is a multiple of 4 use the LDS-staged row loader
// (aligned 16-byte loads); other FP32 widths and FP64 (whose pulls are
// 8-byte loads already) pull directly.
template <typename T>
static hipError_t launch_step_t(const T* fin, T* fout, const Grid& g, const Tiling& t, const StepCoef<T>& c,
                                hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        if (g.nx % 4 == 0 && t.staged)
            return c.unit ? launch_step_v<T, true, true>(fin, fout, g, t, c, s)
                          : launch_step_v<T, false, true>(fin, fout, g, t, c, s);
    }
    return c.unit ? launch_step_v<T, true, false>(fin, fout, g, t, c, s)
                  : launch_step_v<T, false, false>(fin, fout, g, t, c, s);
}

template <typename T, bool UNIT, bool STAGED>
static hipError_t launch_step2_extrap_v(const T* fin, T* fout, const Grid& g, const Tiling& t, const StepCoef<T>& c,
                                        T ext, hipStream_t s) {
    if (t.depth != 2) return hipErrorInvalidValue;
    dim3 grid(t.nblocks);
    switch (t.nt) {
        case 128: step2_extrap<T, 128, UNIT, STAGED><<<grid, 128, 0, s>>>(fin, fout, g, t, c, ext); break;
        case 256: step2_extrap<T, 256, UNIT, STAGED><<<grid, 256, 0, s>>>(fin, fout, g, t, c, ext); break;
        case 512:
            if constexpr (sizeof(T) == 4) {
                step2_extrap<T, 512, UNIT, STAGED><<<grid, 512, 0, s>>>(fin, fout, g, t, c, ext);
                break;
            } else {
                return hipErrorInvalidValue;
            }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_step2_extrap_t(const T* fin, T* fout, const Grid& g, const Tiling& t, const StepCoef<T>& c,
                                        T ext, hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        if (g.nx % 4 == 0 && t.staged)
            return c.unit ? launch_step2_extrap_v<T, true, true>(fin, fout, g, t, c, ext, s)
                          : launch_step2_extrap_v<T, false, true>(fin, fout, g, t, c, ext, s);
    }
    return c.unit ? launch_step2_extrap_v<T, true, false>(fin, fout, g, t, c, ext, s)
                  : launch_step2_extrap_v<T, false, false>(fin, fout, g, t, c, ext, s);
}

hipError_t launch_step2_extrap(int precision, const void* fin, void* fout, const Grid& g, const Tiling& t,
                               const void* coef, double ext, hipStream_t s) {
    if (precision == 0)
        return launch_step2_extrap_t<double>((const double*)fin, (double*)fout, g, t, *(const StepCoef<double>*)coef,
                                             ext, s);
    return launch_step2_extrap_t<float>((const float*)fin, (float*)fout, g, t, *(const StepCoef<float>*)coef,
                                        (float)ext, s);
}

hipError_t launch_step(int precision, const void* fin, void* fout, const Grid& g, const Tiling& t, const void* coef,
                       hipStream_t s) {
    if (precision == 0)
        return launch_step_t<double>((const double*)fin, (double*)fout, g, t, *(const StepCoef<double>*)coef, s);
    return launch_step_t<float>((const float*)fin, (float*)fout, g, t, *(const StepCoef<float>*)coef, s);
}


template <typename T, bool UA, int D>
static hipError_t launch_batch_d(int nt, const T* fin, T* fout, const BatchMember<T>* m, const int* tm, int total,
                                 int nblocks, unsigned long long* ctr, hipStream_t s) {
    switch (nt) {
        case 64:
            if constexpr (D == 1) {
                batch_step<T, 64, UA, D><<<nblocks, 64, 0, s>>>(fin, fout, m, tm, total, ctr);
                break;
            } else {
                return hipErrorInvalidValue;
            }
        case 128: batch_step<T, 128, UA, D><<<nblocks, 128, 0, s>>>(fin, fout, m, tm, total, ctr); break;
        case 256: batch_step<T, 256, UA, D><<<nblocks, 256, 0, s>>>(fin, fout, m, tm, total, ctr); break;
        case 512:
            // the float64 rings of a two-step sweep of 512 lanes exceed the LDS of one workgroup
            if constexpr (D == 1 || sizeof(T) == 4) {
                batch_step<T, 512, UA, D><<<nblocks, 512, 0, s>>>(fin, fout, m, tm, total, ctr);
                break;
            } else {
                return hipErrorInvalidValue;
            }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool UA>
static hipError_t launch_batch_t(int depth, int nt, const T* fin, T* fout, const BatchMember<T>* m, const int* tm,
                                 int total, int nblocks, unsigned long long* ctr, hipStream_t s) {
    if (depth == 2) return launch_batch_d<T, UA, 2>(nt, fin, fout, m, tm, total, nblocks, ctr, s);
    if (depth == 1) return launch_batch_d<T, UA, 1>(nt, fin, fout, m, tm, total, nblocks, ctr, s);
    return hipErrorInvalidValue;
}

hipError_t launch_batch_step(int precision, int depth, int nt, bool unit_all, const void* fin, void* fout,
                             const void* members, const int* tile_member, int total_tiles, int nblocks,
                             unsigned long long* ctr, hipStream_t s) {
    if (precision == 0) {
        auto f = unit_all ? launch_batch_t<double, true> : launch_batch_t<double, false>;
        return f(depth, nt, (const double*)fin, (double*)fout, (const BatchMember<double>*)members, tile_member,
                 total_tiles, nblocks, ctr, s);
    }
    auto f = unit_all ? launch_batch_t<float, true> : launch_batch_t<float, false>;
    return f(depth, nt, (const float*)fin, (float*)fout, (const BatchMember<float>*)members, tile_member, total_tiles,
             nblocks, ctr, s);
}

template <typename T, bool UA, int D>
static int occ_d(int nt) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (nt) {
        case 64:
            if constexpr (D == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_step<T, 64, UA, D>, 64, 0);
            break;
        case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_step<T, 128, UA, D>, 128, 0); break;
        case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_step<T, 256, UA, D>, 256, 0); break;
        case 512:
            if constexpr (D == 1 || sizeof(T) == 4)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_step<T, 512, UA, D>, 512, 0);
            break;
        default: break;
    }
    return (e == hipSuccess && n > 0) ? n : 1;
}

template <typename T, bool UA>
static int occ_t(int depth, int nt) {
    return depth == 2 ? occ_d<T, UA, 2>(nt) : occ_d<T, UA, 1>(nt);
}

int batch_blocks_per_cu(int precision, int depth, int nt, bool unit_all) {
    if (precision == 0) return unit_all ? occ_t<double, true>(depth, nt) : occ_t<double, false>(depth, nt);
    return unit_all ? occ_t<float, true>(depth, nt) : occ_t<float, false>(depth, nt);
}

template <typename T, bool UNIT, bool STAGED>
static int occ_step_t(int depth, int nt) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    if (depth == 2) {
        switch (nt) {
            case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2_fused<T, 128, UNIT, STAGED>, 128, 0); break;
            case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2_fused<T, 256, UNIT, STAGED>, 256, 0); break;
            case 512:
                if constexpr (sizeof(T) == 4)
                    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step2_fused<T, 512, UNIT, STAGED>, 512, 0);
                break;
            default: break;
        }
    } else {
        switch (nt) {
            case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_fused<T, 64, UNIT, STAGED>, 64, 0); break;
            case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_fused<T, 128, UNIT, STAGED>, 128, 0); break;
            case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_fused<T, 256, UNIT, STAGED>, 256, 0); break;
            case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_fused<T, 512, UNIT, STAGED>, 512, 0); break;
            default: break;
        }
    }
    return (e == hipSuccess && n > 0) ? n : 1;
}

int step_blocks_per_cu(int precision, int depth, int nt, bool unit, bool staged) {
    if (precision == 0) return unit ? occ_step_t<double, true, false>(depth, nt) : occ_step_t<double, false, false>(depth, nt);
    if (staged) return unit ? occ_step_t<float, true, true>(depth, nt) : occ_step_t<float, false, true>(depth, nt);
    return unit ? occ_step_t<float, true, false>(depth, nt) : occ_step_t<float, false, false>(depth, nt);
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

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
    zero_u64_k<<<(n + 255) / 256, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s) {
    zero_u32_k<<<(n + 255) / 256, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, long long n, hipStream_t s) {
    fill_zero_k<<<elementwise_blocks(n), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace lbch

// ---------------------------------------------------------------------------
// Streaming copy used only to measure the HBM ceiling and calibrate counters.
// ---------------------------------------------------------------------------
namespace lbch {

__global__ __launch_bounds__(256) void copy16_k(const float4* __restrict__ src, float4* __restrict__ dst, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy16(const void* src, void* dst, long long n16, hipStream_t s) {
    long long b = (n16 + 255) / 256;
    const int nb = (int)(b < 16384 ? (b < 1 ? 1 : b) : 16384);
    copy16_k<<<nb, 256, 0, s>>>((const float4*)src, (float4*)dst, n16);
    return hipGetLastError();
}

}  // namespace lbch

// ---------------------------------------------------------------------------
// Helpers of the hybrid (surrogate jump + lattice Boltzmann correction) schedule.
// ---------------------------------------------------------------------------
namespace lbch {

__global__ __launch_bounds__(kRedThreads) void sum_f32_k(const float* __restrict__ x, long long n,
                                                         double* partials) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int kind[4] = {0, 0, 0, 0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        v[0] += (double)x[i];
    block_reduce_waves<4>(v, kind, partials + 4 * blockIdx.x);
}

// x += (num[0] - den_minus[0]) * inv_n   (exact mass projection: shift by the mean defect)
__global__ void add_f32_k(float* __restrict__ x, long long n, const double* __restrict__ num,
                          const double* __restrict__ den_minus, double inv_n) {
    const float shift = (float)((num[0] - den_minus[0]) * inv_n);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] += shift;
}

// out = base + k (b - a): the rate-extrapolated jump (FP32 arithmetic, k exact in FP32 for integer jumps)
__global__ void extrap_f32_k(const float* base, const float* __restrict__ a, const float* __restrict__ b,
                             float k, long long n, float* out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = base[i] + k * (b[i] - a[i]);
}

// cur += k (cur - prev) over the nine population planes (a projective step of
// the populations themselves; n16 = 16-byte chunks)
template <typename V, typename T>
__global__ void extrap_pop_k(V* __restrict__ cur, const V* __restrict__ prev, T k, long long n16) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n16;
         i += (long long)gridDim.x * blockDim.x) {
        V c = cur[i];
        const V q = prev[i];
        c = c + k * (c - q);
        cur[i] = c;
    }
}

// dst (a window grid) <- the 9 population planes of src at rows y0.., columns x0.. (wrapped)
template <typename T>
__global__ void copy_window_k(const T* __restrict__ src, const Grid sg, int y0, int x0, T* __restrict__ dst,
                              const Grid dg) {
    const long long n = (long long)dg.nx * dg.ny;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(idx / dg.nx), x = (int)(idx % dg.nx);
        int ys = (y0 + y) % sg.ny, xs = (x0 + x) % sg.nx;
        if (ys < 0) ys += sg.ny;
        if (xs < 0) xs += sg.nx;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            dst[i * dg.plane + (long long)y * dg.pitch + x] = src[i * sg.plane + (long long)ys * sg.pitch + xs];
    }
}

// sums of (win - big)^2 and big^2 over the window interior
__global__ __launch_bounds__(kRedThreads) void window_err_k(const float* __restrict__ win, int side,
                                                            const float* __restrict__ big, int ny, int nx, int y0,
                                                            int x0, int margin, int interior, double* partials) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int kind[4] = {0, 0, 0, 0};
    const long long n = (long long)interior * interior;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(i / interior) + margin, c = (int)(i % interior) + margin;
        int yb = (y0 + r) % ny, xb = (x0 + c) % nx;
        if (yb < 0) yb += ny;
        if (xb < 0) xb += nx;
        const double a = win[(long long)r * side + c], b = big[(long long)yb * nx + xb];
        v[0] += (a - b) * (a - b);
        v[1] += b * b;
    }
    block_reduce_waves<4>(v, kind, partials + 4 * blockIdx.x);
}

hipError_t launch_sum_f32(const float* x, long long n, double* partials, double* out, hipStream_t s) {
    sum_f32_k<<<kRedBlocks, kRedThreads, 0, s>>>(x, n, partials);
    const int kinds[4] = {0, 0, 0, 0};
    return launch_finalize(partials, kRedBlocks, 4, kinds, out, s);
}

hipError_t launch_add_f32(float* x, long long n, const double* num, const double* den_minus, double inv_n,
                          hipStream_t s) {
    add_f32_k<<<elementwise_blocks(n), 256, 0, s>>>(x, n, num, den_minus, inv_n);
    return hipGetLastError();
}

hipError_t launch_extrap_f32(const float* base, const float* a, const float* b, float k, long long n, float* out,
                             hipStream_t s) {
    extrap_f32_k<<<elementwise_blocks(n), 256, 0, s>>>(base, a, b, k, n, out);
    return hipGetLastError();
}

hipError_t launch_extrap_pop(int precision, void* cur, const void* prev, double k, long long elems, hipStream_t s) {
    if (precision == 0) {
        const long long n16 = elems / 2;
        extrap_pop_k<f64x2, double><<<elementwise_blocks(n16), 256, 0, s>>>((f64x2*)cur, (const f64x2*)prev, k, n16);
    } else {
        const long long n16 = elems / 4;
        extrap_pop_k<f32x4, float><<<elementwise_blocks(n16), 256, 0, s>>>((f32x4*)cur, (const f32x4*)prev, (float)k,
                                                                           n16);
    }
    return hipGetLastError();
}

hipError_t launch_copy_window(int precision, const void* src, const Grid& sg, int y0, int x0, void* dst,
                              const Grid& dg, hipStream_t s) {
    const int nb = elementwise_blocks((long long)dg.nx * dg.ny);
    if (precision == 0) copy_window_k<double><<<nb, 256, 0, s>>>((const double*)src, sg, y0, x0, (double*)dst, dg);
    else copy_window_k<float><<<nb, 256, 0, s>>>((const float*)src, sg, y0, x0, (float*)dst, dg);
    return hipGetLastError();
}

hipError_t launch_window_err(const float* win, int side, const float* big, int ny, int nx, int y0, int x0, int margin,
                             int interior, double* partials, double* out2, hipStream_t s) {
    window_err_k<<<kRedBlocks, kRedThreads, 0, s>>>(win, side, big, ny, nx, y0, x0, margin, interior, partials);
    const int kinds[4] = {0, 0, 0, 0};
    return launch_finalize(partials, kRedBlocks, 4, kinds, out2, s);
}

}  // namespace lbch
