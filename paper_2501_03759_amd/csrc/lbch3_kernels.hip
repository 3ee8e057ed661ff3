// HIP kernels of the scheme on the three-dimensional D3Q15 lattice (eq 21) for
// gfx950: the same step as the D2Q9 kernels (eqs 17-19, 22, 26, 13, 16), with
// the cubic anisotropy of eq 6 (d = 3).  The moment rows split by parity under
// c -> -c: f_eq is even and the source odd, so with one rate s_e for the even
// rows and one rate s_q for the odd rows other than the fluxes the collision
// of eq 17 is, whatever the rows within each class are,
//   f*_i = f_eq,i + (1 - s_e)(f+_i - f_eq,i) + (1 - s_q) f-_i
//          - (1 - s_q / 2) dt c w_i e_i.g + (s_q - s_j)/10 e_i.(j - (dt c / 6) g)
// (f+-: halves of f_i +- f_opp(i); g = grad mu_beta; 10 = |flux row|^2).  With
// s_e = s_q = 1 (the default) only phi and the flux of each node are needed.
//
// Layout: population plane i holds nz slabs of ny rows of `pitch` elements;
// element (i, z, y, x) is at i * plane + z * slab + y * pitch + x.  The buffer
// holds post-collision populations at the node that produced them; the next
// step pulls f_i(x) = f*_i(x - e_i).
#include "lbch_internal.h"

#include <math.h>

namespace lbch {

namespace {

// D3Q15 directions of eq 21a
__device__ constexpr int kEX[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
__device__ constexpr int kEY[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
__device__ constexpr int kEZ[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};

__device__ __forceinline__ void lds_barrier3() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

template <typename T> __device__ __forceinline__ T recip(T x);
template <> __device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double recip<double>(double x) { return 1.0 / x; }

// gamma of eq 6 (d = 3) and h_a with |grad phi| (P grad_n gamma)_a = p_a h_a:
// n_a^2 = p_a^2 / |p|^2, s4 = sum n_a^4, gamma = 1 + alpha (4 s4 - 3),
// h_a = 16 alpha (n_a^2 - s4).  gamma = 1, h = 0 where |grad phi| <= floor.
template <typename T>
__device__ __forceinline__ void aniso3(T px, T py, T pz, const StepCoef3<T>& c, T& gamma, T& hx, T& hy, T& hz) {
    const T g2 = px * px + py * py + pz * pz;
    gamma = T(1);
    hx = hy = hz = T(0);
    if (g2 > c.floor2) {
        const T inv = recip<T>(g2);
        const T a = px * px * inv, b = py * py * inv, d = pz * pz * inv;
        const T s4 = (a * a + b * b) + d * d;
        gamma = T(1) + c.alpha * (T(4) * s4 - T(3));
        hx = c.alpha16 * (a - s4);
        hy = c.alpha16 * (b - s4);
        hz = c.alpha16 * (d - s4);
    }
}

// Eq 26 on D3Q15 from three padded planes (U = z+1, C = z, D = z-1) at (ly, lx):
// faces (+-x, +-y in C; U, D centres) and the eight body diagonals (corners of U, D).
template <typename T, int RW>
struct Stencil3 {
    const T (*U)[RW];
    const T (*C)[RW];
    const T (*D)[RW];
    __device__ __forceinline__ T gx(int ly, int lx, const StepCoef3<T>& c) const {
        const T dg = ((U[ly + 1][lx + 1] - U[ly + 1][lx - 1]) + (U[ly - 1][lx + 1] - U[ly - 1][lx - 1])) +
                     ((D[ly + 1][lx + 1] - D[ly + 1][lx - 1]) + (D[ly - 1][lx + 1] - D[ly - 1][lx - 1]));
        return c.gf * (C[ly][lx + 1] - C[ly][lx - 1]) + c.gd * dg;
    }
    __device__ __forceinline__ T gy(int ly, int lx, const StepCoef3<T>& c) const {
        const T dg = ((U[ly + 1][lx + 1] - U[ly - 1][lx + 1]) + (U[ly + 1][lx - 1] - U[ly - 1][lx - 1])) +
                     ((D[ly + 1][lx + 1] - D[ly - 1][lx + 1]) + (D[ly + 1][lx - 1] - D[ly - 1][lx - 1]));
        return c.gf * (C[ly + 1][lx] - C[ly - 1][lx]) + c.gd * dg;
    }
    __device__ __forceinline__ T gz(int ly, int lx, const StepCoef3<T>& c) const {
        const T dg = ((U[ly + 1][lx + 1] - D[ly + 1][lx + 1]) + (U[ly + 1][lx - 1] - D[ly + 1][lx - 1])) +
                     ((U[ly - 1][lx + 1] - D[ly - 1][lx + 1]) + (U[ly - 1][lx - 1] - D[ly - 1][lx - 1]));
        return c.gf * (U[ly][lx] - D[ly][lx]) + c.gd * dg;
    }
    __device__ __forceinline__ T lap(int ly, int lx, const StepCoef3<T>& c) const {
        const T faces = ((C[ly][lx + 1] + C[ly][lx - 1]) + (C[ly + 1][lx] + C[ly - 1][lx])) + (U[ly][lx] + D[ly][lx]);
        const T diag = ((U[ly + 1][lx + 1] + U[ly + 1][lx - 1]) + (U[ly - 1][lx + 1] + U[ly - 1][lx - 1])) +
                       ((D[ly + 1][lx + 1] + D[ly + 1][lx - 1]) + (D[ly - 1][lx + 1] + D[ly - 1][lx - 1]));
        return c.lf * faces + c.ld * diag - c.lc * C[ly][lx];
    }
};

// phi and the flux sum_i e_i f_i of one node's fifteen populations, in the
// fixed order both users share (the flux from the four body-diagonal pairs)
template <typename T>
__device__ __forceinline__ void moments15(const T (&f)[15], T (&r)[4]) {
    const T s1 = ((f[1] + f[2]) + (f[3] + f[4])) + (f[5] + f[6]);
    const T s2 = ((f[7] + f[8]) + (f[9] + f[10])) + ((f[11] + f[12]) + (f[13] + f[14]));
    const T d7 = f[7] - f[8], d9 = f[9] - f[10], d11 = f[11] - f[12], d13 = f[13] - f[14];
    r[0] = f[0] + s1 + s2;
    r[1] = (f[1] - f[2]) + ((d7 + d9) + (d11 - d13));
    r[2] = (f[3] - f[4]) + ((d7 + d9) - (d11 - d13));
    r[3] = (f[5] - f[6]) + ((d7 - d9) + (d11 + d13));
}

}  // namespace

// ---------------------------------------------------------------------------
// Fused step on D3Q15.  A workgroup of TX x TY lanes owns an x-y tile
// (lane (tx, ty) -> column x0 - 3 + tx, row y0 - 3 + ty, wrapped) and sweeps
// hz planes along z; iteration j pulls plane a = z0 - 3 + j and runs the four
// stages of the D2Q9 sweep in two phases separated by one barrier, each stage
// reading only planes that an earlier phase finished: phase 1 A (pull, phi,
// flux at a) and C (div Q, lap w -> mu_beta at a-3); phase 2 B (grad phi,
// lap phi, gamma, Q, w, mu_alpha at a-1) and D (grad mu_beta, collision,
// store at a-4).  Two barriers per plane.  Stage outputs live in LDS rings of
// three padded planes, each slot indexed by the iteration that wrote it
// (j mod 3; register rings j mod 6, the plane loop unrolled six times so that
// every slot is static); every lane computes every stage and only the tile
// interior (TX - 6) x (TY - 6) is stored.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY, bool GEN>
__global__ __launch_bounds__(TX * TY) void step3_fused(const T* __restrict__ fin, T* __restrict__ fout,
                                                       const Grid3 g, const Tiling3 tl, const StepCoef3<T> c) {
    constexpr int RW = TX + 2, RH = TY + 2, U = 6;
    __shared__ T s_phi[3][RH][RW];
    __shared__ T s_qx[3][RH][RW];
    __shared__ T s_qy[3][RH][RW];
    __shared__ T s_qz[3][RH][RW];
    __shared__ T s_w[3][RH][RW];
    __shared__ T s_mb[3][RH][RW];
    // block b runs on XCD b % 8; each XCD takes a contiguous range of tiles
    const int tile = (int)(blockIdx.x & 7) * tl.per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= tl.ntiles) return;
    const int tx_i = tile % tl.tiles_x;
    const int rest = tile / tl.tiles_x;
    const int ty_i = rest % tl.tiles_y;
    const int tz_i = rest / tl.tiles_y;
    const int x0 = tx_i * (TX - 6), y0 = ty_i * (TY - 6), z0 = tz_i * tl.hz;
    const int wx = min(TX - 6, g.nx - x0), wy = min(TY - 6, g.ny - y0), hl = min(tl.hz, g.nz - z0);
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int lx = tx + 1, ly = ty + 1;
    const int x = wrapi(x0 - 3 + tx, g.nx), y = wrapi(y0 - 3 + ty, g.ny);
    const bool store_lane = tx >= 3 && tx < 3 + wx && ty >= 3 && ty < 3 + wy;
    // pull sources: column x - e_ix, row y - e_iy (wrapped once per lane)
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    // 32-bit in-slab byte offsets of the nine (x, y) sources (a slab holds
    // fewer than 2^31 / 15 elements); the slab and plane parts of every
    // address are uniform over the workgroup
    constexpr unsigned ES = sizeof(T);
    const unsigned rc = (unsigned)(y * g.pitch), rm = (unsigned)(ym * g.pitch), rp = (unsigned)(yp * g.pitch);
    const unsigned oxy[9] = {(rc + x) * ES,  (rc + xm) * ES, (rc + xp) * ES, (rm + x) * ES, (rp + x) * ES,
                             (rm + xm) * ES, (rp + xp) * ES, (rp + xm) * ES, (rm + xp) * ES};
    // D stores plane a - 4; the last iteration runs only C and D (no stage
    // needs its planes a and a - 1)
    const int niter = hl + 7;

    T red[GEN ? 1 : U][4];  // phi, j_x, j_y, j_z of the pulled node (A -> D, four iterations later)
    T mua[U], tloc[U];  // B -> D (three iterations later), B -> C (two)
    T buf[2][15];       // pulled populations of the next plane in flight
    T fr[GEN ? 15 : 1];  // s_e, s_q != 1: the populations of plane a-4, pulled again

    auto issue = [&](int za, T (&b)[15]) {
        const int zr = wrapi(za, g.nz);
        const int zm = zr == 0 ? g.nz - 1 : zr - 1, zp = zr == g.nz - 1 ? 0 : zr + 1;
#pragma unroll
        for (int i = 0; i < 15; ++i) {
            // source (x - e_ix, y - e_iy): index into oxy
            const int sx = kEX[i] > 0 ? 1 : (kEX[i] < 0 ? 2 : 0);
            const int sy = kEY[i] > 0 ? 1 : (kEY[i] < 0 ? 2 : 0);
            const int k = sy == 0 ? sx : (sx == 0 ? 2 + sy : (sx == sy ? 4 + sx : (sy == 2 ? 7 : 8)));
            const int zs = kEZ[i] > 0 ? zm : (kEZ[i] < 0 ? zp : zr);
            const char* __restrict__ base = (const char*)(fin + ((long long)i * g.plane + (long long)zs * g.slab));
            b[i] = *(const T*)(base + oxy[k]);
        }
    };

    issue(z0 - 3, buf[0]);
    for (int jb = 0; jb < niter; jb += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int j = jb + k;
            if (j < niter) {
                const bool head = j + 1 < niter;
                // LDS slots written by iterations j, j-1, j-2
                const int s0 = k % 3, s1 = (k + 2) % 3, s2 = (k + 1) % 3;
                // ======== phase 1 ========
                // ---- A: plane a ----
                if (head) {
                    // the class-rate collision pulls the node again and takes phi and the
                    // flux from there, so only the unit-rate one keeps them in registers
                    T r[4];
                    moments15<T>(buf[j & 1], r);
                    if constexpr (!GEN) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) red[k][q] = r[q];
                    }
                    s_phi[s0][ly][lx] = r[0];
                }
                if (j + 2 < niter) issue(z0 - 3 + j + 1, buf[(j + 1) & 1]);
                // the addresses stage A read four iterations ago
                if constexpr (GEN) {
                    if (j >= 7) issue(z0 - 7 + j, fr);
                }
                // ---- C: plane a-3; its Q and w planes come from B of iterations j-1 .. j-3 ----
                if (j >= 5) {
                    const Stencil3<T, RW> qx{s_qx[s1], s_qx[s2], s_qx[s0]};
                    const Stencil3<T, RW> qy{s_qy[s1], s_qy[s2], s_qy[s0]};
                    const Stencil3<T, RW> qz{s_qz[s1], s_qz[s2], s_qz[s0]};
                    T mb = tloc[(k + U - 2) % U] - ((qx.gx(ly, lx, c) + qy.gy(ly, lx, c)) + qz.gz(ly, lx, c));
                    if (c.reg != REG_NONE) {
                        const Stencil3<T, RW> ws{s_w[s1], s_w[s2], s_w[s0]};
                        mb += c.eps * ws.lap(ly, lx, c);
                    }
                    s_mb[s0][ly][lx] = mb;
                }
                lds_barrier3();
                // ======== phase 2 ========
                // ---- D: plane a-4; its mu_beta planes come from C of iterations j .. j-2.
                // D goes first so that its stores have B's time to complete before
                // the next iteration waits on its loads (that wait covers every
                // earlier load and store) ----
                if (j >= 7) {
                    const Stencil3<T, RW> ms{s_mb[s0], s_mb[s1], s_mb[s2]};
                    const T gx = ms.gx(ly, lx, c), gy = ms.gy(ly, lx, c), gz = ms.gz(ly, lx, c);
                    T rg[4];
                    if constexpr (GEN) moments15<T>(fr, rg);
                    const T(&r)[4] = GEN ? rg : red[(k + U - 4) % U];
                    const T mu_a = mua[(k + U - 3) % U];
                    // e_i.(j - v g) and e_i.g for every direction
                    const T ax = c.u * (r[1] - c.v * gx), ay = c.u * (r[2] - c.v * gy), az = c.u * (r[3] - c.v * gz);
                    const T bx = c.hd * gx, by = c.hd * gy, bz = c.hd * gz;
                    T o[15];
                    o[0] = r[0] + (c.w0 - T(1)) * mu_a;
                    const T ef = c.wf * mu_a, ed = c.wd * mu_a;
                    if constexpr (!GEN) {
#pragma unroll
                        for (int i = 1; i < 15; ++i) {
                            const T w_i = i < 7 ? c.wf : c.wd;
                            const T eq = i < 7 ? ef : ed;
                            const T ej = T(kEX[i]) * ax + T(kEY[i]) * ay + T(kEZ[i]) * az;
                            const T eg = T(kEX[i]) * bx + T(kEY[i]) * by + T(kEZ[i]) * bz;
                            o[i] = eq - w_i * eg + ej;
                        }
                    } else {
                        o[0] += c.se1 * (fr[0] - o[0]);
                        // direction i + 1 is opposite to i for odd i
#pragma unroll
                        for (int i = 1; i < 15; i += 2) {
                            const T w_i = i < 7 ? c.wf : c.wd;
                            const T eq = i < 7 ? ef : ed;
                            const T ej = T(kEX[i]) * ax + T(kEY[i]) * ay + T(kEZ[i]) * az;
                            const T eg = T(kEX[i]) * bx + T(kEY[i]) * by + T(kEZ[i]) * bz;
                            const T ev = eq + c.se1 * (T(0.5) * (fr[i] + fr[i + 1]) - eq);
                            const T od = c.sq1 * (T(0.5) * (fr[i] - fr[i + 1])) - w_i * eg + ej;
                            o[i] = ev + od;
                            o[i + 1] = ev - od;
                        }
                    }
                    if (store_lane) {
                        const int rd = z0 - 7 + j;
#pragma unroll
                        for (int i = 0; i < 15; ++i) {
                            char* __restrict__ q = (char*)(fout + ((long long)i * g.plane + (long long)rd * g.slab));
                            *(T*)(q + oxy[0]) = o[i];
                        }
                    }
                }
                // ---- B: plane a-1 ----
                if (j >= 2 && head) {
                    const Stencil3<T, RW> st{s_phi[s0], s_phi[s1], s_phi[s2]};
                    const T px = st.gx(ly, lx, c), py = st.gy(ly, lx, c), pz = st.gz(ly, lx, c);
                    const T lap = st.lap(ly, lx, c);
                    const T pC = s_phi[s1][ly][lx];
                    const T fb = c.beta4 * pC * (pC * pC - T(1));
                    T gamma, hx, hy, hz;
                    aniso3<T>(px, py, pz, c, gamma, hx, hy, hz);
                    if (c.qform == 0) {
                        s_qx[s0][ly][lx] = c.kappa * px * (gamma + hx);
                        s_qy[s0][ly][lx] = c.kappa * py * (gamma + hy);
                        s_qz[s0][ly][lx] = c.kappa * pz * (gamma + hz);
                    } else {
                        s_qx[s0][ly][lx] = gamma * c.kappa * px + px * hx;
                        s_qy[s0][ly][lx] = gamma * c.kappa * py + py * hy;
                        s_qz[s0][ly][lx] = gamma * c.kappa * pz + pz * hz;
                    }
                    T w, tl0 = (gamma - T(1)) * fb + c.kappa * lap;
                    if (c.reg == REG_WILLMORE) {
                        w = lap - fb;
                        tl0 -= c.eps * (c.beta4 * (T(3) * pC * pC - T(1))) * w;
                    } else if (c.reg == REG_LINEAR) {
                        w = lap;
                    } else {
                        w = T(0);
                    }
                    s_w[s0][ly][lx] = w;
                    tloc[k] = tl0;
                    mua[k] = fb - c.kappa * lap;
                }
                lds_barrier3();
            }
        }
    }
}

// Equilibrium of eq 18 at phi0 with mu_alpha(phi0), written where the first
// pull reads it (population i of node x at x - e_i).
template <typename T, typename P>
__global__ __launch_bounds__(256) void init3_k(const P* __restrict__ phi0, T* __restrict__ fout, const Grid3 g,
                                               const StepCoef3<T> c, unsigned* bad) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(idx % g.nx);
        const long long r = idx / g.nx;
        const int y = (int)(r % g.ny), z = (int)(r / g.ny);
        auto P0 = [&](int dz, int dy, int dx) {
            const int zz = wrapi(z + dz, g.nz), yy = wrapi(y + dy, g.ny), xx = wrapi(x + dx, g.nx);
            return (T)phi0[((long long)zz * g.ny + yy) * g.nx + xx];
        };
        const T pc = P0(0, 0, 0);
        const T faces = ((P0(0, 0, 1) + P0(0, 0, -1)) + (P0(0, 1, 0) + P0(0, -1, 0))) + (P0(1, 0, 0) + P0(-1, 0, 0));
        const T diag = ((P0(1, 1, 1) + P0(1, 1, -1)) + (P0(1, -1, 1) + P0(1, -1, -1))) +
                       ((P0(-1, 1, 1) + P0(-1, 1, -1)) + (P0(-1, -1, 1) + P0(-1, -1, -1)));
        const T lap = c.lf * faces + c.ld * diag - c.lc * pc;
        const T mua = c.beta4 * pc * (pc * pc - T(1)) - c.kappa * lap;
        if (!isfinite((double)pc)) atomicAdd(bad, 1u);
        for (int i = 0; i < 15; ++i) {
            const T v = i == 0 ? pc + (c.w0 - T(1)) * mua : (i < 7 ? c.wf : c.wd) * mua;
            const int xs = wrapi(x - kEX[i], g.nx), ys = wrapi(y - kEY[i], g.ny), zs = wrapi(z - kEZ[i], g.nz);
            fout[(long long)i * g.plane + (long long)zs * g.slab + (long long)ys * g.pitch + xs] = v;
        }
    }
}

// phi = sum_i f*_i(x - e_i) (eq 22) in float64: optional dense copy [z][y][x]
// and partial {sum, min, max, non-finite count}.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void moments3_k(const T* __restrict__ fin, const Grid3 g, void* phi_out,
                                                          int out_dtype, double* partials) {
    double v[4] = {0.0, INFINITY, -INFINITY, 0.0};
    const int kind[4] = {0, 1, 2, 0};
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(idx % g.nx);
        const long long r = idx / g.nx;
        const int y = (int)(r % g.ny), z = (int)(r / g.ny);
        double phi = 0.0;
        for (int i = 0; i < 15; ++i) {
            const int xs = wrapi(x - kEX[i], g.nx), ys = wrapi(y - kEY[i], g.ny), zs = wrapi(z - kEZ[i], g.nz);
            phi += (double)fin[(long long)i * g.plane + (long long)zs * g.slab + (long long)ys * g.pitch + xs];
        }
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

// Discrete free energy (eq 7, d = 3) from phi [z][y][x] (float64): partials of
// the gradient, bulk and regularisation sums and the non-finite count.
__global__ __launch_bounds__(kRedThreads) void energy3_k(const double* __restrict__ phi, const Grid3 g,
                                                         const StepCoef3<double> c, double* partials) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int kind[4] = {0, 0, 0, 0};
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(idx % g.nx);
        const long long r = idx / g.nx;
        const int y = (int)(r % g.ny), z = (int)(r / g.ny);
        auto P = [&](int dz, int dy, int dx) {
            return phi[((long long)wrapi(z + dz, g.nz) * g.ny + wrapi(y + dy, g.ny)) * g.nx + wrapi(x + dx, g.nx)];
        };
        const double pc = P(0, 0, 0);
        const double px = c.gf * (P(0, 0, 1) - P(0, 0, -1)) +
                          c.gd * (((P(1, 1, 1) - P(1, 1, -1)) + (P(1, -1, 1) - P(1, -1, -1))) +
                                  ((P(-1, 1, 1) - P(-1, 1, -1)) + (P(-1, -1, 1) - P(-1, -1, -1))));
        const double py = c.gf * (P(0, 1, 0) - P(0, -1, 0)) +
                          c.gd * (((P(1, 1, 1) - P(1, -1, 1)) + (P(1, 1, -1) - P(1, -1, -1))) +
                                  ((P(-1, 1, 1) - P(-1, -1, 1)) + (P(-1, 1, -1) - P(-1, -1, -1))));
        const double pz = c.gf * (P(1, 0, 0) - P(-1, 0, 0)) +
                          c.gd * (((P(1, 1, 1) - P(-1, 1, 1)) + (P(1, 1, -1) - P(-1, 1, -1))) +
                                  ((P(1, -1, 1) - P(-1, -1, 1)) + (P(1, -1, -1) - P(-1, -1, -1))));
        const double faces = ((P(0, 0, 1) + P(0, 0, -1)) + (P(0, 1, 0) + P(0, -1, 0))) + (P(1, 0, 0) + P(-1, 0, 0));
        const double diag = ((P(1, 1, 1) + P(1, 1, -1)) + (P(1, -1, 1) + P(1, -1, -1))) +
                            ((P(-1, 1, 1) + P(-1, 1, -1)) + (P(-1, -1, 1) + P(-1, -1, -1)));
        const double lap = c.lf * faces + c.ld * diag - c.lc * pc;
        double gamma, hx, hy, hz;
        aniso3<double>(px, py, pz, c, gamma, hx, hy, hz);
        const double q = pc * pc - 1.0;
        const double Fb = 0.25 * c.beta4 * q * q, fb = c.beta4 * pc * q;
        double G = 0.0;
        if (c.reg == REG_WILLMORE) G = (lap - fb) * (lap - fb);
        else if (c.reg == REG_LINEAR) G = lap * lap;
        const double tg = gamma * 0.5 * c.kappa * (px * px + py * py + pz * pz), tb = gamma * Fb, tr = 0.5 * c.eps * G;
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

// canonical pre-collision populations f_i(x) = f*_i(x - e_i) <-> internal layout
template <typename T>
__global__ __launch_bounds__(256) void gather3_k(const T* __restrict__ fin, const Grid3 g, T* __restrict__ dense) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(idx % g.nx);
        const long long r = idx / g.nx;
        const int y = (int)(r % g.ny), z = (int)(r / g.ny);
        for (int i = 0; i < 15; ++i) {
            const int xs = wrapi(x - kEX[i], g.nx), ys = wrapi(y - kEY[i], g.ny), zs = wrapi(z - kEZ[i], g.nz);
            dense[(long long)i * n + idx] =
                fin[(long long)i * g.plane + (long long)zs * g.slab + (long long)ys * g.pitch + xs];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void scatter3_k(const T* __restrict__ dense, const Grid3 g, T* __restrict__ fout) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(idx % g.nx);
        const long long r = idx / g.nx;
        const int y = (int)(r % g.ny), z = (int)(r / g.ny);
        for (int i = 0; i < 15; ++i) {
            const int xs = wrapi(x - kEX[i], g.nx), ys = wrapi(y - kEY[i], g.ny), zs = wrapi(z - kEZ[i], g.nz);
            fout[(long long)i * g.plane + (long long)zs * g.slab + (long long)ys * g.pitch + xs] =
                dense[(long long)i * n + idx];
        }
    }
}

// ------------------------------------------------------------- launchers
namespace {
int blocks3(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}
}  // namespace

namespace {
template <typename T, int TX, int TY, bool GEN>
int occ3_one() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step3_fused<T, TX, TY, GEN>, TX * TY, 0) != hipSuccess ||
        n < 1) {
        (void)hipGetLastError();
        n = 1;
    }
    return n;
}
template <typename T, int TX, int TY>
int occ3(bool gen) {
    return gen ? occ3_one<T, TX, TY, true>() : occ3_one<T, TX, TY, false>();
}
}  // namespace

// Tile shapes (lanes in x, lanes in y) by workgroup size: 512 = 32 x 16,
// 1024 = 32 x 32 (FP32), 988 = 38 x 26 (FP32: a 32-column interior, so every
// stored row is one whole 128-byte line when nx is a multiple of 32).
bool tile3_shape(int precision, int block_threads, int* tx, int* ty) {
    int x = 0, y = 0;
    if (block_threads == 512) x = 32, y = 16;
    else if (precision == 1 && block_threads == 1024) x = 32, y = 32;
    else if (precision == 1 && block_threads == 988) x = 38, y = 26;
    else return false;
    if (tx) *tx = x;
    if (ty) *ty = y;
    return true;
}

int step3_blocks_per_cu(int precision, int tx, int ty, bool gen) {
    if (precision == 0) return occ3<double, 32, 16>(gen);
    if (tx == 38) return occ3<float, 38, 26>(gen);
    return ty == 32 ? occ3<float, 32, 32>(gen) : occ3<float, 32, 16>(gen);
}

// hz = 0: the sweep length that minimises rounds * (hz + 7), where a round is
// one wave of `slots` resident workgroups and hz + 7 the iterations of a
// sweep (7 start-up slabs), over hz in [4, nz].
Tiling3 make_tiling3(int nx, int ny, int nz, int hz, int slots, int tx, int ty) {
    Tiling3 t{};
    t.tx = tx;
    t.ty = ty;
    t.tiles_x = (nx + tx - 7) / (tx - 6);
    t.tiles_y = (ny + ty - 7) / (ty - 6);
    const long long cols = (long long)t.tiles_x * t.tiles_y;
    if (hz <= 0) {
        if (slots <= 0) slots = 256;
        long long best = -1;
        hz = nz;
        for (int h = nz < 4 ? nz : 4; h <= nz; ++h) {
            const long long tiles = cols * ((nz + h - 1) / h);
            const long long cost = ((tiles + slots - 1) / slots) * (h + 7LL);
            if (best < 0 || cost < best) {
                best = cost;
                hz = h;
            }
        }
    }
    t.hz = hz < nz ? hz : nz;
    t.zchunks = (nz + t.hz - 1) / t.hz;
    t.ntiles = (int)(cols * t.zchunks);
    t.per_xcd = (t.ntiles + 7) / 8;
    t.nblocks = 8 * t.per_xcd;
    return t;
}

hipError_t launch_step3(int precision, const void* fin, void* fout, const Grid3& g, const Tiling3& t,
                        const void* coef, hipStream_t s) {
    int tx = 0, ty = 0;
    if (!tile3_shape(precision, t.tx * t.ty, &tx, &ty) || tx != t.tx || ty != t.ty) return hipErrorInvalidValue;
    if (precision == 0) {
        const auto& c = *(const StepCoef3<double>*)coef;
        if (c.gen)
            step3_fused<double, 32, 16, true><<<t.nblocks, 512, 0, s>>>((const double*)fin, (double*)fout, g, t, c);
        else
            step3_fused<double, 32, 16, false><<<t.nblocks, 512, 0, s>>>((const double*)fin, (double*)fout, g, t, c);
        return hipGetLastError();
    }
    const auto& c = *(const StepCoef3<float>*)coef;
    const float* in = (const float*)fin;
    float* out = (float*)fout;
    if (tx == 38) {
        if (c.gen) step3_fused<float, 38, 26, true><<<t.nblocks, 988, 0, s>>>(in, out, g, t, c);
        else step3_fused<float, 38, 26, false><<<t.nblocks, 988, 0, s>>>(in, out, g, t, c);
    } else if (ty == 32) {
        if (c.gen) step3_fused<float, 32, 32, true><<<t.nblocks, 1024, 0, s>>>(in, out, g, t, c);
        else step3_fused<float, 32, 32, false><<<t.nblocks, 1024, 0, s>>>(in, out, g, t, c);
    } else {
        if (c.gen) step3_fused<float, 32, 16, true><<<t.nblocks, 512, 0, s>>>(in, out, g, t, c);
        else step3_fused<float, 32, 16, false><<<t.nblocks, 512, 0, s>>>(in, out, g, t, c);
    }
    return hipGetLastError();
}

hipError_t launch_init3(int precision, const void* phi0, int phi_dtype, void* fout, const Grid3& g, const void* coef,
                        unsigned* bad, hipStream_t s) {
    const int nb = blocks3((long long)g.nx * g.ny * g.nz);
    if (precision == 0) {
        const auto& c = *(const StepCoef3<double>*)coef;
        if (phi_dtype == 0) init3_k<double, double><<<nb, 256, 0, s>>>((const double*)phi0, (double*)fout, g, c, bad);
        else init3_k<double, float><<<nb, 256, 0, s>>>((const float*)phi0, (double*)fout, g, c, bad);
    } else {
        const auto& c = *(const StepCoef3<float>*)coef;
        if (phi_dtype == 0) init3_k<float, double><<<nb, 256, 0, s>>>((const double*)phi0, (float*)fout, g, c, bad);
        else init3_k<float, float><<<nb, 256, 0, s>>>((const float*)phi0, (float*)fout, g, c, bad);
    }
    return hipGetLastError();
}

hipError_t launch_moments3(int precision, const void* fin, const Grid3& g, void* phi_out, int out_dtype,
                           double* partials, int nparts, hipStream_t s) {
    if (precision == 0)
        moments3_k<double><<<nparts, kRedThreads, 0, s>>>((const double*)fin, g, phi_out, out_dtype, partials);
    else
        moments3_k<float><<<nparts, kRedThreads, 0, s>>>((const float*)fin, g, phi_out, out_dtype, partials);
    return hipGetLastError();
}

hipError_t launch_energy3(const double* phi, const Grid3& g, const StepCoef3<double>& c, double* partials,
                          int nparts, hipStream_t s) {
    energy3_k<<<nparts, kRedThreads, 0, s>>>(phi, g, c, partials);
    return hipGetLastError();
}

hipError_t launch_gather3(int precision, const void* fin, const Grid3& g, void* dense, hipStream_t s) {
    const int nb = blocks3((long long)g.nx * g.ny * g.nz);
    if (precision == 0) gather3_k<double><<<nb, 256, 0, s>>>((const double*)fin, g, (double*)dense);
    else gather3_k<float><<<nb, 256, 0, s>>>((const float*)fin, g, (float*)dense);
    return hipGetLastError();
}

hipError_t launch_scatter3(int precision, const void* dense, const Grid3& g, void* fout, hipStream_t s) {
    const int nb = blocks3((long long)g.nx * g.ny * g.nz);
    if (precision == 0) scatter3_k<double><<<nb, 256, 0, s>>>((const double*)dense, g, (double*)fout);
    else scatter3_k<float><<<nb, 256, 0, s>>>((const float*)dense, g, (float*)fout);
    return hipGetLastError();
}

}  // namespace lbch
