// C-ABI layer of liblbch: parameter handling, buffers, launches, reductions,
// checkpointing.  See include/lbch.h for the contract of every entry point.
#include "../../include/lbch.h"
#include "../../include/lbch_batch.h"
#include "../../include/lbch_diag.h"
#include "lbch_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace lbch;

namespace lbch {

thread_local std::string g_err;

lbch_status fail(lbch_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace lbch

namespace {

lbch_status ok() { return LBCH_OK; }

#define HIP_TRY(expr)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(LBCH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool isfin(double v) { return std::isfinite(v); }

double s_j_of(const lbch_params* p) {
    const double c = p->dx / p->dt;
    const double cs2 = c * c / 3.0;
    return 1.0 / (p->mobility / (cs2 * p->dt) + 0.5);
}

}  // namespace


// ------------------------------------------------------------ host helpers
extern "C" int32_t lbch_abi_version(void) { return LBCH_ABI_VERSION; }

extern "C" const char* lbch_last_error(void) { return g_err.c_str(); }

extern "C" lbch_status lbch_params_default(lbch_params* p) {
    if (!p) return fail(LBCH_E_INVALID, "params pointer is NULL");
    std::memset(p, 0, sizeof *p);
    p->abi_version = LBCH_ABI_VERSION;
    p->lattice = LBCH_D2Q9;
    p->precision = LBCH_FP64;
    p->boundary = LBCH_BC_PERIODIC;
    p->nx = 100;
    p->ny = 100;
    p->nz = 1;
    p->dx = 1.0;
    p->dt = 1.0;
    p->mobility = 0.1;
    for (double& s : p->s) s = 1.0;
    p->alpha = 0.0;
    p->aniso_m = 4;
    p->aniso_theta0 = 0.0;
    p->regularization = LBCH_REG_WILLMORE;
    p->eps_reg = 0.03;
    p->q_form = LBCH_Q_DERIVED;
    p->grad_floor = 1e-10;
    return lbch_params_from_sigma_width(p, 0.01, 5.0);
}

extern "C" lbch_status lbch_params_from_sigma_width(lbch_params* p, double sigma, double width) {
    if (!p) return fail(LBCH_E_INVALID, "params pointer is NULL");
    if (!(sigma > 0) || !(width > 0) || !isfin(sigma) || !isfin(width))
        return fail(LBCH_E_INVALID, "sigma and width must be positive and finite (got %g, %g)", sigma, width);
    // eq 5 inverted: sigma D = 8 kappa / 3 and sigma / D = 4 beta / 3
    p->kappa = 3.0 * sigma * width / 8.0;
    p->beta = 3.0 * sigma / (4.0 * width);
    return ok();
}

extern "C" lbch_status lbch_params_validate(const lbch_params* p) {
    if (!p) return fail(LBCH_E_INVALID, "params pointer is NULL");
    if (p->abi_version != LBCH_ABI_VERSION)
        return fail(LBCH_E_INVALID, "abi_version %d != %d", p->abi_version, LBCH_ABI_VERSION);
    if (p->lattice != LBCH_D2Q9 && p->lattice != LBCH_D3Q15)
        return fail(LBCH_E_INVALID, "unknown lattice %d", p->lattice);
    const bool d3 = p->lattice == LBCH_D3Q15;
    if (p->boundary != LBCH_BC_PERIODIC) return fail(LBCH_E_UNSUPPORTED, "only periodic boundaries are built");
    if (p->precision != LBCH_FP64 && p->precision != LBCH_FP32)
        return fail(LBCH_E_INVALID, "unknown precision %d", p->precision);
    if (p->nx < 1 || p->ny < 1) return fail(LBCH_E_INVALID, "grid %d x %d must be >= 1 x 1", p->nx, p->ny);
    if (!d3 && p->nz != 1) return fail(LBCH_E_INVALID, "nz = %d on the D2Q9 lattice (must be 1)", p->nz);
    if (d3 && p->nz < 1) return fail(LBCH_E_INVALID, "nz = %d must be >= 1", p->nz);
    const long long pitch = ((long long)p->nx + 63) / 64 * 64;
    if (pitch * (long long)p->ny * p->nz * (d3 ? 15 : 9) >= (1LL << 31))
        return fail(LBCH_E_INVALID, "grid %d x %d x %d exceeds 2^31 population entries", p->nx, p->ny, p->nz);
    if (!(p->dx > 0) || !(p->dt > 0) || !isfin(p->dx) || !isfin(p->dt))
        return fail(LBCH_E_INVALID, "dx, dt must be positive and finite");
    if (!(p->mobility > 0) || !isfin(p->mobility)) return fail(LBCH_E_INVALID, "mobility must be > 0");
    const double sj = s_j_of(p);
    if (!(sj > 0 && sj < 2)) return fail(LBCH_E_INVALID, "s_3 = s_5 = %g outside (0, 2)", sj);
    for (int k = 1; k < 9; ++k) {
        if (k == 3 || k == 5) continue;
        if (!(p->s[k] > 0 && p->s[k] < 2)) return fail(LBCH_E_INVALID, "s[%d] = %g outside (0, 2)", k, p->s[k]);
    }
    if (!(p->kappa > 0) || !isfin(p->kappa) || !(p->beta > 0) || !isfin(p->beta))
        return fail(LBCH_E_INVALID, "kappa, beta must be positive and finite");
    if (!(p->alpha >= 0) || !isfin(p->alpha)) return fail(LBCH_E_INVALID, "alpha must be >= 0");
    if (p->aniso_m < 1 || p->aniso_m > 8) return fail(LBCH_E_INVALID, "aniso_m %d outside 1..8", p->aniso_m);
    if (!isfin(p->aniso_theta0)) return fail(LBCH_E_INVALID, "aniso_theta0 not finite");
    if (p->regularization < LBCH_REG_NONE || p->regularization > LBCH_REG_WILLMORE)
        return fail(LBCH_E_INVALID, "unknown regularization %d", p->regularization);
    if (!(p->eps_reg >= 0) || !isfin(p->eps_reg)) return fail(LBCH_E_INVALID, "eps_reg must be >= 0");
    if (p->q_form != LBCH_Q_DERIVED && p->q_form != LBCH_Q_LITERAL)
        return fail(LBCH_E_INVALID, "unknown q_form %d", p->q_form);
    if (!(p->grad_floor >= 0) || !isfin(p->grad_floor)) return fail(LBCH_E_INVALID, "grad_floor must be >= 0");
    if (d3) {
        // D3Q15 takes one rate per parity class: the even D2Q9 slots (e, eps, p_xx, p_xy)
        // give s_e, the odd non-flux slots (q_x, q_y) give s_q
        for (int k : {2, 7, 8})
            if (p->s[k] != p->s[1])
                return fail(LBCH_E_UNSUPPORTED, "D3Q15 needs s[1] = s[2] = s[7] = s[8] (one even-row rate; s[%d] = %g)",
                            k, p->s[k]);
        if (p->s[6] != p->s[4])
            return fail(LBCH_E_UNSUPPORTED, "D3Q15 needs s[4] = s[6] (one rate for the odd non-flux rows)");
        if (p->aniso_m != 4 || p->aniso_theta0 != 0.0)
            return fail(LBCH_E_UNSUPPORTED, "D3Q15 has the cubic anisotropy of eq 6 only (aniso_m 4, theta0 0)");
    }
    return ok();
}

extern "C" lbch_status lbch_relaxation_rates(const lbch_params* p, double s_out[9]) {
    if (!p || !s_out) return fail(LBCH_E_INVALID, "NULL argument");
    for (int k = 0; k < 9; ++k) s_out[k] = p->s[k];
    s_out[3] = s_out[5] = s_j_of(p);
    return ok();
}

extern "C" lbch_status lbch_params_set_collision(lbch_params* p, int32_t model, double magic) {
    if (!p) return fail(LBCH_E_INVALID, "params pointer is NULL");
    if (!(p->mobility > 0) || !(p->dx > 0) || !(p->dt > 0) || !isfin(p->mobility) || !isfin(p->dx) ||
        !isfin(p->dt))
        return fail(LBCH_E_INVALID, "mobility, dx, dt must be positive and finite");
    const double sj = s_j_of(p);
    double s[9];
    if (model == LBCH_COLLISION_MRT) {
        for (double& v : s) v = 1.0;
    } else if (model == LBCH_COLLISION_SRT) {
        for (double& v : s) v = sj;
    } else if (model == LBCH_COLLISION_TRT) {
        if (!(magic > 0) || !isfin(magic)) return fail(LBCH_E_INVALID, "magic = %g must be > 0", magic);
        const double sp = 1.0 / (0.5 + magic / (1.0 / sj - 0.5));
        if (!(sp > 0 && sp < 2)) return fail(LBCH_E_INVALID, "TRT rate s_+ = %g outside (0, 2)", sp);
        const double tr[9] = {sp, sp, sp, sj, sj, sj, sj, sp, sp};
        for (int k = 0; k < 9; ++k) s[k] = tr[k];
    } else {
        return fail(LBCH_E_INVALID, "unknown collision model %d", model);
    }
    if (!(sj > 0 && sj < 2)) return fail(LBCH_E_INVALID, "s_j = %g outside (0, 2)", sj);
    for (int k = 0; k < 9; ++k) p->s[k] = s[k];
    return ok();
}

// ---------------------------------------------------------------- helpers
namespace lbch {

template <typename T>
void fill_coef(const lbch_params* p, StepCoef<T>& c) {
    const double dx = p->dx, dt = p->dt, cc = dx / dt;
    double s[9];
    lbch_relaxation_rates(p, s);
    c.g3 = (T)(1.0 / 3.0 / dx);
    c.g12 = (T)(1.0 / 12.0 / dx);
    c.l23 = (T)(2.0 / 3.0 / (dx * dx));
    c.l16 = (T)(1.0 / 6.0 / (dx * dx));
    c.l103 = (T)(10.0 / 3.0 / (dx * dx));
    c.kappa = (T)p->kappa;
    c.beta4 = (T)(4.0 * p->beta);
    c.eps = (T)(p->regularization == LBCH_REG_NONE ? 0.0 : p->eps_reg);
    c.alpha = (T)p->alpha;
    c.floor2 = (T)(p->grad_floor * p->grad_floor);
    c.rot_c = (T)std::cos(p->aniso_m * p->aniso_theta0);
    c.rot_s = (T)std::sin(p->aniso_m * p->aniso_theta0);
    c.alpha_m = (T)(p->alpha * p->aniso_m);
    const double nrm[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};
    c.cs1 = (T)(s[1] / nrm[1]);
    c.cs2 = (T)(s[2] / nrm[2]);
    c.cs3 = (T)(s[3] / nrm[3]);
    c.cs4 = (T)(s[4] / nrm[4]);
    c.cs5 = (T)(s[5] / nrm[5]);
    c.cs6 = (T)(s[6] / nrm[6]);
    c.cs7 = (T)(s[7] / nrm[7]);
    c.cs8 = (T)(s[8] / nrm[8]);
    // F_m = (c/3) (0,0,0,-gx,gx,-gy,gy,0,0); Delta_k = s_k (m_k - meq_k) - dt (1 - s_k/2) F_k
    c.cf3 = (T)(dt * (1.0 - s[3] / 2.0) * (cc / 3.0) / nrm[3]);
    c.cf4 = (T)(dt * (1.0 - s[4] / 2.0) * (cc / 3.0) / nrm[4]);
    c.cf5 = (T)(dt * (1.0 - s[5] / 2.0) * (cc / 3.0) / nrm[5]);
    c.cf6 = (T)(dt * (1.0 - s[6] / 2.0) * (cc / 3.0) / nrm[6]);
    c.u3 = (T)((1.0 - s[3]) / nrm[3]);
    c.u5 = (T)((1.0 - s[5]) / nrm[5]);
    c.v4 = (T)(dt * 0.5 * (cc / 3.0) / nrm[4]);
    c.v6 = (T)(dt * 0.5 * (cc / 3.0) / nrm[6]);
    c.m = p->aniso_m;
    c.reg = p->regularization;
    c.qform = p->q_form;
    c.unit = 1;
    for (int k : {1, 2, 4, 6, 7, 8})
        if (s[k] != 1.0) c.unit = 0;
}

void fill_red(const lbch_params* p, RedCoef& r) {
    const double dx = p->dx;
    r.g3 = 1.0 / 3.0 / dx;
    r.g12 = 1.0 / 12.0 / dx;
    r.l23 = 2.0 / 3.0 / (dx * dx);
    r.l16 = 1.0 / 6.0 / (dx * dx);
    r.l103 = 10.0 / 3.0 / (dx * dx);
    r.kappa = p->kappa;
    r.beta = p->beta;
    r.eps = p->regularization == LBCH_REG_NONE ? 0.0 : p->eps_reg;
    r.alpha = p->alpha;
    r.floor2 = p->grad_floor * p->grad_floor;
    r.rot_c = std::cos(p->aniso_m * p->aniso_theta0);
    r.rot_s = std::sin(p->aniso_m * p->aniso_theta0);
    r.area = dx * dx;
    r.m = p->aniso_m;
    r.reg = p->regularization;
}

// Grids this small default to one time step per launch.
static bool small_grid(long long nx, long long ny) { return nx * ny <= 512LL * 512; }

// Default lane count: at depth 1 the fewest lanes over the row (ties to the
// larger block); at depth 2 the shape with the most resident waves per CU on
// large grids (256 lanes in FP32, whose LDS rings allow 3 workgroups per CU;
// 128 in FP64).
static int default_nt(int nx, int depth, int esize) {
    if (depth == 2) return (esize == 4 && nx >= 192) ? 256 : 128;
    const int cand[4] = {64, 128, 256, 512};
    long long best = -1;
    int nt = 64;
    for (int k = 0; k < 4; ++k) {
        const int W = cand[k] - 8;
        const long long cost = (long long)((nx + W - 1) / W) * cand[k];
        if (best < 0 || cost <= best) {
            best = cost;
            nt = cand[k];
        }
    }
    return nt;
}

// slots: workgroups resident on the whole device at once (0 = unknown).
Tiling make_tiling(int nx, int ny, int nt, int hc, int depth, int esize, int slots, int cus) {
    if (nt == 0) nt = default_nt(nx, depth, esize);
    Tiling t{};
    t.nt = nt;
    t.depth = depth;
    t.W = nt - 8 * depth;  // multiple of 8: strips start on 32-byte boundaries
    t.strips = (nx + t.W - 1) / t.W;
    const int hmin = depth == 1 ? 16 : 32;
    if (hc == 0 && cus > 0 && (long long)t.strips * ((ny + hmin - 1) / hmin) < cus) {
        // small grids: fewer tiles than CUs even at the usual shortest chunk, so a
        // launch lasts one chunk's sweep; take the shortest chunk (>= 4 rows) that
        // keeps at most 2.5 workgroups per CU (measured on 100^2 to 1024^2: beyond
        // that the CUs' shared throughput outweighs the shorter sweep)
        for (int h = 4; h <= hmin; ++h)
            if ((long long)t.strips * ((ny + h - 1) / h) * 2 <= 5LL * cus) {
                hc = h;
                break;
            }
    }
    if (hc == 0) {
        if (depth == 1) {
            // short sweeps measured fastest on 8192^2 (more resident
            // workgroups; the extra halo rows mostly hit L2): about 8 tiles
            // per CU, >= 16 rows
            long long want = (long long)t.strips * ny / 8192;
            hc = (int)(want < 16 ? 16 : (want > 256 ? 256 : want));
        } else if (ny <= 32 || slots <= 0) {
            long long want = (long long)t.strips * ny / 2048;
            hc = (int)(want < 32 ? 32 : (want > 512 ? 512 : want));
        } else {
            // a chunk of h rows costs h + 17 iterations of the two-step
            // sweep (17 start-up rows); the launch takes ceil(tiles / slots)
            // rounds of the longest chunk: minimise rounds * (h + 17)
            long long best = -1;
            const int hmax = ny < 512 ? ny : 512;
            for (int h = 32; h <= hmax; ++h) {
                const long long tiles = (long long)t.strips * ((ny + h - 1) / h);
                const long long cost = ((tiles + slots - 1) / slots) * (h + 17LL);
                if (best < 0 || cost < best) {
                    best = cost;
                    hc = h;
                }
            }
        }
    }
    t.hc = hc < ny ? hc : ny;
    t.chunks = (ny + t.hc - 1) / t.hc;
    t.ntiles = t.strips * t.chunks;
    t.per_xcd = (t.ntiles + 7) / 8;
    t.nblocks = 8 * t.per_xcd;
    t.staged = 1;
    return t;
}

// Tiling of the given depth for sim s (nt, hc = 0: defaults), with the
// sim's row-loader choice and the device's resident-workgroup count.
static Tiling sim_tiling(const lbch_sim* s, int depth, int nt, int hc) {
    if (nt == 0) nt = default_nt(s->g.nx, depth, (int)s->esize);
    const bool staged = s->user_loader == 0 && s->precision == LBCH_FP32 && s->g.nx % 4 == 0;
    const bool unit = s->precision == LBCH_FP32 ? s->cf.unit != 0 : s->cd.unit != 0;
    const int slots = s->cus * step_blocks_per_cu(s->precision, depth, nt, unit, staged);
    Tiling t = make_tiling(s->g.nx, s->g.ny, nt, hc, depth, (int)s->esize, slots, s->cus);
    t.staged = s->user_loader == 0;
    return t;
}

template <typename T>
void fill_coef3(const lbch_params* p, StepCoef3<T>& c) {
    const double dx = p->dx, dt = p->dt, cc = dx / dt;
    c.gf = (T)(1.0 / 3.0 / dx);
    c.gd = (T)(1.0 / 24.0 / dx);
    c.lf = (T)(2.0 / 3.0 / (dx * dx));
    c.ld = (T)(1.0 / 12.0 / (dx * dx));
    c.lc = (T)(14.0 / 3.0 / (dx * dx));
    c.kappa = (T)p->kappa;
    c.beta4 = (T)(4.0 * p->beta);
    c.eps = (T)(p->regularization == LBCH_REG_NONE ? 0.0 : p->eps_reg);
    c.alpha = (T)p->alpha;
    c.alpha16 = (T)(16.0 * p->alpha);
    c.floor2 = (T)(p->grad_floor * p->grad_floor);
    // D3Q15 rate classes: s_e from the even D2Q9 slots (s[1]), s_q from the odd non-flux ones (s[4])
    const double se = p->s[1], sq = p->s[4];
    c.u = (T)((sq - s_j_of(p)) / 10.0);
    c.v = (T)(dt * cc / 6.0);
    c.hd = (T)((1.0 - 0.5 * sq) * dt * cc);
    c.w0 = (T)(2.0 / 9.0);
    c.wf = (T)(1.0 / 9.0);
    c.wd = (T)(1.0 / 72.0);
    c.se1 = (T)(1.0 - se);
    c.sq1 = (T)(1.0 - sq);
    c.reg = p->regularization;
    c.qform = p->q_form;
    c.gen = se != 1.0 || sq != 1.0;
}

// D3Q15 tiling: block_threads 512 = 32 x 16 lanes, 1024 = 32 x 32 and
// 988 = 38 x 26 (FP32 only); 0 = the default of the precision.  hz = 0: the
// sweep-length model.  block_threads must be one tile3_shape accepts.
static Tiling3 sim_tiling3(const lbch_sim* s, int block_threads, int hz) {
    if (block_threads == 0) block_threads = s->precision == LBCH_FP32 ? 1024 : 512;
    int tx = 32, ty = 16;
    tile3_shape(s->precision, block_threads, &tx, &ty);
    return make_tiling3(s->g3.nx, s->g3.ny, s->g3.nz, hz,
                        s->cus * step3_blocks_per_cu(s->precision, tx, ty, s->c3d.gen != 0), tx, ty);
}

template void fill_coef<double>(const lbch_params*, StepCoef<double>&);
template void fill_coef<float>(const lbch_params*, StepCoef<float>&);
template void fill_coef3<double>(const lbch_params*, StepCoef3<double>&);
template void fill_coef3<float>(const lbch_params*, StepCoef3<float>&);

}  // namespace lbch

namespace {

const void* coef_ptr(const lbch_sim* s) {
    if (s->d3) return s->precision == LBCH_FP64 ? (const void*)&s->c3d : (const void*)&s->c3f;
    return s->precision == LBCH_FP64 ? (const void*)&s->cd : (const void*)&s->cf;
}

lbch_status step_launch(lbch_sim* s, const Tiling& t) {
    hipError_t e = s->d3 ? launch_step3(s->precision, s->f[s->cur], s->f[s->cur ^ 1], s->g3, s->t3, coef_ptr(s),
                                        s->stream)
                         : launch_step(s->precision, s->f[s->cur], s->f[s->cur ^ 1], s->g, t, coef_ptr(s), s->stream);
    if (e != hipSuccess) return fail(LBCH_E_DEVICE, "step launch failed: %s", hipGetErrorString(e));
    return LBCH_OK;
}

lbch_status check_sim(const lbch_sim* s) {
    if (!s) return fail(LBCH_E_INVALID, "simulation handle is NULL");
    return ok();
}

lbch_status check_init(const lbch_sim* s) {
    if (!s) return fail(LBCH_E_INVALID, "simulation handle is NULL");
    if (!s->initialized) return fail(LBCH_E_STATE, "simulation not initialised (call lbch_init first)");
    return ok();
}

void free_all(lbch_sim* s) {
    if (s->hyb_win) (void)lbch_batch_destroy(s->hyb_win);
    for (void* p : {(void*)s->f[0], (void*)s->f[1], (void*)s->phi64, (void*)s->partials, (void*)s->result,
                    (void*)s->bad, s->hyb_snap, (void*)s->hyb_phi[0], (void*)s->hyb_phi[1], (void*)s->hyb_phi[2],
                    (void*)s->hyb_dsum, (void*)s->hyb_part, (void*)s->hyb_wphi})
        if (p) (void)hipFree(p);
}

struct StateHeader {
    char magic[8];            // "LBCHST01"
    int32_t abi_version;
    int32_t precision;
    int32_t nx, ny;
    int64_t step;
    lbch_params params;
};

}  // namespace

// ------------------------------------------------------------- lifecycle
extern "C" lbch_status lbch_create(const lbch_params* p, void* hip_stream, lbch_sim** out) {
    if (!out) return fail(LBCH_E_INVALID, "out pointer is NULL");
    lbch_status st = lbch_params_validate(p);
    if (st != LBCH_OK) return st;
    lbch_sim* s = new (std::nothrow) lbch_sim();
    if (!s) return fail(LBCH_E_OOM, "host allocation failed");
    s->p = *p;
    s->precision = p->precision;
    s->esize = p->precision == LBCH_FP64 ? 8 : 4;
    s->stream = (hipStream_t)hip_stream;
    s->g.nx = p->nx;
    s->g.ny = p->ny;
    s->g.pitch = (p->nx + 63) / 64 * 64;
    s->g.pad_ = 0;
    // planes padded by 256 elements so that the population planes do not
    // alias in the same DRAM channel at power-of-two sizes
    s->g.plane = (long long)s->g.pitch * p->ny + 256;
    s->d3 = p->lattice == LBCH_D3Q15;
    s->nq = s->d3 ? 15 : 9;
    s->nodes = (long long)p->nx * p->ny * p->nz;
    fill_coef<double>(p, s->cd);
    fill_coef<float>(p, s->cf);
    fill_red(p, s->rc);
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            s->cus = cus;
        (void)hipGetLastError();
    }
    long long plane = s->g.plane;
    if (s->d3) {
        s->g3.nx = p->nx;
        s->g3.ny = p->ny;
        s->g3.nz = p->nz;
        s->g3.pitch = s->g.pitch;
        s->g3.slab = (long long)s->g.pitch * p->ny;
        s->g3.plane = s->g3.slab * p->nz + 256;
        plane = s->g3.plane;
        fill_coef3<double>(p, s->c3d);
        fill_coef3<float>(p, s->c3f);
        s->t3 = sim_tiling3(s, 0, 0);
        s->t1.depth = 1;
        s->t.depth = 1;
    } else {
        // two steps per launch by default (each population crosses HBM once
        // per two updates); single-step launches finish odd step counts.  On
        // grids of at most 512^2 nodes a launch is latency-bound and one step
        // per launch is faster (7 start-up rows per chunk instead of 14:
        // measured 11.5 against 15 us per step from 64^2 to 512^2)
        const int d0 = small_grid(p->nx, p->ny) ? 1 : 2;
        s->t1 = sim_tiling(s, 1, 0, 0);
        s->t = sim_tiling(s, d0, 0, 0);
    }
    const size_t fbytes = (size_t)plane * s->nq * s->esize;
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&s->f[0], fbytes)) != hipSuccess || (e = hipMalloc(&s->f[1], fbytes)) != hipSuccess ||
        (e = hipMalloc((void**)&s->phi64, (size_t)s->nodes * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&s->partials, (size_t)kRedBlocks * 4 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&s->result, 8 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&s->bad, sizeof(unsigned))) != hipSuccess) {
        free_all(s);
        delete s;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? LBCH_E_OOM : LBCH_E_DEVICE, "device allocation failed: %s",
                    hipGetErrorString(e));
    }
    *out = s;
    return ok();
}

extern "C" lbch_status lbch_destroy(lbch_sim* s) {
    if (!s) return ok();
    (void)hipStreamSynchronize(s->stream);
    free_all(s);
    delete s;
    return ok();
}

extern "C" lbch_status lbch_init_device(lbch_sim* s, const void* phi0_dev, int32_t dtype, int64_t n) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (!phi0_dev) return fail(LBCH_E_INVALID, "phi0 pointer is NULL");
    if (dtype != LBCH_FP64 && dtype != LBCH_FP32) return fail(LBCH_E_INVALID, "unknown dtype %d", dtype);
    if (n != (int64_t)s->nodes)
        return fail(LBCH_E_INVALID, "n = %lld but the grid has %lld nodes", (long long)n, (long long)s->nodes);
    HIP_TRY(launch_zero_u32(s->bad, 1, s->stream));
    if (s->d3) HIP_TRY(launch_init3(s->precision, phi0_dev, dtype, s->f[0], s->g3, coef_ptr(s), s->bad, s->stream));
    else HIP_TRY(launch_init(s->precision, phi0_dev, dtype, s->f[0], s->g, coef_ptr(s), s->bad, s->stream));
    s->cur = 0;
    s->step = 0;
    s->initialized = true;
    return ok();
}

extern "C" lbch_status lbch_init(lbch_sim* s, const double* phi0, int64_t n) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (!phi0) return fail(LBCH_E_INVALID, "phi0 pointer is NULL");
    const int64_t nn = (int64_t)s->nodes;
    if (n != nn) return fail(LBCH_E_INVALID, "n = %lld but the grid has %lld nodes", (long long)n, (long long)nn);
    for (int64_t i = 0; i < nn; ++i)
        if (!std::isfinite(phi0[i])) return fail(LBCH_E_INVALID, "phi0[%lld] is not finite", (long long)i);
    // stage through the reduction scratch (float64, one value per node)
    HIP_TRY(hipMemcpyAsync(s->phi64, phi0, (size_t)nn * sizeof(double), hipMemcpyHostToDevice, s->stream));
    st = lbch_init_device(s, s->phi64, LBCH_FP64, n);
    if (st != LBCH_OK) return st;
    HIP_TRY(hipStreamSynchronize(s->stream));
    return ok();
}

extern "C" lbch_status lbch_step(lbch_sim* s, int64_t nsteps) {
    lbch_status st = check_init(s);
    if (st != LBCH_OK) return st;
    if (nsteps < 0) return fail(LBCH_E_INVALID, "nsteps = %lld < 0", (long long)nsteps);
    int64_t k = 0;
    if (s->t.depth == 2) {
        for (; k + 2 <= nsteps; k += 2) {
            if ((st = step_launch(s, s->t)) != LBCH_OK) return st;
            s->cur ^= 1;
            s->step += 2;
        }
    }
    for (; k < nsteps; ++k) {
        if ((st = step_launch(s, s->t1)) != LBCH_OK) return st;
        s->cur ^= 1;
        s->step += 1;
    }
    return ok();
}

extern "C" lbch_status lbch_step_extrapolated(lbch_sim* s, double ext) {
    lbch_status st = check_init(s);
    if (st != LBCH_OK) return st;
    if (!std::isfinite(ext)) return fail(LBCH_E_INVALID, "ext = %g is not finite", ext);
    if (s->d3) return fail(LBCH_E_UNSUPPORTED, "the extrapolating step is built for D2Q9");
    if (s->t.depth != 2) return fail(LBCH_E_UNSUPPORTED, "the extrapolating step needs two steps per launch");
    hipError_t e = launch_step2_extrap(s->precision, s->f[s->cur], s->f[s->cur ^ 1], s->g, s->t, coef_ptr(s), ext,
                                       s->stream);
    if (e != hipSuccess) return fail(LBCH_E_DEVICE, "step launch failed: %s", hipGetErrorString(e));
    s->cur ^= 1;
    s->step += 2;
    return ok();
}

extern "C" lbch_status lbch_get_step(const lbch_sim* s, int64_t* step) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (!step) return fail(LBCH_E_INVALID, "step pointer is NULL");
    *step = s->step;
    return ok();
}

extern "C" lbch_status lbch_synchronize(lbch_sim* s) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    HIP_TRY(hipStreamSynchronize(s->stream));
    return ok();
}

// ------------------------------------------------------------ reductions
namespace {

// phi (float64) into s->phi64 and {sum, min, max, nonfinite} into host out4.
lbch_status phi_reduce(lbch_sim* s, double out4[4]) {
    if (s->d3)
        HIP_TRY(launch_moments3(s->precision, s->f[s->cur], s->g3, s->phi64, 0, s->partials, kRedBlocks, s->stream));
    else
        HIP_TRY(launch_moments(s->precision, s->f[s->cur], s->g, s->phi64, 0, s->partials, kRedBlocks, s->stream));
    const int kinds[4] = {0, 1, 2, 0};
    HIP_TRY(launch_finalize(s->partials, kRedBlocks, 4, kinds, s->result, s->stream));
    HIP_TRY(hipMemcpyAsync(out4, s->result, 4 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    unsigned bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, s->bad, sizeof bad, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (bad) out4[3] += bad;
    return ok();
}

}  // namespace

extern "C" lbch_status lbch_moments(lbch_sim* s, double* phi_out, double* mass, double* phi_min, double* phi_max) {
    lbch_status st = check_init(s);
    if (st != LBCH_OK) return st;
    double r[4];
    st = phi_reduce(s, r);
    if (st != LBCH_OK) return st;
    if (phi_out) HIP_TRY(hipMemcpy(phi_out, s->phi64, (size_t)s->nodes * sizeof(double), hipMemcpyDeviceToHost));
    if (mass) *mass = r[0] * s->p.dx * s->p.dx * (s->d3 ? s->p.dx : 1.0);
    if (phi_min) *phi_min = r[1];
    if (phi_max) *phi_max = r[2];
    if (r[3] != 0.0) return fail(LBCH_E_NONFINITE, "state holds %.0f non-finite phi values", r[3]);
    return ok();
}

extern "C" lbch_status lbch_free_energy(lbch_sim* s, double* energy, double* terms4) {
    lbch_status st = check_init(s);
    if (st != LBCH_OK) return st;
    double r[4];
    st = phi_reduce(s, r);
    if (st != LBCH_OK) return st;
    if (s->d3) HIP_TRY(launch_energy3(s->phi64, s->g3, s->c3d, s->partials, kRedBlocks, s->stream));
    else HIP_TRY(launch_energy(s->phi64, s->g, s->rc, s->partials, kRedBlocks, s->stream));
    const int kinds[4] = {0, 0, 0, 0};
    HIP_TRY(launch_finalize(s->partials, kRedBlocks, 4, kinds, s->result, s->stream));
    double e[4];
    HIP_TRY(hipMemcpyAsync(e, s->result, 4 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const double a = s->rc.area * (s->d3 ? s->p.dx : 1.0);   // dx^2 or dx^3
    const double tg = e[0] * a, tb = e[1] * a, tr = e[2] * a;
    if (energy) *energy = tg + tb + tr;
    if (terms4) {
        terms4[0] = tg;
        terms4[1] = tb;
        terms4[2] = tr;
        terms4[3] = tg + tb + tr;
    }
    if (r[3] != 0.0 || e[3] != 0.0) return fail(LBCH_E_NONFINITE, "free energy of a non-finite state");
    return ok();
}

extern "C" lbch_status lbch_phi_device(lbch_sim* s, void* dst, int32_t dtype) {
    lbch_status st = check_init(s);
    if (st != LBCH_OK) return st;
    if (!dst) return fail(LBCH_E_INVALID, "dst is NULL");
    if (dtype != LBCH_FP64 && dtype != LBCH_FP32) return fail(LBCH_E_INVALID, "unknown dtype %d", dtype);
    if (s->d3) HIP_TRY(launch_moments3(s->precision, s->f[s->cur], s->g3, dst, dtype, s->partials, kRedBlocks,
                                       s->stream));
    else HIP_TRY(launch_moments(s->precision, s->f[s->cur], s->g, dst, dtype, s->partials, kRedBlocks, s->stream));
    return ok();
}

// ---------------------------------------------------------- checkpointing
extern "C" lbch_status lbch_state_bytes(const lbch_sim* s, int64_t* bytes) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (!bytes) return fail(LBCH_E_INVALID, "bytes pointer is NULL");
    *bytes = (int64_t)sizeof(StateHeader) + (int64_t)s->nq * s->nodes * (int64_t)s->esize;
    return ok();
}

extern "C" lbch_status lbch_save_state(lbch_sim* s, void* dst, int32_t dst_is_device) {
    lbch_status st = check_init(s);
    if (st != LBCH_OK) return st;
    if (!dst) return fail(LBCH_E_INVALID, "dst is NULL");
    StateHeader h{};
    std::memcpy(h.magic, "LBCHST01", 8);
    h.abi_version = LBCH_ABI_VERSION;
    h.precision = s->precision;
    h.nx = s->g.nx;
    h.ny = s->g.ny;
    h.step = s->step;
    h.params = s->p;
    const size_t body = (size_t)s->nq * s->nodes * s->esize;
    // the idle population buffer holds the dense copy
    void* tmp = s->f[s->cur ^ 1];
    if (s->d3) HIP_TRY(launch_gather3(s->precision, s->f[s->cur], s->g3, tmp, s->stream));
    else HIP_TRY(launch_gather(s->precision, s->f[s->cur], s->g, tmp, s->stream));
    if (dst_is_device) {
        HIP_TRY(hipMemcpyAsync(dst, &h, sizeof h, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipMemcpyAsync((char*)dst + sizeof h, tmp, body, hipMemcpyDeviceToDevice, s->stream));
    } else {
        std::memcpy(dst, &h, sizeof h);
        HIP_TRY(hipMemcpyAsync((char*)dst + sizeof h, tmp, body, hipMemcpyDeviceToHost, s->stream));
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return ok();
}

extern "C" lbch_status lbch_load_state(lbch_sim* s, const void* src, int32_t src_is_device) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (!src) return fail(LBCH_E_INVALID, "src is NULL");
    StateHeader h{};
    if (src_is_device) HIP_TRY(hipMemcpy(&h, src, sizeof h, hipMemcpyDeviceToHost));
    else std::memcpy(&h, src, sizeof h);
    if (std::memcmp(h.magic, "LBCHST01", 8) != 0) return fail(LBCH_E_INVALID, "not an lbch state (bad magic)");
    if (h.abi_version != LBCH_ABI_VERSION) return fail(LBCH_E_INVALID, "state ABI %d", h.abi_version);
    if (h.precision != s->precision || h.nx != s->g.nx || h.ny != s->g.ny || h.params.lattice != s->p.lattice ||
        h.params.nz != s->p.nz)
        return fail(LBCH_E_INVALID,
                    "state is %dx%dx%d lattice %d precision %d, simulation is %dx%dx%d lattice %d precision %d", h.nx,
                    h.ny, h.params.nz, h.params.lattice, h.precision, s->g.nx, s->g.ny, s->p.nz, s->p.lattice,
                    s->precision);
    const size_t body = (size_t)s->nq * s->nodes * s->esize;
    void* tmp = s->f[s->cur ^ 1];
    HIP_TRY(hipMemcpyAsync(tmp, (const char*)src + sizeof h, body,
                           src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
    if (s->d3) HIP_TRY(launch_scatter3(s->precision, tmp, s->g3, s->f[s->cur], s->stream));
    else HIP_TRY(launch_scatter(s->precision, tmp, s->g, s->f[s->cur], s->stream));
    HIP_TRY(launch_zero_u32(s->bad, 1, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->step = h.step;
    s->initialized = true;
    return ok();
}

// ---------------------------------------------------------------- tiling
extern "C" lbch_status lbch_set_time_blocking(lbch_sim* s, int32_t depth) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (depth != 1 && depth != 2) return fail(LBCH_E_INVALID, "time-blocking depth %d not in {1, 2}", depth);
    if (s->d3) {
        if (depth != 1) return fail(LBCH_E_UNSUPPORTED, "D3Q15 steps one time step per launch");
        return ok();
    }
    s->t = sim_tiling(s, depth, 0, 0);
    if (depth == 1) s->t1 = s->t;
    return ok();
}

extern "C" lbch_status lbch_get_time_blocking(const lbch_sim* s, int32_t* depth) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (!depth) return fail(LBCH_E_INVALID, "depth pointer is NULL");
    *depth = s->t.depth;
    return ok();
}

extern "C" lbch_status lbch_set_tiling(lbch_sim* s, int32_t block_threads, int32_t rows_per_block) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (s->d3) {
        if (block_threads != 0 && !tile3_shape(s->precision, block_threads, nullptr, nullptr))
            return fail(LBCH_E_INVALID, "D3Q15 block_threads %d not in {0, 512%s}", block_threads,
                        s->precision == LBCH_FP32 ? ", 988, 1024" : "");
        if (rows_per_block < 0) return fail(LBCH_E_INVALID, "rows_per_block %d < 0", rows_per_block);
        s->t3 = sim_tiling3(s, block_threads, rows_per_block);
        return ok();
    }
    const int depth = s->t.depth;
    if (block_threads != 0 && block_threads != 64 && block_threads != 128 && block_threads != 256 &&
        block_threads != 512)
        return fail(LBCH_E_INVALID, "block_threads %d not in {64, 128, 256, 512}", block_threads);
    if (depth == 2 && (block_threads == 64 || (s->esize == 8 && block_threads == 512)))
        return fail(LBCH_E_INVALID, "block_threads %d not available at time-blocking depth 2 in %s", block_threads,
                    s->esize == 8 ? "FP64" : "FP32");
    if (rows_per_block < 0) return fail(LBCH_E_INVALID, "rows_per_block %d < 0", rows_per_block);
    s->user_nt = block_threads;
    s->user_hc = rows_per_block;
    s->t = sim_tiling(s, depth, block_threads, rows_per_block);
    if (depth == 1) s->t1 = s->t;
    return ok();
}

extern "C" lbch_status lbch_set_row_loader(lbch_sim* s, int32_t mode) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (mode != 0 && mode != 1) return fail(LBCH_E_INVALID, "row loader mode %d not in {0, 1}", mode);
    s->user_loader = mode;
    s->t.staged = mode == 0;
    s->t1.staged = mode == 0;
    return ok();
}

extern "C" lbch_status lbch_get_tiling(const lbch_sim* s, int32_t* block_threads, int32_t* rows_per_block) {
    lbch_status st = check_sim(s);
    if (st != LBCH_OK) return st;
    if (block_threads) *block_threads = s->d3 ? s->t3.tx * s->t3.ty : s->t.nt;
    if (rows_per_block) *rows_per_block = s->d3 ? s->t3.hz : s->t.hc;
    return ok();
}

// ------------------------------------------------------------ diagnostics
extern "C" lbch_status lbch_diag_copy(const void* src, void* dst, int64_t bytes, void* hip_stream) {
    if (!src || !dst) return fail(LBCH_E_INVALID, "NULL pointer");
    if (bytes <= 0 || bytes % 16 != 0) return fail(LBCH_E_INVALID, "bytes = %lld must be a positive multiple of 16",
                                                   (long long)bytes);
    if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return fail(LBCH_E_INVALID, "pointers must be 16-byte aligned");
    HIP_TRY(launch_copy16(src, dst, bytes / 16, (hipStream_t)hip_stream));
    return ok();
}

// ------------------------------------------------------------- autotuner
namespace {

// D3Q15: every built tile shape x sweep lengths {4, 8, 16, 32, 64, 128, model}
// (capped at nz), timed like the D2Q9 trials (idle buffer written, state kept).
// The sweep-length model counts rounds of resident workgroups; measured, the
// step is closer to bound by the total work (tiles x (hz + 7)), so the trials
// decide.
lbch_status autotune3(lbch_sim* s, int steps_per_trial, int32_t* block_threads, int32_t* rows_per_block,
                      double* ms_per_step) {
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    float best = -1.0f;
    Tiling3 best_t = s->t3;
    const int shapes[3] = {512, 988, 1024};
    const int hzs[7] = {0, 4, 8, 16, 32, 64, 128};
    for (int bt : shapes) {
        if (!tile3_shape(s->precision, bt, nullptr, nullptr)) continue;
        for (int hz : hzs) {
            if (hz > s->g3.nz) continue;
            const Tiling3 t = sim_tiling3(s, bt, hz);
            hipError_t e = launch_step3(s->precision, s->f[s->cur], s->f[s->cur ^ 1], s->g3, t, coef_ptr(s),
                                        s->stream);
            if (e == hipSuccess) e = hipEventRecord(a, s->stream);
            for (int k = 0; e == hipSuccess && k < steps_per_trial; ++k)
                e = launch_step3(s->precision, s->f[s->cur], s->f[s->cur ^ 1], s->g3, t, coef_ptr(s), s->stream);
            if (e == hipSuccess) e = hipEventRecord(b, s->stream);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e != hipSuccess) {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
                return fail(LBCH_E_DEVICE, "autotune trial failed: %s", hipGetErrorString(e));
            }
            if (best < 0.0f || ms < best) {
                best = ms;
                best_t = t;
            }
        }
    }
    s->t3 = best_t;
    // the winner timed once more on its own (as for D2Q9)
    float ms = 0.0f;
    hipError_t e = hipEventRecord(a, s->stream);
    for (int k = 0; e == hipSuccess && k < steps_per_trial; ++k)
        e = launch_step3(s->precision, s->f[s->cur], s->f[s->cur ^ 1], s->g3, s->t3, coef_ptr(s), s->stream);
    if (e == hipSuccess) e = hipEventRecord(b, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(LBCH_E_DEVICE, "autotune trial failed: %s", hipGetErrorString(e));
    if (block_threads) *block_threads = best_t.tx * best_t.ty;
    if (rows_per_block) *rows_per_block = best_t.hz;
    if (ms_per_step) *ms_per_step = ms / steps_per_trial;
    return LBCH_OK;
}

}  // namespace

extern "C" lbch_status lbch_autotune(lbch_sim* s, int32_t steps_per_trial, int32_t* block_threads,
                                     int32_t* rows_per_block, double* ms_per_step) {
    lbch_status st = check_init(s);
    if (st != LBCH_OK) return st;
    if (steps_per_trial < 1) return fail(LBCH_E_INVALID, "steps_per_trial %d < 1", steps_per_trial);
    if (s->d3) return autotune3(s, steps_per_trial, block_threads, rows_per_block, ms_per_step);
    // Trials read the current state and write the idle buffer, so the state is untouched.
    // chunk heights: 0 = the launch model's own choice (the default tiling, small-grid rule
    // included), then fixed heights
    const int nts[4] = {64, 128, 256, 512};
    const int hcs[8] = {0, 8, 16, 32, 64, 128, 256, 512};
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    float best[2] = {-1.0f, -1.0f};          // per step, per depth
    Tiling best_t[2] = {s->t1, s->t};
    const int staged = s->t.staged;
    for (int depth = 1; depth <= 2; ++depth) {
        for (int nt : nts) {
            if (nt > 128 && s->g.nx < nt / 2) continue;          // mostly idle lanes
            if (depth == 2 && (nt == 64 || (s->esize == 8 && nt == 512))) continue;
            for (int hc : hcs) {
                if (hc > 8 && hc > s->g.ny) continue;
                if (depth == 2 && hc > 0 && hc < 32) continue;   // 17 start-up rows per chunk
                Tiling t = hc == 0 ? sim_tiling(s, depth, nt, 0)
                                   : make_tiling(s->g.nx, s->g.ny, nt, hc, depth, (int)s->esize);
                t.staged = staged;
                hipError_t e =
                    launch_step(s->precision, s->f[s->cur], s->f[s->cur ^ 1], s->g, t, coef_ptr(s), s->stream);
                if (e == hipSuccess) e = hipEventRecord(a, s->stream);
                for (int k = 0; e == hipSuccess && k < steps_per_trial; ++k)
                    e = launch_step(s->precision, s->f[s->cur], s->f[s->cur ^ 1], s->g, t, coef_ptr(s), s->stream);
                if (e == hipSuccess) e = hipEventRecord(b, s->stream);
                if (e == hipSuccess) e = hipEventSynchronize(b);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                if (e != hipSuccess) {
                    (void)hipEventDestroy(a);
                    (void)hipEventDestroy(b);
                    return fail(LBCH_E_DEVICE, "autotune trial failed: %s", hipGetErrorString(e));
                }
                ms /= (float)depth;
                if (best[depth - 1] < 0.0f || ms < best[depth - 1]) {
                    best[depth - 1] = ms;
                    best_t[depth - 1] = t;
                }
            }
        }
    }
    s->t1 = best_t[0];
    const int d = (best[1] >= 0.0f && best[1] < best[0]) ? 2 : 1;
    s->t = best_t[d - 1];
    s->user_nt = s->t.nt;
    s->user_hc = s->t.hc;
    // the winner timed once more on its own: the minimum over many trials is biased low, and
    // the GPU is left running the chosen kernel (its clocks settle over ~20 launches after a
    // change of load)
    float ms = 0.0f;
    hipError_t e = hipEventRecord(a, s->stream);
    for (int k = 0; e == hipSuccess && k < steps_per_trial; ++k)
        e = launch_step(s->precision, s->f[s->cur], s->f[s->cur ^ 1], s->g, s->t, coef_ptr(s), s->stream);
    if (e == hipSuccess) e = hipEventRecord(b, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(LBCH_E_DEVICE, "autotune trial failed: %s", hipGetErrorString(e));
    if (block_threads) *block_threads = s->t.nt;
    if (rows_per_block) *rows_per_block = s->t.hc;
    if (ms_per_step) *ms_per_step = ms / (float)d / (float)steps_per_trial;
    return ok();
}
