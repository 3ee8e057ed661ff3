// Surrogate jump + lattice Boltzmann correction / rejection (include/lbch_hybrid.h).
#include "../../include/lbch_batch.h"
#include "../../include/lbch_hybrid.h"
#include "lbch_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <random>
#include <vector>

using namespace lbch;

#define HIP_TRY(expr)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(LBCH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define ST_TRY(expr)                      \
    do {                                  \
        lbch_status s_ = (expr);          \
        if (s_ != LBCH_OK) return s_;     \
    } while (0)

extern "C" lbch_status lbch_hybrid_default_opts(lbch_hybrid_opts* o) {
    if (!o) return fail(LBCH_E_INVALID, "NULL argument");
    std::memset(o, 0, sizeof *o);
    o->jump = 200;
    o->correct_steps = 10;
    o->tol_energy = 1e-6;
    o->windows = 4;
    o->window_interior = 192;
    o->window_margin = 64;
    o->tol_window = 1e-2;
    o->check_every = 1;
    o->seed = 1;
    o->ncond = 0;
    return LBCH_OK;
}

namespace {

// The schedule's workspace, kept with the simulation (freed by lbch_destroy):
// allocated by the first call, the window ensemble again only when the window
// count or size changes.
lbch_status ensure_workspace(lbch_sim* sim, const lbch_hybrid_opts* o, int side) {
    const size_t fbytes = (size_t)sim->g.plane * 9 * sim->esize;
    const size_t nbytes = (size_t)sim->g.nx * sim->g.ny * sizeof(float);
    auto get = [](void** p, size_t bytes) -> hipError_t { return *p ? hipSuccess : hipMalloc(p, bytes); };
    HIP_TRY(get(&sim->hyb_snap, fbytes));
    for (float*& q : sim->hyb_phi) HIP_TRY(get((void**)&q, nbytes));
    HIP_TRY(get((void**)&sim->hyb_dsum, 8 * sizeof(double)));
    HIP_TRY(get((void**)&sim->hyb_part, (size_t)kRedBlocks * 4 * sizeof(double)));
    if (o->windows > 0 && (sim->hyb_windows != o->windows || sim->hyb_side != side)) {
        if (sim->hyb_win) {
            (void)lbch_batch_destroy(sim->hyb_win);
            sim->hyb_win = nullptr;
        }
        if (sim->hyb_wphi && sim->hyb_side != side) {
            (void)hipFree(sim->hyb_wphi);
            sim->hyb_wphi = nullptr;
        }
        sim->hyb_windows = sim->hyb_side = 0;
        HIP_TRY(get((void**)&sim->hyb_wphi, (size_t)side * side * sizeof(float)));
        std::vector<lbch_params> mp(o->windows, sim->p);
        for (auto& q : mp) q.nx = q.ny = side;
        ST_TRY(lbch_batch_create(mp.data(), o->windows, sim->stream, &sim->hyb_win));
        sim->hyb_windows = o->windows;
        sim->hyb_side = side;
    }
    return LBCH_OK;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    void start() { (void)hipEventRecord(a, s); }
    double stop() {
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
};

}  // namespace

extern "C" lbch_status lbch_hybrid_advance(lbch_sim* sim, lbsg_net* net, const lbch_hybrid_opts* o, int64_t nsteps,
                                           lbch_hybrid_stats* stats) {
    if (!sim || !o || (!net && !o->dry_run && !o->extrapolate)) return fail(LBCH_E_INVALID, "NULL argument");
    if (!sim->initialized) return fail(LBCH_E_STATE, "simulation not initialised");
    if (sim->d3) return fail(LBCH_E_UNSUPPORTED, "the hybrid schedule runs on D2Q9 simulations only");
    if (o->jump < 1 || o->correct_steps < 0 || !(o->tol_energy >= 0) || o->windows < 0 || o->window_interior < 1 ||
        o->window_margin < 0 || !(o->tol_window > 0) || o->check_every < 1 || o->ncond < 0 || o->ncond > 8 ||
        o->inner_steps < 0 || o->inner_jump < 0 || nsteps < 0)
        return fail(LBCH_E_INVALID, "invalid hybrid options");
    const int nx = sim->g.nx, ny = sim->g.ny;
    const long long N = (long long)nx * ny;
    const int side = o->window_interior + 2 * o->window_margin;
    if (o->windows > 0 && (side > nx || side > ny)) return fail(LBCH_E_INVALID, "window larger than the grid");
    hipStream_t s = sim->stream;
    // The projective difference of the correction phase spans the last launch, which must
    // advance two steps (a one-step difference amplifies the flux mode, eigenvalue -0.25 of
    // the linearised step): run at two steps per launch, and give the caller's tiling back.
    struct TilingGuard {
        lbch_sim* sim;
        lbch::Tiling t;
        ~TilingGuard() { sim->t = t; }
    } tiling_guard{sim, sim->t};
    if (o->inner_steps > 0 && o->inner_jump > 0 && sim->t.depth != 2) ST_TRY(lbch_set_time_blocking(sim, 2));
    lbch_hybrid_stats st{};
    ST_TRY(ensure_workspace(sim, o, side));
    void *snap = sim->hyb_snap, *phi = sim->hyb_phi[0], *phin = sim->hyb_phi[1], *phi1 = sim->hyb_phi[2],
         *dsum = sim->hyb_dsum, *part = sim->hyb_part, *wphi = sim->hyb_wphi;
    lbch_batch* win = o->windows > 0 ? sim->hyb_win : nullptr;
    const size_t fbytes = (size_t)sim->g.plane * 9 * sim->esize;
    // Three population buffers rotate: the simulation's pair f[cur], f[cur ^ 1] and one
    // outside it, which holds the snapshot of the cycle's start state while a cycle runs
    // (no copy): the first write of a cycle goes to a pair buffer that is not the snapshot,
    // and the snapshot is then taken out of the pair.  On exit the simulation gets its own
    // two buffers back (one copy when its state sits in the third).
    struct PairGuard {
        lbch_sim* sim;
        void* own0;       // the simulation's own buffers
        void* own1;
        void* third;
        size_t bytes;
        hipStream_t s;
        ~PairGuard() {
            void*& cur = sim->f[sim->cur];
            void*& oth = sim->f[sim->cur ^ 1];
            if (cur == third) {
                void* dst = (oth == own0) ? own1 : own0;
                (void)hipMemcpyAsync(dst, third, bytes, hipMemcpyDeviceToDevice, s);
                (void)hipStreamSynchronize(s);
                cur = dst;
            }
            oth = (cur == own0) ? own1 : own0;
        }
    } pair_guard{sim, sim->f[0], sim->f[1], snap, fbytes, s};
    void* spare = snap;     // the buffer outside the pair
    std::mt19937_64 rng(o->seed);
    Timer tm(s);
    const int64_t cyc = (int64_t)o->jump + o->correct_steps;
    int64_t left = nsteps;
    // correction phase: plain steps, optionally with projective steps of the populations
    const size_t pop_elems = (size_t)sim->g.plane * 9;
    auto correct = [&](int64_t n) -> lbch_status {
        int64_t done = 0;
        if (o->inner_steps > 0 && o->inner_jump > 0) {
            // the difference spans the last launch: two steps when the plain steps run two per launch
            const int span = (sim->t.depth == 2 && o->inner_steps % 2 == 0) ? 2 : 1;
            // with two steps per launch the extrapolation is stored by the last launch itself
            const bool fused = span == 2 && !sim->d3;
            while (done + 2LL * o->inner_steps + o->inner_jump <= n) {
                if (fused) {
                    lbch_status ls = lbch_step(sim, o->inner_steps - 2);
                    if (ls != LBCH_OK) return ls;
                    ls = lbch_step_extrapolated(sim, (double)o->inner_jump / span);
                    if (ls != LBCH_OK) return ls;
                } else {
                    lbch_status ls = lbch_step(sim, o->inner_steps);
                    if (ls != LBCH_OK) return ls;
                    HIP_TRY(launch_extrap_pop(sim->precision, sim->f[sim->cur], sim->f[sim->cur ^ 1],
                                              (double)o->inner_jump / span, (long long)pop_elems, s));
                }
                sim->step += o->inner_jump;
                done += o->inner_steps + o->inner_jump;
            }
        }
        return lbch_step(sim, n - done);
    };
    double E0 = 0.0, E1 = 0.0;
    bool have_e0 = false;             // E0 known: the state is the one an accepted cycle ended in
    while (left >= cyc) {
        st.cycles += 1;
        if (!have_e0) {
            lbch_status est = lbch_free_energy(sim, &E0, nullptr);
            if (est != LBCH_OK) return est;
        }
        const int64_t step0 = sim->step;
        // snapshot (the start state's buffer leaves the pair), jump, mass projection,
        // re-initialisation
        tm.start();
        void* const saved = sim->f[sim->cur];
        if (o->dry_run) {
            HIP_TRY(hipMemcpyAsync(spare, saved, fbytes, hipMemcpyDeviceToDevice, s));
            sim->f[sim->cur] = spare;
            spare = saved;
        } else {
            ST_TRY(lbch_phi_device(sim, phi, LBCH_FP32));
            if (o->extrapolate) {
                // rate from one plain step (the state is re-initialised below); it reads the
                // saved buffer and writes the other one, then the saved buffer leaves the pair
                ST_TRY(lbch_step(sim, 1));
                sim->f[sim->cur ^ 1] = spare;
                spare = saved;
                ST_TRY(lbch_phi_device(sim, phi1, LBCH_FP32));
                const float* base = (const float*)phi;
                if (net) {
                    ST_TRY(lbsg_predict(net, (const float*)phi, o->cond, o->ncond, ny, nx, (float*)phin));
                    base = (const float*)phin;
                }
                HIP_TRY(launch_extrap_f32(base, (const float*)phi, (const float*)phi1, (float)o->jump, N,
                                          (float*)phin, s));
            } else {
                ST_TRY(lbsg_predict(net, (const float*)phi, o->cond, o->ncond, ny, nx, (float*)phin));
                sim->f[sim->cur] = spare;     // the re-initialisation writes outside the snapshot
                spare = saved;
            }
            HIP_TRY(launch_sum_f32((const float*)phi, N, (double*)part, (double*)dsum, s));
            HIP_TRY(launch_sum_f32((const float*)phin, N, (double*)part, (double*)dsum + 1, s));
            HIP_TRY(launch_add_f32((float*)phin, N, (const double*)dsum, (const double*)dsum + 1, 1.0 / (double)N, s));
            ST_TRY(lbch_init_device(sim, phin, LBCH_FP32, N));
        }
        st.ms_surrogate += tm.stop();
        tm.start();
        if (o->dry_run) {
            ST_TRY(lbch_step(sim, cyc));
        } else {
            ST_TRY(correct(o->correct_steps));
        }
        st.ms_correct += tm.stop();
        sim->step = step0 + cyc;
        // checks
        tm.start();
        bool accept = true;
        lbch_status est = lbch_free_energy(sim, &E1, nullptr);
        if (est != LBCH_OK && est != LBCH_E_NONFINITE) return est;
        if (est == LBCH_E_NONFINITE || !(E1 <= E0 * (1.0 + o->tol_energy))) {
            accept = false;
            st.rejected_energy += 1;
        }
        if (accept && o->windows > 0 && (st.cycles - 1) % o->check_every == 0) {
            // shadow windows from the snapshot (swap it in temporarily as the state to read)
            std::vector<std::pair<int, int>> pos(o->windows);
            void* live = sim->f[sim->cur];
            sim->f[sim->cur] = saved;
            for (int w = 0; w < o->windows; ++w) {
                pos[w] = {(int)(rng() % (uint64_t)ny), (int)(rng() % (uint64_t)nx)};
                lbch_status ls = lbch_batch_load_window(win, w, sim, pos[w].first, pos[w].second);
                if (ls != LBCH_OK) {
                    sim->f[sim->cur] = live;
                    return ls;
                }
            }
            sim->f[sim->cur] = live;
            ST_TRY(lbch_batch_step(win, cyc));
            ST_TRY(lbch_phi_device(sim, phi, LBCH_FP32));
            double worst = 0.0;
            for (int w = 0; w < o->windows; ++w) {
                ST_TRY(lbch_batch_phi_device(win, w, wphi, LBCH_FP32));
                HIP_TRY(launch_window_err((const float*)wphi, side, (const float*)phi, ny, nx, pos[w].first,
                                          pos[w].second, o->window_margin, o->window_interior, (double*)part,
                                          (double*)dsum + 2, s));
                double e2[2];
                HIP_TRY(hipMemcpyAsync(e2, (double*)dsum + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                const double rel = std::sqrt(e2[0] / (e2[1] > 0 ? e2[1] : 1e-300));
                if (rel > worst) worst = rel;
            }
            if (worst > st.max_window_err) st.max_window_err = worst;
            if (worst > o->tol_window) {
                accept = false;
                st.rejected_window += 1;
            }
        }
        st.ms_checks += tm.stop();
        if (accept) {
            st.accepted += 1;
            st.last_energy = E1;
            E0 = E1;
            have_e0 = true;       // the snapshot's buffer (spare) is free again
        } else {
            have_e0 = false;
            tm.start();
            // back to the start state: its buffer returns to the pair
            spare = sim->f[sim->cur];
            sim->f[sim->cur] = saved;
            sim->step = step0;
            ST_TRY(lbch_step(sim, cyc));
            st.plain_steps += cyc;
            st.ms_plain += tm.stop();
        }
        left -= cyc;
    }
    if (left > 0) {
        tm.start();
        ST_TRY(lbch_step(sim, left));
        st.plain_steps += left;
        st.ms_plain += tm.stop();
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (stats) *stats = st;
    return LBCH_OK;
}

extern "C" lbch_status lbch_extrapolate(const float* base, const float* phi_t, const float* phi_t1, double k,
                                        int64_t n, float* out, void* hip_stream) {
    if (!base || !phi_t || !phi_t1 || !out) return fail(LBCH_E_INVALID, "NULL argument");
    if (n < 0) return fail(LBCH_E_INVALID, "n = %lld < 0", (long long)n);
    if (!std::isfinite(k)) return fail(LBCH_E_INVALID, "k is not finite");
    if (n == 0) return LBCH_OK;
    HIP_TRY(launch_extrap_f32(base, phi_t, phi_t1, (float)k, n, out, (hipStream_t)hip_stream));
    return LBCH_OK;
}
