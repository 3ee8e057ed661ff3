/*
 * lbch_hybrid.h — jump-accelerated time stepping with the lattice Boltzmann
 * scheme as fallback and reference.
 *
 * One cycle advances a simulation by jump + correct_steps time steps:
 *   1. free energy E0 of the current state (eq 7, discrete; the E1 of the
 *      previous cycle when that cycle was accepted);
 *   2. snapshot of the populations;
 *   3. the jump, phi(t) -> phi'(t + jump), in one of two forms:
 *      extrapolate = 0: phi' = surrogate(phi, conditioning) (the network was
 *        trained to map phi(t) to phi(t + jump));
 *      extrapolate = 1: one plain step gives the rate r = phi(t+1) - phi(t);
 *        phi' = phi(t) + jump * r, plus, when a network is given, its
 *        residual surrogate(phi(t)) - phi(t) (the network was trained on
 *        phi(t + jump) - jump * r as the target);
 *   4. exact mass projection: phi' += (sum phi - sum phi') / N;
 *   5. the populations are re-initialised at the equilibrium of eq 18 at
 *      phi' (as lbch_init_device) and correct_steps plain steps follow
 *      (optionally accelerated themselves by short projective steps of the
 *      populations, inner_steps / inner_jump below);
 *   6. checks: reject if E1 > E0 (1 + tol_energy); on every check_every-th
 *      cycle also run `windows` shadow windows (interior + margin on each
 *      side, random positions) with the plain scheme for jump + correct_steps
 *      steps from the snapshot and reject if the relative L2 difference of
 *      their interiors to the hybrid state exceeds tol_window;
 *   7. on rejection the snapshot is restored and the cycle's steps are run
 *      with the plain scheme.
 * Steps that do not fill a cycle are plain steps.  A run whose every jump is
 * rejected is bitwise identical to a plain run.
 *
 * The extrapolated jump is a projective step: the correction steps must damp
 * what the extrapolation amplifies (a mode decaying by mu per step grows by
 * |1 - jump mu| per jump and shrinks by (1 - mu)^correct_steps), which needs
 * correct_steps of the order of jump / 3; the energy and window checks reject
 * cycles that violate it.
 *
 * Conventions as in lbch.h.  The simulation and the network must share the
 * same stream.
 */
#ifndef LBCH_HYBRID_H
#define LBCH_HYBRID_H

#include <stdint.h>

#include "lbch.h"
#include "lbsg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbch_hybrid_opts {
    int32_t jump;             /* steps covered by one surrogate application (> 0) */
    int32_t correct_steps;    /* plain steps after each re-initialisation (>= 0) */
    double tol_energy;        /* relative free-energy increase allowed per cycle (>= 0) */
    int32_t windows;          /* shadow windows per checked cycle (0 = no window check) */
    int32_t window_interior;  /* interior side of a window (>= 1) */
    int32_t window_margin;    /* margin on each side (>= 0) */
    double tol_window;        /* relative L2 tolerance of the window interiors (> 0) */
    int32_t check_every;      /* window check on every check_every-th cycle (>= 1) */
    uint64_t seed;            /* window placement */
    int32_t ncond;            /* conditioning values of the surrogate (= its in_ch - 1) */
    float cond[8];
    int32_t dry_run;          /* nonzero: no surrogate; each cycle runs the plain scheme and the
                                 window check measures the windows' own error (calibration) */
    int32_t extrapolate;      /* 0: the network maps phi(t) -> phi(t + jump); 1: rate extrapolation
                                 from one plain step, plus the network's residual if one is given */
    int32_t inner_steps;      /* > 0: the correction phase runs in inner cycles of inner_steps plain
                                 steps followed by a projective step of the populations over
                                 inner_jump steps (f += inner_jump / d (f_n - f_(n-d)), d = 2 when
                                 inner_steps is even, else 1), repeated while at least inner_steps
                                 plain steps remain after it; the rest are plain steps.  With inner
                                 steps the simulation runs two steps per launch during the call
                                 (its tiling is restored on return): only a two-step difference is
                                 stable (the flux mode of a one-step difference grows). */
    int32_t inner_jump;       /* >= 0 */
} lbch_hybrid_opts;

typedef struct lbch_hybrid_stats {
    int64_t cycles, accepted, rejected_energy, rejected_window;
    int64_t plain_steps;      /* steps run by the plain scheme (rejections and remainder) */
    double max_window_err;    /* largest window relative L2 difference seen */
    double last_energy;
    double ms_surrogate, ms_correct, ms_checks, ms_plain;   /* device time split */
} lbch_hybrid_stats;

/* jump 200, correct_steps 10, tol_energy 1e-6, 4 windows of 192 + 2 x 64,
 * tol_window 1e-2, check_every 1, seed 1, ncond 0, dry_run 0, extrapolate 0,
 * inner_steps 0, inner_jump 0. */
lbch_status lbch_hybrid_default_opts(lbch_hybrid_opts* opts);

/* Advances sim by nsteps (>= 0) with the cycle above; stats (nullable) are
 * filled (not accumulated).  net may be NULL only with dry_run or
 * extrapolate.  Synchronises.  The first call on a simulation allocates the
 * schedule's workspace, which stays with the simulation until lbch_destroy: a
 * third population buffer (the snapshot), three FP32 fields of the grid and
 * the shadow-window ensemble; later calls allocate nothing unless the window
 * count or size changes (then the ensemble is rebuilt).  A failed allocation
 * returns LBCH_E_DEVICE before the state is touched. */
lbch_status lbch_hybrid_advance(lbch_sim* sim, lbsg_net* net, const lbch_hybrid_opts* opts, int64_t nsteps,
                                lbch_hybrid_stats* stats);

/* out[i] = base[i] + k (phi_t1[i] - phi_t[i]) for i < n, all FP32 device
 * arrays (out may alias base): the extrapolated jump of step 3, and the
 * residual target phi(t + jump) - jump r of the training data (base =
 * phi(t + jump), k = -jump).  Stream-ordered.
 * NULL pointer or n < 0 -> LBCH_E_INVALID. */
lbch_status lbch_extrapolate(const float* base, const float* phi_t, const float* phi_t1, double k, int64_t n,
                             float* out, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBCH_HYBRID_H */
