/*
 * lbch_hybrid.h — surrogate-accelerated time stepping with the lattice
 * Boltzmann scheme as fallback and judge.
 *
 * One cycle advances a simulation by jump + correct_steps time steps:
 *   1. free energy E0 of the current state (eq 7, discrete);
 *   2. snapshot of the populations;
 *   3. phi' = surrogate(phi, conditioning)  (the net was trained to map
 *      phi(t) to phi(t + jump));
 *   4. exact mass projection: phi' += (sum phi - sum phi') / N;
 *   5. the populations are re-initialised at the equilibrium of eq 18 at
 *      phi' (as lbch_init_device) and correct_steps plain steps follow;
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
} lbch_hybrid_opts;

typedef struct lbch_hybrid_stats {
    int64_t cycles, accepted, rejected_energy, rejected_window;
    int64_t plain_steps;      /* steps run by the plain scheme (rejections and remainder) */
    double max_window_err;    /* largest window relative L2 difference seen */
    double last_energy;
    double ms_surrogate, ms_correct, ms_checks, ms_plain;   /* device time split */
} lbch_hybrid_stats;

/* jump 200, correct_steps 10, tol_energy 1e-6, 4 windows of 192 + 2 x 64,
 * tol_window 1e-2, check_every 1, seed 1, ncond 0, dry_run 0. */
lbch_status lbch_hybrid_default_opts(lbch_hybrid_opts* opts);

/* Advances sim by nsteps (>= 0) with the cycle above; stats (nullable) are
 * filled (not accumulated).  net may be NULL only with dry_run.  Synchronises. */
lbch_status lbch_hybrid_advance(lbch_sim* sim, lbsg_net* net, const lbch_hybrid_opts* opts, int64_t nsteps,
                                lbch_hybrid_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* LBCH_HYBRID_H */
