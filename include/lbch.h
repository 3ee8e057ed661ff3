/*
 * lbch.h — C ABI of the MI355X (gfx950) lattice Boltzmann solver for the
 * anisotropic Cahn–Hilliard equation of Liu, Wang & Liu, "Modelling
 * anisotropic Cahn-Hilliard equation with the lattice Boltzmann method"
 * (arXiv 2501.03759).
 *
 * One simulation = one periodic D2Q9 grid (or one D3Q15 box, eq 21) whose
 * populations live in HBM in the library's own buffers.  Every call returns an lbch_status (0 = OK,
 * < 0 = error); no C++ exception crosses the ABI and lbch_last_error()
 * returns a thread-local message describing the last failure.
 *
 * Units: lattice spacing dx and time step dt are parameters (default 1);
 * c = dx/dt and c_s^2 = c^2/3 (Section 3, below eq 21).
 *
 * Ownership: the library owns all device memory it allocates; host arrays
 * passed in are copied and never retained; device pointers passed in must
 * stay valid until the work queued on the simulation's stream completes.
 *
 * Streams: each simulation is bound to one HIP stream (NULL = the null
 * stream).  Calls that only enqueue work return before it completes;
 * calls that return host data synchronise that stream.  A simulation must
 * not be used from two threads at once; distinct simulations are
 * independent.
 */
#ifndef LBCH_H
#define LBCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBCH_ABI_VERSION 2

typedef enum lbch_status {
    LBCH_OK = 0,
    LBCH_E_INVALID = -1,      /* bad argument or parameter */
    LBCH_E_UNSUPPORTED = -2,  /* valid in the paper but not built (non-periodic, 3D options below) */
    LBCH_E_OOM = -3,          /* device or host allocation failed */
    LBCH_E_DEVICE = -4,       /* HIP runtime error */
    LBCH_E_NONFINITE = -5,    /* the state holds NaN/Inf (results still written) */
    LBCH_E_STATE = -6         /* call out of order (e.g. step before init) */
} lbch_status;

enum { LBCH_D2Q9 = 0 /* eq 20 */, LBCH_D3Q15 = 1 /* eq 21 (see below) */ };
enum { LBCH_FP64 = 0, LBCH_FP32 = 1 };
enum { LBCH_BC_PERIODIC = 0 /* Section 4: periodic boundaries */ };
enum {
    LBCH_REG_NONE = 0,
    LBCH_REG_LINEAR = 1,      /* eq 8 / eq 12: eps * Delta^2 phi                     */
    LBCH_REG_WILLMORE = 2     /* eq 9 / eq 13: eps (Delta - f')(Delta phi - f)        */
};
enum {
    LBCH_Q_DERIVED = 0,       /* Q = kappa (gamma grad phi + |grad phi| P grad_n gamma):
                                 eq 14 with F ~ kappa |grad phi|^2 / 2 (default)      */
    LBCH_Q_LITERAL = 1        /* Q = gamma kappa grad phi + |grad phi| P grad_n gamma:
                                 eq 15 exactly as printed                             */
};

/*
 * Problem statement (Sections 2-3).  Fill with lbch_params_default() and
 * override fields.
 *   nx, ny, nz    grid nodes (>= 1 each); nz = 1 on D2Q9.  Fields are
 *                 row-major [ny][nx] (D2Q9) or [nz][ny][nx] (D3Q15); the
 *                 row-padded population storage must stay below 2^31 entries.
 *   dx, dt        lattice spacing and time step (> 0).
 *   mobility      M of eq 10 (> 0); sets s_3 = s_5 = 1/(M/(c_s^2 dt) + 1/2)
 *                 (relation stated after eq 38), which must lie in (0, 2).
 *   s[9]          relaxation rates of eq 25 for the other moments; s[0] is
 *                 irrelevant (phi is conserved), s[3] and s[5] are ignored.
 *                 The paper does not give them; default 1.  Each in (0, 2).
 *   kappa, beta   gradient and double-well coefficients (eq 1, eq 4), > 0.
 *                 lbch_params_from_sigma_width() sets them from eq 5.
 *   alpha         anisotropy strength of eq 6 (>= 0).
 *   aniso_m       fold of the anisotropy, 1..8 (eq 6 is m = 4): gamma =
 *                 1 + alpha cos(m (theta - theta0)).
 *   aniso_theta0  orientation of the anisotropy (eq 6 is theta0 = 0).
 *   regularization, eps_reg   eq 7-9 and eqs 12/13; eps_reg >= 0.
 *   q_form        LBCH_Q_DERIVED or LBCH_Q_LITERAL (see above).
 *   grad_floor    |grad phi| <= grad_floor  =>  gamma = 1 and no tangential
 *                 term (the normal of eq 2 is undefined); >= 0.
 *
 * D3Q15 (eq 21: velocities 0, the six faces, the eight body diagonals;
 * weights 2/9, 1/9, 1/72).  The same step on a periodic nx x ny x nz box:
 * eq 26 stencils over the 15 velocities, the cubic anisotropy of eq 6 with
 * d = 3, gamma = 1 + alpha (4 sum_a n_a^4 - 3), and the MRT collision on the
 * 15-moment basis obtained by Gram-Schmidt orthogonalisation of 1, |c|^2,
 * |c|^4, c_x, |c|^2 c_x, c_y, |c|^2 c_y, c_z, |c|^2 c_z, 3c_x^2 - |c|^2,
 * c_y^2 - c_z^2, c_x c_y, c_y c_z, c_x c_z, c_x c_y c_z, whose flux rows relax
 * at s_j from the mobility.  The other rates come one per parity class under
 * c -> -c from the D2Q9 slots of the same class: the eight even rows (|c|^2,
 * |c|^4 and the five second-order rows) relax at s_e = s[1], which must equal
 * s[2], s[7] and s[8]; the four odd non-flux rows (|c|^2 c_a, c_x c_y c_z) at
 * s_q = s[4], which must equal s[6] (else LBCH_E_UNSUPPORTED).  The presets
 * of lbch_params_set_collision satisfy this.  s_e = s_q = 1 (the default)
 * runs a collision that reads only phi and the flux of each node; other
 * rates re-read the pulled populations in the collision.  aniso_m must be 4
 * with aniso_theta0 = 0.  One
 * launch per step (time-blocking depth 1); ensembles and the hybrid schedule
 * return LBCH_E_UNSUPPORTED for D3Q15.
 */
typedef struct lbch_params {
    int32_t abi_version;      /* must equal LBCH_ABI_VERSION */
    int32_t lattice;          /* LBCH_D2Q9 or LBCH_D3Q15 */
    int32_t precision;        /* LBCH_FP64 (verification) or LBCH_FP32 (production) */
    int32_t boundary;         /* LBCH_BC_PERIODIC */
    int32_t nx, ny;
    double dx, dt;
    double mobility;
    double s[9];
    double kappa, beta;
    double alpha;
    int32_t aniso_m;
    int32_t regularization;
    double aniso_theta0;
    double eps_reg;
    int32_t q_form;
    int32_t nz;               /* 1 on D2Q9 */
    double grad_floor;
} lbch_params;

typedef struct lbch_sim lbch_sim;   /* opaque; owned by the caller until lbch_destroy */

/* Host-only helpers (no GPU needed). ---------------------------------------- */

/* Paper defaults of eq 39: M = 0.1, eps = 0.03 (Willmore), D = 5, sigma = 0.01
 * (kappa = 0.01875, beta = 0.0015), 100 x 100 grid, alpha = 0, FP64, free
 * rates 1.  NULL -> LBCH_E_INVALID. */
lbch_status lbch_params_default(lbch_params* p);

/* kappa and beta from surface tension sigma and interface width D by
 * inverting eq 5: kappa = 3 sigma D / 8, beta = 3 sigma / (4 D).
 * sigma, D > 0 and finite, else LBCH_E_INVALID (p unchanged). */
lbch_status lbch_params_from_sigma_width(lbch_params* p, double sigma, double width);

/* Checks every field; LBCH_OK, LBCH_E_INVALID or LBCH_E_UNSUPPORTED with the
 * reason in lbch_last_error(). */
lbch_status lbch_params_validate(const lbch_params* p);

/* The nine relaxation rates actually used (s_3 = s_5 from the mobility). */
lbch_status lbch_relaxation_rates(const lbch_params* p, double s_out[9]);

/* Collision variants (Section 3: the paper chooses MRT for its stability and
 * shows no alternative).  All three are rate choices of eq 17 / eq 25 on D2Q9:
 *   LBCH_COLLISION_MRT  the free rates s[1], s[2], s[4], s[6], s[7], s[8] = 1;
 *   LBCH_COLLISION_SRT  every rate = s_j (single relaxation time, BGK);
 *   LBCH_COLLISION_TRT  the moments even under c -> -c (e, eps, p_xx, p_xy:
 *                       s[1], s[2], s[7], s[8]) at s_+, the odd ones (s[4],
 *                       s[6], and the fluxes) at s_j, where magic > 0 is
 *                       Lambda = (1/s_+ - 1/2)(1/s_j - 1/2).
 * s_j comes from the mobility, dx and dt already in p (set them first).
 * magic is read for TRT only.  Unknown model, magic <= 0 or non-finite, or a
 * resulting rate outside (0, 2) -> LBCH_E_INVALID (p unchanged).  On D3Q15
 * the same three presets apply class by class (see the D3Q15 paragraph of
 * lbch_params). */
enum { LBCH_COLLISION_MRT = 0, LBCH_COLLISION_SRT = 1, LBCH_COLLISION_TRT = 2 };
lbch_status lbch_params_set_collision(lbch_params* p, int32_t model, double magic);

/* Library ABI version (LBCH_ABI_VERSION it was built with). */
int32_t lbch_abi_version(void);

/* Thread-local description of the last error ("" if none).  Valid until the
 * next failing call on this thread. */
const char* lbch_last_error(void);

/* Simulation lifecycle. ------------------------------------------------------ */

/* Validates p, allocates two population buffers (9 or 15 planes, structure of
 * arrays, rows padded) plus reduction scratch on the current HIP device and
 * binds the simulation to hip_stream (a hipStream_t; NULL = null stream).
 * *out is set only on success. */
lbch_status lbch_create(const lbch_params* p, void* hip_stream, lbch_sim** out);

/* Frees everything the simulation owns (waits for its stream first). NULL is
 * accepted. */
lbch_status lbch_destroy(lbch_sim* sim);

/* Sets the populations to the equilibrium of eq 18 at the initial order
 * parameter phi0 (host, float64, row-major [ny][nx] or [nz][ny][nx],
 * n = nx*ny*nz entries),
 * with mu_alpha of eq 16 evaluated by the eq 26b stencil and no source term
 * (the paper does not state the initial populations).  Resets the step
 * counter to 0.  Non-finite phi0 -> LBCH_E_INVALID.  Synchronises. */
lbch_status lbch_init(lbch_sim* sim, const double* phi0, int64_t n);

/* Same from device memory: phi0_dev holds nx*ny*nz values of dtype LBCH_FP64
 * or LBCH_FP32, dense row-major.  Stream-ordered, does not synchronise and
 * does not inspect the values (a non-finite input surfaces as
 * LBCH_E_NONFINITE from the next lbch_moments). */
lbch_status lbch_init_device(lbch_sim* sim, const void* phi0_dev, int32_t dtype, int64_t n);

/* Advances nsteps (>= 0) time steps of eq 17: per node phi (eq 22), the
 * eq 26 stencils, the anisotropic chemical potential (eqs 13/15/16), the
 * modified equilibrium (eq 18), the source (eq 19), the MRT collision in
 * moment space (eqs 17, 23, 25) and periodic streaming.  Fused kernel
 * launches enqueued on the simulation's stream, each advancing the time
 * blocking depth of steps (lbch_set_time_blocking: two steps per launch by
 * default on D2Q9 grids above 512^2 nodes, one otherwise; an odd remainder is
 * one single-step launch); returns without waiting.  Before init ->
 * LBCH_E_STATE. */
lbch_status lbch_step(lbch_sim* sim, int64_t nsteps);

/* Two time steps in one two-step launch, storing the populations
 * f_{n+2} + ext (f_{n+2} - f_n) elementwise instead of f_{n+2}: a projective
 * step of the populations (the correction phase of lbch_hybrid_advance uses
 * it with ext = inner_jump / 2) folded into the launch that reads f_n.  The
 * step count advances by 2.  Needs two steps per launch
 * (lbch_set_time_blocking 2) and D2Q9, else LBCH_E_UNSUPPORTED; non-finite
 * ext -> LBCH_E_INVALID; before init -> LBCH_E_STATE.  Stream-ordered. */
lbch_status lbch_step_extrapolated(lbch_sim* sim, double ext);

/* Steps taken since the last init / load. */
lbch_status lbch_get_step(const lbch_sim* sim, int64_t* step);

/* Waits for all work queued on the simulation's stream. */
lbch_status lbch_synchronize(lbch_sim* sim);

/* Reductions (synchronise). -------------------------------------------------- */

/* phi = sum_i f_i (eq 22) of the current state.  phi_out (host, nullable)
 * receives nx*ny*nz float64 values row-major; mass = sum phi dx^d (d = 2 or
 * 3; conserved, eq 34); phi_min / phi_max.  Sums are accumulated in float64 in a fixed
 * order (deterministic).  Any pointer may be NULL.  A non-finite value in
 * the state -> LBCH_E_NONFINITE (outputs still written). */
lbch_status lbch_moments(lbch_sim* sim, double* phi_out, double* mass,
                         double* phi_min, double* phi_max);

/* Discrete free energy of eq 7 at the current phi: sum over nodes of
 * dx^d [gamma (kappa/2 |grad phi|^2 + F(phi)) + eps/2 G(phi)] with the
 * eq 26 stencils, F of eq 4 and G of eq 8 / eq 9.  terms4 (nullable)
 * receives {gradient, bulk, regularisation, total}.  float64 throughout.
 * Non-finite -> LBCH_E_NONFINITE. */
lbch_status lbch_free_energy(lbch_sim* sim, double* energy, double* terms4);

/* Writes phi of the current state to device memory (dtype LBCH_FP64 or
 * LBCH_FP32, nx*ny*nz dense row-major).  Stream-ordered, no synchronisation. */
lbch_status lbch_phi_device(lbch_sim* sim, void* dst_dev, int32_t dtype);

/* Checkpoint / resume. ------------------------------------------------------- */

/* Size in bytes of a saved state: a fixed header (magic, ABI version, grid,
 * precision, step, parameters) followed by the pre-collision populations
 * f_i(x, t) of eq 17 as dense planes [9][ny][nx] (D2Q9) or [15][nz][ny][nx]
 * (D3Q15, directions in the order of eq 21a) in the simulation's precision. */
lbch_status lbch_state_bytes(const lbch_sim* sim, int64_t* bytes);

/* Saves to dst (host memory if dst_is_device == 0, else device memory), which
 * must hold lbch_state_bytes() bytes.  Synchronises. */
lbch_status lbch_save_state(lbch_sim* sim, void* dst, int32_t dst_is_device);

/* Restores a state saved from a simulation with the same grid and precision;
 * the step counter is restored; other parameters are those of sim (so a run
 * can be resumed with changed physics).  Mismatch -> LBCH_E_INVALID.
 * Synchronises. */
lbch_status lbch_load_state(lbch_sim* sim, const void* src, int32_t src_is_device);

/* Launch shape of the fused step kernel. -------------------------------------- */

/* Time steps per kernel launch (temporal blocking): 1, or 2 (each launch
 * reads the populations once, keeps the first step's post-collision rows on
 * chip and writes the state two steps later; lbch_step with an odd count
 * finishes with one single-step launch).  Results are bitwise identical for
 * both depths.  Default 2, and 1 on grids of at most 512^2 nodes, where a
 * launch is latency-bound and the single-step sweep's shorter start-up wins
 * (measured).  Changing the depth restores the default tiling
 * of that depth.  depth not in {1, 2} -> LBCH_E_INVALID; D3Q15 runs depth 1
 * only (2 -> LBCH_E_UNSUPPORTED). */
lbch_status lbch_set_time_blocking(lbch_sim* sim, int32_t depth);
lbch_status lbch_get_time_blocking(const lbch_sim* sim, int32_t* depth);

/* Tiling of the current depth.  block_threads in {64, 128, 256, 512} at
 * depth 1 and {128, 256, 512} at depth 2 (at most 256 in FP64): each
 * workgroup owns a strip of block_threads - 8 * depth columns;
 * rows_per_block >= 1 rows of that strip are swept per workgroup.  The
 * result is bitwise independent of the choice.  0 for either argument
 * restores the built-in default for the grid (for grids with fewer tiles than
 * CUs at the usual chunk, the shortest chunk of at least 4 rows that keeps at
 * most 2.5 tiles per CU).  D3Q15: block_threads is 512
 * (32 x 16 lanes storing 26 x 10 nodes) or, in FP32, 1024 (32 x 32 lanes
 * storing 26 x 26; the FP32 default) or 988 (38 x 26 lanes storing 32 x 20:
 * whole 128-byte rows when nx is a multiple of 32) and rows_per_block is the
 * number of z slabs swept per workgroup. */
lbch_status lbch_set_tiling(lbch_sim* sim, int32_t block_threads, int32_t rows_per_block);
lbch_status lbch_get_tiling(const lbch_sim* sim, int32_t* block_threads, int32_t* rows_per_block);

/* Times the step kernel over depth in {1, 2} x block_threads x
 * rows_per_block in {the launch model's own height (the default tiling),
 * 8, ..., 512} (steps_per_trial launches each, reading
 * the current state and writing the idle buffer, so the state and the step
 * counter are unchanged), keeps the fastest per step (depth and tiling),
 * times it once more (steps_per_trial launches) and returns its tiling
 * (rows_per_block: the height in use) and that time per step.  Synchronises.  Before init ->
 * LBCH_E_STATE.  D3Q15: every tile shape of lbch_set_tiling x z-sweep lengths
 * {model default, 4, 8, ..., 128} (at most nz). */
lbch_status lbch_autotune(lbch_sim* sim, int32_t steps_per_trial, int32_t* block_threads,
                          int32_t* rows_per_block, double* ms_per_step);

/* How the step kernel reads a row of populations: 0 = automatic (FP32 grids
 * with nx % 4 == 0 fetch aligned 16-byte chunks into LDS and read the pulled
 * values from there; otherwise one load per population and lane), 1 = always
 * the per-lane loads.  Results are bitwise identical either way. */
lbch_status lbch_set_row_loader(lbch_sim* sim, int32_t mode);

#ifdef __cplusplus
}
#endif

#endif /* LBCH_H */
