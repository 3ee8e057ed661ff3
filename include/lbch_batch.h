/*
 * lbch_batch.h — ensembles of independent simulations advanced together.
 *
 * A batch holds `count` periodic D2Q9 grids of the anisotropic Cahn-Hilliard
 * lattice Boltzmann scheme (each member with its own grid size and its own
 * physical parameters of Sections 2-3, all in one precision) and advances all
 * of them with ONE persistent kernel launch per time step, or per two time
 * steps (the default, as lbch_set_time_blocking); chunks of launches are
 * replayed from a captured HIP graph when the batch has its own stream.  The
 * update applied to every member is exactly the lbch_step update (include
 * /lbch.h): a member's result is bitwise identical to a standalone simulation
 * with the same parameters and initial field.
 *
 * Conventions (status codes, ownership, streams, errors) are those of lbch.h.
 * `member` arguments index 0 .. count-1; out of range -> LBCH_E_INVALID.
 */
#ifndef LBCH_BATCH_H
#define LBCH_BATCH_H

#include <stdint.h>

#include "lbch.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbch_batch lbch_batch;   /* opaque; owned by the caller until lbch_batch_destroy */

/* members[count] (count >= 1) are validated as by lbch_params_validate and
 * must share `precision`.  Allocates one pair of population buffers for all
 * members plus reduction scratch.  hip_stream NULL = null stream (then no
 * graph capture). */
lbch_status lbch_batch_create(const lbch_params* members, int32_t count, void* hip_stream, lbch_batch** out);
lbch_status lbch_batch_destroy(lbch_batch* batch);

/* Initial field of one member (host float64 row-major [ny][nx], n = nx*ny),
 * as lbch_init: equilibrium of eq 18, step counter reset for the batch when
 * every member has been initialised.  Non-finite -> LBCH_E_INVALID. */
lbch_status lbch_batch_init(lbch_batch* batch, int32_t member, const double* phi0, int64_t n);

/* Same from device memory (LBCH_FP64 / LBCH_FP32 values), stream-ordered. */
lbch_status lbch_batch_init_device(lbch_batch* batch, int32_t member, const void* phi0_dev, int32_t dtype,
                                   int64_t n);

/* Advances every member nsteps time steps (one launch per step over all
 * members' tiles).  Before every member is initialised -> LBCH_E_STATE. */
lbch_status lbch_batch_step(lbch_batch* batch, int64_t nsteps);

lbch_status lbch_batch_get_step(const lbch_batch* batch, int64_t* step);
lbch_status lbch_batch_synchronize(lbch_batch* batch);

/* Per-member reductions, as lbch_moments / lbch_free_energy / lbch_phi_device. */
lbch_status lbch_batch_moments(lbch_batch* batch, int32_t member, double* phi_out, double* mass,
                               double* phi_min, double* phi_max);
lbch_status lbch_batch_free_energy(lbch_batch* batch, int32_t member, double* energy, double* terms4);
lbch_status lbch_batch_phi_device(lbch_batch* batch, int32_t member, void* dst_dev, int32_t dtype);

/* Time steps per launch, 1 or 2 (default 2, and 1 for ensembles of at most
 * 512^2 nodes in all, as for one simulation; an odd remainder of
 * lbch_batch_step runs one single-step launch).  Bitwise identical results.
 * depth not in {1, 2} -> LBCH_E_INVALID. */
lbch_status lbch_batch_set_time_blocking(lbch_batch* batch, int32_t depth);
lbch_status lbch_batch_get_time_blocking(const lbch_batch* batch, int32_t* depth);

/* Launch shape of the current depth: block_threads in {64, 128, 256, 512}
 * ({128, 256, 512} at depth 2, at most 256 in FP64) for every member,
 * rows_per_block >= 1 rows per tile (0 = default: 64 at depth 2, 32 at
 * depth 1, or for ensembles with fewer tiles than CUs the shortest chunk of
 * at least 4 rows that keeps at most 2.5 tiles per CU), persistent_blocks
 * workgroups in the persistent grid (0 = fill every CU).  Bitwise
 * independent of the choice.  lbch_batch_get_tiling reports the chunk
 * height in use. */
lbch_status lbch_batch_set_tiling(lbch_batch* batch, int32_t block_threads, int32_t rows_per_block,
                                  int32_t persistent_blocks);
lbch_status lbch_batch_get_tiling(const lbch_batch* batch, int32_t* block_threads, int32_t* rows_per_block,
                                  int32_t* persistent_blocks, int32_t* total_tiles);

/* Times launch shapes (depth x block_threads x rows_per_block, the heights
 * being the default rule's own and 16 .. 128) for this batch with
 * steps_per_trial launches each (writing the idle buffer: the state and step
 * counter are unchanged), keeps the fastest per step (and the fastest
 * single-step shape for odd remainders); rows_per_block returns the height in
 * use.  Synchronises. */
lbch_status lbch_batch_autotune(lbch_batch* batch, int32_t steps_per_trial, int32_t* block_threads,
                                int32_t* rows_per_block, double* ms_per_step);

/* Total lattice nodes over all members (for throughput accounting). */
lbch_status lbch_batch_nodes(const lbch_batch* batch, int64_t* nodes);

#ifdef __cplusplus
}
#endif

#endif /* LBCH_BATCH_H */
