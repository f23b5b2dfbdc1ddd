/* Batched Crank-Nicolson steps: many independent problems (2D and 3D, any
 * supported sizes, PCG or PGMRES, float64 or mixed precision) advanced
 * together on one GPU.
 *
 * Each problem is a full fsd_problem (fsd.h) bound to its own slice of one
 * caller-owned workspace.  The batch owns a native executor: `lanes`
 * host worker threads, each with its own HIP stream (caller-provided), so
 * that the device-resident Krylov loops of different problems overlap on
 * the GPU instead of running one after the other.  Problems are assigned
 * to lanes by longest-processing-time-first on a cost estimate
 * (unknowns x line length x log2 line length x expected iterations), and
 * each lane runs its problems in that order every step.  The iteration
 * counts of a step feed the estimate of the next one.
 *
 * fsd_batch_autotune tunes the engine (tile shape) of every pass of every
 * problem (fsd_autotune), then times one step for each lane count 1, 2, 4,
 * ... up to the number of streams, with direct kernel launches and with
 * launch graphs of the Krylov iteration chunks (fsd_set_graphs), and keeps
 * the fastest combination.
 *
 * Results are bitwise those of calling fsd_cn_step on each problem alone:
 * the executor changes only which stream and thread run a problem.
 *
 * Errors: FSD_EINVAL (bad arguments, any invalid parameter set: the index
 * is in fsd_last_error()), FSD_ESMALLWS, FSD_ENOTBOUND, FSD_EHIP; a failed
 * or non-converged solve reports its status in its fsd_stats entry and
 * the call returns the first non-OK status in problem order. */
#ifndef FSD_BATCH_H
#define FSD_BATCH_H

#include "fsd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsd_batch_s* fsd_batch;

/* Validate and plan `count` problems (host only). */
fsd_status fsd_batch_create(const fsd_params* params, int count, fsd_batch* out);
void fsd_batch_destroy(fsd_batch batch);

/* Total workspace (the per-problem workspaces, each 256-byte aligned), and
 * problem i's offset inside it. */
size_t fsd_batch_workspace_bytes(fsd_batch batch);
size_t fsd_batch_offset(fsd_batch batch, int i);

/* Bind the workspace and `nstreams` >= 1 HIP streams (hipStream_t passed as
 * void*); the executor uses min(nstreams, count) lanes until
 * fsd_batch_autotune or fsd_batch_set_lanes changes it. */
fsd_status fsd_batch_bind(fsd_batch batch, void* d_ws, size_t bytes, void* const* streams,
                          int nstreams);

fsd_status fsd_batch_set_lanes(fsd_batch batch, int lanes);
int fsd_batch_lanes(fsd_batch batch);

/* Launch graphs for every problem of the batch (fsd_set_graphs), and the
 * current setting. */
fsd_status fsd_batch_set_graphs(fsd_batch batch, int on);
int fsd_batch_graphs(fsd_batch batch);

/* One CN step of every problem: d_u_prev[i], d_F[i] (may be NULL: f = 0),
 * d_guess[i] (read in EXTERNAL / GUARDED mode; the array itself may be
 * NULL otherwise), d_u_next[i]; stats: `count` entries or NULL.  Returns
 * after every lane has enqueued its problems' work and finished their
 * host-side convergence checks; the streams are synchronised. */
fsd_status fsd_batch_cn_step(fsd_batch batch, const double* const* d_u_prev,
                             const double* const* d_F, const double* const* d_guess,
                             double* const* d_u_next, fsd_stats* stats);

/* Tune the engines of every problem's passes (fsd_autotune), then try lane
 * counts 1, 2, 4, ... <= nstreams, first with direct launches and
 * then with launch graphs, with one CN step each (outputs to d_u_next,
 * inputs unchanged; the time history of FSD_X0_EXTRAP is reset afterwards)
 * and keep the fastest combination (fsd_batch_lanes, fsd_batch_graphs).
 * ms_out (optional, >= 2 (log2(nstreams) + 1) entries) receives the step
 * time of each candidate, direct launches first; returns the chosen lane
 * count or a negative status. */
int fsd_batch_autotune(fsd_batch batch, const double* const* d_u_prev, const double* const* d_F,
                       double* const* d_u_next, double* ms_out);

/* Problem i's handle (owned by the batch), e.g. for fsd_get_coefficients. */
fsd_problem fsd_batch_problem(fsd_batch batch, int i);

#ifdef __cplusplus
}
#endif

#endif
