// The engine's batched mode, used by the serving loop (serve.cpp): a
// handle whose device memory comes from a caller's arena, whose pinned
// scalars and stream are the server's, and whose P-LBFGS iteration advances
// as a state machine, one evaluation per round of segmented launches.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/scvt.h"

namespace scvt {

struct Round;

// Bytes of pinned host memory a batched handle uses for its scalars.
constexpr size_t kBatchPinnedBytes = 64 * sizeof(double);

// Create a handle for cfg (P-LBFGS with at most 16 pairs) in the device
// memory [arena, arena + arena_bytes) (at least scvt_footprint bytes) with
// the pinned scalars `pinned` (kBatchPinnedBytes) on stream `stream`.  The
// generators z0 (host, n x 3) are copied in and the set-up kernels issued;
// the first evaluation happens in the handle's first round.  Nothing is
// allocated.  Errors: SCVT_E_INVALID (configuration not served in batches),
// SCVT_E_OOM (arena too small), SCVT_E_HIP.
int batch_create(const scvt_config* cfg, const double* z0, void* arena, size_t arena_bytes,
                 double* pinned, void* stream, int64_t max_iter, double tol, scvt_handle** out);

// Record the handle's launches of the next round into r (r also receives
// the launches of a history push that batch_finish left for it).
int batch_plan(scvt_handle* h, Round& r);

// After the round ran: take its scalars and advance the state machine;
// launches of the next step that must precede everything else in the next
// round (the history push) go into `next`.  Returns SCVT_PENDING while the
// solve goes on, else its final status (SCVT_OK converged, SCVT_NOT_CONVERGED
// at max_iter, or an error).
int batch_finish(scvt_handle* h, Round& next);

// The handle's record (as scvt_solve fills it) with the given status.
void batch_info(scvt_handle* h, scvt_info* info, int status);

// Release a batched handle (its arena and pinned memory stay the caller's).
void batch_destroy(scvt_handle* h);

}  // namespace scvt
