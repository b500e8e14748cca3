/*
 * ctserve.h -- C ABI of the projector serving engine (continuous batching on one device).
 *
 * A server accepts forward (A x) and back projection (A^T y) requests for any number of plans
 * (ctproj.h) as they arrive, and runs them on one device while others are still running:
 *
 *   - Memory.  The caller hands the server one device arena (its HBM budget).  Every admitted
 *     call takes from it the outputs of its requests (one block, placed from the bottom of the
 *     arena) and its scratch -- the workspace of the call (ctp_workspace_bytes) and, when
 *     several requests are merged, a staging copy of their inputs (one block, placed from the
 *     top, freed when the call completes).  A request is admitted only when those blocks fit;
 *     until then it waits in the queue.  Outputs stay resident in the arena until released, so
 *     a client that holds results can keep later requests waiting (a wait then times out).
 *   - Order.  When a slot is free the server picks the head of the next call: requests that
 *     have waited at least age_cap_us come first, oldest first; the others follow in order of
 *     their work (voxel-view updates: n_vox x n_views of the plan), smallest first, so short
 *     requests are not held behind long ones.  A head whose call does not fit in the arena is
 *     passed over in favour of the next one unless it has reached the age cap, in which case
 *     nothing else starts until it fits.  age_cap_us = 0 gives strict first come, first served.
 *   - Batching.  The head is admitted together with the other queued requests that share its
 *     plan, direction and storage types (at most max_batch, in arrival order; the paper's
 *     batched, channelled tensors, Section 1 and 2.4: one plan serves the whole batch).  If the
 *     merged call does not fit, fewer requests are merged.
 *   - Overlap.  Each slot owns a HIP stream; up to n_slots calls run concurrently.  Optionally
 *     the last slot is an express lane for short requests (express_work below): it never takes
 *     a long call, and the other slots still take short ones.  A kernel launch keeps the
 *     compute units it holds until its work-groups drain, and while two long launches run the
 *     units that one frees go to the other first; so with an express lane long calls run one
 *     at a time, and launch_work splits each call into short launches between which the other
 *     streams' kernels start.
 *
 * Results are those of ctp_project / ctp_backproject with batch = the merged count.  Every
 * batch item's result is bitwise independent of the other items of its call (the forward
 * projector's fixed-point scale is chosen per item, the back projector is a per-voxel gather),
 * so a request gets the same bits alone and in the mix.
 *
 * The server runs one host thread of its own.  While calls are in flight it looks at their
 * completion events every 50 us (a timed sleep that a submission, release or cancellation ends
 * early); when the server is idle it sleeps until the next submission.
 * All functions return a ctp_status; ctp_last_error() holds the detail.
 */
#ifndef CTSERVE_H
#define CTSERVE_H

#include "ctproj.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ctp_server ctp_server;   /* opaque */

typedef struct {
    void *arena;          /* device memory on the current device, 256-byte aligned, owned by the
                             caller and unused by it while the server lives */
    size_t arena_bytes;   /* the HBM budget */
    int32_t n_slots;      /* concurrent calls (streams), 1..16 */
    int32_t max_batch;    /* most requests merged into one call, 1..1024 */
    int64_t age_cap_us;   /* wait after which a request is served in arrival order (>= 0;
                             0 = strict first come, first served) */
    double express_work;  /* with n_slots >= 2 and express_work > 0, the last slot runs only
                             calls whose requests' work (voxel-view updates) is at most this,
                             and merges at most express_work of it into one call, so short
                             requests never wait behind a device full of long calls; calls of
                             longer requests then run one at a time;
                             0 = every slot takes every call */
    double launch_work;   /* > 0: a call is split into kernel launches over consecutive view
                             ranges of at most this many voxel-view updates each (at least one
                             view), so that other slots' work starts between them; the result
                             has the same bits.  0 = one launch per call */
} ctp_server_config;

/* Host-clock times (steady clock, ns) and placement of one request. */
typedef struct {
    int64_t submit_ns;    /* ctp_server_submit returned */
    int64_t admit_ns;     /* its call was launched */
    int64_t done_ns;      /* the server saw its call complete */
    int32_t batch;        /* requests in its call */
    int32_t slot;         /* stream slot of its call */
} ctp_request_info;

typedef struct {
    int64_t submitted, completed, failed, calls;
    int64_t cancelled;    /* requests removed from the queue by ctp_server_cancel */
    int32_t max_running;  /* most calls in flight at once */
    int32_t max_batch_seen;
    size_t arena_peak;    /* most arena bytes in use at once */
} ctp_server_stats;

/* Start a server on the current device.  Errors: CTP_EINVAL (NULL config or arena, sizes out of
 * range, misaligned arena), CTP_EDEVICE (stream / event creation), CTP_ENOMEM. */
ctp_status ctp_server_create(const ctp_server_config *cfg, ctp_server **out);

/* Queue one request: out = A in (dir = CTP_FORWARD, in is one volume) or out = A^T in
 * (CTP_BACKWARD, in is one sinogram), layouts as in ctproj.h, batch 1.  `input` is device memory
 * that must stay valid and unchanged until the request completes; `ready` is the stream whose
 * work so far produces it (the server's call waits for it; 0 = the null stream).  The plan must
 * outlive the request and belong to the server's device.  Returns at once with a ticket (> 0).
 * Errors: CTP_EINVAL (NULL arguments, unknown direction or dtype, plan of another device),
 * CTP_ENOMEM (the request alone can never fit in the arena), CTP_EDEVICE. */
ctp_status ctp_server_submit(ctp_server *srv, const ctp_plan *plan, ctp_direction dir,
                             const void *input, ctp_dtype in_dtype, ctp_dtype out_dtype,
                             hipStream_t ready, uint64_t *ticket);

/* Wait until the request is done (timeout_us < 0: no limit).  On success *result (if not NULL)
 * is the device address of its output inside the arena, complete and valid until released.
 * Errors: CTP_EINVAL (unknown or released ticket), CTP_ETIMEOUT (not done within timeout_us;
 * the request goes on), CTP_ECANCELED (cancelled), or the status of its failed call
 * (CTP_EINVAL / CTP_EDEVICE, with the call's message). */
ctp_status ctp_server_wait(ctp_server *srv, uint64_t ticket, int64_t timeout_us, void **result);

/* Non-blocking: *done = 1 and *result set when complete, else *done = 0. */
ctp_status ctp_server_query(ctp_server *srv, uint64_t ticket, int *done, void **result);

/* Times and placement of a request (valid until it is released). */
ctp_status ctp_server_info(ctp_server *srv, uint64_t ticket, ctp_request_info *info);

/* Remove a queued request (one whose call has not been admitted).  Its wait and query then
 * report CTP_ECANCELED, and the ticket must still be released.  Errors: CTP_EINVAL for an
 * unknown or released ticket and for a request that is already running or finished. */
ctp_status ctp_server_cancel(ctp_server *srv, uint64_t ticket);

/* Give the request's output back to the arena.  `consumer` is the stream on which the caller's
 * last use of the output was enqueued: the memory is reused only after that work has run.
 * A queued or running request cannot be released (CTP_EINVAL); the ticket is forgotten. */
ctp_status ctp_server_release(ctp_server *srv, uint64_t ticket, hipStream_t consumer);

ctp_status ctp_server_get_stats(ctp_server *srv, ctp_server_stats *stats);

/* Wait for every queued and running request, then stop the thread and free the streams and
 * events.  The arena is not freed (it is the caller's).  NULL is accepted. */
ctp_status ctp_server_destroy(ctp_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* CTSERVE_H */
