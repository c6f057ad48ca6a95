/*
 * swept.h -- C interface of libswept.so: swept and classic time-space
 * decompositions of explicit 1D stencil time-stepping on an AMD MI355X (gfx950).
 *
 * The problem statement follows the paper (Magee & Niemeyer, "Accelerating
 * solutions of one-dimensional unsteady PDEs with GPU-based swept time-space
 * decomposition"): a scheme, a grid of n points, dt and dx, a number of
 * timesteps and a boundary type (Sec. 4.1 experimental method, Sec. 5.2 test
 * cases, Appendices B-D).  Schemes:
 *   SW_HEAT   heat equation, forward-time central-space     (Appendix B, Eq. Heatdisc)
 *   SW_KS     Kuramoto-Sivashinsky, 5-point central + RK2   (Appendix C, Eqs. KSDisc, RKm, RKf)
 *   SW_EULER  1D Euler, 2nd-order finite volume, limiter, Roe-averaged spectral-radius flux, RK2
 *             (Appendix D)
 *
 * Every solve computes, in IEEE binary64, exactly the classic level-by-level
 * result: the swept rule performs the same operations in a different order and
 * place (Sec. 2).  Each product that the canonical update rules fuse into a sum
 * is one correctly rounded fused multiply-add; nothing else is contracted.
 * swept_solve and classic_solve return bit-identical states for the same plan
 * and input.
 *
 * Conventions
 *  - State layout: caller-owned DEVICE memory, float64, structure of arrays
 *    [nvars][n] (nvars = 1 for heat/KS, 3 = (rho, rho*u, E) for Euler), contiguous.
 *    On entry it holds the initial condition; on completion the state after
 *    nsteps timesteps.  The update is in place.  Host pointers are rejected.
 *  - Asynchrony: solves are enqueued on `hip_stream` (a hipStream_t, or NULL for
 *    the default stream) and return before the work finishes; the caller keeps
 *    the state buffer alive until the stream has drained.
 *  - Ownership: a plan owns its scratch memory (edge buffers, ping-pong buffer)
 *    and its cached HIP graphs; one solve at a time per plan.
 *  - Errors: every entry point returns SW_OK (0) or a negative SW_E* code, never
 *    aborts or throws, and writes out-parameters only on success.  A
 *    human-readable detail of the last failure on the calling thread is
 *    available from sw_last_error().
 */
#ifndef SWEPT_H
#define SWEPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define SW_OK            0
#define SW_EINVAL       -1   /* bad argument (also: host pointer given as state) */
#define SW_ENOMEM       -2   /* device or host allocation failed */
#define SW_EDEVICE      -3   /* HIP runtime error; detail in sw_last_error() */
#define SW_EUNSUPPORTED -4   /* swept decomposition impossible for this n (no legal tile width divides n) */
#define SW_EBUSY        -5   /* plan already in use / batch memory budget or slots exhausted */
#define SW_ENOTREADY    -6   /* ticket still running */
#define SW_ENAN         -7   /* optional post-solve check found a non-finite value */

/* ---- problem description ---------------------------------------------- */
#define SW_HEAT   0
#define SW_KS     1
#define SW_EULER  2

#define SW_PERIODIC   0      /* stencil wraps around the ends (Appendix C) */
#define SW_DIRICHLET  1      /* r ghost points per end held at bc_left / bc_right at every level */
#define SW_REFLECTIVE 2      /* insulated ends, heat only (Appendix B, Eq. heatcond):
                                T_{-1} = T_1, T_n = T_{n-2} for points 0..n-1 */

/* sw_problem.flags */
#define SW_PROBLEM_LIMITER_RECIPROCAL 1u  /* Euler: take the limiter ratio backward/forward
                                             instead of the orientation printed in Eqs.
                                             limitleft/limitright */

typedef struct {
    int32_t scheme;        /* SW_HEAT, SW_KS or SW_EULER */
    int32_t bc;            /* SW_PERIODIC, SW_DIRICHLET or SW_REFLECTIVE */
    int64_t n;             /* grid points (heat, KS) or cells (Euler), >= 1 */
    int64_t nsteps;        /* full timesteps, >= 0 (0 = no-op) */
    double  dt, dx;        /* > 0 */
    double  alpha;         /* heat diffusivity: Fo = (alpha*dt)/(dx*dx) */
    double  gamma;         /* Euler heat-capacity ratio (> 1) */
    double  bc_left[3];    /* Dirichlet ghost values, per variable (Euler: conserved) */
    double  bc_right[3];
    uint32_t flags;        /* SW_PROBLEM_* */
    uint32_t reserved;     /* must be 0 */
} sw_problem;

/* Tile shape.  threads = work-group size (a multiple of 64, at most 1024; at
 * most 512 with 8 or more points per lane, Euler: 512, and 256 with 8 points per
 * lane); width = points per swept tile = points_per_lane * threads, with
 * points_per_lane in {1, 2, 4, 8, 16} and at least the stencil radius (Euler:
 * at most 8).  classic_threads = work-group size of the classic kernel (one
 * point per lane; a multiple of 64 in [64, 1024]); the paper takes the best time
 * over block sizes (Sec. 4.1, experimental method), and the tuning table holds
 * the measured best per scheme and size class.  Zeros ask for the tuned or
 * default choice (classic default 256). */
#define SW_TUNE_NO_GRAPH  1   /* enqueue kernels one by one instead of replaying a HIP graph */
#define SW_TUNE_CHECK_NAN 2   /* after a solve, synchronise and report SW_ENAN on non-finite output */
#define SW_TUNE_HYBRID    4   /* Hybrid variant (Sec. 5.1): for Dirichlet and reflective problems,
                                 the host CPU computes the tile that straddles the domain boundary
                                 in every shifted phase while the GPU computes the others; its two
                                 edge slots travel through pinned host memory.  Bit-identical
                                 results; phases are enqueued one by one (no graph), and a solve
                                 first waits on the host for the plan's previous solve.  No
                                 effect for periodic problems. */
#define SW_TUNE_LDS       8   /* Shared variant (Sec. 5.1): each tile's two-row working array lives
                                 in LDS and the work-group's threads stride over every level's
                                 points, one barrier per level, instead of the register kernel.
                                 The width may be any multiple of 4 r up to 64 points per thread
                                 whose rows, 2 nvars (width + 2 r) doubles, fit in 160 KB of LDS
                                 (heat and KS: width <= 10,236; Euler: <= 3,408); otherwise
                                 SW_EINVAL.  Bit-identical results.  Not with SW_TUNE_HYBRID or
                                 swept_solve_noalloc. */
typedef struct {
    int32_t width;
    int32_t threads;
    int32_t flags;           /* SW_TUNE_* */
    int32_t classic_threads;
} sw_tuning;

typedef struct {
    int32_t width;            /* w: points per tile */
    int32_t threads;          /* work-group size */
    int32_t points_per_lane;  /* w / threads */
    int32_t radius;           /* r: stencil radius per sub-step (1 heat, 2 KS/Euler) */
    int32_t substeps;         /* S: sub-steps per timestep (1 heat, 2 KS/Euler) */
    int32_t nvars;            /* variables per point */
    int32_t swept_ok;         /* 1 if swept_solve can run (width divides n) */
    int32_t classic_threads;  /* work-group size of the classic kernel */
    int64_t nodes;            /* K = n / w tiles per phase */
    int64_t levels;           /* S * nsteps sub-step levels */
    int64_t levels_per_phase; /* H = w / (2 r) */
    int64_t full_phases;      /* Q = levels / H */
    int64_t remainder;        /* levels - Q*H, done by one extra Up/Down pair */
    int64_t swept_launches;   /* kernels per swept solve */
    int64_t classic_launches; /* kernels per classic solve (one per sub-step) */
    int64_t scratch_bytes;    /* device scratch owned by the plan */
} sw_plan_info;

typedef struct sw_plan sw_plan;

/* Validate a problem and build a plan: derive r, S, nvars and the canonical
 * constants, pick the tile shape (tuning may be NULL), allocate scratch on the
 * current device.  SW_EINVAL for an invalid problem or tile shape. */
int swept_plan(const sw_problem *problem, const sw_tuning *tuning, sw_plan **out);

/* Geometry and launch counts of a plan. */
int swept_plan_info(const sw_plan *plan, sw_plan_info *out);

/* Swept decomposition (Sec. 4.2-4.3): an Up-triangle launch, alternating-offset
 * Diamond launches, a Down-triangle launch, plus one Up/Down pair for a
 * remainder of fewer levels than a phase.  Each tile advances w/(2r) levels per
 * launch in on-chip memory and exchanges only its edges through HBM.
 * SW_EUNSUPPORTED if no legal width divides n (classic_solve still works). */
int swept_solve(sw_plan *plan, double *d_state, void *hip_stream);

/* Classic decomposition (Sec. 5.1, the Classic listing): one kernel launch per
 * sub-timestep, ping-ponging through global memory. */
int classic_solve(sw_plan *plan, double *d_state, void *hip_stream);

/* Free a plan (waits for its in-flight work first).  NULL is a no-op. */
void swept_plan_destroy(sw_plan *plan);

/* Measurement hook: enqueue `reps` launches of one swept phase kind on
 * `hip_stream` between two HIP events and return their mean duration in
 * microseconds (synchronous).  kind: 0 = Up triangle, 1 = Diamond (offsets
 * alternate as in a solve), 2 = Down triangle, each over all K tiles with the
 * full H levels.  The launches reuse the plan's edge buffer; afterwards the
 * contents of d_state and of the edges are unspecified (run it on a scratch
 * state).  SW_EUNSUPPORTED if the plan cannot run swept. */
int swept_profile_phase(sw_plan *plan, double *d_state, int32_t kind, int32_t reps,
                        void *hip_stream, double *avg_us);

/* ---- allocation-free solve --------------------------------------------- */
/* For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The same swept solve as
 * swept_solve on a plan of this problem and tile shape (bit-identical results),
 * but its edge slots live in a static device array of SW_NOALLOC_SCRATCH_BYTES
 * that the library holds on every device it runs on until the process ends, and
 * its phases are enqueued one by one on hip_stream (no graph is built).  The call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine (the
 * first call on a device only resolves that device's copy of the array).
 *  - problem, tuning: as for swept_plan (tuning may be NULL; its only accepted
 *    flag is SW_TUNE_NO_GRAPH).  d_state: caller-owned device state, as for
 *    swept_solve.  Asynchronous on hip_stream.
 *  - The edge scratch needs nvars * (2 n + 4 K r) doubles (K = n / width); a
 *    problem needing more than SW_NOALLOC_SCRATCH_BYTES is rejected with
 *    SW_EINVAL before anything is enqueued (32 MiB: heat and KS up to n = 2^20,
 *    Euler up to n = 2^19).  SW_EUNSUPPORTED if no legal width divides n.
 *  - Every call on one device shares that device's array and leaves its last
 *    contents behind (nothing in it has to start at zero: each solve's first
 *    phase writes every slot before any is read).  Calls that overlap on one
 *    device -- on different streams, or from different threads -- race on it and
 *    must be serialised by the caller. */
#define SW_NOALLOC_SCRATCH_BYTES (32ll << 20)
int swept_solve_noalloc(const sw_problem *problem, const sw_tuning *tuning, double *d_state,
                        void *hip_stream);

/* ---- batched / served solves ------------------------------------------- */
/* Many independent solves share launches.  The paper runs one solve at a time;
 * batching many solves of uneven n into shared phase launches, and serving
 * them continuously, are this library's additions around its swept phases.
 * Each solve keeps the exact results of swept_solve on the same problem. */
#define SW_BATCH_SERVE      1     /* a worker thread admits and advances solves continuously */
#define SW_BATCH_PERSISTENT 2     /* ensemble: one persistent launch per tile group in which work-groups
                                     take tiles from a device queue and wait on device-side completion
                                     counters of the tiles they depend on, instead of one launch per
                                     phase index (Sec. 7 suggests GPU-side synchronisation) */
typedef struct {
    int64_t budget_bytes;     /* device bytes the batch may hold for resident solves: each is charged
                                 its state plus its edge slots rounded up to 256 bytes (swept), or
                                 twice its state (classic fallback); batch_ticket_info reports it */
    int32_t max_slots;        /* maximum resident solves (0 = unlimited) */
    int32_t flags;            /* SW_BATCH_SERVE or SW_BATCH_PERSISTENT (ensemble), or 0 */
    int32_t points_per_lane;  /* batched tiles are one wave wide; points per lane (1, 2, 4 or 8, at
                                 most what divides n / 64) or 0 for the tuned choice per size class */
    int32_t reserved;         /* must be 0 */
} sw_batch_config;

typedef struct {
    int32_t status;           /* SW_TICKET_* */
    int32_t swept;            /* 1: swept phases in shared launches; 0: classic fallback */
    int32_t width;            /* tile width used (swept) */
    int32_t phases;           /* swept phases of the solve */
    double  submit_s, start_s, end_s;  /* host steady-clock seconds: submitted, admitted, finished */
    int64_t resident_bytes;   /* device bytes charged against the batch budget while resident */
} sw_ticket_info;

typedef struct sw_batch sw_batch;

/* Ticket status values reported by batch_poll. */
#define SW_TICKET_QUEUED   0
#define SW_TICKET_RUNNING  1
#define SW_TICKET_DONE     2
#define SW_TICKET_FAILED   3
#define SW_TICKET_CANCELLED 4

/* Create a batch on the current device.  With SW_BATCH_SERVE a worker thread
 * starts at once. */
int  batch_create(const sw_batch_config *config, sw_batch **out);
/* Queue one solve on caller-owned device state (layout as above; the caller keeps
 * it alive and untouched until the ticket is done).  The initial state must already
 * be complete on the device when batch_submit is called (the batch runs on streams
 * of its own: synchronise the stream that wrote the state first, or use
 * batch_submit_async).  SW_EBUSY if the solve alone exceeds the budget.
 * Thread-safe. */
int  batch_submit(sw_batch *batch, const sw_problem *problem, double *d_state, uint64_t *ticket);
/* As batch_submit, but the state may still be being written by work queued on
 * hip_stream: the library records an event on that stream now, and the solve's
 * first launch waits for it. */
int  batch_submit_async(sw_batch *batch, const sw_problem *problem, double *d_state, void *hip_stream,
                        uint64_t *ticket);
/* Ensemble mode: run every queued solve to completion, then return
 * (synchronous).  Solves are admitted in submission order in waves that fit the
 * budget and slot limit; each wave runs as one HIP graph launch holding one
 * batched launch per phase index and tile-width group, each group's chain of
 * launches on a parallel branch of the graph. */
int  batch_run(sw_batch *batch, void *hip_stream);
int  batch_poll(sw_batch *batch, uint64_t ticket, int32_t *status_out);
/* Block until the ticket is done, cancelled or failed, or timeout_us passes
 * (negative: no limit).  SW_ENOTREADY on timeout. */
int  batch_wait(sw_batch *batch, uint64_t ticket, int64_t timeout_us);
/* Cancel a ticket that has not started (SW_EBUSY once it runs). */
int  batch_cancel(sw_batch *batch, uint64_t ticket);
/* Status and timing of one ticket. */
int  batch_ticket_info(sw_batch *batch, uint64_t ticket, sw_ticket_info *out);
/* Stop the worker (served mode; queued tickets are cancelled, running ones
 * finish), free the batch's device memory. */
void batch_destroy(sw_batch *batch);

/* ---- diagnostics ------------------------------------------------------- */
const char *sw_strerror(int status);
const char *sw_last_error(void);   /* thread-local detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* SWEPT_H */
