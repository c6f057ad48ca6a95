// C interface of libswept.so (declared in include/swept.h): plans, swept and
// classic solves, error reporting.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "api_internal.hpp"
#include "kernels.hpp"
#include "plan_core.hpp"
#include "tune.hpp"
#include "swept.h"

using namespace sw;

namespace sw {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return SW_EDEVICE;
}

int check_device_ptr(const void *p)
{
    if (!p) return fail(SW_EINVAL, "state pointer is NULL");
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SW_EINVAL, "state pointer is not device memory");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(SW_EINVAL, "state pointer is not device memory");
    return SW_OK;
}

}  // namespace sw

#define HIP_TRY(expr)                                        \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return sw::hip_fail(_e, #expr); \
    } while (0)

namespace {

constexpr size_t kMaxGraphPhases = 4096;   // larger launch lists are replayed in chunks
constexpr int64_t kDiamondChunk = 2048;    // diamonds per replayed chunk (even: offsets 1,0,...)
constexpr int64_t kClassicChunkSteps = 256;  // timesteps per replayed classic chunk (even)

bool uses_hybrid(const sw_plan *p)
{
    return (p->tflags & SW_TUNE_HYBRID) && p->geom.swept_ok && p->geom.bc != SW_PERIODIC;
}

// Pinned doubles for the straddling tile: its two slots and one top level.
size_t hybrid_doubles(const Geom &g) { return (size_t)g.nv * (2 * 2 * (size_t)g.E + (size_t)g.w); }

void release_hybrid(sw_plan *p)
{
    if (p->hyb_done) (void)hipEventDestroy(p->hyb_done);
    if (p->hyb_ready) (void)hipEventDestroy(p->hyb_ready);
    if (p->hyb_stream) (void)hipStreamDestroy(p->hyb_stream);
    if (p->h_hybrid) (void)hipHostFree(p->h_hybrid);
    p->hyb_done = p->hyb_ready = nullptr;
    p->hyb_stream = nullptr;
    p->h_hybrid = nullptr;
    p->hyb_tiles.clear();
}

int ensure_device(sw_plan *p)
{
    if (p->device >= 0) return SW_OK;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const Geom &g = p->geom;
    const size_t state_bytes = (size_t)g.n * g.nv * sizeof(double);
    // on any failure, release what this call allocated so a later call starts clean
    auto undo = [p](int code, const char *msg) {
        (void)hipGetLastError();
        if (p->done) (void)hipEventDestroy(p->done);
        if (p->cap) (void)hipStreamDestroy(p->cap);
        (void)hipFree(p->d_flag);
        (void)hipFree(p->d_tmp);
        (void)hipFree(p->d_edges);
        release_hybrid(p);
        p->done = nullptr;
        p->cap = nullptr;
        p->d_flag = nullptr;
        p->d_tmp = p->d_edges = nullptr;
        return fail(code, msg);
    };
    if (g.swept_ok && g.edge_doubles > 0 &&
        hipMalloc(&p->d_edges, (size_t)g.edge_doubles * sizeof(double)) != hipSuccess)
        return undo(SW_ENOMEM, "edge buffer allocation failed");
    if (hipMalloc(&p->d_tmp, state_bytes) != hipSuccess)
        return undo(SW_ENOMEM, "classic scratch allocation failed");
    if (hipMalloc(&p->d_flag, sizeof(int)) != hipSuccess) return undo(SW_ENOMEM, "flag allocation failed");
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
        return undo(SW_EDEVICE, "capture stream creation failed");
    if (hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess)
        return undo(SW_EDEVICE, "event creation failed");
    if (uses_hybrid(p)) {
        if (hipHostMalloc((void **)&p->h_hybrid, hybrid_doubles(g) * sizeof(double), 0) != hipSuccess)
            return undo(SW_ENOMEM, "pinned host buffer allocation failed");
        if (hipStreamCreateWithFlags(&p->hyb_stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->hyb_ready, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&p->hyb_done, hipEventDisableTiming) != hipSuccess)
            return undo(SW_EDEVICE, "hybrid stream or event creation failed");
        p->hyb_tiles.assign(p->phases.size(), HybridTile{});
    }
    p->device = dev;
    return SW_OK;
}

// One swept phase of the plan's kernel: the register tile, or the Shared variant.
hipError_t launch_plan_phase(const Geom &g, const TileArgs &a, hipStream_t st, int64_t tiles = -1)
{
    if (g.lds) return launch_lds_phase(g.scheme, g.threads, a, st, tiles);
    return launch_swept_phase(g.scheme, g.P, g.threads, a, st, tiles);
}

int enqueue_phases(sw_plan *p, double *state, size_t first, size_t count, hipStream_t st)
{
    const Geom &g = p->geom;
    for (size_t i = first; i < first + count; ++i) {
        TileArgs a = make_tile_args(g, p->consts, p->phases[i], state, p->d_edges);
        hipError_t e = launch_plan_phase(g, a, st);
        if (e != hipSuccess) return hip_fail(e, "swept kernel launch");
    }
    return SW_OK;
}

// Capture `count` phases starting at `first` into an executable graph.
int capture_phases(sw_plan *p, double *state, size_t first, size_t count, hipGraphExec_t *out)
{
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_phases(p, state, first, count, p->cap);
    hipError_t e = hipStreamEndCapture(p->cap, &graph);
    if (rc != SW_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return SW_OK;
}

void drop_swept_graphs(sw_plan *p)
{
    for (hipGraphExec_t x : {p->swept_exec, p->swept_body, p->swept_tail})
        if (x) (void)hipGraphExecDestroy(x);
    p->swept_exec = p->swept_body = p->swept_tail = nullptr;
    p->swept_state = nullptr;
}

void hybrid_callback(void *ud) { hybrid_tile_host(*static_cast<HybridTile *>(ud)); }

// Hybrid variant: every shifted phase runs tiles 0 .. K-2 on the GPU while the host
// computes the straddling tile K-1 (slots 2K-1 and 0) on the plan's copy stream.
int run_hybrid(sw_plan *p, double *state, hipStream_t st)
{
    const Geom &g = p->geom;
    const size_t slot_doubles = (size_t)g.nv * 2 * g.E;
    double *ha = p->h_hybrid, *hb = ha + slot_doubles, *htop = hb + slot_doubles;
    hipStream_t cs = p->hyb_stream;
    const int half = g.w / 2;
    for (size_t i = 0; i < p->phases.size(); ++i) {
        const Phase &ph = p->phases[i];
        const TileArgs a = make_tile_args(g, p->consts, ph, state, p->d_edges);
        if (ph.offset == 0) {
            hipError_t e = launch_swept_phase(g.scheme, g.P, g.threads, a, st);
            if (e != hipSuccess) return hip_fail(e, "swept kernel launch");
            continue;
        }
        HIP_TRY(hipEventRecord(p->hyb_ready, st));   // the phase's inputs are complete
        hipError_t e = launch_swept_phase(g.scheme, g.P, g.threads, a, st, g.K - 1);
        if (e != hipSuccess) return hip_fail(e, "swept kernel launch");
        double *da = p->d_edges + (size_t)(2 * g.K - 1) * slot_doubles, *db = p->d_edges;
        HIP_TRY(hipStreamWaitEvent(cs, p->hyb_ready, 0));
        HIP_TRY(hipMemcpyAsync(ha, da, slot_doubles * sizeof(double), hipMemcpyDeviceToHost, cs));
        HIP_TRY(hipMemcpyAsync(hb, db, slot_doubles * sizeof(double), hipMemcpyDeviceToHost, cs));
        HybridTile &ht = p->hyb_tiles[i];
        ht.a = a;
        ht.scheme = g.scheme;
        ht.slot_a = ha;
        ht.slot_b = hb;
        ht.top = htop;
        HIP_TRY(hipLaunchHostFunc(cs, hybrid_callback, &ht));
        if (ph.kind != PH_DOWN) {
            HIP_TRY(hipMemcpyAsync(da, ha, slot_doubles * sizeof(double), hipMemcpyHostToDevice, cs));
            HIP_TRY(hipMemcpyAsync(db, hb, slot_doubles * sizeof(double), hipMemcpyHostToDevice, cs));
        } else {
            // the top level's points [lo, hi): the tile's left half is the domain's last w/2
            // points, its right half the first w/2
            const int lo = half - g.r * ph.levels, hi = half + g.r * ph.levels;
            for (int v = 0; v < g.nv; ++v) {
                const double *src = htop + (size_t)v * g.w;
                double *dst = state + (size_t)v * g.n;
                const int l1 = lo, h1 = hi < half ? hi : half, l2 = lo > half ? lo : half, h2 = hi;
                if (h1 > l1)
                    HIP_TRY(hipMemcpyAsync(dst + g.n - half + l1, src + l1, (size_t)(h1 - l1) * sizeof(double),
                                           hipMemcpyHostToDevice, cs));
                if (h2 > l2)
                    HIP_TRY(hipMemcpyAsync(dst + (l2 - half), src + l2, (size_t)(h2 - l2) * sizeof(double),
                                           hipMemcpyHostToDevice, cs));
            }
        }
        HIP_TRY(hipEventRecord(p->hyb_done, cs));
        HIP_TRY(hipStreamWaitEvent(st, p->hyb_done, 0));   // the next phase reads the tile's output
    }
    return SW_OK;
}

int run_swept(sw_plan *p, double *state, hipStream_t st)
{
    const size_t n = p->phases.size();
    if (p->geom.lds && !p->lds_ready) {   // before any launch is captured
        HIP_TRY(prepare_lds_phase(p->geom.scheme));
        p->lds_ready = true;
    }
    if (uses_hybrid(p)) {
        // the previous solve's host callbacks read the per-phase records rewritten here
        HIP_TRY(hipEventSynchronize(p->done));
        return run_hybrid(p, state, st);
    }
    if (p->tflags & SW_TUNE_NO_GRAPH) return enqueue_phases(p, state, 0, n, st);
    if (p->swept_state != state) {
        drop_swept_graphs(p);
        int rc;
        if (n <= kMaxGraphPhases) {
            if ((rc = capture_phases(p, state, 0, n, &p->swept_exec))) return rc;
        } else {
            // phases: [Up] [Diamond x (Q-1)] [Down] [Up Down]?; replay the diamonds in chunks
            const int64_t diamonds = p->geom.Q - 1;
            p->body_reps = diamonds / kDiamondChunk;
            p->tail_first = 1 + (size_t)(p->body_reps * kDiamondChunk);
            if ((rc = capture_phases(p, state, 1, (size_t)kDiamondChunk, &p->swept_body))) return rc;
            if ((rc = capture_phases(p, state, p->tail_first, n - p->tail_first, &p->swept_tail))) return rc;
        }
        p->swept_state = state;
    }
    if (p->swept_exec) {
        HIP_TRY(hipGraphLaunch(p->swept_exec, st));
        return SW_OK;
    }
    int rc = enqueue_phases(p, state, 0, 1, st);
    if (rc) return rc;
    for (int64_t r = 0; r < p->body_reps; ++r) HIP_TRY(hipGraphLaunch(p->swept_body, st));
    HIP_TRY(hipGraphLaunch(p->swept_tail, st));
    return SW_OK;
}

// Classic time-stepping of `steps` timesteps, the first being timestep `step0`
// (heat alternates state <-> tmp by step parity; RK2 schemes write the
// predictor to tmp and the final stage back into the state).
int enqueue_classic(sw_plan *p, double *state, int64_t steps, int64_t step0, hipStream_t st)
{
    const Geom &g = p->geom;
    const int dir = g.bc;  // BcKind
    for (int64_t m = 0; m < steps; ++m) {
        hipError_t e;
        if (g.S == 1) {
            const bool even = ((step0 + m) & 1) == 0;
            const double *src = even ? state : p->d_tmp;
            double *dst = even ? p->d_tmp : state;
            e = launch_classic_level(g.scheme, src, dst, g.n, dir, 0, p->consts, g.classic_threads, st);
        } else {
            e = launch_classic_level(g.scheme, state, p->d_tmp, g.n, dir, 1, p->consts, g.classic_threads, st);
            if (e == hipSuccess)
                e = launch_classic_level(g.scheme, p->d_tmp, state, g.n, dir, 0, p->consts, g.classic_threads, st);
        }
        if (e != hipSuccess) return hip_fail(e, "classic kernel launch");
    }
    return SW_OK;
}

int run_classic(sw_plan *p, double *state, hipStream_t st)
{
    const Geom &g = p->geom;
    const int64_t steps = g.nsteps;
    int64_t done = 0;
    if (!(p->tflags & SW_TUNE_NO_GRAPH) && steps >= kClassicChunkSteps) {
        if (p->classic_state != state) {
            if (p->classic_exec) (void)hipGraphExecDestroy(p->classic_exec);
            p->classic_exec = nullptr;
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_classic(p, state, kClassicChunkSteps, 0, p->cap);
            hipError_t e = hipStreamEndCapture(p->cap, &graph);
            if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&p->classic_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            p->classic_state = state;
        }
        const int64_t reps = steps / kClassicChunkSteps;
        for (int64_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(p->classic_exec, st));
        done = reps * kClassicChunkSteps;
    }
    int rc = enqueue_classic(p, state, steps - done, done, st);
    if (rc) return rc;
    if (g.S == 1 && (steps & 1))
        HIP_TRY(hipMemcpyAsync(state, p->d_tmp, (size_t)g.n * g.nv * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
    return SW_OK;
}

int check_nan(sw_plan *p, const double *state, hipStream_t st)
{
    int host = 0;
    HIP_TRY(hipMemsetAsync(p->d_flag, 0, sizeof(int), st));
    hipError_t e = launch_nonfinite_scan(state, p->geom.n * p->geom.nv, p->d_flag, st);
    if (e != hipSuccess) return hip_fail(e, "nonfinite scan launch");
    HIP_TRY(hipMemcpyAsync(&host, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return host ? fail(SW_ENAN, "non-finite value in the solution") : SW_OK;
}

template <class F>
int solve_common(sw_plan *p, double *state, void *stream, F &&body)
{
    if (!p) return fail(SW_EINVAL, "plan is NULL");
    std::unique_lock<std::mutex> lk(p->mu, std::try_to_lock);
    if (!lk.owns_lock()) return fail(SW_EBUSY, "plan is in use by another thread");
    int rc = check_device_ptr(state);
    if (rc) return rc;
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(SW_EDEVICE, "cannot select the plan's device");
    if ((rc = ensure_device(p))) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipStreamWaitEvent(st, p->done, 0));
    rc = body(st);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(p->done, st));
    if (p->tflags & SW_TUNE_CHECK_NAN) return check_nan(p, state, st);
    return SW_OK;
}

}  // namespace

extern "C" {

int swept_plan(const sw_problem *problem, const sw_tuning *tuning, sw_plan **out)
{
    if (!out) return fail(SW_EINVAL, "out is NULL");
    std::string err;
    int rc = validate_problem(problem, &err);
    if (rc) return fail(rc, err);
    int width = tuning ? tuning->width : 0;
    int threads = tuning ? tuning->threads : 0;
    if ((width == 0) != (threads == 0)) return fail(SW_EINVAL, "give both width and threads, or neither");
    if (width == 0) {
        if (!tuned_shape(*problem, &width, &threads)) default_shape(*problem, &width, &threads);
    }
    const int32_t tflags = tuning ? tuning->flags : 0;
    if (tflags & ~(SW_TUNE_NO_GRAPH | SW_TUNE_CHECK_NAN | SW_TUNE_HYBRID | SW_TUNE_LDS))
        return fail(SW_EINVAL, "unknown tuning flags");
    const bool lds = (tflags & SW_TUNE_LDS) != 0;
    if (lds && (tflags & SW_TUNE_HYBRID)) return fail(SW_EINVAL, "SW_TUNE_LDS and SW_TUNE_HYBRID exclude each other");
    Geom g;
    if ((rc = make_geom(*problem, width, threads, &g, &err, lds))) return fail(rc, err);
    if (lds && lds_tile_bytes(g.nv, g.r, g.w) > kLdsTileMaxBytes)
        return fail(SW_EINVAL, "the Shared variant's rows do not fit in 160 KB of LDS at this width");

    if (tuning && tuning->width && !g.swept_ok)
        return fail(SW_EINVAL, "tile width does not divide n");
    int ct = tuning ? tuning->classic_threads : 0;
    if (ct == 0 && !tuned_classic_threads(*problem, &ct)) ct = 256;
    if (!legal_threads(ct)) return fail(SW_EINVAL, "classic_threads must be a multiple of 64 in [64, 1024]");
    g.classic_threads = ct;
    sw_plan *p = new (std::nothrow) sw_plan();
    if (!p) return fail(SW_ENOMEM, "plan allocation failed");
    p->prob = *problem;
    p->geom = g;
    p->consts = make_consts(*problem);
    if (g.swept_ok) p->phases = build_phases(g);
    p->tflags = tflags;
    *out = p;
    return SW_OK;
}

int swept_plan_info(const sw_plan *p, sw_plan_info *out)
{
    if (!p || !out) return fail(SW_EINVAL, "NULL argument");
    const Geom &g = p->geom;
    sw_plan_info i;
    std::memset(&i, 0, sizeof(i));
    i.width = g.w; i.threads = g.threads; i.points_per_lane = g.P;
    i.radius = g.r; i.substeps = g.S; i.nvars = g.nv; i.swept_ok = g.swept_ok ? 1 : 0;
    i.classic_threads = g.classic_threads;
    i.nodes = g.K; i.levels = g.levels; i.levels_per_phase = g.H;
    i.full_phases = g.Q; i.remainder = g.rem;
    i.swept_launches = (int64_t)p->phases.size();
    i.classic_launches = g.levels;
    i.scratch_bytes = (g.edge_doubles + g.n * g.nv) * (int64_t)sizeof(double);
    *out = i;
    return SW_OK;
}

int swept_solve(sw_plan *p, double *d_state, void *hip_stream)
{
    if (p && !p->geom.swept_ok)
        return fail(SW_EUNSUPPORTED, "no legal swept tile width divides n; use classic_solve");
    return solve_common(p, d_state, hip_stream, [&](hipStream_t st) {
        if (p->phases.empty()) return (int)SW_OK;
        return run_swept(p, d_state, st);
    });
}

int classic_solve(sw_plan *p, double *d_state, void *hip_stream)
{
    return solve_common(p, d_state, hip_stream, [&](hipStream_t st) {
        if (p->geom.nsteps == 0) return (int)SW_OK;
        return run_classic(p, d_state, st);
    });
}

int swept_profile_phase(sw_plan *p, double *d_state, int32_t kind, int32_t reps, void *hip_stream,
                        double *avg_us)
{
    if (!p || !avg_us || reps < 1 || kind < PH_UP || kind > PH_DOWN)
        return fail(SW_EINVAL, "invalid profiling request");
    if (!p->geom.swept_ok) return fail(SW_EUNSUPPORTED, "plan cannot run swept");
    double us = 0.0;
    int rc = solve_common(p, d_state, hip_stream, [&](hipStream_t st) -> int {
        if (p->geom.lds && !p->lds_ready) {
            HIP_TRY(prepare_lds_phase(p->geom.scheme));
            p->lds_ready = true;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        int r = SW_OK;
        hipError_t he = hipEventRecord(e0, st);
        for (int32_t i = 0; i < reps && r == SW_OK && he == hipSuccess; ++i) {
            Phase ph{kind, p->geom.H, kind == PH_UP ? 0 : (int32_t)((i + 1) & 1)};
            TileArgs a = make_tile_args(p->geom, p->consts, ph, d_state, p->d_edges);
            hipError_t le = launch_plan_phase(p->geom, a, st);
            if (le != hipSuccess) r = hip_fail(le, "profiled launch");
        }
        if (he == hipSuccess) he = hipEventRecord(e1, st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (r) return r;
        if (he != hipSuccess) return hip_fail(he, "profiling events");
        us = 1000.0 * (double)ms / reps;
        return (int)SW_OK;
    });
    if (rc) return rc;
    *avg_us = us;
    return SW_OK;
}

void swept_plan_destroy(sw_plan *p)
{
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        if (p->device >= 0) {
            DeviceGuard guard(p->device);
            (void)hipEventSynchronize(p->done);
            drop_swept_graphs(p);
            if (p->classic_exec) (void)hipGraphExecDestroy(p->classic_exec);
            if (p->hyb_stream) (void)hipStreamSynchronize(p->hyb_stream);
            (void)hipFree(p->d_edges);
            (void)hipFree(p->d_tmp);
            (void)hipFree(p->d_flag);
            (void)hipEventDestroy(p->done);
            (void)hipStreamDestroy(p->cap);
            release_hybrid(p);
        }
    }
    delete p;
}

const char *sw_strerror(int status)
{
    switch (status) {
    case SW_OK: return "ok";
    case SW_EINVAL: return "invalid argument";
    case SW_ENOMEM: return "out of memory";
    case SW_EDEVICE: return "HIP runtime error";
    case SW_EUNSUPPORTED: return "unsupported";
    case SW_EBUSY: return "busy";
    case SW_ENOTREADY: return "not ready";
    case SW_ENAN: return "non-finite result";
    default: return "unknown status";
    }
}

const char *sw_last_error(void) { return sw::g_last_error.c_str(); }

}  // extern "C"
