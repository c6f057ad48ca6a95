// Test-only CPU build of the library's batched and served solve scheduler.
//
// batch.hip (the batch_* entry points of include/swept.h) is compiled unchanged
// against the CPU stand-in runtime in fakehip/, with the batch kernels replaced by
// host functions that run each (solve, tile) item through the tile emulator
// (tile_emu.hpp) when its stream gets to it.  The CPU tests drive the real admission,
// tick, table and retirement logic with this library and compare every result
// with the oracle.  It is never linked into libswept.so; classic fallbacks (solves
// no tile width divides) are not available here.
#include <chrono>
#include <cstring>
#include <string>

#include "../../paper_1705_03162_amd/csrc/batch.hip"
#include "../../paper_1705_03162_amd/csrc/tune.cpp"
#include "tile_emu.hpp"

namespace sw {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t, const char *where)
{
    g_last_error = std::string(where) + ": CPU stand-in runtime error";
    return SW_EDEVICE;
}

int check_device_ptr(const void *p) { return p ? SW_OK : fail(SW_EINVAL, "state pointer is NULL"); }

namespace {

template <class Sch, int P>
void run_items(const SolveDesc *desc, const int2 *items, int64_t nitems, int global_phase)
{
    for (int64_t i = 0; i < nitems; ++i) {
        const int2 it = items[i];
        const SolveDesc &d = desc[it.x];
        const int p = global_phase >= 0 ? global_phase : d.phase;
        if (p >= d.nphases) continue;
        TileArgs a{};
        a.state = d.state;
        a.edges = d.edges;
        a.n = d.n;
        a.K = d.K;
        a.w = d.w;
        a.H = d.H;
        a.E = d.E;
        a.bc = d.bc;
        a.ends = 0;
        a.c = d.c;
        phase_at(d.Q, d.rem, d.H, p, a.kind, a.levels, a.offset);
        emu::emulate_tile<Sch, P>(a, (int64_t)it.y, 1);
    }
}

template <class Sch>
bool run_items_p(int P, const SolveDesc *desc, const int2 *items, int64_t nitems, int global_phase)
{
    switch (P) {
    case 1: run_items<Sch, 1>(desc, items, nitems, global_phase); return true;
    case 2: run_items<Sch, 2>(desc, items, nitems, global_phase); return true;
    case 4: run_items<Sch, 4>(desc, items, nitems, global_phase); return true;
    case 8: run_items<Sch, 8>(desc, items, nitems, global_phase); return true;
    default: return false;
    }
}

}  // namespace

hipError_t launch_batch_phase(int scheme, int P, const SolveDesc *desc, const int2 *items, int64_t nitems,
                              int global_phase, int grid, hipStream_t st)
{
    if (grid < 1 || nitems < 0 || (P != 1 && P != 2 && P != 4 && P != 8)) return hipErrorInvalidValue;
    fakehip::enqueue(st, [=] {
        if (scheme == SW_HEAT) run_items_p<Heat>(P, desc, items, nitems, global_phase);
        else if (scheme == SW_KS) run_items_p<KS>(P, desc, items, nitems, global_phase);
        else run_items_p<Euler>(P, desc, items, nitems, global_phase);
    });
    return hipSuccess;
}

hipError_t launch_advance_phases(SolveDesc *desc, int64_t n, hipStream_t st)
{
    fakehip::enqueue(st, [=] {
        for (int64_t i = 0; i < n; ++i)
            if (desc[i].phase < desc[i].nphases) desc[i].phase += 1;
    });
    return hipSuccess;
}

hipError_t launch_stamp(uint64_t *stamps, int idx, hipStream_t st)
{
    fakehip::enqueue(st, [=] {
        const auto ns = std::chrono::duration_cast<std::chrono::nanoseconds>(
                            std::chrono::steady_clock::now().time_since_epoch()).count();
        stamps[idx] = (uint64_t)ns / 10;   // the stand-in wall clock runs at 100 MHz
    });
    return hipSuccess;
}

int batch_blocks_per_cu(int, int) { return 2; }
int persistent_blocks_per_cu(int, int) { return 2; }

hipError_t launch_zero_words(void *p, int64_t count, hipStream_t st)
{
    fakehip::enqueue(st, [=] { std::memset(p, 0, (size_t)count * 4); });
    return hipSuccess;
}

// The persistent launch, run by one stand-in work-group: it takes the queue entries
// in order (phase-major, so every dependency is already done when an entry runs),
// checks the dependency counters as the device kernel waits on them, and keeps the
// same completion counters and per-solve stamps.
template <class Sch>
void run_persistent(int P, PersistArgs q)
{
    const int64_t total = q.phase_start[q.max_phases];
    for (int64_t i = 0; i < total; ++i) {
        int p = 0;
        while (p + 1 <= q.max_phases && q.phase_start[p + 1] <= i) ++p;
        const int64_t r = i - q.phase_start[p];
        const int2 it = q.items[r];
        const SolveDesc &d = q.desc[it.x];
        const int64_t base = r - it.y;
        if (p > 0) {
            int64_t deps[2];
            const int nd = phase_deps(d.Q, d.rem, d.H, d.K, p, it.y, deps);
            for (int k = 0; k < nd; ++k)
                if (q.done[base + deps[k]] < p) *q.error = 1;   // would wait forever
        }
        TileArgs a{};
        a.state = d.state;
        a.edges = d.edges;
        a.n = d.n;
        a.K = d.K;
        a.w = d.w;
        a.H = d.H;
        a.E = d.E;
        a.bc = d.bc;
        a.ends = 0;
        a.c = d.c;
        phase_at(d.Q, d.rem, d.H, p, a.kind, a.levels, a.offset);
        switch (P) {
        case 1: emu::emulate_tile<Sch, 1>(a, (int64_t)it.y, 1); break;
        case 2: emu::emulate_tile<Sch, 2>(a, (int64_t)it.y, 1); break;
        case 4: emu::emulate_tile<Sch, 4>(a, (int64_t)it.y, 1); break;
        default: emu::emulate_tile<Sch, 8>(a, (int64_t)it.y, 1); break;
        }
        q.done[r] = p + 1;
        if (p + 1 == d.nphases && ++q.finished[it.x] == d.K) {
            const auto ns = std::chrono::duration_cast<std::chrono::nanoseconds>(
                                std::chrono::steady_clock::now().time_since_epoch()).count();
            q.stamps[it.x] = (uint64_t)ns / 10;
        }
    }
    *q.next = (unsigned long long)total;
}

hipError_t launch_persistent_batch(int scheme, int P, const PersistArgs &q, int grid, hipStream_t st)
{
    if (grid < 1 || (P != 1 && P != 2 && P != 4 && P != 8)) return hipErrorInvalidValue;
    fakehip::enqueue(st, [=] {
        if (scheme == SW_HEAT) run_persistent<Heat>(P, q);
        else if (scheme == SW_KS) run_persistent<KS>(P, q);
        else run_persistent<Euler>(P, q);
    });
    return hipSuccess;
}

}  // namespace sw

extern "C" {

// Classic plans are not part of this build: batches here hold swept solves only.
int swept_plan(const sw_problem *, const sw_tuning *, sw_plan **) { return SW_EUNSUPPORTED; }
int classic_solve(sw_plan *, double *, void *) { return SW_EUNSUPPORTED; }
void swept_plan_destroy(sw_plan *) {}

const char *sw_strerror(int status) { return status == SW_OK ? "ok" : "error"; }
const char *sw_last_error(void) { return sw::g_last_error.c_str(); }

// A stand-in stream and a copy queued on it (it runs when something waits for it):
// lets a test write a solve's initial state "asynchronously" before submitting.
void *servesim_stream_create(void)
{
    hipStream_t s = nullptr;
    (void)hipStreamCreateWithFlags(&s, 0);
    return s;
}
void servesim_enqueue_copy(void *stream, void *dst, const void *src, size_t bytes)
{
    (void)hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, (hipStream_t)stream);
}
void servesim_stream_destroy(void *stream) { (void)hipStreamDestroy((hipStream_t)stream); }

// Ticks of a served batch so far (test introspection).
int64_t servesim_ticks(sw_batch *b)
{
    std::lock_guard<std::mutex> lk(b->mu);
    return b->ticks;
}

}  // extern "C"
