// Batched solves (batch_* entry points of include/swept.h).
//
// Ensemble mode (batch_run): queued solves are grouped by (scheme, points per
// lane); each group advances all its solves together, one launch per phase
// index covering every tile of every solve still running.  Solves are sorted
// by phase count, so the solves still running at phase p are always a prefix of
// the group's (solve, tile) table and one table serves every launch.  The
// launches of all groups (and timing events) are captured into one HIP graph
// and replayed with a single launch.  Kernel boundaries order the phases, which
// keeps edge data coherent across the MI355X's eight XCD-private L2 caches
// without device-side flags.
//
// Served mode (flags SW_BATCH_SERVE): a worker thread admits queued solves as
// memory and slots free up and runs ticks; each tick advances every resident
// solve by one phase with one launch per group (continuous batching).
//
// Admission is by a device-memory budget: a resident solve holds its state plus
// its edge slots (about 3 n nvars doubles).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "api_internal.hpp"
#include "kernels.hpp"
#include "plan_core.hpp"
#include "swept.h"
#include "tune.hpp"

using namespace sw;

#define BHIP(expr)                                            \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return sw::hip_fail(_e, #expr); \
    } while (0)

namespace {

using Clock = std::chrono::steady_clock;

double now_s()
{
    return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

struct Ticket {
    uint64_t id = 0;
    sw_problem prob{};
    double *state = nullptr;
    int32_t status = SW_TICKET_QUEUED;
    int64_t bytes = 0;
    double t_submit = 0, t_start = 0, t_end = 0;
    // swept geometry when batched
    bool swept = false;
    int P = 0;
    Geom geom;
    double *edges = nullptr;
    int32_t phase = 0;
    int32_t nphases = 0;
    int64_t admit_tick = -1;   // served: first tick of its group that includes it
    hipEvent_t ready = nullptr;   // batch_submit_async: the state is complete on the device
    sw_plan *plan = nullptr;      // served classic fallback in flight
    hipEvent_t finished = nullptr;
};

// Make `st` wait until the ticket's initial state is complete (batch_submit_async).
hipError_t wait_ready(const Ticket &t, hipStream_t st)
{
    return t.ready ? hipStreamWaitEvent(st, t.ready, 0) : hipSuccess;
}

void release_events(Ticket *t)
{
    if (t->ready) (void)hipEventDestroy(t->ready);
    if (t->finished) (void)hipEventDestroy(t->finished);
    t->ready = t->finished = nullptr;
}

constexpr size_t kArenaAlign = 256;

// Device bytes a resident solve holds in the batch: its state plus, batched, its edge
// slots as the arena hands them out (rounded to the arena's alignment), or, solved
// classically, the plan's scratch (a second state array).
int64_t resident_bytes(const sw_problem &p, bool swept, const Geom &g)
{
    const int64_t state = p.n * (int64_t)scheme_nvars(p.scheme) * (int64_t)sizeof(double);
    if (!swept) return 2 * state;
    const int64_t edges = g.edge_doubles * (int64_t)sizeof(double);
    return state + (edges + (int64_t)kArenaAlign - 1) / (int64_t)kArenaAlign * (int64_t)kArenaAlign;
}

// Tile shape for a batched solve: one-wave tiles (no barriers), the most points
// per lane that divide n up to a cap -- the caller's points_per_lane, else the
// tuned value for the size class, else 8.
bool batch_shape(const sw_problem &p, int forced, int *P, Geom *g)
{
    int cap = 8;
    if (forced > 0) cap = forced;
    else if (int t = 0; tuned_batch_points(p, &t) && t > 0) cap = t;
    for (int pp = 8; pp >= 1; pp /= 2) {
        if (pp > cap) continue;
        if (!legal_points_per_lane(p.scheme, pp)) continue;
        const int w = 64 * pp;
        if (p.n % w != 0) continue;
        std::string err;
        if (make_geom(p, w, 64, g, &err) != SW_OK) continue;
        *P = pp;
        return true;
    }
    return false;
}

// Device arena: large chunks, first-fit sub-allocation, freed only on destroy.
struct Arena {
    struct Chunk { char *base; size_t size; std::map<size_t, size_t> free; };  // offset -> size
    std::vector<Chunk> chunks;
    static constexpr size_t kChunk = (size_t)256 << 20;
    static constexpr size_t kAlign = kArenaAlign;

    void *alloc(size_t bytes)
    {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (Chunk &c : chunks) {
            for (auto it = c.free.begin(); it != c.free.end(); ++it) {
                if (it->second >= bytes) {
                    size_t off = it->first, sz = it->second;
                    c.free.erase(it);
                    if (sz > bytes) c.free[off + bytes] = sz - bytes;
                    return c.base + off;
                }
            }
        }
        size_t sz = std::max(kChunk, bytes);
        void *p = nullptr;
        if (hipMalloc(&p, sz) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
        Chunk c{(char *)p, sz, {}};
        if (sz > bytes) c.free[bytes] = sz - bytes;
        chunks.push_back(std::move(c));
        return p;
    }
    void release(void *p, size_t bytes)
    {
        if (!p) return;
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (Chunk &c : chunks) {
            char *cp = (char *)p;
            if (cp < c.base || cp >= c.base + c.size) continue;
            size_t off = (size_t)(cp - c.base);
            auto nx = c.free.lower_bound(off);
            // merge with the following block
            if (nx != c.free.end() && nx->first == off + bytes) { bytes += nx->second; nx = c.free.erase(nx); }
            // merge with the preceding block
            if (nx != c.free.begin()) {
                auto pv = std::prev(nx);
                if (pv->first + pv->second == off) { pv->second += bytes; return; }
            }
            c.free[off] = bytes;
            return;
        }
    }
    void destroy()
    {
        for (Chunk &c : chunks) (void)hipFree(c.base);
        chunks.clear();
    }
};

// Device copy of one group's descriptors and (solve, tile) items.
struct GroupBuf {
    int scheme = 0, P = 1;
    std::vector<Ticket *> members;  // solves in table order
    std::vector<SolveDesc> desc;
    std::vector<int2> items;
    std::vector<int64_t> prefix;   // items of the first k solves
    SolveDesc *d_desc = nullptr;
    int2 *d_items = nullptr;
    int grid_cap = 1;
};

SolveDesc make_desc(const Ticket &t)
{
    SolveDesc d{};
    d.state = t.state;
    d.edges = t.edges;
    d.n = t.geom.n;
    d.K = t.geom.K;
    d.Q = t.geom.Q;
    d.rem = t.geom.rem;
    d.w = t.geom.w;
    d.H = t.geom.H;
    d.E = t.geom.E;
    d.bc = t.geom.bc;
    d.nphases = phase_count(t.geom.Q, t.geom.rem);
    d.phase = t.phase;
    d.c = make_consts(t.prob);
    return d;
}

int num_cus()
{
    static int cached = 0;
    if (!cached) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            cached = n;
        else
            cached = 256;
    }
    return cached;
}

}  // namespace

struct sw_batch {
    sw_batch_config cfg{};
    std::deque<Ticket> tickets;    // indexable by id - 1; push_back keeps references valid,
                                   // so the served worker may hold Ticket pointers
    uint64_t next_id = 1;
    std::mutex mu;
    std::condition_variable cv;
    Arena arena;
    // served mode
    bool serve = false;
    bool stop = false;
    std::thread worker;
    hipStream_t stream = nullptr;
    int device = -1;
    std::deque<uint64_t> queue;    // waiting tickets (served mode)
    int64_t resident = 0;
    int nresident = 0;
    int64_t ticks = 0;
    std::string worker_error;
};

namespace {

Ticket *find_ticket(sw_batch *b, uint64_t id)
{
    if (id == 0 || id > b->tickets.size()) return nullptr;
    return &b->tickets[id - 1];
}

// Device resources of one ensemble wave; release() frees whatever was allocated.
struct EnsembleRun {
    std::vector<GroupBuf> gb;
    std::vector<void *> dev;           // device allocations
    std::vector<hipStream_t> streams;  // one per tile group: the graph's parallel branches
    std::vector<hipEvent_t> events;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;

    hipError_t alloc(void **p, size_t bytes)
    {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) dev.push_back(*p);
        return e;
    }
    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipStream_t s : streams) (void)hipStreamDestroy(s);
        if (cap) (void)hipStreamDestroy(cap);
        for (void *p : dev) (void)hipFree(p);
        exec = nullptr;
        events.clear();
        streams.clear();
        cap = nullptr;
        dev.clear();
    }
};

// Relative cost of a point-level (for splitting the persistent grid between groups).
double level_weight(int scheme) { return scheme == SW_EULER ? 20.0 : (scheme == SW_KS ? 2.0 : 1.0); }

// Capture the phase-index launches of every group: each group's chain of launches (one
// per phase index, then a timing stamp) on a parallel branch of the graph, so a group of
// short phases runs beside the others instead of waiting for each phase index of all.
int capture_lockstep(EnsembleRun &run, uint64_t *d_stamps, const std::vector<size_t> &soff, hipGraph_t *graph)
{
    BHIP(hipStreamBeginCapture(run.cap, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_stamp(d_stamps, 0, run.cap);
    hipEvent_t fork = run.events[0];
    if (le == hipSuccess) le = hipEventRecord(fork, run.cap);
    for (size_t g = 0; g < run.gb.size() && le == hipSuccess; ++g) {
        GroupBuf &gb = run.gb[g];
        hipStream_t s = run.streams[g];
        if ((le = hipStreamWaitEvent(s, fork, 0)) != hipSuccess) break;
        const int gp = gb.desc.empty() ? 0 : gb.desc.front().nphases;   // sorted: the largest first
        size_t a = gb.desc.size();
        for (int p = 0; p < gp && le == hipSuccess; ++p) {
            // solves still running at phase p: a prefix of the sorted group
            while (a > 0 && gb.desc[a - 1].nphases <= p) --a;
            const int64_t nitems = gb.prefix[a];
            const int grid = (int)std::min<int64_t>(nitems, gb.grid_cap);
            le = launch_batch_phase(gb.scheme, gb.P, gb.d_desc, gb.d_items, nitems, p, grid, s);
            if (le == hipSuccess) le = launch_stamp(d_stamps, (int)(soff[g] + (size_t)p), s);
        }
        if (le != hipSuccess) break;
        if ((le = hipEventRecord(run.events[g + 1], s)) != hipSuccess) break;
        le = hipStreamWaitEvent(run.cap, run.events[g + 1], 0);
    }
    hipError_t ce = hipStreamEndCapture(run.cap, graph);
    if (le != hipSuccess) return hip_fail(le, "batched phase launch");
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    return SW_OK;
}

// Per-group device state of the persistent launch.
struct PersistGroup {
    PersistArgs q{};
    int grid = 1;
    int64_t nsolves = 0;
    std::vector<int64_t> phase_start;
};

// Capture one persistent launch per group, the groups on parallel branches of the graph
// (each with its share of the resident work-groups), after a stamp of the start time.
int capture_persistent(EnsembleRun &run, std::vector<PersistGroup> &pg, uint64_t *d_t0, hipGraph_t *graph)
{
    BHIP(hipStreamBeginCapture(run.cap, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_stamp(d_t0, 0, run.cap);
    hipEvent_t fork = run.events[0];
    if (le == hipSuccess) le = hipEventRecord(fork, run.cap);
    for (size_t g = 0; g < pg.size() && le == hipSuccess; ++g) {
        hipStream_t s = run.streams[g];
        hipEvent_t join = run.events[g + 1];
        const PersistArgs &q = pg[g].q;
        const int64_t items = pg[g].phase_start.empty() ? 0 : (int64_t)run.gb[g].items.size();
        if ((le = hipStreamWaitEvent(s, fork, 0)) != hipSuccess) break;
        // counters start at zero (a fill kernel, not a memset node, inside a graph)
        if ((le = launch_zero_words(q.done, items, s)) != hipSuccess) break;
        if ((le = launch_zero_words(q.finished, pg[g].nsolves, s)) != hipSuccess) break;
        if ((le = launch_zero_words(q.next, 2, s)) != hipSuccess) break;
        if ((le = launch_zero_words(q.error, 1, s)) != hipSuccess) break;
        if ((le = launch_persistent_batch(run.gb[g].scheme, run.gb[g].P, q, pg[g].grid, s)) != hipSuccess) break;
        if ((le = hipEventRecord(join, s)) != hipSuccess) break;
        le = hipStreamWaitEvent(run.cap, join, 0);
    }
    hipError_t ce = hipStreamEndCapture(run.cap, graph);
    if (le != hipSuccess) return hip_fail(le, "persistent batched launch");
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    return SW_OK;
}

// Run a set of admitted swept tickets to completion as one graph (ensemble mode):
// one launch per phase index and group, or (SW_BATCH_PERSISTENT) one persistent
// launch per group.  Every exit goes through one cleanup: device buffers freed,
// edges returned to the arena, tickets DONE or FAILED.
int run_ensemble(sw_batch *b, std::vector<Ticket *> &ts, hipStream_t st)
{
    EnsembleRun run;
    int rc = SW_OK;
    const bool persistent = (b->cfg.flags & SW_BATCH_PERSISTENT) != 0;
    std::vector<PersistGroup> pg;
    // timing stamps: [0] = start, then per group from soff[g]: one per phase index
    // (lock-step) or one per solve (persistent)
    std::vector<size_t> soff;
    uint64_t *d_stamps = nullptr;
    std::vector<uint64_t> stamps;
    int clock_khz = 0;
    double t0 = 0.0;
    auto finish = [&](int code) {
        if (code == SW_OK) {
            const double tick_s = clock_khz > 0 ? 1.0 / (1000.0 * clock_khz) : 0.0;
            for (size_t g = 0; g < run.gb.size(); ++g)
                for (size_t i = 0; i < run.gb[g].members.size(); ++i) {
                    Ticket *t = run.gb[g].members[i];
                    const size_t np = (size_t)phase_count(t->geom.Q, t->geom.rem);
                    const uint64_t end = persistent ? stamps[soff[g] + i] : (np ? stamps[soff[g] + np - 1] : stamps[0]);
                    t->t_end = t0 + (double)(end - stamps[0]) * tick_s;
                    t->status = SW_TICKET_DONE;
                }
        } else {
            const double t = now_s();
            for (Ticket *x : ts) { x->status = SW_TICKET_FAILED; x->t_end = t; }
        }
        run.release();
        for (Ticket *t : ts) {
            b->arena.release(t->edges, (size_t)t->geom.edge_doubles * sizeof(double));
            t->edges = nullptr;
            release_events(t);
        }
        return code;
    };
    for (Ticket *t : ts) {
        t->phase = 0;
        t->edges = (double *)b->arena.alloc((size_t)t->geom.edge_doubles * sizeof(double));
        if (!t->edges) return finish(fail(SW_ENOMEM, "edge arena allocation failed"));
    }
    // group by (scheme, P), sort by phase count (descending)
    std::map<std::pair<int, int>, std::vector<Ticket *>> groups;
    for (Ticket *t : ts) groups[{t->prob.scheme, t->P}].push_back(t);
    for (auto &kv : groups) {
        auto &v = kv.second;
        std::stable_sort(v.begin(), v.end(), [](const Ticket *x, const Ticket *y) {
            return phase_count(x->geom.Q, x->geom.rem) > phase_count(y->geom.Q, y->geom.rem);
        });
        GroupBuf g;
        g.scheme = kv.first.first;
        g.P = kv.first.second;
        g.members = v;
        g.prefix.push_back(0);
        for (size_t s = 0; s < v.size(); ++s) {
            g.desc.push_back(make_desc(*v[s]));
            for (int64_t j = 0; j < v[s]->geom.K; ++j) g.items.push_back(make_int2((int)s, (int)j));
            g.prefix.push_back((int64_t)g.items.size());
        }
        g.grid_cap = batch_blocks_per_cu(g.scheme, g.P) * num_cus();
        run.gb.push_back(std::move(g));
    }
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
            return finish(fail(SW_EDEVICE, "device clock rate"));
    }
    size_t nstamps = 1;
    soff.assign(run.gb.size(), 0);
    for (size_t g = 0; g < run.gb.size(); ++g) {
        soff[g] = nstamps;
        nstamps += persistent ? run.gb[g].desc.size()
                              : (run.gb[g].desc.empty() ? 0 : (size_t)run.gb[g].desc.front().nphases);
    }
    stamps.assign(nstamps, 0);
    if (run.alloc((void **)&d_stamps, nstamps * sizeof(uint64_t)) != hipSuccess)
        return finish(fail(SW_ENOMEM, "stamp buffer allocation failed"));
    for (GroupBuf &g : run.gb) {
        if (run.alloc((void **)&g.d_desc, g.desc.size() * sizeof(SolveDesc)) != hipSuccess ||
            run.alloc((void **)&g.d_items, g.items.size() * sizeof(int2)) != hipSuccess)
            return finish(fail(SW_ENOMEM, "batch table allocation failed"));
        if (hipMemcpyAsync(g.d_desc, g.desc.data(), g.desc.size() * sizeof(SolveDesc), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(g.d_items, g.items.data(), g.items.size() * sizeof(int2), hipMemcpyHostToDevice, st) != hipSuccess)
            return finish(fail(SW_EDEVICE, "batch table upload"));
    }
    if (persistent) {
        // queue layout, counters, and each group's share of the resident work-groups
        double total_work = 0.0;
        std::vector<double> work(run.gb.size(), 0.0);
        for (size_t g = 0; g < run.gb.size(); ++g) {
            for (const Ticket *t : run.gb[g].members)
                work[g] += (double)t->geom.n * (double)t->geom.levels * level_weight(t->prob.scheme);
            total_work += work[g];
        }
        pg.resize(run.gb.size());
        for (size_t g = 0; g < run.gb.size(); ++g) {
            GroupBuf &gb = run.gb[g];
            PersistGroup &x = pg[g];
            int gp = gb.desc.empty() ? 0 : gb.desc.front().nphases;   // sorted: the largest first
            x.phase_start.assign((size_t)gp + 1, 0);
            size_t a = gb.desc.size();
            for (int p = 0; p < gp; ++p) {
                while (a > 0 && gb.desc[a - 1].nphases <= p) --a;
                x.phase_start[(size_t)p + 1] = x.phase_start[(size_t)p] + gb.prefix[a];
            }
            x.nsolves = (int64_t)gb.desc.size();
            int64_t *d_ps = nullptr;
            int32_t *d_done = nullptr, *d_fin = nullptr, *d_err = nullptr;
            unsigned long long *d_next = nullptr;
            if (run.alloc((void **)&d_ps, x.phase_start.size() * sizeof(int64_t)) != hipSuccess ||
                run.alloc((void **)&d_done, std::max<size_t>(gb.items.size(), 1) * sizeof(int32_t)) != hipSuccess ||
                run.alloc((void **)&d_fin, std::max<size_t>(gb.desc.size(), 1) * sizeof(int32_t)) != hipSuccess ||
                run.alloc((void **)&d_next, sizeof(unsigned long long)) != hipSuccess ||
                run.alloc((void **)&d_err, sizeof(int32_t)) != hipSuccess)
                return finish(fail(SW_ENOMEM, "persistent batch allocation failed"));
            if (hipMemcpyAsync(d_ps, x.phase_start.data(), x.phase_start.size() * sizeof(int64_t),
                               hipMemcpyHostToDevice, st) != hipSuccess)
                return finish(fail(SW_EDEVICE, "persistent queue upload"));
            x.q.desc = gb.d_desc;
            x.q.items = gb.d_items;
            x.q.phase_start = d_ps;
            x.q.done = d_done;
            x.q.finished = d_fin;
            x.q.stamps = d_stamps + soff[g];
            x.q.next = d_next;
            x.q.error = d_err;
            x.q.max_phases = gp;
            x.q.spin_limit = (int64_t)1 << 22;   // a few seconds of polling
            const int occ = persistent_blocks_per_cu(gb.scheme, gb.P) * num_cus();
            const double share = total_work > 0.0 ? work[g] / total_work : 1.0;
            x.grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)(occ * share + 0.5),
                                                                 std::max<int64_t>(x.phase_start.back(), 1)));
        }
    }
    {   // fork streams and events of the parallel branches
        run.streams.assign(run.gb.size(), nullptr);
        run.events.assign(run.gb.size() + 1, nullptr);
        for (hipStream_t &s : run.streams)
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) { s = nullptr; return finish(fail(SW_EDEVICE, "stream creation")); }
        for (hipEvent_t &e : run.events)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { e = nullptr; return finish(fail(SW_EDEVICE, "event creation")); }
    }
    if (hipStreamSynchronize(st) != hipSuccess) return finish(fail(SW_EDEVICE, "batch table upload"));
    if (hipStreamCreateWithFlags(&run.cap, hipStreamNonBlocking) != hipSuccess) {
        run.cap = nullptr;
        return finish(fail(SW_EDEVICE, "capture stream creation"));
    }
    hipGraph_t graph = nullptr;
    rc = persistent ? capture_persistent(run, pg, d_stamps, &graph) : capture_lockstep(run, d_stamps, soff, &graph);
    if (rc == SW_OK) {
        hipError_t e = hipGraphInstantiate(&run.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { run.exec = nullptr; rc = hip_fail(e, "hipGraphInstantiate"); }
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) return finish(rc);
    for (Ticket *t : ts)
        if (wait_ready(*t, st) != hipSuccess) return finish(fail(SW_EDEVICE, "waiting for the submitted states"));
    t0 = now_s();
    for (Ticket *t : ts) { t->status = SW_TICKET_RUNNING; t->t_start = t0; }
    hipError_t e = hipGraphLaunch(run.exec, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return finish(hip_fail(e, "batched graph"));
    if (hipMemcpy(stamps.data(), d_stamps, stamps.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return finish(fail(SW_EDEVICE, "reading completion timestamps"));
    for (const PersistGroup &x : pg) {
        int32_t err = 0;
        if (hipMemcpy(&err, x.q.error, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess)
            return finish(fail(SW_EDEVICE, "reading the persistent batch status"));
        if (err) return finish(fail(SW_EDEVICE, "persistent batch: a dependency wait gave up"));
    }
    return finish(SW_OK);
}

// Solves no swept tile width divides: classic time-stepping through a plan.
int run_classic_ticket(Ticket &t, hipStream_t st)
{
    sw_plan *plan = nullptr;
    int rc = swept_plan(&t.prob, nullptr, &plan);
    if (rc) { t.status = SW_TICKET_FAILED; return rc; }
    t.status = SW_TICKET_RUNNING;
    t.t_start = now_s();
    if (wait_ready(t, st) != hipSuccess) rc = fail(SW_EDEVICE, "waiting for the submitted state");
    if (rc == SW_OK) rc = classic_solve(plan, t.state, st);
    if (rc == SW_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(SW_EDEVICE, "classic batch solve");
    swept_plan_destroy(plan);
    t.t_end = now_s();
    t.status = rc == SW_OK ? SW_TICKET_DONE : SW_TICKET_FAILED;
    return rc;
}

// ---------------------------------------------------------------- served mode

// One group (scheme, points per lane) of a served batch.  Each group ticks on
// its own stream, so a group of short phases advances as often as its launches
// allow.  Its device table of (solve, tile) items grows by appending admitted
// solves at tick boundaries and is rebuilt only when more than half of its
// items belong to finished solves; a device kernel advances every solve's phase
// after each tick, so no table is re-sent per tick.  Up to two ticks are in
// flight per group while the host admits, appends and retires.
struct ServeGroup {
    int scheme = 0, P = 1;
    hipStream_t stream = nullptr;
    SolveDesc *h_desc = nullptr, *d_desc = nullptr;   // pinned staging, device table
    int2 *h_items = nullptr, *d_items = nullptr;
    size_t cap_desc = 0, cap_items = 0;
    size_t ndesc = 0, nitems = 0, dead_items = 0;
    std::vector<Ticket *> members;     // desc index -> solve (finished ones stay until a rebuild)
    std::vector<Ticket *> pending;     // admitted, not yet in the table
    std::deque<hipEvent_t> inflight;   // completion events of enqueued ticks, oldest first
    std::vector<hipEvent_t> spare;
    int64_t enqueued = 0, done = 0;    // ticks
    int64_t active = 0;                // members still running
    int grid_cap = 1;

    static constexpr int kMaxInflight = 2;

    hipError_t init(int sch, int p)
    {
        scheme = sch;
        P = p;
        grid_cap = batch_blocks_per_cu(sch, p) * num_cus();
        return hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    }
    // Capacity for nd descriptors and ni items; reallocation waits for the stream
    // and drops the table contents (the caller rebuilds).
    hipError_t reserve(size_t nd, size_t ni, bool *reallocated)
    {
        *reallocated = false;
        if (nd <= cap_desc && ni <= cap_items) return hipSuccess;
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        const size_t cd = std::max<size_t>(std::max(nd, 2 * cap_desc), 64);
        const size_t ci = std::max<size_t>(std::max(ni, 2 * cap_items), 4096);
        release_tables();
        ndesc = nitems = dead_items = 0;
        *reallocated = true;
        // capacities are recorded only once every buffer exists
        if ((e = hipHostMalloc((void **)&h_desc, cd * sizeof(SolveDesc), 0)) == hipSuccess &&
            (e = hipMalloc(&d_desc, cd * sizeof(SolveDesc))) == hipSuccess &&
            (e = hipHostMalloc((void **)&h_items, ci * sizeof(int2), 0)) == hipSuccess &&
            (e = hipMalloc(&d_items, ci * sizeof(int2))) == hipSuccess) {
            cap_desc = cd;
            cap_items = ci;
            return hipSuccess;
        }
        release_tables();
        return e;
    }
    void release_tables()
    {
        if (h_desc) (void)hipHostFree(h_desc);
        if (d_desc) (void)hipFree(d_desc);
        if (h_items) (void)hipHostFree(h_items);
        if (d_items) (void)hipFree(d_items);
        h_desc = d_desc = nullptr;
        h_items = d_items = nullptr;
        cap_desc = cap_items = 0;
    }
    void destroy()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        for (hipEvent_t e : inflight) (void)hipEventDestroy(e);
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
        inflight.clear();
        spare.clear();
        release_tables();
        if (stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
    }
};

// The phase a solve runs at tick `tick` of its group.
int32_t phase_at_tick(const Ticket &t, int64_t tick)
{
    const int64_t p = tick - t.admit_tick;
    return (int32_t)std::min<int64_t>(std::max<int64_t>(p, 0), t.nphases);
}

void write_entries(ServeGroup &g, Ticket *t)
{
    SolveDesc d = make_desc(*t);
    d.phase = phase_at_tick(*t, g.enqueued);
    const int s = (int)g.ndesc;
    g.h_desc[g.ndesc++] = d;
    for (int64_t j = 0; j < t->geom.K; ++j) g.h_items[g.nitems++] = make_int2(s, (int)j);
}

// Put pending solves into the table before the next tick: append them, or
// rebuild the table without finished solves (after the stream drains) when
// those hold more than half of its items or the capacity must grow.
hipError_t prepare_table(ServeGroup &g)
{
    size_t add_d = g.pending.size(), add_i = 0;
    for (Ticket *t : g.pending) add_i += (size_t)t->geom.K;
    const bool compact = g.dead_items * 2 > g.nitems && g.dead_items > 0;
    if (add_d == 0 && !compact) return hipSuccess;
    hipError_t e;
    for (Ticket *t : g.pending) {
        t->admit_tick = g.enqueued;
        if ((e = wait_ready(*t, g.stream)) != hipSuccess) return e;   // before its first tick
    }
    bool realloc = false;
    if (!compact && (e = g.reserve(g.ndesc + add_d, g.nitems + add_i, &realloc)) != hipSuccess) return e;
    if (!compact && !realloc) {
        const size_t d0 = g.ndesc, i0 = g.nitems;
        for (Ticket *t : g.pending) { write_entries(g, t); g.members.push_back(t); }
        g.pending.clear();
        // appended ranges only; in-flight ticks read [0, d0) and [0, i0), which stay untouched
        if ((e = hipMemcpyAsync(g.d_desc + d0, g.h_desc + d0, (g.ndesc - d0) * sizeof(SolveDesc),
                                hipMemcpyHostToDevice, g.stream)) != hipSuccess) return e;
        return hipMemcpyAsync(g.d_items + i0, g.h_items + i0, (g.nitems - i0) * sizeof(int2),
                              hipMemcpyHostToDevice, g.stream);
    }
    // rebuild: the staging buffers are rewritten, so nothing may still read them
    if ((e = hipStreamSynchronize(g.stream)) != hipSuccess) return e;
    std::vector<Ticket *> keep;
    size_t nd = add_d, ni = add_i;
    for (Ticket *t : g.members)
        if (t->status == SW_TICKET_RUNNING) { keep.push_back(t); ++nd; ni += (size_t)t->geom.K; }
    if ((e = g.reserve(nd, ni, &realloc)) != hipSuccess) return e;
    g.ndesc = g.nitems = g.dead_items = 0;
    g.members.clear();
    for (Ticket *t : keep) { write_entries(g, t); g.members.push_back(t); }
    for (Ticket *t : g.pending) { write_entries(g, t); g.members.push_back(t); }
    g.pending.clear();
    if ((e = hipMemcpyAsync(g.d_desc, g.h_desc, g.ndesc * sizeof(SolveDesc), hipMemcpyHostToDevice,
                            g.stream)) != hipSuccess) return e;
    return hipMemcpyAsync(g.d_items, g.h_items, g.nitems * sizeof(int2), hipMemcpyHostToDevice, g.stream);
}

hipError_t enqueue_tick(ServeGroup &g)
{
    hipError_t e = launch_batch_phase(g.scheme, g.P, g.d_desc, g.d_items, (int64_t)g.nitems, -1,
                                      (int)std::min<int64_t>((int64_t)g.nitems, g.grid_cap), g.stream);
    if (e == hipSuccess) e = launch_advance_phases(g.d_desc, (int64_t)g.ndesc, g.stream);
    if (e != hipSuccess) return e;
    hipEvent_t ev;
    if (!g.spare.empty()) { ev = g.spare.back(); g.spare.pop_back(); }
    else if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev, g.stream)) != hipSuccess) { g.spare.push_back(ev); return e; }
    g.inflight.push_back(ev);
    g.enqueued += 1;
    return hipSuccess;
}

void retire(sw_batch *b, Ticket *t, int32_t status, double t_done)
{
    t->status = status;
    t->t_end = t_done;
    release_events(t);
    b->arena.release(t->edges, (size_t)t->geom.edge_doubles * sizeof(double));
    t->edges = nullptr;
    b->resident -= t->bytes;
    b->nresident -= 1;
}

// Collect finished ticks; solves whose last phase has run are done.  Returns
// true if anything finished.  Called with b->mu held.
bool reap(sw_batch *b, ServeGroup &g, hipError_t *err)
{
    bool any = false;
    while (!g.inflight.empty()) {
        hipError_t q = hipEventQuery(g.inflight.front());
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) { *err = q; break; }
        g.spare.push_back(g.inflight.front());
        g.inflight.pop_front();
        g.done += 1;
        any = true;
    }
    if (!any) return false;
    const double t_done = now_s();
    for (Ticket *t : g.members) {
        if (t->status != SW_TICKET_RUNNING || t->admit_tick + t->nphases > g.done) continue;
        retire(b, t, SW_TICKET_DONE, t_done);
        g.dead_items += (size_t)t->geom.K;
        g.active -= 1;
    }
    return true;
}

void fail_group(sw_batch *b, ServeGroup &g, hipError_t e)
{
    // nothing queued on the group may still write edges that are about to be reused
    (void)hipStreamSynchronize(g.stream);
    for (hipEvent_t ev : g.inflight) g.spare.push_back(ev);
    g.inflight.clear();
    const double t = now_s();
    for (Ticket *x : g.members)
        if (x->status == SW_TICKET_RUNNING) retire(b, x, SW_TICKET_FAILED, t);
    for (Ticket *x : g.pending)
        if (x->status == SW_TICKET_RUNNING) retire(b, x, SW_TICKET_FAILED, t);
    g.members.clear();
    g.pending.clear();
    g.active = 0;
    g.ndesc = g.nitems = g.dead_items = 0;
    b->worker_error = hipGetErrorString(e);
}

void serve_loop(sw_batch *b)
{
    (void)hipSetDevice(b->device);
    std::map<std::pair<int, int>, ServeGroup> groups;
    std::vector<Ticket *> classic_running;   // classic fallbacks in flight on b->stream
    for (;;) {
        std::vector<Ticket *> classic_now;
        bool stopping = false, busy = false;
        {
            std::lock_guard<std::mutex> lk(b->mu);
            // admit in arrival order while memory and slots allow (head-of-line blocking keeps FIFO)
            while (!b->queue.empty()) {
                Ticket *t = find_ticket(b, b->queue.front());
                if (!t || t->status != SW_TICKET_QUEUED) { b->queue.pop_front(); continue; }
                const bool slots_full = b->cfg.max_slots > 0 && b->nresident >= b->cfg.max_slots;
                if (slots_full || b->resident + t->bytes > b->cfg.budget_bytes) break;
                if (!t->swept) {   // classic fallback: admitted like the others, run beside them
                    t->status = SW_TICKET_RUNNING;
                    t->t_start = now_s();
                    b->resident += t->bytes;
                    b->nresident += 1;
                    classic_now.push_back(t);
                    b->queue.pop_front();
                    continue;
                }
                t->edges = (double *)b->arena.alloc((size_t)t->geom.edge_doubles * sizeof(double));
                if (!t->edges) break;  // retry when memory frees up
                t->nphases = phase_count(t->geom.Q, t->geom.rem);
                t->status = SW_TICKET_RUNNING;
                t->t_start = now_s();
                b->resident += t->bytes;
                b->nresident += 1;
                ServeGroup &g = groups[{t->prob.scheme, t->P}];
                if (!g.stream) {
                    hipError_t e = g.init(t->prob.scheme, t->P);
                    if (e != hipSuccess) { retire(b, t, SW_TICKET_FAILED, now_s()); b->worker_error = hipGetErrorString(e); b->queue.pop_front(); continue; }
                }
                g.pending.push_back(t);
                g.active += 1;
                b->queue.pop_front();
            }
            stopping = b->stop;
        }
        // classic fallbacks run on the batch's own stream, in flight beside the groups' ticks
        for (Ticket *t : classic_now) {
            int rc = swept_plan(&t->prob, nullptr, &t->plan);
            if (rc == SW_OK && wait_ready(*t, b->stream) != hipSuccess) rc = SW_EDEVICE;
            if (rc == SW_OK) rc = classic_solve(t->plan, t->state, b->stream);
            if (rc == SW_OK && (hipEventCreateWithFlags(&t->finished, hipEventDisableTiming) != hipSuccess ||
                                hipEventRecord(t->finished, b->stream) != hipSuccess))
                rc = SW_EDEVICE;
            std::lock_guard<std::mutex> lk(b->mu);
            if (rc == SW_OK) {
                classic_running.push_back(t);
            } else {
                (void)hipStreamSynchronize(b->stream);
                swept_plan_destroy(t->plan);
                t->plan = nullptr;
                retire(b, t, SW_TICKET_FAILED, now_s());
                b->cv.notify_all();
            }
        }
        for (size_t k = 0; k < classic_running.size();) {
            Ticket *t = classic_running[k];
            const hipError_t q = hipEventQuery(t->finished);
            if (q == hipErrorNotReady) { ++k; continue; }
            swept_plan_destroy(t->plan);
            t->plan = nullptr;
            std::lock_guard<std::mutex> lk(b->mu);
            retire(b, t, q == hipSuccess ? SW_TICKET_DONE : SW_TICKET_FAILED, now_s());
            b->cv.notify_all();
            classic_running.erase(classic_running.begin() + (long)k);
            classic_now.push_back(t);   // counts as progress
        }
        bool progressed = !classic_now.empty();
        for (auto &kv : groups) {
            ServeGroup &g = kv.second;
            hipError_t e = hipSuccess;
            {
                std::lock_guard<std::mutex> lk(b->mu);
                if (reap(b, g, &e)) { progressed = true; b->ticks += 1; b->cv.notify_all(); }
                if (e != hipSuccess) { fail_group(b, g, e); b->cv.notify_all(); continue; }
            }
            while ((int)g.inflight.size() < ServeGroup::kMaxInflight && g.active > 0) {
                e = prepare_table(g);
                if (e == hipSuccess) e = enqueue_tick(g);
                if (e != hipSuccess) {
                    std::lock_guard<std::mutex> lk(b->mu);
                    fail_group(b, g, e);
                    b->cv.notify_all();
                    break;
                }
                progressed = true;
            }
            if (!g.inflight.empty() || g.active > 0) busy = true;
        }
        if (!classic_running.empty()) busy = true;
        if (!busy) {
            std::unique_lock<std::mutex> lk(b->mu);
            if (b->queue.empty() && (stopping || b->stop)) break;
            if (b->queue.empty()) b->cv.wait_for(lk, std::chrono::milliseconds(2));
        } else if (!progressed) {
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    for (auto &kv : groups) kv.second.destroy();
}

int serve_start(sw_batch *b)
{
    BHIP(hipGetDevice(&b->device));
    BHIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    b->worker = std::thread(serve_loop, b);
    return SW_OK;
}

void serve_stop(sw_batch *b)
{
    {
        std::lock_guard<std::mutex> lk(b->mu);
        b->stop = true;
        // queued tickets that never started are cancelled
        for (uint64_t id : b->queue) {
            Ticket *t = find_ticket(b, id);
            if (t && t->status == SW_TICKET_QUEUED) t->status = SW_TICKET_CANCELLED;
        }
        b->queue.clear();
        b->cv.notify_all();
    }
    if (b->worker.joinable()) b->worker.join();
    if (b->stream) (void)hipStreamDestroy(b->stream);
    b->stream = nullptr;
}

}  // namespace

extern "C" {

int batch_create(const sw_batch_config *config, sw_batch **out)
{
    if (!config || !out) return fail(SW_EINVAL, "NULL argument");
    if (config->budget_bytes <= 0 || config->max_slots < 0 ||
        (config->flags & ~(SW_BATCH_SERVE | SW_BATCH_PERSISTENT)) != 0 || config->reserved != 0 ||
        ((config->flags & SW_BATCH_SERVE) && (config->flags & SW_BATCH_PERSISTENT)))
        return fail(SW_EINVAL, "invalid batch configuration");
    const int ppl = config->points_per_lane;
    if (ppl != 0 && ppl != 1 && ppl != 2 && ppl != 4 && ppl != 8)
        return fail(SW_EINVAL, "points_per_lane must be 0, 1, 2, 4 or 8");
    sw_batch *b = new (std::nothrow) sw_batch();
    if (!b) return fail(SW_ENOMEM, "batch allocation failed");
    b->cfg = *config;
    b->serve = (config->flags & SW_BATCH_SERVE) != 0;
    if (b->serve) {
        int rc = serve_start(b);
        if (rc) { delete b; return rc; }
    }
    *out = b;
    return SW_OK;
}

namespace {

int submit_ticket(sw_batch *b, const sw_problem *problem, double *d_state, hipStream_t *ready_on,
                  uint64_t *ticket)
{
    if (!b || !ticket) return fail(SW_EINVAL, "NULL argument");
    std::string err;
    int rc = validate_problem(problem, &err);
    if (rc) return fail(rc, err);
    if ((rc = check_device_ptr(d_state))) return rc;
    Ticket t;
    t.swept = batch_shape(*problem, b->cfg.points_per_lane, &t.P, &t.geom) && problem->nsteps > 0;
    const int64_t bytes = resident_bytes(*problem, t.swept, t.geom);
    if (bytes > b->cfg.budget_bytes) return fail(SW_EBUSY, "solve larger than the batch memory budget");
    if (ready_on) {
        // the solve's first launch waits for the work the caller has queued on its stream
        if (hipEventCreateWithFlags(&t.ready, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SW_EDEVICE, "event creation failed");
        }
        if (hipEventRecord(t.ready, *ready_on) != hipSuccess) {
            (void)hipEventDestroy(t.ready);
            return fail(SW_EDEVICE, "recording the submitting stream failed");
        }
    }
    std::lock_guard<std::mutex> lk(b->mu);
    t.id = b->next_id++;
    t.prob = *problem;
    t.state = d_state;
    t.bytes = bytes;
    t.t_submit = now_s();
    b->tickets.push_back(t);
    *ticket = t.id;
    if (b->serve) {
        b->queue.push_back(t.id);
        b->cv.notify_all();
    }
    return SW_OK;
}

}  // namespace

int batch_submit(sw_batch *b, const sw_problem *problem, double *d_state, uint64_t *ticket)
{
    return submit_ticket(b, problem, d_state, nullptr, ticket);
}

int batch_submit_async(sw_batch *b, const sw_problem *problem, double *d_state, void *hip_stream,
                       uint64_t *ticket)
{
    hipStream_t st = (hipStream_t)hip_stream;
    return submit_ticket(b, problem, d_state, &st, ticket);
}

int batch_run(sw_batch *b, void *hip_stream)
{
    if (!b) return fail(SW_EINVAL, "NULL batch");
    if (b->serve) return fail(SW_EINVAL, "batch_run is for ensemble batches; served batches run by themselves");
    std::lock_guard<std::mutex> lk(b->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    int rc_all = SW_OK;
    // admit queued tickets in submission order, in waves that fit the budget and slots
    size_t i = 0;
    while (i < b->tickets.size()) {
        std::vector<Ticket *> wave;
        int64_t used = 0;
        for (; i < b->tickets.size(); ++i) {
            Ticket &t = b->tickets[i];
            if (t.status != SW_TICKET_QUEUED) continue;
            if (!t.swept) {
                if (t.prob.nsteps == 0) { t.status = SW_TICKET_DONE; t.t_start = t.t_end = now_s(); continue; }
                int rc = run_classic_ticket(t, st);
                release_events(&t);
                if (rc && rc_all == SW_OK) rc_all = rc;
                continue;
            }
            const bool slots_full = b->cfg.max_slots > 0 && (int)wave.size() >= b->cfg.max_slots;
            if (!wave.empty() && (slots_full || used + t.bytes > b->cfg.budget_bytes)) break;
            wave.push_back(&t);
            used += t.bytes;
        }
        if (!wave.empty()) {
            int rc = run_ensemble(b, wave, st);
            if (rc && rc_all == SW_OK) rc_all = rc;
        }
    }
    return rc_all;
}

int batch_poll(sw_batch *b, uint64_t ticket, int32_t *status_out)
{
    if (!b || !status_out) return fail(SW_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(b->mu);
    Ticket *t = find_ticket(b, ticket);
    if (!t) return fail(SW_EINVAL, "unknown ticket");
    *status_out = t->status;
    return SW_OK;
}

int batch_ticket_info(sw_batch *b, uint64_t ticket, sw_ticket_info *out)
{
    if (!b || !out) return fail(SW_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(b->mu);
    Ticket *t = find_ticket(b, ticket);
    if (!t) return fail(SW_EINVAL, "unknown ticket");
    sw_ticket_info i;
    std::memset(&i, 0, sizeof(i));
    i.status = t->status;
    i.swept = t->swept ? 1 : 0;
    i.width = t->swept ? t->geom.w : 0;
    i.phases = t->swept ? phase_count(t->geom.Q, t->geom.rem) : 0;
    i.submit_s = t->t_submit;
    i.start_s = t->t_start;
    i.end_s = t->t_end;
    i.resident_bytes = t->bytes;
    *out = i;
    return SW_OK;
}

int batch_wait(sw_batch *b, uint64_t ticket, int64_t timeout_us)
{
    if (!b) return fail(SW_EINVAL, "NULL batch");
    const auto t0 = Clock::now();
    std::unique_lock<std::mutex> lk(b->mu);
    for (;;) {
        Ticket *t = find_ticket(b, ticket);
        if (!t) return fail(SW_EINVAL, "unknown ticket");
        if (t->status == SW_TICKET_DONE || t->status == SW_TICKET_CANCELLED) return SW_OK;
        if (t->status == SW_TICKET_FAILED) return fail(SW_EDEVICE, "ticket failed");
        if (!b->serve && t->status == SW_TICKET_QUEUED)
            return fail(SW_ENOTREADY, "ticket is queued; call batch_run");
        const auto waited = std::chrono::duration_cast<std::chrono::microseconds>(Clock::now() - t0).count();
        if (timeout_us >= 0 && waited >= timeout_us) return fail(SW_ENOTREADY, "ticket not finished");
        b->cv.wait_for(lk, std::chrono::microseconds(200));
    }
}

int batch_cancel(sw_batch *b, uint64_t ticket)
{
    if (!b) return fail(SW_EINVAL, "NULL batch");
    std::lock_guard<std::mutex> lk(b->mu);
    Ticket *t = find_ticket(b, ticket);
    if (!t) return fail(SW_EINVAL, "unknown ticket");
    if (t->status != SW_TICKET_QUEUED) return fail(SW_EBUSY, "ticket already started");
    t->status = SW_TICKET_CANCELLED;
    if (b->serve) {
        auto it = std::find(b->queue.begin(), b->queue.end(), ticket);
        if (it != b->queue.end()) b->queue.erase(it);
    }
    b->cv.notify_all();
    return SW_OK;
}

void batch_destroy(sw_batch *b)
{
    if (!b) return;
    if (b->serve) serve_stop(b);
    {
        std::lock_guard<std::mutex> lk(b->mu);
        for (Ticket &t : b->tickets) release_events(&t);
        b->arena.destroy();
    }
    delete b;
}

}  // extern "C"
