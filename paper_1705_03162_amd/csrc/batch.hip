// Batched solves (batch_* entry points of include/swept.h).
//
// A batch holds tickets for independent solves on caller-owned device states.
// Admission is by a device-memory budget: a resident solve holds its state plus
// its edge slots and scratch (about 3 n nvars doubles).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "api_internal.hpp"
#include "plan_core.hpp"
#include "swept.h"

using namespace sw;

namespace {

struct Ticket {
    uint64_t id = 0;
    sw_problem prob{};
    double *state = nullptr;
    int32_t status = SW_TICKET_QUEUED;
    int64_t bytes = 0;
    sw_plan *plan = nullptr;
};

int64_t resident_bytes(const sw_problem &p)
{
    return 3 * p.n * (int64_t)scheme_nvars(p.scheme) * (int64_t)sizeof(double);
}

}  // namespace

struct sw_batch {
    sw_batch_config cfg{};
    std::vector<Ticket> tickets;
    uint64_t next_id = 1;
    std::mutex mu;
};

extern "C" {

int batch_create(const sw_batch_config *config, sw_batch **out)
{
    if (!config || !out) return fail(SW_EINVAL, "NULL argument");
    if (config->budget_bytes <= 0 || config->max_slots < 0 || config->flags != 0)
        return fail(SW_EINVAL, "invalid batch configuration");
    sw_batch *b = new (std::nothrow) sw_batch();
    if (!b) return fail(SW_ENOMEM, "batch allocation failed");
    b->cfg = *config;
    *out = b;
    return SW_OK;
}

int batch_submit(sw_batch *b, const sw_problem *problem, double *d_state, uint64_t *ticket)
{
    if (!b || !ticket) return fail(SW_EINVAL, "NULL argument");
    std::string err;
    int rc = validate_problem(problem, &err);
    if (rc) return fail(rc, err);
    if ((rc = check_device_ptr(d_state))) return rc;
    const int64_t bytes = resident_bytes(*problem);
    if (bytes > b->cfg.budget_bytes) return fail(SW_EBUSY, "solve larger than the batch memory budget");
    std::lock_guard<std::mutex> lk(b->mu);
    Ticket t;
    t.id = b->next_id++;
    t.prob = *problem;
    t.state = d_state;
    t.bytes = bytes;
    b->tickets.push_back(t);
    *ticket = t.id;
    return SW_OK;
}

int batch_run(sw_batch *b, void *hip_stream)
{
    if (!b) return fail(SW_EINVAL, "NULL batch");
    std::lock_guard<std::mutex> lk(b->mu);
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<Ticket *> running;
    int64_t in_use = 0;
    auto drain = [&]() -> int {
        if (running.empty()) return SW_OK;
        hipError_t e = hipStreamSynchronize(st);
        for (Ticket *t : running) {
            swept_plan_destroy(t->plan);
            t->plan = nullptr;
            t->status = e == hipSuccess ? SW_TICKET_DONE : SW_TICKET_FAILED;
        }
        running.clear();
        in_use = 0;
        return e == hipSuccess ? SW_OK : hip_fail(e, "batch solve");
    };
    for (Ticket &t : b->tickets) {
        if (t.status != SW_TICKET_QUEUED) continue;
        const bool slots_full = b->cfg.max_slots > 0 && (int)running.size() >= b->cfg.max_slots;
        if (slots_full || in_use + t.bytes > b->cfg.budget_bytes) {
            int rc = drain();
            if (rc) return rc;
        }
        int rc = swept_plan(&t.prob, nullptr, &t.plan);
        if (rc) { t.status = SW_TICKET_FAILED; continue; }
        t.status = SW_TICKET_RUNNING;
        sw_plan_info info;
        swept_plan_info(t.plan, &info);
        rc = info.swept_ok ? swept_solve(t.plan, t.state, st) : classic_solve(t.plan, t.state, st);
        if (rc) { t.status = SW_TICKET_FAILED; swept_plan_destroy(t.plan); t.plan = nullptr; continue; }
        running.push_back(&t);
        in_use += t.bytes;
    }
    return drain();
}

int batch_poll(sw_batch *b, uint64_t ticket, int32_t *status_out)
{
    if (!b || !status_out) return fail(SW_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(b->mu);
    for (const Ticket &t : b->tickets)
        if (t.id == ticket) { *status_out = t.status; return SW_OK; }
    return fail(SW_EINVAL, "unknown ticket");
}

int batch_wait(sw_batch *b, uint64_t ticket, int64_t timeout_us)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        int32_t s = 0;
        int rc = batch_poll(b, ticket, &s);
        if (rc) return rc;
        if (s == SW_TICKET_DONE || s == SW_TICKET_CANCELLED) return SW_OK;
        if (s == SW_TICKET_FAILED) return fail(SW_EDEVICE, "ticket failed");
        const auto us = std::chrono::duration_cast<std::chrono::microseconds>(
                            std::chrono::steady_clock::now() - t0).count();
        if (timeout_us >= 0 && us >= timeout_us) return fail(SW_ENOTREADY, "ticket not finished");
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

int batch_cancel(sw_batch *b, uint64_t ticket)
{
    if (!b) return fail(SW_EINVAL, "NULL batch");
    std::lock_guard<std::mutex> lk(b->mu);
    for (Ticket &t : b->tickets)
        if (t.id == ticket) {
            if (t.status == SW_TICKET_QUEUED) { t.status = SW_TICKET_CANCELLED; return SW_OK; }
            return fail(SW_EBUSY, "ticket already started");
        }
    return fail(SW_EINVAL, "unknown ticket");
}

void batch_destroy(sw_batch *b)
{
    if (!b) return;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        for (Ticket &t : b->tickets) swept_plan_destroy(t.plan);
    }
    delete b;
}

}  // extern "C"
