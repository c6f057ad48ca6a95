// Internal declarations shared by the C-interface translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "hybrid.hpp"
#include "plan_core.hpp"
#include "swept.h"

struct sw_plan {
    sw_problem prob{};
    sw::Geom geom;
    sw::Consts consts{};
    std::vector<sw::Phase> phases;
    int tflags = 0;
    bool lds_ready = false;       // Shared variant: kernel's LDS limit raised
    int device = -1;              // device of the scratch buffers (set on first solve)
    double *d_edges = nullptr;    // 2K edge slots
    double *d_tmp = nullptr;      // classic ping-pong / predictor buffer
    int *d_flag = nullptr;        // non-finite check
    hipStream_t cap = nullptr;    // private stream used only for graph capture
    hipEvent_t done = nullptr;    // completion of the last solve enqueued with this plan
    hipGraphExec_t swept_exec = nullptr, swept_body = nullptr, swept_tail = nullptr;
    const double *swept_state = nullptr;  // state pointer baked into the swept graphs
    int64_t body_reps = 0;
    size_t tail_first = 0;
    hipGraphExec_t classic_exec = nullptr;
    const double *classic_state = nullptr;
    // Hybrid variant (SW_TUNE_HYBRID): pinned host copies of the straddling tile (slot a,
    // slot b, top level), the stream that moves them and runs the host computation, and
    // one host-tile record per phase (read by the host callbacks)
    double *h_hybrid = nullptr;
    hipStream_t hyb_stream = nullptr;
    hipEvent_t hyb_ready = nullptr, hyb_done = nullptr;
    std::vector<sw::HybridTile> hyb_tiles;
    std::mutex mu;
};

namespace sw {

extern thread_local std::string g_last_error;
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *where);
int check_device_ptr(const void *p);

// Makes `dev` the current device for the guard's lifetime (no-op for dev < 0).
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (dev < 0) return;
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace sw
