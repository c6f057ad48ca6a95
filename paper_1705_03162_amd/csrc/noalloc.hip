// Allocation-free swept solve (swept_solve_noalloc in include/swept.h).
//
// The swept decomposition needs device memory beyond the caller's state only for
// its edge slots.  Here they live in a file-scope device array of fixed size
// instead of a plan's hipMalloc'd buffer, and the phases are enqueued straight
// onto the caller's stream (no graph is instantiated), so the call allocates
// nothing on the device or through a library.  Each device holds its own copy of
// the array for the life of the process; every call on a device shares it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "api_internal.hpp"
#include "kernels.hpp"
#include "plan_core.hpp"
#include "swept.h"
#include "tune.hpp"

using namespace sw;

namespace {

constexpr int64_t kScratchBytes = SW_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

// Edge slots of swept_solve_noalloc.  In host code this name is only a stand-in:
// kernels receive the device address taken once per device below.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved on the first call
// per device (the device must be current).
int scratch_address(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(SW_EDEVICE, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        }
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SW_OK;
}

}  // namespace

extern "C" int swept_solve_noalloc(const sw_problem *problem, const sw_tuning *tuning, double *d_state,
                                   void *hip_stream)
{
    std::string err;
    int rc = validate_problem(problem, &err);
    if (rc) return fail(rc, err);
    if (tuning && (tuning->flags & ~SW_TUNE_NO_GRAPH))
        return fail(SW_EINVAL, "swept_solve_noalloc takes no flags but SW_TUNE_NO_GRAPH (it never builds a graph)");
    int width = tuning ? tuning->width : 0;
    int threads = tuning ? tuning->threads : 0;
    if ((width == 0) != (threads == 0)) return fail(SW_EINVAL, "give both width and threads, or neither");
    if (width == 0 && !tuned_shape(*problem, &width, &threads)) default_shape(*problem, &width, &threads);
    Geom g;
    if ((rc = make_geom(*problem, width, threads, &g, &err))) return fail(rc, err);
    if (!g.swept_ok) return fail(SW_EUNSUPPORTED, "no legal swept tile width divides n");
    const int64_t need = g.edge_doubles * (int64_t)sizeof(double);
    if (need > kScratchBytes)
        return fail(SW_EINVAL, "problem needs " + std::to_string(need) + " bytes of edge scratch; the static scratch of "
                                   "swept_solve_noalloc holds " + std::to_string(kScratchBytes) + " (use swept_plan)");
    if ((rc = check_device_ptr(d_state))) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    double *edges = nullptr;
    if ((rc = scratch_address(dev, &edges))) return rc;
    if (g.levels == 0) return SW_OK;
    const Consts c = make_consts(*problem);
    hipStream_t st = (hipStream_t)hip_stream;
    const int count = phase_count(g.Q, g.rem);
    for (int p = 0; p < count; ++p) {
        Phase ph;
        phase_at(g.Q, g.rem, g.H, p, ph.kind, ph.levels, ph.offset);
        const TileArgs a = make_tile_args(g, c, ph, d_state, edges);
        e = launch_swept_phase(g.scheme, g.P, g.threads, a, st);
        if (e != hipSuccess) return hip_fail(e, "swept kernel launch");
    }
    return SW_OK;
}
