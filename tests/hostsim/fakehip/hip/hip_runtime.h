// Test-only stand-in for the HIP runtime, so that the library's host code (the
// batched and served solve scheduler in batch.hip) can be compiled with g++ and
// run on a CPU.  "Device" memory is host memory.  Streams are lazy: work enqueued
// on a stream runs only when the host waits for it (stream or event
// synchronisation, or an event query, which runs one queued item per call), so
// up to several ticks are genuinely in flight while the host keeps scheduling,
// and an asynchronous copy reads its source when it runs, not when it was
// enqueued.  Graph capture records a stream's work and replays it on launch.
#pragma once

#include <chrono>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <vector>

typedef int hipError_t;
enum : int {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
};
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount, hipDeviceAttributeWallClockRate };
enum : unsigned { hipStreamNonBlocking = 1u, hipEventDisableTiming = 2u };

struct int2 { int x, y; };
inline int2 make_int2(int x, int y) { return int2{x, y}; }

namespace fakehip {

using Work = std::function<void()>;

struct Stream {
    std::deque<Work> queue;
    uint64_t issued = 0, executed = 0;
    bool capturing = false;
    std::vector<Work> captured;
    Stream *capture_into = nullptr;    // joined another stream's capture (fork by event)
    std::vector<Stream *> joined;      // streams that joined this stream's capture
};
// An event recorded during a capture only orders captured work; the stand-in
// graph runs its work in capture order, which is one valid order of the forks.
struct Event { Stream *stream = nullptr; uint64_t ticket = 0; Stream *capture_origin = nullptr; };
struct Graph { std::vector<Work> work; };

inline std::recursive_mutex &lock()
{
    static std::recursive_mutex m;
    return m;
}
inline Stream *resolve(Stream *s)
{
    static Stream null_stream;
    return s ? s : &null_stream;
}
inline void run_one(Stream *s)
{
    Work w = std::move(s->queue.front());
    s->queue.pop_front();
    w();
    s->executed += 1;
}
inline void run_until(Stream *s, uint64_t ticket)
{
    while (s->executed < ticket && !s->queue.empty()) run_one(s);
}
inline void enqueue(Stream *s, Work w)
{
    std::lock_guard<std::recursive_mutex> lk(lock());
    s = resolve(s);
    if (s->capture_into) { s->capture_into->captured.push_back(std::move(w)); return; }
    if (s->capturing) { s->captured.push_back(std::move(w)); return; }
    s->queue.push_back(std::move(w));
    s->issued += 1;
}

}  // namespace fakehip

typedef fakehip::Stream *hipStream_t;
typedef fakehip::Event *hipEvent_t;
typedef fakehip::Graph *hipGraph_t;
typedef fakehip::Graph *hipGraphExec_t;

inline const char *hipGetErrorString(hipError_t) { return "error (CPU stand-in runtime)"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int)
{
    *v = a == hipDeviceAttributeMultiprocessorCount ? 4 : 100000;   // CUs; wall clock in kHz
    return hipSuccess;
}

inline hipError_t hipMalloc(void **p, size_t bytes)
{
    *p = std::aligned_alloc(256, (bytes + 255) / 256 * 256 + 256);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
template <class T> inline hipError_t hipMalloc(T **p, size_t bytes) { return hipMalloc((void **)p, bytes); }
inline hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostMalloc(void **p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
inline hipError_t hipHostFree(void *p) { return hipFree(p); }

inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = new fakehip::Stream(); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> lk(fakehip::lock());
    s = fakehip::resolve(s);
    fakehip::run_until(s, s->issued);
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s)
{
    if (!s) return hipSuccess;
    hipStreamSynchronize(s);
    delete s;
    return hipSuccess;
}

inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = new fakehip::Event(); return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) { return hipEventCreateWithFlags(e, 0); }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> lk(fakehip::lock());
    s = fakehip::resolve(s);
    if (s->capturing || s->capture_into) {
        e->stream = nullptr;
        e->capture_origin = s->capturing ? s : s->capture_into;
        return hipSuccess;
    }
    e->capture_origin = nullptr;
    e->stream = s;
    e->ticket = s->issued;
    return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t e)
{
    std::lock_guard<std::recursive_mutex> lk(fakehip::lock());
    if (!e->stream || e->stream->executed >= e->ticket) return hipSuccess;
    fakehip::run_one(e->stream);   // one queued item per query: the work completes over time
    return e->stream->executed >= e->ticket ? hipSuccess : hipErrorNotReady;
}
inline hipError_t hipEventSynchronize(hipEvent_t e)
{
    std::lock_guard<std::recursive_mutex> lk(fakehip::lock());
    if (e->stream) fakehip::run_until(e->stream, e->ticket);
    return hipSuccess;
}
inline hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned)
{
    std::lock_guard<std::recursive_mutex> lk(fakehip::lock());
    s = fakehip::resolve(s);
    if (e->capture_origin) {   // fork: s joins the capture; join back into the origin: nothing to do
        if (s != e->capture_origin && !s->capture_into) {
            s->capture_into = e->capture_origin;
            e->capture_origin->joined.push_back(s);
        }
        return hipSuccess;
    }
    return hipEventSynchronize(e);
}

inline hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s)
{
    fakehip::enqueue(s, [=] { std::memcpy(dst, src, bytes); });
    return hipSuccess;
}
inline hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind k)
{
    hipMemcpyAsync(dst, src, bytes, k, nullptr);
    return hipStreamSynchronize(nullptr);
}

inline hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    s = fakehip::resolve(s);
    s->capturing = true;
    s->captured.clear();
    return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g)
{
    s = fakehip::resolve(s);
    *g = new fakehip::Graph{std::move(s->captured)};
    s->captured.clear();
    s->capturing = false;
    for (fakehip::Stream *j : s->joined) j->capture_into = nullptr;
    s->joined.clear();
    return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, char *, size_t)
{
    *x = new fakehip::Graph(*g);
    return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s)
{
    for (const fakehip::Work &w : x->work) fakehip::enqueue(s, w);
    return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t x) { delete x; return hipSuccess; }
