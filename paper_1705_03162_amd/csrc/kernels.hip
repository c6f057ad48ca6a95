// HIP kernels for gfx950 besides the swept tile kernel: the classic
// one-sub-step-per-launch kernel, the Shared-variant swept tile (lds_tile.hpp), the
// served-batch phase counter, the device clock stamp and the non-finite scan, plus the
// dispatch of every launch by scheme.  The swept tile kernel and its batched form are in swept_tile.hpp,
// instantiated per scheme in tiles_heat.hip, tiles_ks.hip and tiles_euler.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "lds_tile.hpp"

namespace sw {

namespace {

// Classic: one thread per point, one launch per sub-step (Sec. 5.1).  For the
// final RK2 stage `dst` holds u^m and is updated in place (the listing's +=).
// MAXT bounds the work-group size it is compiled for (256, or 1024 for larger
// blocks, which leaves each lane fewer registers).
template <class Sch, int MAXT>
__global__ __launch_bounds__(MAXT) void classic_level(const double *__restrict__ src, double *dst,
                                                     int64_t n, int bc, int predictor, Consts c)
{
    constexpr int NV = Sch::NV, R = Sch::R;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ext[NV][1 + 2 * R];
    const bool tiny = n <= 2 * R;  // the stencil may wrap more than once
#pragma unroll
    for (int d = 0; d < 2 * R + 1; ++d) {
        int64_t jj = i - R + d;
        const bool inside = jj >= 0 && jj < n;
        const bool dirichlet = bc == BC_DIRICHLET;
        if (dirichlet) jj = jj < 0 ? 0 : (jj >= n ? n - 1 : jj);
        else if (bc == BC_REFLECTIVE) jj = jj < 0 ? -jj : (jj >= n ? 2 * (n - 1) - jj : jj);  // R == 1, n >= 2
        else if (tiny) jj = ((jj % n) + n) % n;
        else jj = jj < 0 ? jj + n : (jj >= n ? jj - n : jj);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double val = src[(int64_t)v * n + jj];
            ext[v][d] = (inside || !dirichlet) ? val : (d < R ? c.ghost_l[v] : c.ghost_r[v]);
        }
    }
    double out[NV][1];
    const bool in_place = Sch::S == 2 && !predictor;
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v][0] = in_place ? dst[(int64_t)v * n + i] : 0.0;
    const bool all[1] = {true};
    Sch::template level<1>(out, ext, predictor != 0, c, all);
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[(int64_t)v * n + i] = out[v][0];
}

// Served batches: after a tick, every solve in the table moves to its next phase.
__global__ void advance_phases(SolveDesc *desc, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && desc[i].phase < desc[i].nphases) desc[i].phase += 1;
}

__global__ void zero_words(uint32_t *p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void stamp_kernel(uint64_t *stamps, int idx)
{
    if (threadIdx.x == 0) stamps[idx] = wall_clock64();
}

// Flag non-finite values (optional post-solve check).
__global__ void nonfinite_scan(const double *x, int64_t count, int *flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_swept_phase(int scheme, int P, int threads, const TileArgs &a, hipStream_t st, int64_t tiles)
{
    if (tiles < 0 || tiles > a.K) tiles = a.K;
    if (tiles <= 0) return hipSuccess;
    if (scheme == 0) return swept_phase_for<Heat>(P, threads, a, st, tiles);
    if (scheme == 1) return swept_phase_for<KS>(P, threads, a, st, tiles);
    return swept_phase_for<Euler>(P, threads, a, st, tiles);
}

hipError_t prepare_lds_phase(int scheme)
{
    if (scheme == 0) return lds_prepare_for<Heat>();
    if (scheme == 1) return lds_prepare_for<KS>();
    return lds_prepare_for<Euler>();
}

hipError_t launch_lds_phase(int scheme, int threads, const TileArgs &a, hipStream_t st, int64_t tiles)
{
    if (tiles < 0 || tiles > a.K) tiles = a.K;
    if (tiles <= 0) return hipSuccess;
    if (scheme == 0) return lds_phase_for<Heat>(threads, a, st, tiles);
    if (scheme == 1) return lds_phase_for<KS>(threads, a, st, tiles);
    return lds_phase_for<Euler>(threads, a, st, tiles);
}

template <class Sch>
void classic_launch_t(const double *src, double *dst, int64_t n, int bc, int predictor, const Consts &c,
                      int T, hipStream_t st)
{
    const unsigned blocks = (unsigned)((n + T - 1) / T);
    if (T <= 256)
        hipLaunchKernelGGL((classic_level<Sch, 256>), dim3(blocks), dim3(T), 0, st, src, dst, n, bc, predictor, c);
    else
        hipLaunchKernelGGL((classic_level<Sch, 1024>), dim3(blocks), dim3(T), 0, st, src, dst, n, bc, predictor, c);
}

hipError_t launch_classic_level(int scheme, const double *src, double *dst, int64_t n, int bc,
                                int predictor, const Consts &c, int threads, hipStream_t st)
{
    if (threads < 64 || threads > 1024 || threads % 64 != 0) return hipErrorInvalidValue;
    if (scheme == 0) classic_launch_t<Heat>(src, dst, n, bc, predictor, c, threads, st);
    else if (scheme == 1) classic_launch_t<KS>(src, dst, n, bc, predictor, c, threads, st);
    else classic_launch_t<Euler>(src, dst, n, bc, predictor, c, threads, st);
    return hipGetLastError();
}

hipError_t launch_batch_phase(int scheme, int P, const SolveDesc *desc, const int2 *items, int64_t nitems,
                              int global_phase, int grid, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    if (scheme == 0) return batch_phase_for<Heat>(P, desc, items, nitems, global_phase, grid, st);
    if (scheme == 1) return batch_phase_for<KS>(P, desc, items, nitems, global_phase, grid, st);
    return batch_phase_for<Euler>(P, desc, items, nitems, global_phase, grid, st);
}

int batch_blocks_per_cu(int scheme, int P)
{
    if (scheme == 0) return batch_blocks_for<Heat>(P);
    if (scheme == 1) return batch_blocks_for<KS>(P);
    return batch_blocks_for<Euler>(P);
}

hipError_t launch_persistent_batch(int scheme, int P, const PersistArgs &q, int grid, hipStream_t st)
{
    if (scheme == 0) return persistent_phase_for<Heat>(P, q, grid, st);
    if (scheme == 1) return persistent_phase_for<KS>(P, q, grid, st);
    return persistent_phase_for<Euler>(P, q, grid, st);
}

int persistent_blocks_per_cu(int scheme, int P)
{
    if (scheme == 0) return persistent_blocks_for<Heat>(P);
    if (scheme == 1) return persistent_blocks_for<KS>(P);
    return persistent_blocks_for<Euler>(P);
}

hipError_t launch_zero_words(void *p, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_words, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)p, count);
    return hipGetLastError();
}

hipError_t launch_advance_phases(SolveDesc *desc, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(advance_phases, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, desc, n);
    return hipGetLastError();
}

hipError_t launch_stamp(uint64_t *stamps, int idx, hipStream_t st)
{
    hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, st, stamps, idx);
    return hipGetLastError();
}

hipError_t launch_nonfinite_scan(const double *x, int64_t count, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(nonfinite_scan, dim3(1024), dim3(256), 0, st, x, count, flag);
    return hipGetLastError();
}

}  // namespace sw
