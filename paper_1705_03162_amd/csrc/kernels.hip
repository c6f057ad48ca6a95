// HIP kernels for gfx950: the swept tile kernel (Up / Diamond / Down phases)
// and the classic one-sub-step-per-launch kernel.
//
// Swept tile kernel.  One work-group is one node of the swept rule (the paper's
// Shared variant maps a node to a block, Sec. 4.1), but the two-row working
// array lives in VGPRs instead of shared memory: lane g owns P consecutive
// points of both rows.  Per level a lane needs r points of the source row from
// each neighbouring lane; inside a wave they arrive through DPP row moves across
// the whole wave (wave_shr:1 / wave_shl:1), between waves through a small
// double-buffered LDS exchange with one barrier per level.  A one-wave tile
// therefore runs barrier-free.  There is no contraction anywhere, so MFMA has no
// role; the kernel is bound by FP64 VALU issue.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sw {

namespace {

constexpr int DPP_WAVE_SHL1 = 0x130;  // lane i receives lane i+1
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane i receives lane i-1

// Move a double across lanes with a DPP control; lanes whose source lane lies
// outside the wave keep `old`.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double old, double v)
{
    const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
    const unsigned long long x = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)x, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(x >> 32), CTRL,
                                               0xF, 0xF, false);
    const unsigned long long r = ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo;
    return __builtin_bit_cast(double, r);
}

template <class Sch, int P, bool ODD>
__device__ __forceinline__ void level_step(const TileArgs &a, int g, int NW, int s,
                                           const double (&src)[Sch::NV][P], double (&dst)[Sch::NV][P],
                                           const double (&hl)[Sch::NV][Sch::R],
                                           const double (&hr)[Sch::NV][Sch::R], bool wall,
                                           double (*xch)[16][2][Sch::NV][Sch::R])
{
    constexpr int NV = Sch::NV, R = Sch::R;
    double ext[NV][P + 2 * R];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int k = 0; k < P; ++k) ext[v][R + k] = src[v][k];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            // wave-edge lanes get the tile's outer halo; interior lanes their neighbour's points
            ext[v][i] = dpp_move<DPP_WAVE_SHR1>(hl[v][i], src[v][P - R + i]);
            ext[v][R + P + i] = dpp_move<DPP_WAVE_SHL1>(hr[v][i], src[v][i]);
        }
    }
    if (NW > 1) {
        const int lane = g & 63, wave = g >> 6, buf = s & 1;
        if (lane == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i) xch[buf][wave][0][v][i] = src[v][i];
        }
        if (lane == 63) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i) xch[buf][wave][1][v][i] = src[v][P - R + i];
        }
        __syncthreads();
        if (lane == 0 && wave > 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i) ext[v][i] = xch[buf][wave - 1][1][v][i];
        }
        if (lane == 63 && wave < NW - 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i) ext[v][R + P + i] = xch[buf][wave + 1][0][v][i];
        }
    }
    if (wall) {
        const int gw = a.w / (2 * P) - 1;  // last lane left of the wall
        if (g == gw) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i) ext[v][R + P + i] = a.c.ghost_r[v];
        }
        if (g == gw + 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i) ext[v][i] = a.c.ghost_l[v];
        }
    }
    int klo, khi;
    lane_bounds(a, s, g, P, R, klo, khi);
    Sch::template level<P>(dst, ext, ODD, a.c, klo, khi);
}

template <class Sch, int P, int MAXT>
__global__ __launch_bounds__(MAXT) void swept_tile(TileArgs a)
{
    constexpr int NV = Sch::NV, R = Sch::R;
    __shared__ double xch[2][16][2][NV][R];
    const int g = threadIdx.x;
    const int NW = blockDim.x >> 6;
    const int64_t j = blockIdx.x;
    double r0[NV][P], r1[NV][P], hl[NV][R], hr[NV][R];
    lane_load<Sch, P>(a, j, g, r0, r1, hl, hr);
    const int nlev = tile_levels(a);
    const bool wall = straddles_wall(a, j);
    int s = 1;
    for (; s + 1 <= nlev; s += 2) {
        level_step<Sch, P, true>(a, g, NW, s, r0, r1, hl, hr, wall, xch);
        level_step<Sch, P, false>(a, g, NW, s + 1, r1, r0, hl, hr, wall, xch);
    }
    if (s <= nlev) level_step<Sch, P, true>(a, g, NW, s, r0, r1, hl, hr, wall, xch);
    if (NW > 1) __syncthreads();  // every wave has read its inputs before any slot is rewritten
    lane_store<Sch, P>(a, j, g, r0, r1);
}

// Classic: one thread per point, one launch per sub-step (Sec. 4.1).  For the
// final RK2 stage `dst` holds u^m and is updated in place (the listing's +=).
template <class Sch>
__global__ __launch_bounds__(256) void classic_level(const double *__restrict__ src, double *dst,
                                                     int64_t n, int dirichlet, int predictor, Consts c)
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
        if (dirichlet) jj = jj < 0 ? 0 : (jj >= n ? n - 1 : jj);
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
    Sch::template level<1>(out, ext, predictor != 0, c, 0, 1);
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[(int64_t)v * n + i] = out[v][0];
}

// Flag non-finite values (optional post-solve check).
__global__ void nonfinite_scan(const double *x, int64_t count, int *flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) atomicOr(flag, 1);
}

template <class Sch, int P>
hipError_t launch_tile(const TileArgs &a, int threads, hipStream_t st)
{
    constexpr int MAXT = max_threads_for(Sch::NV, P);
    if (threads > MAXT) return hipErrorInvalidValue;
    hipLaunchKernelGGL((swept_tile<Sch, P, MAXT>), dim3((unsigned)a.K), dim3(threads), 0, st, a);
    return hipGetLastError();
}

template <class Sch>
hipError_t launch_tile_p(const TileArgs &a, int P, int threads, hipStream_t st)
{
    switch (P) {
    case 1: if constexpr (Sch::R <= 1) return launch_tile<Sch, 1>(a, threads, st); break;
    case 2: return launch_tile<Sch, 2>(a, threads, st);
    case 4: return launch_tile<Sch, 4>(a, threads, st);
    case 8: return launch_tile<Sch, 8>(a, threads, st);
    case 16: if constexpr (Sch::NV == 1) return launch_tile<Sch, 16>(a, threads, st); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_swept_phase(int scheme, int P, int threads, const TileArgs &a, hipStream_t st)
{
    if (a.K <= 0) return hipSuccess;
    if (scheme == 0) return launch_tile_p<Heat>(a, P, threads, st);
    if (scheme == 1) return launch_tile_p<KS>(a, P, threads, st);
    return launch_tile_p<Euler>(a, P, threads, st);
}

hipError_t launch_classic_level(int scheme, const double *src, double *dst, int64_t n, int dirichlet,
                                int predictor, const Consts &c, hipStream_t st)
{
    const int T = 256;
    const unsigned blocks = (unsigned)((n + T - 1) / T);
    if (scheme == 0)
        hipLaunchKernelGGL(classic_level<Heat>, dim3(blocks), dim3(T), 0, st, src, dst, n, dirichlet, predictor, c);
    else if (scheme == 1)
        hipLaunchKernelGGL(classic_level<KS>, dim3(blocks), dim3(T), 0, st, src, dst, n, dirichlet, predictor, c);
    else
        hipLaunchKernelGGL(classic_level<Euler>, dim3(blocks), dim3(T), 0, st, src, dst, n, dirichlet, predictor, c);
    return hipGetLastError();
}

hipError_t launch_nonfinite_scan(const double *x, int64_t count, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(nonfinite_scan, dim3(1024), dim3(256), 0, st, x, count, flag);
    return hipGetLastError();
}

}  // namespace sw
