// The paper's Shared variant of the swept tile (Sec. 5.1): one work-group per node,
// the two-row working array in LDS, the work-group's threads striding over the
// computed set of each level and one barrier per level.  Every point is one call of
// the scheme's per-point rule on a halo read from LDS, so a point-level moves
// (2r + 2) NV doubles through LDS; the register kernel (swept_tile.hpp) keeps the rows
// in VGPRs instead.  The width is bounded only by the LDS a work-group may hold, so
// this is the "largest triangle that fits" design, measured beside the register one.
// Same slots, same boundary treatment and the same rules as swept_tile, so results
// are bit-identical.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sw {

namespace {

template <class Sch>
__global__ __launch_bounds__(1024) void lds_tile(TileArgs args)
{
    constexpr int NV = Sch::NV, R = Sch::R;
    extern __shared__ double rows[];
    const int64_t j = blockIdx.x;
    TileArgs a = args;
    a.ends = tile_ends(args, j);
    const int w = a.w, half = w >> 1, span = w + 2 * R, T = blockDim.x, t = threadIdx.x;
    // tile position x of row q of variable v, x in [-R, w + R)
    auto at = [&](int v, int q, int x) -> double & { return rows[(2 * v + q) * span + R + x]; };

    if (a.kind == PH_UP) {
        const int64_t g0 = tile_start(a, j);
        for (int x = t; x < w; x += T)
            for (int v = 0; v < NV; ++v) {
                at(v, 0, x) = a.state[(int64_t)v * a.n + g0 + x];
                at(v, 1, x) = 0.0;
            }
        if (t < R)
            for (int v = 0; v < NV; ++v)
                for (int q = 0; q < 2; ++q) { at(v, q, t - R) = 0.0; at(v, q, w + t) = 0.0; }
    } else {
        // left half from slot a (an R slot: points [-r, w/2)), right half from slot b
        // (an L slot: points [w/2, w + r)); the previous triangles' tips beyond the tile
        // go to the halo of row 1, which the widest level reads
        const double *sa = a.edges + slot_base<Sch>(a, slot_a(a, j));
        const double *sb = a.edges + slot_base<Sch>(a, slot_b(a, j));
        for (int x = t; x < w; x += T) {
            const double *src = x < half ? sa + x + R : sb + x - half;
            for (int v = 0; v < NV; ++v)
                for (int q = 0; q < 2; ++q) at(v, q, x) = src[(v * 2 + q) * a.E];
        }
        if (t < R) {
            const bool dl = a.bc == BC_DIRICHLET && a.offset == 0 && j == 0;   // the unshifted
            const bool dr = a.bc == BC_DIRICHLET && a.offset == 0 && j == a.K - 1;   // tiles at the walls
            for (int v = 0; v < NV; ++v) {
                at(v, 1, t - R) = dl ? a.c.ghost_l[v] : sa[(v * 2 + 1) * a.E + t];
                at(v, 1, w + t) = dr ? a.c.ghost_r[v] : sb[(v * 2 + 1) * a.E + half + t];
                at(v, 0, t - R) = 0.0;
                at(v, 0, w + t) = 0.0;
            }
        }
    }
    __syncthreads();

    const bool wall = straddles_wall(a, j);
    const bool refl = a.bc == BC_REFLECTIVE;   // heat only: R == 1
    const int nlev = tile_levels(a);
    for (int s = 1; s <= nlev; ++s) {
        const int m = half_width(a, s);
        const int q = s & 1, p = q ^ 1;
        const bool widest = s == a.H && a.kind != PH_UP;
        for (int x = half - R * m + t; x < half + R * m; x += T) {
            double ext[NV][1 + 2 * R];
            for (int v = 0; v < NV; ++v)
                for (int d = 0; d <= 2 * R; ++d) ext[v][d] = at(v, p, x - R + d);
            if (refl) {
                if constexpr (R == 1) {
                    // insulated domain ends at the widest level, and the two ends that meet
                    // at the centre of the wall-straddling tile: T_{-1} = T_1, T_n = T_{n-2}
                    if ((widest && (a.ends & 1) && x == 0) || (wall && x == half)) ext[0][0] = ext[0][2];
                    if ((widest && (a.ends & 2) && x == w - 1) || (wall && x == half - 1)) ext[0][2] = ext[0][0];
                }
            } else if (wall) {   // Dirichlet wall at the tile centre: across it lie the ghost values
                for (int v = 0; v < NV; ++v)
                    for (int d = 0; d <= 2 * R; ++d) {
                        const int pos = x - R + d;
                        if (x >= half && pos < half) ext[v][d] = a.c.ghost_l[v];
                        if (x < half && pos >= half) ext[v][d] = a.c.ghost_r[v];
                    }
            }
            double dst[NV][1];
            for (int v = 0; v < NV; ++v) dst[v][0] = at(v, q, x);   // u^m for a final stage
            const bool in[1] = {true};
            Sch::template level<1, false>(dst, ext, (s & 1) != 0, a.c, in);
            for (int v = 0; v < NV; ++v) at(v, q, x) = dst[v][0];
        }
        __syncthreads();
    }

    // new L slot into a (points [0, w/2 + r)), new R slot into b (points [w/2 - r, w))
    if (a.kind != PH_DOWN) {
        double *sa = a.edges + slot_base<Sch>(a, slot_a(a, j));
        double *sb = a.edges + slot_base<Sch>(a, slot_b(a, j));
        for (int x = t; x < w; x += T)
            for (int v = 0; v < NV; ++v)
                for (int q = 0; q < 2; ++q) {
                    const double val = at(v, q, x);
                    if (x < half + R) sa[(v * 2 + q) * a.E + x] = val;
                    if (x >= half - R) sb[(v * 2 + q) * a.E + x - (half - R)] = val;
                }
    }
    int lo, hi;
    const int topl = store_top_level<Sch>(a, lo, hi);
    if (topl < 0) return;
    const int64_t g0 = tile_start(a, j);
    for (int x = lo + t; x < hi; x += T)
        for (int v = 0; v < NV; ++v) a.state[(int64_t)v * a.n + wrap_once(g0 + x, a.n)] = at(v, topl & 1, x);
}

// Allow the kernel all the dynamic LDS a work-group may have (once per process, before
// any launch is captured).
template <class Sch>
hipError_t lds_prepare_for()
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&lds_tile<Sch>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsTileMaxBytes);
}

template <class Sch>
hipError_t lds_phase_for(int threads, const TileArgs &a, hipStream_t st, int64_t tiles)
{
    const int64_t bytes = lds_tile_bytes(Sch::NV, Sch::R, a.w);
    if (bytes > kLdsTileMaxBytes || threads < 64 || threads > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lds_tile<Sch>, dim3((unsigned)tiles), dim3((unsigned)threads), (size_t)bytes, st, a);
    return hipGetLastError();
}

}  // namespace

}  // namespace sw
