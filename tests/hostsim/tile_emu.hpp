// Test-only host emulation of one swept tile (one work-group of one phase).
//
// Runs the library's own tile geometry (lane_load / lane_bounds / lane_store) and
// per-point rules (schemes.hpp) on the CPU, with a software work-group standing in
// for the GPU lanes: each lane's halo is read straight from its neighbours' rows
// instead of through DPP moves and LDS.  Shared by the schedule emulator
// (hostsim.cpp) and the served-batch emulator (servesim.cpp).
#pragma once

#include <stdexcept>
#include <vector>

#include "plan_core.hpp"

namespace sw {
namespace emu {

template <class Sch, int P>
void emulate_tile(const TileArgs &a, int64_t j, int NW)
{
    constexpr int NV = Sch::NV, R = Sch::R;
    const int lanes = 64 * NW;
    struct Lane { double r0[NV][P], r1[NV][P], hl[NV][R], hr[NV][R]; };
    std::vector<Lane> L(lanes);
    {
        for (int l = 0; l < lanes; ++l) lane_load<Sch, P>(a, j, l, L[l].r0, L[l].r1, L[l].hl, L[l].hr);
        const int nlev = tile_levels(a);
        const bool wall = straddles_wall(a, j);
        for (int s = 1; s <= nlev; ++s) {
            const bool odd = (s & 1) != 0;
            // like the kernel: the points just outside the tile are supplied only at the
            // widest level of a Diamond/Down (the only level whose stencil reaches them)
            const bool outer = s == a.H && a.kind != PH_UP;
            for (int l = 0; l < lanes; ++l) {
                double (&src)[NV][P] = odd ? L[l].r0 : L[l].r1;
                double (&dst)[NV][P] = odd ? L[l].r1 : L[l].r0;
                double ext[NV][P + 2 * R];
                for (int v = 0; v < NV; ++v) {
                    for (int k = 0; k < P; ++k) ext[v][R + k] = src[v][k];
                    for (int i = 0; i < R; ++i) {
                        // halo points by position: q < 0 / q >= w lie outside the tile
                        const int ql = l * P - R + i, qr = l * P + P + i;
                        ext[v][i] = ql >= 0 ? (odd ? L[ql / P].r0 : L[ql / P].r1)[v][ql % P]
                                            : (outer ? L[0].hl[v][ql + R] : 0.0);
                        ext[v][R + P + i] = qr < a.w ? (odd ? L[qr / P].r0 : L[qr / P].r1)[v][qr % P]
                                                     : (outer ? L[0].hr[v][qr - a.w] : 0.0);
                        if (a.bc == BC_DIRICHLET) {
                            // Dirichlet wall at the tile centre: across it lie the ghosts
                            if (wall && l * P >= a.w / 2 && ql < a.w / 2) ext[v][i] = a.c.ghost_l[v];
                            if (wall && l * P < a.w / 2 && qr >= a.w / 2) ext[v][R + P + i] = a.c.ghost_r[v];
                        }
                    }
                }
                if (a.bc == BC_REFLECTIVE) {
                    // insulated ends: the point beyond an end takes the value one point
                    // inside it (domain point -1 <- 1, n <- n-2), by tile position
                    auto at = [&](int q) { return (odd ? L[q / P].r0 : L[q / P].r1)[0][q % P]; };
                    const int ends = tile_ends(a, j), half = a.w / 2;
                    const int ql = l * P - 1, qr = l * P + P;
                    if (outer && (ends & 1) && ql == -1) ext[0][0] = at(1);
                    if (outer && (ends & 2) && qr == a.w) ext[0][P + 1] = at(a.w - 2);
                    if (wall && l * P == half) ext[0][0] = at(half + 1);
                    if (wall && qr == half) ext[0][P + 1] = at(half - 2);
                }
                // element masks exactly as the kernel derives them (residues from s mod G)
                const int m = half_width(a, s);
                const int lo = a.w / 2 - R * m, hi = a.w / 2 + R * m;
                const int smod = s % group_len(P, R);
                bool in[P];
                for (int k = 0; k < P; ++k) {
                    int la, lb;
                    element_lane_bounds(P, R, level_widening(a, s), smod, lo, hi, 0, k, la, lb);
                    in[k] = l >= la && l < lb;
                }
                int klo, khi;  // cross-check against the direct bounds
                lane_bounds(a, s, l, P, R, klo, khi);
                for (int k = 0; k < P; ++k)
                    if (in[k] != (k >= klo && k < khi)) throw std::logic_error("element mask mismatch");
                int lmin, lmax;  // lanes the kernel does not skip
                element_lane_span(P, R, level_widening(a, s), smod, lo, hi, 0, lmin, lmax);
                if (klo < khi && !(l >= lmin && l < lmax)) throw std::logic_error("skipped an active lane");
                if (klo >= khi && l >= lmin && l < lmax && (l == lmin || l == lmax - 1) && lmax - lmin > 2)
                    throw std::logic_error("lane span not tight");
                Sch::template level<P>(dst, ext, odd, a.c, in);
            }
        }
        for (int l = 0; l < lanes; ++l) lane_store<Sch, P>(a, j, l, L[l].r0, L[l].r1);
    }
}


}  // namespace emu
}  // namespace sw
