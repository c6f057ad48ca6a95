// Test-only host emulation of the swept tile schedule.
//
// Runs the library's own launch sequence (build_phases), tile geometry
// (lane_load / lane_bounds / lane_store) and per-point rules (schemes.hpp) on
// the CPU, with a software work-group standing in for the GPU lanes: each lane's
// halo is read straight from its neighbours' rows instead of through DPP moves
// and LDS.  The CPU tests compare it bit for bit with the oracle, which checks
// the decomposition's geometry (edges, offsets, remainders, walls) without a
// GPU.  It is never linked into libswept.so.
#include <math.h>
#include <stdint.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "plan_core.hpp"

using namespace sw;

namespace {

template <class Sch, int P>
void run_phase(const Geom &g, const TileArgs &a)
{
    constexpr int NV = Sch::NV, R = Sch::R;
    const int lanes = 64 * g.NW;
    struct Lane { double r0[NV][P], r1[NV][P], hl[NV][R], hr[NV][R]; };
    std::vector<Lane> L(lanes);
    for (int64_t j = 0; j < a.K; ++j) {
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

template <class Sch>
int run_all(const Geom &g, const Consts &c, double *state)
{
    std::vector<double> edges((size_t)g.edge_doubles, 0.0);
    for (const Phase &ph : build_phases(g)) {
        TileArgs a = make_tile_args(g, c, ph, state, edges.data());
        switch (g.P) {
        case 1: run_phase<Sch, 1>(g, a); break;
        case 2: run_phase<Sch, 2>(g, a); break;
        case 4: run_phase<Sch, 4>(g, a); break;
        case 8: run_phase<Sch, 8>(g, a); break;
        case 16: run_phase<Sch, 16>(g, a); break;
        default: return SW_EINVAL;
        }
    }
    return SW_OK;
}

}  // namespace

extern "C" int hostsim_swept(const sw_problem *p, int width, int threads, double *state)
{
    std::string err;
    int rc = validate_problem(p, &err);
    if (rc) return rc;
    Geom g;
    if ((rc = make_geom(*p, width, threads, &g, &err))) return rc;
    if (!g.swept_ok) return SW_EUNSUPPORTED;
    Consts c = make_consts(*p);
    try {
        if (p->scheme == SW_HEAT) return run_all<Heat>(g, c, state);
        if (p->scheme == SW_KS) return run_all<KS>(g, c, state);
        return run_all<Euler>(g, c, state);
    } catch (const std::exception &) {
        return -100;  // internal consistency check failed
    }
}

// Launch sequence of a plan: out[3*i .. 3*i+2] = (kind, levels, offset).
extern "C" int hostsim_phases(const sw_problem *p, int width, int threads, int32_t *out, int max)
{
    std::string err;
    int rc = validate_problem(p, &err);
    if (rc) return rc;
    Geom g;
    if ((rc = make_geom(*p, width, threads, &g, &err))) return rc;
    std::vector<Phase> ph = build_phases(g);
    int cnt = 0;
    for (const Phase &x : ph) {
        if (cnt < max) { out[3 * cnt] = x.kind; out[3 * cnt + 1] = x.levels; out[3 * cnt + 2] = x.offset; }
        ++cnt;
    }
    return cnt;
}
