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
#include "tile_emu.hpp"

using namespace sw;

namespace {

template <class Sch, int P>
void run_phase(const Geom &g, const TileArgs &a)
{
    for (int64_t j = 0; j < a.K; ++j) emu::emulate_tile<Sch, P>(a, j, g.NW);
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
