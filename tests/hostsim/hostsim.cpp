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

#include "hybrid.hpp"
#include "plan_core.hpp"
#include "tile_emu.hpp"

using namespace sw;

namespace {

template <class Sch, int P>
void run_phase(const Geom &g, const TileArgs &a, int64_t tiles)
{
    for (int64_t j = 0; j < tiles; ++j) emu::emulate_tile<Sch, P>(a, j, g.NW);
}

// Hybrid variant: the straddling tile of a shifted non-periodic phase is computed by
// the library's host routine (hybrid_tile_host) on copies of its two slots, the way
// the library's hybrid solve moves them through pinned memory.
template <class Sch>
void hybrid_straddling_tile(const Geom &g, const TileArgs &a, std::vector<double> &edges, double *state)
{
    const size_t slot = (size_t)g.nv * 2 * g.E;
    std::vector<double> sa(edges.begin() + (2 * g.K - 1) * slot, edges.begin() + 2 * g.K * slot);
    std::vector<double> sb(edges.begin(), edges.begin() + slot);
    std::vector<double> top((size_t)g.nv * g.w, 0.0);
    HybridTile t{a, g.scheme, sa.data(), sb.data(), top.data()};
    hybrid_tile_host(t);
    if (a.kind != PH_DOWN) {
        std::copy(sa.begin(), sa.end(), edges.begin() + (2 * g.K - 1) * slot);
        std::copy(sb.begin(), sb.end(), edges.begin());
        return;
    }
    const int half = g.w / 2;
    for (int x = half - g.r * a.levels; x < half + g.r * a.levels; ++x)
        for (int v = 0; v < g.nv; ++v)
            state[(int64_t)v * g.n + (x < half ? g.n - half + x : x - half)] = top[(size_t)v * g.w + x];
}

template <class Sch>
int run_all(const Geom &g, const Consts &c, double *state, bool hybrid = false)
{
    std::vector<double> edges((size_t)g.edge_doubles, 0.0);
    for (const Phase &ph : build_phases(g)) {
        TileArgs a = make_tile_args(g, c, ph, state, edges.data());
        const bool split = hybrid && g.bc != SW_PERIODIC && ph.offset == 1;
        const int64_t tiles = split ? a.K - 1 : a.K;
        switch (g.P) {
        case 1: run_phase<Sch, 1>(g, a, tiles); break;
        case 2: run_phase<Sch, 2>(g, a, tiles); break;
        case 4: run_phase<Sch, 4>(g, a, tiles); break;
        case 8: run_phase<Sch, 8>(g, a, tiles); break;
        case 16: run_phase<Sch, 16>(g, a, tiles); break;
        default: return SW_EINVAL;
        }
        if (split) hybrid_straddling_tile<Sch>(g, a, edges, state);
    }
    return SW_OK;
}

}  // namespace

extern "C" int hostsim_swept_mode(const sw_problem *p, int width, int threads, double *state, int hybrid)
{
    std::string err;
    int rc = validate_problem(p, &err);
    if (rc) return rc;
    Geom g;
    if ((rc = make_geom(*p, width, threads, &g, &err))) return rc;
    if (!g.swept_ok) return SW_EUNSUPPORTED;
    Consts c = make_consts(*p);
    try {
        if (p->scheme == SW_HEAT) return run_all<Heat>(g, c, state, hybrid != 0);
        if (p->scheme == SW_KS) return run_all<KS>(g, c, state, hybrid != 0);
        return run_all<Euler>(g, c, state, hybrid != 0);
    } catch (const std::exception &) {
        return -100;  // internal consistency check failed
    }
}

// Dataflow order: tiles run one at a time in a seeded random order that respects only
// phase_deps (the rule the persistent batched kernel waits on), not the phase order.
template <class Sch, int P>
int run_dataflow(const Geom &g, const Consts &c, double *state, uint64_t seed)
{
    std::vector<double> edges((size_t)g.edge_doubles, 0.0);
    const std::vector<Phase> ph = build_phases(g);
    const int np = (int)ph.size();
    std::vector<int> done((size_t)g.K, 0);   // phases completed per tile
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
    for (;;) {
        std::vector<int64_t> ready;
        for (int64_t j = 0; j < g.K; ++j) {
            const int p = done[(size_t)j];
            if (p >= np) continue;
            bool ok = true;
            if (p > 0) {
                int64_t deps[2];
                const int nd = phase_deps(g.Q, g.rem, g.H, g.K, p, j, deps);
                for (int k = 0; k < nd; ++k) ok = ok && done[(size_t)deps[k]] >= p;
            }
            if (ok) ready.push_back(j);
        }
        if (ready.empty()) break;
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;
        const int64_t j = ready[(size_t)(x % ready.size())];
        const int p = done[(size_t)j];
        TileArgs a = make_tile_args(g, c, ph[(size_t)p], state, edges.data());
        emu::emulate_tile<Sch, P>(a, j, g.NW);
        done[(size_t)j] = p + 1;
    }
    for (int64_t j = 0; j < g.K; ++j)
        if (done[(size_t)j] != np) return -101;   // some tile never became ready
    return SW_OK;
}

template <class Sch>
int dataflow_for(const Geom &g, const Consts &c, double *state, uint64_t seed)
{
    switch (g.P) {
    case 1: return run_dataflow<Sch, 1>(g, c, state, seed);
    case 2: return run_dataflow<Sch, 2>(g, c, state, seed);
    case 4: return run_dataflow<Sch, 4>(g, c, state, seed);
    case 8: return run_dataflow<Sch, 8>(g, c, state, seed);
    case 16: return run_dataflow<Sch, 16>(g, c, state, seed);
    default: return SW_EINVAL;
    }
}

extern "C" int hostsim_dataflow(const sw_problem *p, int width, int threads, double *state, uint64_t seed)
{
    std::string err;
    int rc = validate_problem(p, &err);
    if (rc) return rc;
    Geom g;
    if ((rc = make_geom(*p, width, threads, &g, &err))) return rc;
    if (!g.swept_ok) return SW_EUNSUPPORTED;
    Consts c = make_consts(*p);
    try {
        if (p->scheme == SW_HEAT) return dataflow_for<Heat>(g, c, state, seed);
        if (p->scheme == SW_KS) return dataflow_for<KS>(g, c, state, seed);
        return dataflow_for<Euler>(g, c, state, seed);
    } catch (const std::exception &) {
        return -100;
    }
}

extern "C" int hostsim_swept(const sw_problem *p, int width, int threads, double *state)
{
    return hostsim_swept_mode(p, width, threads, state, 0);
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
