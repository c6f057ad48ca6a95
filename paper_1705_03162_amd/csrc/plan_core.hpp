// Host-side plan geometry: problem validation, canonical constants, legal tile
// shapes and the launch sequence of a swept solve.
//
// Launch sequence (Sec. 4.2): an Up triangle, then Diamonds at alternating
// offsets (0 and w/2, the zig-zag of the node locations), then a Down triangle
// that completes a full level; each phase advances H = w/(2r) levels.  A final
// remainder of h < H levels is done with one more Up/Down pair whose Up stops at
// level h and writes its top directly.
#pragma once

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "swept.h"
#include "tile.hpp"

namespace sw {

struct Phase {
    int32_t kind;    // PhaseKind
    int32_t levels;  // levels advanced (Up/Down); 2H-1 computed levels for a Diamond
    int32_t offset;  // 0 or 1 (tiles shifted by w/2)
};

struct Geom {
    int scheme = 0, bc = 0, r = 1, S = 1, nv = 1;
    int64_t n = 0, nsteps = 0, levels = 0;
    int w = 0, threads = 0, P = 0, NW = 0, H = 0, E = 0;
    int classic_threads = 256;   // work-group size of the classic kernel
    int64_t K = 0, Q = 0, rem = 0;
    bool swept_ok = false;
    bool lds = false;   // Shared variant: the rows in LDS, threads striding over the points
    int64_t edge_doubles = 0;
};

inline int scheme_radius(int scheme) { return scheme == SW_HEAT ? 1 : 2; }
inline int scheme_substeps(int scheme) { return scheme == SW_HEAT ? 1 : 2; }
inline int scheme_nvars(int scheme) { return scheme == SW_EULER ? 3 : 1; }

// Points per lane for which kernels are instantiated.
inline bool legal_points_per_lane(int scheme, int P)
{
    if (P != 1 && P != 2 && P != 4 && P != 8 && P != 16) return false;
    if (scheme == SW_EULER && P > 8) return false;    // register budget of the flux stencil
    return true;
}

inline bool legal_threads(int threads) { return threads >= 64 && threads <= 1024 && threads % 64 == 0; }

inline int validate_problem(const sw_problem *p, std::string *err)
{
    if (!p) { *err = "problem is NULL"; return SW_EINVAL; }
    if (p->scheme < SW_HEAT || p->scheme > SW_EULER) { *err = "unknown scheme"; return SW_EINVAL; }
    if (p->bc != SW_PERIODIC && p->bc != SW_DIRICHLET && p->bc != SW_REFLECTIVE) {
        *err = "unknown boundary type"; return SW_EINVAL;
    }
    if (p->bc == SW_REFLECTIVE && (p->scheme != SW_HEAT || p->n < 2)) {
        *err = "reflective ends are defined for the heat equation (Appendix B) with n >= 2";
        return SW_EINVAL;
    }
    if (p->n < 1) { *err = "n must be >= 1"; return SW_EINVAL; }
    if (p->nsteps < 0) { *err = "nsteps must be >= 0"; return SW_EINVAL; }
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) { *err = "dt must be finite and > 0"; return SW_EINVAL; }
    if (!(p->dx > 0.0) || !std::isfinite(p->dx)) { *err = "dx must be finite and > 0"; return SW_EINVAL; }
    if (p->scheme == SW_HEAT && !std::isfinite(p->alpha)) { *err = "alpha must be finite"; return SW_EINVAL; }
    if (p->scheme == SW_EULER && !(p->gamma > 1.0 && std::isfinite(p->gamma))) {
        *err = "gamma must be finite and > 1"; return SW_EINVAL;
    }
    if ((p->flags & ~SW_PROBLEM_LIMITER_RECIPROCAL) != 0 || p->reserved != 0) {
        *err = "unknown problem flags"; return SW_EINVAL;
    }
    for (int v = 0; v < 3; ++v)
        if (!std::isfinite(p->bc_left[v]) || !std::isfinite(p->bc_right[v])) {
            *err = "boundary values must be finite"; return SW_EINVAL;
        }
    if (p->nsteps > (int64_t)1 << 40) { *err = "nsteps too large"; return SW_EINVAL; }
    return SW_OK;
}

// Constants in the canonical order (every solver path uses exactly these).
inline Consts make_consts(const sw_problem &p)
{
    Consts c{};
    c.fo = (p.alpha * p.dt) / (p.dx * p.dx);
    c.c0 = 1.0 - 2.0 * c.fo;
    c.c1 = 1.0 / (4.0 * p.dx);
    c.c2 = 1.0 / (p.dx * p.dx);
    c.c4 = c.c2 * c.c2;
    c.k1 = c.c2 - 4.0 * c.c4;
    c.k0 = 6.0 * c.c4 - 2.0 * c.c2;
    c.hdt = 0.5 * p.dt;
    c.dt = p.dt;
    c.gm1 = p.gamma - 1.0;
    c.gamma = p.gamma;
    c.lam = p.dt / p.dx;
    c.hlam = 0.5 * c.lam;
    c.limiter = (p.flags & SW_PROBLEM_LIMITER_RECIPROCAL) ? 1 : 0;
    for (int v = 0; v < 3; ++v) {
        c.ghost_l[v] = p.bc_left[v];
        c.ghost_r[v] = p.bc_right[v];
    }
    return c;
}

// Geometry for an explicit tile shape (width = P * threads).  lds: the Shared variant,
// whose threads stride over the tile's points in LDS (any 1 <= P <= 64; the caller
// checks the LDS the rows take).
inline int make_geom(const sw_problem &p, int width, int threads, Geom *g, std::string *err, bool lds = false)
{
    Geom q;
    q.scheme = p.scheme; q.bc = p.bc;
    q.r = scheme_radius(p.scheme);
    q.S = scheme_substeps(p.scheme);
    q.nv = scheme_nvars(p.scheme);
    q.n = p.n; q.nsteps = p.nsteps; q.levels = (int64_t)q.S * p.nsteps;
    if (!legal_threads(threads)) { *err = "threads must be a multiple of 64 in [64, 1024]"; return SW_EINVAL; }
    if (width <= 0 || width % threads != 0) { *err = "width must be a positive multiple of threads"; return SW_EINVAL; }
    q.P = width / threads;
    q.lds = lds;
    if (lds) {
        if (q.P > 64 || width % (4 * q.r) != 0) {
            *err = "Shared-variant width must be at most 64 points per thread and a multiple of 4 r";
            return SW_EINVAL;
        }
    } else if (!legal_points_per_lane(p.scheme, q.P)) {
        *err = "width/threads must be 1, 2, 4, 8 or 16 points per lane, at least the stencil radius (Euler: at most 8)";
        return SW_EINVAL;
    }
    if (!lds && threads > max_threads_for(scheme_nvars(p.scheme), q.P)) {
        *err = "threads too large for this scheme and points per lane";
        return SW_EINVAL;
    }
    q.w = width; q.threads = threads; q.NW = threads / 64;
    q.H = q.w / (2 * q.r);
    q.E = q.w / 2 + q.r;
    q.swept_ok = (p.n % q.w) == 0;
    q.K = q.swept_ok ? p.n / q.w : 0;
    q.Q = q.levels / q.H;
    q.rem = q.levels - q.Q * q.H;
    q.edge_doubles = q.swept_ok ? 2 * q.K * (int64_t)q.nv * 2 * q.E : 0;
    *g = q;
    return SW_OK;
}

inline std::vector<Phase> build_phases(const Geom &g)
{
    std::vector<Phase> ph;
    if (g.levels == 0) return ph;
    const int cnt = phase_count(g.Q, g.rem);
    ph.reserve((size_t)cnt);
    for (int p = 0; p < cnt; ++p) {
        Phase x;
        phase_at(g.Q, g.rem, g.H, p, x.kind, x.levels, x.offset);
        ph.push_back(x);
    }
    return ph;
}

inline TileArgs make_tile_args(const Geom &g, const Consts &c, const Phase &ph, double *state,
                               double *edges)
{
    TileArgs a{};
    a.state = state; a.edges = edges;
    a.n = g.n; a.K = g.K; a.w = g.w; a.H = g.H; a.E = g.E;
    a.kind = ph.kind; a.levels = ph.levels; a.offset = ph.offset;
    a.bc = g.bc;
    a.ends = 0;
    a.c = c;
    return a;
}

// Default tile shape when neither the caller nor the tuning table gives one:
// the largest legal width that divides n while leaving at least `min_tiles`
// tiles (so that every CU holds several work-groups); otherwise the smallest
// legal width that divides n.
inline bool default_shape(const sw_problem &p, int *width, int *threads)
{
    const int pref_P = p.scheme == SW_EULER ? 4 : 8;
    const int64_t min_tiles = 1024;
    int best_w = 0, best_t = 0;
    // candidates in order of preference
    for (int NW = 1; NW <= 4; NW *= 2) {
        for (int P = pref_P; P >= 1; P /= 2) {
            if (!legal_points_per_lane(p.scheme, P)) continue;
            if (64 * NW > max_threads_for(scheme_nvars(p.scheme), P)) continue;
            int w = 64 * NW * P;
            if (p.n % w != 0) continue;
            if (p.n / w >= min_tiles && w > best_w) { best_w = w; best_t = 64 * NW; }
        }
    }
    if (best_w == 0) {
        for (int P = 1; P <= 16 && best_w == 0; P *= 2) {
            if (!legal_points_per_lane(p.scheme, P)) continue;
            int w = 64 * P;
            if (p.n % w == 0) { best_w = w; best_t = 64; }
        }
    }
    if (best_w == 0) {
        // swept impossible for this n; keep a legal shape for bookkeeping
        int P = scheme_radius(p.scheme) == 1 ? 1 : 2;
        *width = 64 * P; *threads = 64;
        return false;
    }
    *width = best_w; *threads = best_t;
    return true;
}

}  // namespace sw
