// Geometry of one swept tile: which points a lane owns, where its two working
// rows come from and go to, and which points each level computes.
//
// Swept rule on a 1D grid (Sec. 4.2, Fig. 1 and 2; Sec. 4.3 for two sub-steps):
// a node of w points advances every level its domain of dependence allows.  A
// stencil of radius r shrinks the computable set by r per side per level, so an
// Up triangle computes levels 1..H-1 on [r s, w - r s) with H = w / (2 r).  The
// two edges it cannot finish travel to the neighbours; the next launch, offset
// by w/2, fills the gap between two triangles (a Diamond: widening for H levels,
// narrowing for H-1 more), and a final Down triangle completes a full level.
//
// Working array (Sec. 4.2): two rows, row 0 for even and row 1 for odd levels,
// overwritten in place; the edges left behind in the rows are exactly the values
// the neighbour needs.  Here the two rows of a tile live in registers: lane g of
// the work-group owns the P consecutive points [g P, g P + P) of both rows.
//
// Edge slots: the edge buffer holds 2K slots, each two rows of E = w/2 + r
// points per variable, stored [var][row][e].  An "L" slot holds tile points
// [0, w/2 + r) of a node, an "R" slot its points [w/2 - r, w); the r points
// around the middle (the triangle tip) appear in both, as the paper copies the
// tips into both edge arrays.  In a phase with offset o (0, or 1 for w/2), tile
// j reads slot a = 2j + o (an R slot: its points [-r, w/2)) and slot
// b = 2j + o + 1 (an L slot: its points [w/2, w + r)), and writes its own L and R
// slots back into a and b: each slot is read and rewritten by exactly one tile
// per launch (the L/R swap of Sec. 4.2).
//
// Relative levels start at an even absolute level in every phase (H is even), so
// odd relative levels are the odd absolute levels: predictors for RK2 schemes.
#pragma once

#include "schemes.hpp"

namespace sw {

enum PhaseKind : int32_t { PH_UP = 0, PH_DIAMOND = 1, PH_DOWN = 2 };
// Boundary types (the values of SW_PERIODIC, SW_DIRICHLET, SW_REFLECTIVE).
enum BcKind : int32_t { BC_PERIODIC = 0, BC_DIRICHLET = 1, BC_REFLECTIVE = 2 };

// Largest work-group for which a tile kernel is compiled: the two rows take
// 2*nv*P doubles per lane, and the register file must hold them for every wave.
constexpr int max_threads_for(int nv, int P) { return nv > 1 ? (P >= 8 ? 256 : 512) : (P >= 8 ? 512 : 1024); }

struct TileArgs {
    double *state;     // [nv][n]
    double *edges;     // 2K slots of nv*2*E doubles
    int64_t n;         // grid points
    int64_t K;         // tiles per phase (n / w)
    int32_t w;         // tile width
    int32_t H;         // w / (2 r)
    int32_t E;         // w/2 + r
    int32_t kind;      // PhaseKind
    int32_t levels;    // Up/Down: levels to advance (<= H); Diamond: ignored (2H - 1)
    int32_t offset;    // 0, or 1 for tiles shifted by w/2
    int32_t bc;        // BC_PERIODIC, BC_DIRICHLET or BC_REFLECTIVE
    int32_t ends;      // set per tile: bit 0 = its left edge is the domain's left end,
                       // bit 1 = its right edge is the right end (non-periodic only)
    Consts c;
};

// One solve inside a batch: its buffers, geometry and current phase.
struct SolveDesc {
    double *state;
    double *edges;
    int64_t n, K, Q, rem;
    int32_t w, H, E, bc;
    int32_t nphases;   // phase_count(Q, rem)
    int32_t phase;     // next phase to run (served batches advance solves independently)
    Consts c;
};

SW_HD int64_t tile_start(const TileArgs &a, int64_t j) { return j * a.w + (a.offset ? a.w / 2 : 0); }
SW_HD int64_t wrap_once(int64_t x, int64_t n) { return x >= n ? x - n : x; }
SW_HD int64_t slot_a(const TileArgs &a, int64_t j)
{
    int64_t s = 2 * j + a.offset;
    return s >= 2 * a.K ? s - 2 * a.K : s;
}
SW_HD int64_t slot_b(const TileArgs &a, int64_t j)
{
    int64_t s = 2 * j + a.offset + 1;
    return s >= 2 * a.K ? s - 2 * a.K : s;
}
template <class Sch>
SW_HD int64_t slot_base(const TileArgs &a, int64_t s) { return s * (int64_t)Sch::NV * 2 * a.E; }

// Phase p of a solve with Q full phases of H levels and a remainder of rem
// levels: Up(H), Diamond x (Q-1) at offsets 1, 0, 1, ..., Down(H) at offset
// Q mod 2, then Up(rem), Down(rem) at offsets 0, 1 (Sec. 4.2's zig-zag).
SW_HD int phase_count(int64_t Q, int64_t rem) { return (int)((Q >= 1 ? Q + 1 : 0) + (rem > 0 ? 2 : 0)); }
SW_HD void phase_at(int64_t Q, int64_t rem, int H, int64_t p, int32_t &kind, int32_t &levels,
                    int32_t &offset)
{
    if (Q >= 1 && p <= Q) {
        if (p == 0) { kind = PH_UP; levels = H; offset = 0; }
        else if (p < Q) { kind = PH_DIAMOND; levels = 2 * H - 1; offset = (int32_t)(p & 1); }
        else { kind = PH_DOWN; levels = H; offset = (int32_t)(Q & 1); }
        return;
    }
    const int64_t q = p - (Q >= 1 ? Q + 1 : 0);  // 0: remainder Up, 1: remainder Down
    kind = q == 0 ? PH_UP : PH_DOWN;
    levels = (int32_t)rem;
    offset = q == 0 ? 0 : 1;
}

// Tiles of phase p - 1 (p >= 1) whose outputs tile j of phase p reads, written to
// deps[0..count).  A Diamond or Down tile at offset o reads slots 2j + o and
// 2j + o + 1, written by the previous phase (offset 1 - o) as tiles j, j + 1
// (o = 1) or j - 1, j (o = 0).  A remainder Up reads the state, whose points
// [j w, j w + w) the previous Down wrote as tile j (offset 0) or tiles j - 1, j
// (offset 1).  The same tiles were the last to read the slots and points that
// tile j rewrites, so these are also its write-after-read dependencies.
SW_HD int phase_deps(int64_t Q, int64_t rem, int H, int64_t K, int64_t p, int64_t j, int64_t deps[2])
{
    int32_t kind, levels, off, kind0, levels0, off0;
    phase_at(Q, rem, H, p, kind, levels, off);
    phase_at(Q, rem, H, p - 1, kind0, levels0, off0);
    const int64_t left = j == 0 ? K - 1 : j - 1, right = j + 1 == K ? 0 : j + 1;
    if (kind == PH_UP) {
        if (off0 == 0) { deps[0] = j; return 1; }
        deps[0] = left; deps[1] = j;
        return 2;
    }
    if (off == 1) { deps[0] = j; deps[1] = right; }
    else { deps[0] = left; deps[1] = j; }
    return 2;
}

// Number of levels a tile computes in this launch.
SW_HD int tile_levels(const TileArgs &a)
{
    if (a.kind == PH_UP) return a.levels < a.H ? a.levels : a.H - 1;
    if (a.kind == PH_DIAMOND) return 2 * a.H - 1;
    return a.levels;
}

// Half-width (in units of r) of the set of points computed at relative level s;
// the set is [w/2 - r m, w/2 + r m).
SW_HD int half_width(const TileArgs &a, int s)
{
    if (a.kind == PH_UP) return a.H - s;
    if (a.kind == PH_DOWN) return s;
    return s < 2 * a.H - s ? s : 2 * a.H - s;
}

// With Dirichlet ends, the tile of an offset phase that wraps past the end of
// the grid has the wall at its centre: left half = the last w/2 points, right
// half = the first w/2 points, each seeing ghost values across the wall.
SW_HD bool straddles_wall(const TileArgs &a, int64_t j)
{
    return a.bc != BC_PERIODIC && a.offset == 1 && j == a.K - 1;
}

// In unshifted phases of a non-periodic problem, the first tile's left edge and
// the last tile's right edge are the ends of the domain.
SW_HD int32_t tile_ends(const TileArgs &a, int64_t j)
{
    if (a.bc == BC_PERIODIC || a.offset != 0) return 0;
    return (j == 0 ? 1 : 0) | (j == a.K - 1 ? 2 : 0);
}

// Reflective (insulated) ends, heat only (r = 1): the ghost beyond an end mirrors
// the point one inside it (T_{-1} = T_1, T_N = T_{N-2}).  For a lane whose first
// point is the domain's first point, its left halo entry i mirrors ext index
// 2R - i; for a lane whose last point is the domain's last, its right halo entry
// i mirrors ext index P + R - 2 - i (ext covers the lane's points and R halo
// points per side).
SW_HD constexpr int mirror_left_src(int R, int i) { return 2 * R - i; }
SW_HD constexpr int mirror_right_src(int P, int R, int i) { return P + R - 2 - i; }

// Load lane g's rows.  Up: row 0 = the current full level from the state.
// Diamond/Down: both rows from the two source slots, plus the r points just
// outside the tile on each side (row 1: the previous triangles' tips, read once
// at the widest level).
template <class Sch, int P>
SW_HD void lane_load(const TileArgs &a, int64_t j, int g, double (&r0)[Sch::NV][P],
                     double (&r1)[Sch::NV][P], double (&hl)[Sch::NV][Sch::R],
                     double (&hr)[Sch::NV][Sch::R])
{
    constexpr int NV = Sch::NV, R = Sch::R;
    const int half = a.w / 2;
    const int x0 = g * P;
    if (a.kind == PH_UP) {
        const int64_t g0 = tile_start(a, j);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                r0[v][k] = a.state[(int64_t)v * a.n + g0 + x0 + k];
                r1[v][k] = 0.0;
            }
#pragma unroll
            for (int i = 0; i < R; ++i) { hl[v][i] = 0.0; hr[v][i] = 0.0; }
        }
        return;
    }
    const double *sa = a.edges + slot_base<Sch>(a, slot_a(a, j));
    const double *sb = a.edges + slot_base<Sch>(a, slot_b(a, j));
    const bool left = x0 < half;
    const double *src = left ? sa : sb;
    const int e0 = left ? x0 + R : x0 - half;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            r0[v][k] = src[(v * 2 + 0) * a.E + e0 + k];
            r1[v][k] = src[(v * 2 + 1) * a.E + e0 + k];
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            hl[v][i] = sa[(v * 2 + 1) * a.E + i];
            hr[v][i] = sb[(v * 2 + 1) * a.E + half + i];
        }
    }
    // Dirichlet: in unshifted phases the first tile starts at the left wall and
    // the last ends at the right wall, so the points beyond them are ghosts.
    if (a.bc == BC_DIRICHLET && a.offset == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                if (j == 0) hl[v][i] = a.c.ghost_l[v];
                if (j == a.K - 1) hr[v][i] = a.c.ghost_r[v];
            }
        }
    }
}

// Where a tile's final rows go.  Up and Diamond write the new L slot (into a:
// positions x < w/2 + r) and R slot (into b: x >= w/2 - r) of both rows; an Up
// that stops below the triangle tip, and every Down, also write their top
// level's computed points [lo, hi) to the state.
template <class Sch>
SW_HD void store_edge_point(const TileArgs &a, double *sa, double *sb, int v, int x, double row0,
                            double row1)
{
    constexpr int R = Sch::R;
    const int half = a.w / 2;
    if (x < half + R) {
        sa[(v * 2 + 0) * a.E + x] = row0;
        sa[(v * 2 + 1) * a.E + x] = row1;
    }
    if (x >= half - R) {
        sb[(v * 2 + 0) * a.E + x - (half - R)] = row0;
        sb[(v * 2 + 1) * a.E + x - (half - R)] = row1;
    }
}

// Top level written to the state by this phase (-1: none) and its computed set.
template <class Sch>
SW_HD int store_top_level(const TileArgs &a, int &lo, int &hi)
{
    constexpr int R = Sch::R;
    int top = -1;
    if (a.kind == PH_DOWN) top = a.levels;
    else if (a.kind == PH_UP && a.levels < a.H) top = a.levels;
    const int m = a.kind == PH_DOWN ? top : a.H - top;
    lo = a.w / 2 - R * m;
    hi = a.w / 2 + R * m;
    return top;
}

// Top-level value of tile position x written to the state (x in [lo, hi)).
template <class Sch>
SW_HD void store_top_point(const TileArgs &a, int64_t g0, int top, int v, int x, double row0, double row1)
{
    a.state[(int64_t)v * a.n + wrap_once(g0 + x, a.n)] = (top & 1) ? row1 : row0;
}

// Store lane g's rows (its P points at positions g P + k).
template <class Sch, int P>
SW_HD void lane_store(const TileArgs &a, int64_t j, int g, const double (&r0)[Sch::NV][P],
                      const double (&r1)[Sch::NV][P])
{
    constexpr int NV = Sch::NV;
    const int x0 = g * P;
    if (a.kind != PH_DOWN) {
        double *sa = a.edges + slot_base<Sch>(a, slot_a(a, j));
        double *sb = a.edges + slot_base<Sch>(a, slot_b(a, j));
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int k = 0; k < P; ++k) store_edge_point<Sch>(a, sa, sb, v, x0 + k, r0[v][k], r1[v][k]);
    }
    int lo, hi;
    const int top = store_top_level<Sch>(a, lo, hi);
    if (top < 0) return;
    const int64_t g0 = tile_start(a, j);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (x0 + k >= lo && x0 + k < hi) store_top_point<Sch>(a, g0, top, v, x0 + k, r0[v][k], r1[v][k]);
}

// ---- per-element lane bounds with residues fixed by the level's position ----
//
// The computed set [lo, hi) moves by exactly r per level, so lo and hi modulo P
// depend only on s modulo G = max(P/r, 2) and on whether the set is widening
// (Down, lower half of a Diamond: lo = w/2 - r s) or narrowing (Up, upper half of
// a Diamond: lo = w/2 - r (H - s) or w/2 - r (2H - s)).  With levels unrolled in
// groups that start at s = 1 mod G, the residues are compile-time constants and
// element k of lane l is computed iff la <= l < lb below.
SW_HD constexpr int group_len(int P, int R) { return P / R < 2 ? 2 : P / R; }
SW_HD constexpr int pos_mod(int x, int m) { return ((x % m) + m) % m; }
SW_HD bool level_widening(const TileArgs &a, int s)
{
    return a.kind == PH_DOWN || (a.kind == PH_DIAMOND && s <= a.H);
}
SW_HD void element_lane_bounds(int P, int R, bool widening, int s_mod, int lo, int hi, int base,
                               int k, int &la, int &lb)
{
    const int ra = pos_mod(widening ? -R * s_mod : R * s_mod, P);  // lo mod P
    const int rb = pos_mod(widening ? R * s_mod : -R * s_mod, P);  // hi mod P
    // 0 <= lo <= hi <= w (the computed set never leaves the tile): plain shifts
    const int qa = (int)((unsigned)lo / (unsigned)P) - base, qb = (int)((unsigned)hi / (unsigned)P) - base;
    la = k >= ra ? qa : qa + 1;
    lb = k < rb ? qb + 1 : qb;
}

// Lanes (numbered from `base`) that hold at least one computed point: [lmin, lmax).
SW_HD void element_lane_span(int P, int R, bool widening, int s_mod, int lo, int hi, int base,
                             int &lmin, int &lmax)
{
    const int rb = pos_mod(widening ? R * s_mod : -R * s_mod, P);
    lmin = (int)((unsigned)lo / (unsigned)P) - base;                     // element P-1 is past lo's residue
    lmax = (int)((unsigned)hi / (unsigned)P) - base + (rb > 0 ? 1 : 0);  // element 0 is below hi's residue
}

// Lane-local bounds [klo, khi) of the points computed at relative level s.
SW_HD void lane_bounds(const TileArgs &a, int s, int g, int P, int R, int &klo, int &khi)
{
    const int m = half_width(a, s);
    const int half = a.w / 2;
    int lo = half - R * m - g * P, hi = half + R * m - g * P;
    klo = lo < 0 ? 0 : (lo > P ? P : lo);
    khi = hi < 0 ? 0 : (hi > P ? P : hi);
}

}  // namespace sw
