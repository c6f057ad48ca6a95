// Device code of the swept tile kernel (Up / Diamond / Down phases) and of its
// batched form, with their per-scheme launchers.  Each scheme's kernels are
// instantiated in a translation unit of their own (tiles_heat.hip,
// tiles_ks.hip, tiles_euler.hip), which keeps the unrolled level loops of the
// three schemes compiling in parallel.
//
// One work-group is one node of the swept rule (the paper's Shared variant maps
// a node to a block, Sec. 5.1), but the two-row working array lives in VGPRs
// instead of shared memory: lane g owns P consecutive points of both rows.  Per
// level a lane needs r points of the source row from each neighbouring lane;
// inside a wave they arrive through DPP row moves across the whole wave
// (wave_shr:1 / wave_shl:1), between waves through a small double-buffered LDS
// exchange with one barrier per level.  A one-wave tile therefore runs
// barrier-free.  A stencil update is no matrix product, so MFMA has no role; the
// kernel is bound by FP64 VALU issue (fused multiply-adds where the canonical
// rules write them, nothing contracted implicitly).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "kernels.hpp"

namespace sw {

namespace {

constexpr int DPP_WAVE_SHL1 = 0x130;  // lane i receives lane i+1
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane i receives lane i-1

// Zero-filling DPP move: lanes whose source lies outside the wave read 0.
template <int CTRL>
__device__ __forceinline__ double dpp_zero(double v)
{
    const unsigned long long x = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)x, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(x >> 32), CTRL, 0xF, 0xF, true);
    const unsigned long long r = ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo;
    return __builtin_bit_cast(double, r);
}

// A level of a scheme whose per-cell quantities neighbouring lanes share (Euler):
// each lane evaluates the pressures, pressure ratios and right-interface fluxes of
// its own P cells only and takes the three it lacks from outside its run -- the
// pressures of cells -1 and P, the ratio of cell P and the flux through its left
// interface -- from the neighbouring lanes through DPP.  Every value is the same
// operation on the same operands as in Sch::level, so the result is identical; a
// lane evaluates P of each quantity instead of P + 4 pressures, P + 2 ratios and
// P + 1 fluxes.  Valid where no halo is patched into the level (one-wave tiles off
// the walls, below the widest level): there the wave's edge lanes, which receive
// zeros, hold no computed point, just as with the halo gather.
template <class Sch, int P, bool SEL>
__device__ __forceinline__ void level_exchange(double (&dst)[Sch::NV][P], const double (&ext)[Sch::NV][P + 2 * Sch::R],
                                               bool predictor, const Consts &c, const bool (&in)[P])
{
    constexpr int NV = Sch::NV, R = Sch::R;
    static_assert(NV == 3 && R == 2, "laid out for the Euler rule");
    double pres[P + 2];  // pres[k + 1]: own cell k; pres[0]: cell -1; pres[P + 1]: cell P
#pragma unroll
    for (int k = 0; k < P; ++k) pres[k + 1] = Sch::pressure(ext[0][R + k], ext[1][R + k], ext[2][R + k], c);
    pres[0] = dpp_zero<DPP_WAVE_SHR1>(pres[P]);
    pres[P + 1] = dpp_zero<DPP_WAVE_SHL1>(pres[1]);
    double pr[P + 1];  // pr[k]: ratio at cell k, k = 0 .. P
#pragma unroll
    for (int k = 0; k < P; ++k) pr[k] = Sch::pratio(pres[k], pres[k + 1], pres[k + 2]);
    pr[P] = dpp_zero<DPP_WAVE_SHL1>(pr[0]);
    // The last cell's right-interface flux first: the right neighbour needs it as its
    // left-interface flux.  The others are evaluated as the update streams over the cells.
    double flast[3];
    {
        const double qb[3] = {ext[0][R + P - 1], ext[1][R + P - 1], ext[2][R + P - 1]};
        const double qc[3] = {ext[0][R + P], ext[1][R + P], ext[2][R + P]};
        Sch::flux(qb, qc, pr[P - 1], pr[P], c, flast);
    }
    double fprev[3];  // flux through the interface between cells -1 and 0
#pragma unroll
    for (int v = 0; v < 3; ++v) fprev[v] = dpp_zero<DPP_WAVE_SHR1>(flast[v]);
    const double coef = predictor ? c.hlam : c.lam;
    double val[NV][P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double fnext[3];  // flux through the interface between cells k and k + 1
        if (k == P - 1) {
#pragma unroll
            for (int v = 0; v < 3; ++v) fnext[v] = flast[v];
        } else {
            const double qb[3] = {ext[0][R + k], ext[1][R + k], ext[2][R + k]};
            const double qc[3] = {ext[0][R + k + 1], ext[1][R + k + 1], ext[2][R + k + 1]};
            Sch::flux(qb, qc, pr[k], pr[k + 1], c, fnext);
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const double base = predictor ? ext[v][R + k] : dst[v][k];
            val[v][k] = sw_fma(coef, fprev[v] - fnext[v], base);
            if (!SEL && in[k]) dst[v][k] = val[v][k];
            fprev[v] = fnext[v];
        }
    }
    if (SEL) {
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 3; ++v) dst[v][k] = in[k] ? val[v][k] : dst[v][k];
    }
}

// Select-free narrowing (see level_step) in class P of a one-wave tile, for schemes that
// enable it, where it issues fewer instructions per level than selecting the computed
// set: 4r boundary points, each a scalar lane mask, an address select and NV LDS stores,
// against two selects per point and variable (heat: P = 8 and 16; the lanes' points must
// not straddle a 16-point LDS block, so P divides 16).
template <class Sch, int P>
constexpr bool free_class()
{
    return Sch::FREE_ONE_WAVE && 16 % P == 0 && 4 * Sch::R * (2 + Sch::NV) < 2 * P * Sch::NV;
}

// Select-free widening in the select-free classes where it pays: 4r points restored per
// level, each a lane compare, two selects and one LDS load per variable (heat: P = 16).
template <class Sch, int P>
constexpr bool free_widen_class()
{
    return free_class<Sch, P>() && 4 * Sch::R * (1 + 3 * Sch::NV) < 2 * P * Sch::NV;
}

// LDS rows of a one-wave tile: tile point x at x + x/16 (one padding double per 16,
// which keeps the stride-P accesses of every class layout and the point-major passes
// free of bank conflicts).  Tiles of 8 or more points per lane also hold a sink in each
// row for stores that no lane needs: one double per lane, the padding double after
// 16-point block l for lane l when the row has 64 blocks (w = 1024), else 64 doubles
// appended to the row.
constexpr int wave_span(int P0) { return 68 * P0 + (P0 == 8 ? 64 : 0); }
__device__ __forceinline__ int lds_pos(int x) { return x + (x >> 4); }
template <int P0>
__device__ __forceinline__ int lds_sink(int lane)
{
    static_assert(P0 == 8 || P0 == 16, "the LDS rows hold a sink at 8 and 16 points per lane");
    if constexpr (P0 == 16) return 17 * lane + 16;
    else return 68 * P0 + lane;
}

constexpr int floor_div(int x, int m) { return x >= 0 ? x / m : -((-x + m - 1) / m); }

// f(std::integral_constant<int, i>) for i = 0 .. N-1, the index a compile-time constant.
template <class F, int... I>
__device__ __forceinline__ void unroll_seq(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll(F &&f)
{
    unroll_seq(f, std::make_integer_sequence<int, N>{});
}

// Lane l (wave-uniform, 0 <= l < 64) as a per-lane condition: one scalar shift builds the
// mask, and selects take it as their condition operand (no vector compare).
__device__ __forceinline__ bool is_lane(int l)
{
    return __builtin_amdgcn_inverse_ballot_w64(1ull << l);
}

// One level of a tile: gather the source row with halos, then update the points
// of the computed set [w/2 - r m, w/2 + r m).  Element k of the wave's lanes is
// inside for a contiguous range of lanes whose ends take only two values each
// over k (their residues are compile-time), so a level needs four lane compares
// however many points a lane holds.  A wave with no point inside skips the level
// (after publishing its boundary values for its neighbours), which recovers most
// of the idle half of a triangle in multi-wave tiles.
//
// qa, qb: the wave-uniform lane quotients of the set's ends relative to the first point
// the lanes hold, lo = P qa + ra and hi = P qb + rb with the compile-time residues ra,
// rb; run_group derives them from one pair per group of levels, so a level spends no
// scalar arithmetic on them and its lane compares repeat within the group.
//
// Narrowing levels of a one-wave class layout where free_class holds (P0 > 0: the tile's
// points per lane; `stage` its LDS rows) update every point of the layout unconditionally:
// nothing outside the computed set is read again, but a level's boundary points
// [lo, lo + 2r) and [hi - 2r, hi) are final in its row (the next level of the same
// parity is narrower by 2r per side), so the level after it stores them from its source
// row to the LDS rows, before the level after that overwrites them; the other lanes
// store to their sink, so the store needs no branch.  The last level's points are
// parked with its row, and a Diamond's first narrowing level stores the widest level's.
//
// WIDE: the level may be the widest one of a Diamond or Down (the only level that reads
// the tile's outer halo); one-wave segments that cannot reach it compile the test out.
template <class Sch, int P, bool ODD, bool MULTI, bool WALL, bool INC, int SMOD, int P0 = 0, bool WIDE = true>
__device__ __forceinline__ void level_step(const TileArgs &a, int g, int NW, int s, int org, int qa, int qb,
                                           const double (&src)[Sch::NV][P], double (&dst)[Sch::NV][P],
                                           const double (&hl)[Sch::NV][Sch::R],
                                           const double (&hr)[Sch::NV][Sch::R],
                                           double (*xch)[16][2][Sch::NV][Sch::R], double *stage = nullptr)
{
    constexpr bool FREE = !MULTI && P0 > 0 && !INC && free_class<Sch, P>();
    constexpr bool FREE_W = !MULTI && P0 > 0 && INC && free_widen_class<Sch, P>();
    constexpr int NV = Sch::NV, R = Sch::R;
    const int lane = g & 63, wave = g >> 6, buf = s & 1;
    if (MULTI) {
        // publish this wave's first and last R points (wave positions p = lane P + k)
        if (lane * P < R) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int k = 0; k < P; ++k)
                    if (lane * P + k < R) xch[buf][wave][0][v][lane * P + k] = src[v][k];
        }
        if (lane * P + P > 64 * P - R) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int k = 0; k < P; ++k)
                    if (lane * P + k >= 64 * P - R) xch[buf][wave][1][v][lane * P + k - (64 * P - R)] = src[v][k];
        }
        __syncthreads();
    }
    const int half = a.w >> 1;
    constexpr int RA = pos_mod(INC ? -R * SMOD : R * SMOD, P);   // lo mod P
    constexpr int RB = pos_mod(INC ? R * SMOD : -R * SMOD, P);   // hi mod P
    // first lane of this wave (a one-wave tile is lane 0 onwards)
    const int base = MULTI ? __builtin_amdgcn_readfirstlane(g & ~63) : 0;
    // select-free widening: the next level's halo [lo - 2r, lo) and [hi, hi + 2r) of the row
    // being written keeps its inserted values, read from the LDS row before the update
    // (every lane reads its own element, inside the layout) and selected back after it
    double keep[2][2 * R][NV];
    if constexpr (FREE_W) {
        constexpr int SPAN = wave_span(P0);
        const double *own = stage + (ODD ? SPAN : 0) + lds_pos(org + g * P);
        unroll<2 * R>([&](auto I) {
            constexpr int kl = pos_mod(RA - 2 * R + decltype(I)::value, P);
            constexpr int kr = pos_mod(RB + decltype(I)::value, P);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                keep[0][decltype(I)::value][v] = own[2 * v * SPAN + kl];
                keep[1][decltype(I)::value][v] = own[2 * v * SPAN + kr];
            }
        });
    }

    if (MULTI) {
        // lanes of this wave holding at least one computed point: [lmin, lmax); a
        // one-wave tile always holds some (the computed set is never empty)
        const int lmin = qa - base, lmax = qb - base + (RB > 0 ? 1 : 0);
        if (!(lmin < 64 && lmax > 0 && lmin < lmax)) return;
    }

    // ext[v][i] holds tile position g P - R + i, ext[v][R + P + i] position g P + P + i.
    static_assert(P >= R || P == 1, "a lane's halo spans at most its neighbours, or one point per lane");
    double ext[NV][P + 2 * R];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int k = 0; k < P; ++k) ext[v][R + k] = src[v][k];
        if constexpr (P >= R) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                ext[v][i] = dpp_zero<DPP_WAVE_SHR1>(src[v][P - R + i]);
                ext[v][R + P + i] = dpp_zero<DPP_WAVE_SHL1>(src[v][i]);
            }
        } else {  // one point per lane: points further away pass through successive lanes
            ext[v][R - 1] = dpp_zero<DPP_WAVE_SHR1>(src[v][0]);
#pragma unroll
            for (int i = R - 2; i >= 0; --i) ext[v][i] = dpp_zero<DPP_WAVE_SHR1>(ext[v][i + 1]);
            ext[v][R + 1] = dpp_zero<DPP_WAVE_SHL1>(src[v][0]);
#pragma unroll
            for (int i = 1; i < R; ++i) ext[v][R + 1 + i] = dpp_zero<DPP_WAVE_SHL1>(ext[v][R + i]);
        }
    }
    const int x0 = org + g * P;  // first tile position of this lane
    // The tile's outer halo is read by the widest level of a Diamond/Down only, once
    // per launch: the hint keeps the common path free of taken branches.
    const bool widest = WIDE && s == a.H && a.kind != PH_UP;
    if (__builtin_expect(widest, 0)) {
        const bool refl = a.bc == BC_REFLECTIVE;  // heat only: R == 1
        if (x0 < R) {
            if (refl && (a.ends & 1)) {
                if constexpr (R == 1)
                    if (x0 == 0) ext[0][0] = ext[0][mirror_left_src(R, 0)];
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (x0 - R + i < 0) ext[v][i] = hl[v][x0 + i];
            }
        }
        if (x0 + P + R > a.w) {
            if (refl && (a.ends & 2)) {
                if constexpr (R == 1)
                    if (x0 + P == a.w) ext[0][R + P] = ext[0][mirror_right_src(P, R, 0)];
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (x0 + P + i >= a.w) ext[v][R + P + i] = hr[v][x0 + P + i - a.w];
            }
        }
    }
    if (MULTI) {
        if (lane * P < R && wave > 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (lane * P - R + i < 0) ext[v][i] = xch[buf][wave - 1][1][v][lane * P + i];
        }
        if (lane * P + P + R > 64 * P && wave < NW - 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (lane * P + P + i >= 64 * P)
                        ext[v][R + P + i] = xch[buf][wave + 1][0][v][lane * P + P + i - 64 * P];
        }
    }
    if (WALL && a.bc == BC_REFLECTIVE) {  // insulated ends meet at the tile centre (heat, R == 1)
        if constexpr (R == 1) {
            if (x0 == half) ext[0][0] = ext[0][mirror_left_src(R, 0)];
            if (x0 + P == half) ext[0][R + P] = ext[0][mirror_right_src(P, R, 0)];
        }
    } else if (WALL) {  // Dirichlet wall at the tile centre: across it lie the ghost values
        if (x0 >= half && x0 - R < half) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (x0 - R + i < half) ext[v][i] = a.c.ghost_l[v];
        }
        if (x0 < half && x0 + P + R > half) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (x0 + P + i >= half) ext[v][R + P + i] = a.c.ghost_r[v];
        }
    }
    if constexpr (FREE) {
        // the previous level's boundary points, [lo', lo' + 2r) and [hi' - 2r, hi') with
        // lo' = lo - r and hi' = hi + r, are final in the source row: into its LDS row
        // before the level after this one overwrites them (the values are long computed,
        // so the stores do not wait on this level's arithmetic)
        constexpr int SPAN = wave_span(P0);
        double *own = stage + (ODD ? 0 : SPAN) + lds_pos(x0);
        double *sink = stage + (ODD ? 0 : SPAN) + lds_sink<P0>(lane);
        unroll<2 * R>([&](auto I) {
            constexpr int xl = RA - R + decltype(I)::value, xr = RB - R + decltype(I)::value;
            constexpr int kl = pos_mod(xl, P), kr = pos_mod(xr, P);
            double *pl = is_lane(qa + floor_div(xl, P)) ? own + kl : sink;
            double *pr = is_lane(qb + floor_div(xr, P)) ? own + kr : sink;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                pl[2 * v * SPAN] = src[v][kl];
                pr[2 * v * SPAN] = src[v][kr];
            }
        });
    }
    bool in[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        // element k is computed on lanes [la, lb); la, lb take two values each over k
        const int la = (k >= RA ? qa : qa + 1) - base, lb = (k < RB ? qb + 1 : qb) - base;
        in[k] = FREE || FREE_W || (lane >= la && lane < lb);
    }
    constexpr bool SEL = !FREE && !FREE_W && (MULTI || Sch::SELECT_ONE_WAVE);
    if constexpr (Sch::LANE_EXCHANGE && !MULTI && !WALL) {
        if (__builtin_expect(!widest, 1))   // the widest level reads the patched halo
            level_exchange<Sch, P, SEL>(dst, ext, ODD, a.c, in);
        else
            Sch::template level<P, SEL>(dst, ext, ODD, a.c, in);
    } else {
        Sch::template level<P, SEL>(dst, ext, ODD, a.c, in);
    }
    if constexpr (FREE_W) {
        // lanes outside [0, 64) hold none of these points (the class's last level: the
        // next level fetches a wider layout from LDS)
        unroll<2 * R>([&](auto I) {
            constexpr int xl = RA - 2 * R + decltype(I)::value, xr = RB + decltype(I)::value;
            constexpr int kl = pos_mod(xl, P), kr = pos_mod(xr, P);
            const bool tl = lane == qa + floor_div(xl, P), tr = lane == qb + floor_div(xr, P);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                dst[v][kl] = tl ? keep[0][decltype(I)::value][v] : dst[v][kl];
                dst[v][kr] = tr ? keep[1][decltype(I)::value][v] : dst[v][kr];
            }
        });
    }
}


// One-wave level loops that cannot reach the widest level compile its test out, and the
// widest level runs on its own.  Not for the scheme whose levels exchange per-cell
// quantities between lanes (Euler): without the test the compiler schedules those
// levels one at a time instead of interleaving two, and the Sod Diamond ran 17 % slower.
template <class Sch>
constexpr bool peel_widest() { return !Sch::LANE_EXCHANGE; }

// Levels s0 + U, s0 + U + 1, ... of one aligned group (widening: m = s and s0 = A
// mod G; narrowing: m = mtop - s and m = -A mod G at s0; so the row parity and the
// residues of the computed set are compile-time).  The set's ends move by r
// per level, so their lane quotients at level s0 + U are the group's (qa0, qb0)
// plus compile-time offsets.
template <class Sch, int P, bool MULTI, bool WALL, bool INC, int A, int U, int G, int P0, bool WIDE>
__device__ __forceinline__ void run_group(const TileArgs &a, int g, int NW, int s0, int s_last, int qa0, int qb0,
                                          int org, bool full, double (&r0)[Sch::NV][P], double (&r1)[Sch::NV][P],
                                          const double (&hl)[Sch::NV][Sch::R],
                                          const double (&hr)[Sch::NV][Sch::R],
                                          double (*xch)[16][2][Sch::NV][Sch::R], double *stage)
{
    if constexpr (U < G) {
        const int s = s0 + U;
        if (full || s <= s_last) {
            constexpr int R = Sch::R, SMOD = (A + U) % G, S0 = A % G;
            constexpr int RA0 = pos_mod(INC ? -R * S0 : R * S0, P), RB0 = pos_mod(INC ? R * S0 : -R * S0, P);
            constexpr int RA = pos_mod(INC ? -R * SMOD : R * SMOD, P), RB = pos_mod(INC ? R * SMOD : -R * SMOD, P);
            constexpr int D = INC ? -R * U : R * U;   // lo has moved by D since s0, hi by -D
            static_assert((RA0 + D - RA) % P == 0 && (RB0 - D - RB) % P == 0, "ends stay on their residues");
            constexpr int DA = (RA0 + D - RA) / P, DB = (RB0 - D - RB) / P;
            if constexpr (((A + U) & 1) != 0)
                level_step<Sch, P, true, MULTI, WALL, INC, SMOD, P0, WIDE>(a, g, NW, s, org, qa0 + DA, qb0 + DB, r0,
                                                                           r1, hl, hr, xch, stage);
            else
                level_step<Sch, P, false, MULTI, WALL, INC, SMOD, P0, WIDE>(a, g, NW, s, org, qa0 + DA, qb0 + DB, r1,
                                                                            r0, hl, hr, xch, stage);
            run_group<Sch, P, MULTI, WALL, INC, A, U + 1, G, P0, WIDE>(a, g, NW, s0, s_last, qa0, qb0, org, full,
                                                                       r0, r1, hl, hr, xch, stage);
        }
    }
}

// Levels [s_first, s_last] (aligned to residue A as in run_group) in full groups plus
// one partial group.
// P0 > 0: a one-wave class layout of a tile with P0 points per lane, LDS rows `stage`.
template <class Sch, int P, bool MULTI, bool WALL, bool INC, int A = 1, int P0 = 0, bool WIDE = true>
__device__ __forceinline__ void run_segment(const TileArgs &a, int g, int NW, int s_first, int s_last,
                                            int mtop, double (&r0)[Sch::NV][P], double (&r1)[Sch::NV][P],
                                            const double (&hl)[Sch::NV][Sch::R],
                                            const double (&hr)[Sch::NV][Sch::R],
                                            double (*xch)[16][2][Sch::NV][Sch::R], int org = 0,
                                            double *stage = nullptr)
{
    constexpr int R = Sch::R, G = group_len(P, R), S0 = A % G;
    constexpr int RA0 = pos_mod(INC ? -R * S0 : R * S0, P), RB0 = pos_mod(INC ? R * S0 : -R * S0, P);
    const int half = a.w >> 1;
    // the computed set [lo, hi) relative to the first point the lanes hold (org: 0 for
    // the whole tile, w/2 - 32 P for a one-wave layout packed around the tile centre)
    // lies inside the lanes' points, so lo - ra and hi - rb are non-negative multiples of P
    auto quotients = [&](int s0, int &qa0, int &qb0) {
        const int m0 = INC ? s0 : mtop - s0;
        qa0 = __builtin_amdgcn_readfirstlane((int)((unsigned)(half - R * m0 - org - RA0) / P));
        qb0 = __builtin_amdgcn_readfirstlane((int)((unsigned)(half + R * m0 - org - RB0) / P));
    };
    int s0 = s_first, qa0, qb0;
    for (; s0 + G - 1 <= s_last; s0 += G) {
        quotients(s0, qa0, qb0);
        run_group<Sch, P, MULTI, WALL, INC, A, 0, G, P0, WIDE>(a, g, NW, s0, s_last, qa0, qb0, org, true, r0, r1,
                                                               hl, hr, xch, stage);
    }
    if (s0 <= s_last) {
        quotients(s0, qa0, qb0);
        run_group<Sch, P, MULTI, WALL, INC, A, 0, G, P0, WIDE>(a, g, NW, s0, s_last, qa0, qb0, org, false, r0, r1,
                                                               hl, hr, xch, stage);
    }
}

template <class Sch, int P, bool MULTI, bool WALL>
__device__ __forceinline__ void run_levels(const TileArgs &a, int g, int NW, double (&r0)[Sch::NV][P],
                                           double (&r1)[Sch::NV][P], const double (&hl)[Sch::NV][Sch::R],
                                           const double (&hr)[Sch::NV][Sch::R],
                                           double (*xch)[16][2][Sch::NV][Sch::R])
{
    const int nlev = tile_levels(a);
    if (a.kind == PH_UP) {
        run_segment<Sch, P, MULTI, WALL, false>(a, g, NW, 1, nlev, a.H, r0, r1, hl, hr, xch);
    } else if (a.kind == PH_DOWN) {
        run_segment<Sch, P, MULTI, WALL, true>(a, g, NW, 1, nlev, 0, r0, r1, hl, hr, xch);
    } else {
        run_segment<Sch, P, MULTI, WALL, true>(a, g, NW, 1, a.H, 0, r0, r1, hl, hr, xch);
        run_segment<Sch, P, MULTI, WALL, false>(a, g, NW, a.H + 1, nlev, 2 * a.H, r0, r1, hl, hr, xch);
    }
}

// ---- one-wave tiles: the computed set packed into as few points per lane as it needs ----
//
// A triangle's computed set narrows (and a Diamond's lower half widens) by r
// points per side per level, so a fixed layout of P0 points per lane leaves half
// of the lanes idle on average (the idle threads of the paper's Results).  A
// one-wave tile therefore keeps both rows of the whole tile in LDS and holds in
// registers only a class layout: the 64 P points [w/2 - 32 P, w/2 + 32 P) centred
// in the tile, lane g owning P consecutive ones, with P the smallest class (1, 2, 4, 8,
// and for 16-point tiles 12 and 16) whose layout holds the level's computed set and
// its halo, r m + r <= 32 P.  At a change of class the lanes park their rows in LDS and fetch
// the next layout; positions outside the layout keep their values there (inserted
// edges not yet reached by a widening set, finished values left behind by a
// narrowing one).  The computed set then covers about four fifths of the lane slots
// instead of half.  Row loads and stores go through the same LDS copy,
// point-major, so every global access instruction moves 64 consecutive doubles.
//
// LDS position of tile point x: x + x/16 (one padding double per 16), which keeps
// the stride-P accesses of every class layout and the point-major passes free of
// bank conflicts.
constexpr int kMinClass = 1;   // the narrowest levels (r m + r <= 32) run one point per lane
// The classes above and below P.  Tiles of 16 points per lane of a scheme with CLASS12
// have a 12-point class between 8 and 16: the levels with 256 < r m + r <= 384 then run
// at three quarters of the widest class's lane slots.
template <class Sch>
constexpr int next_class(int P0, int P)
{
    return Sch::CLASS12 && P0 == 16 && P == 8 ? 12 : (P == 12 ? 16 : 2 * P);
}
template <class Sch>
constexpr int prev_class(int P0, int P)
{
    return Sch::CLASS12 && P0 == 16 && P == 16 ? 12 : (P == 12 ? 8 : P / 2);
}

// Widening from class P: the next class up starts at level m = 32 P / r (the first one
// class P cannot hold) or a few levels earlier, at a multiple of its group length, so
// that its levels keep compile-time residues from residue 0.
template <class Sch, int P0, int P>
constexpr int widen_switch()
{
    constexpr int x = 32 * P / Sch::R, G = group_len(next_class<Sch>(P0, P), Sch::R);
    return x - x % G;
}

// Narrowing from class P (m = mtop - s): the next class down holds the levels with
// m <= 32 Pp / r - 1 and starts at the first of them, where m = -1 modulo its group
// length.  Narrowing segments take their compile-time residues from m (the residue A = 1
// means m = -A at the segment's first level), which holds whatever mtop is modulo the
// group length; mtop is even, so the row parity follows m's as well.
template <class Sch, int P0, int P>
__device__ __forceinline__ int narrow_switch(int mtop)
{
    return mtop - 32 * prev_class<Sch>(P0, P) / Sch::R + 1;
}

template <class Sch, int P, int SPAN>
__device__ __forceinline__ void fetch_rows(const double *stage, int org, int lane, double (&r0)[Sch::NV][P],
                                           double (&r1)[Sch::NV][P])
{
#pragma unroll
    for (int v = 0; v < Sch::NV; ++v)
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int i = lds_pos(org + lane * P + k);
            r0[v][k] = stage[(2 * v + 0) * SPAN + i];
            r1[v][k] = stage[(2 * v + 1) * SPAN + i];
        }
}

// Park the rows in LDS at the end of a class.  After select levels the registers mirror
// LDS outside the computed sets and the whole layout is written back; after select-free
// levels only the rows' computed sets are valid: row q of the last level s on the set
// of level s, the other row on the set of level s - 1 (everything else in LDS is already
// current, and a widening run leaves nothing else behind either).
template <class Sch, int P, int P0>
__device__ __forceinline__ void park_rows(const TileArgs &a, double *stage, int org, int lane, int s_last,
                                          const double (&r0)[Sch::NV][P], const double (&r1)[Sch::NV][P])
{
    constexpr int R = Sch::R, SPAN = wave_span(P0);
    const int half = a.w >> 1;
    const int mq = half_width(a, s_last), mp = half_width(a, s_last - 1);
    // relative to the layout: [lo, hi) of the last level's row and of the other row
    const int lo_q = half - R * mq - org, hi_q = half + R * mq - org;
    const int lo_p = half - R * mp - org, hi_p = half + R * mp - org;
    const bool q1 = (s_last & 1) != 0;   // the last level wrote row 1
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int x = lane * P + k;
        const int i = lds_pos(org + x);
        bool in0 = true, in1 = true;
        if constexpr (free_class<Sch, P>()) {
            const bool in_q = x >= lo_q && x < hi_q, in_p = x >= lo_p && x < hi_p;
            in0 = q1 ? in_p : in_q;
            in1 = q1 ? in_q : in_p;
        }
#pragma unroll
        for (int v = 0; v < Sch::NV; ++v) {
            if (in0) stage[(2 * v + 0) * SPAN + i] = r0[v][k];
            if (in1) stage[(2 * v + 1) * SPAN + i] = r1[v][k];
        }
    }
    __syncthreads();
}

// Narrowing levels [s, s_last] (m = mtop - s) from class P downwards, each class
// handing over to the next one down at narrow_switch.
template <class Sch, int P, int P0, bool WALL>
__device__ __forceinline__ void wave_narrow(const TileArgs &a, int lane, double *stage, int s, int s_last,
                                            int mtop, const double (&hl)[Sch::NV][Sch::R],
                                            const double (&hr)[Sch::NV][Sch::R])
{
    constexpr int NV = Sch::NV, R = Sch::R, SPAN = wave_span(P0);
    int s_next = s_last + 1;   // first level of the class below
    if constexpr (P > kMinClass) s_next = narrow_switch<Sch, P0, P>(mtop);
    const int cap = s_last < s_next - 1 ? s_last : s_next - 1;
    if (s <= cap) {
        const int org = (a.w >> 1) - 32 * P;
        double r0[NV][P], r1[NV][P];
        fetch_rows<Sch, P, SPAN>(stage, org, lane, r0, r1);
        run_segment<Sch, P, false, WALL, false, 1, P0, !peel_widest<Sch>()>(a, lane, 1, s, cap, mtop, r0, r1, hl,
                                                                             hr, nullptr, org, stage);
        park_rows<Sch, P, P0>(a, stage, org, lane, cap, r0, r1);
    }
    if constexpr (P > kMinClass) {
        if (s_last >= s_next)
            wave_narrow<Sch, prev_class<Sch>(P0, P), P0, WALL>(a, lane, stage, s > s_next ? s : s_next, s_last, mtop,
                                                          hl, hr);
    }
}

// Widening levels [s, top] (m = s) from class P upwards; class P holds them while
// r m + r <= 32 P, and the next class starts at widen_switch (0 modulo its group
// length; the smallest class starts at level 1).  The full-width class P0 also runs
// a Diamond's narrowing levels [top + 1, n_last] before handing over to the classes
// below it.
template <class Sch, int P, int P0, bool WALL>
__device__ __forceinline__ void wave_widen(const TileArgs &a, int lane, double *stage, int s, int top,
                                           int n_last, const double (&hl)[Sch::NV][Sch::R],
                                           const double (&hr)[Sch::NV][Sch::R])
{
    constexpr int NV = Sch::NV, R = Sch::R, SPAN = wave_span(P0);
    constexpr int A = P == kMinClass ? 1 : 0;
    const int org = (a.w >> 1) - 32 * P;
    if constexpr (P < P0) {
        constexpr int last = widen_switch<Sch, P0, P>() - 1;
        const int cap = top < last ? top : last;
        if (s <= cap) {
            double r0[NV][P], r1[NV][P];
            fetch_rows<Sch, P, SPAN>(stage, org, lane, r0, r1);
            run_segment<Sch, P, false, WALL, true, A, P0, !peel_widest<Sch>()>(a, lane, 1, s, cap, 0, r0, r1, hl,
                                                                               hr, nullptr, org, stage);
            park_rows<Sch, P, P0>(a, stage, org, lane, cap, r0, r1);
        }
        if (cap < top) wave_widen<Sch, next_class<Sch>(P0, P), P0, WALL>(a, lane, stage, cap + 1, top, n_last, hl, hr);
    } else {
        double r0[NV][P], r1[NV][P];
        fetch_rows<Sch, P, SPAN>(stage, org, lane, r0, r1);
        if constexpr (A == 0 && peel_widest<Sch>()) {
            // the widest level H = 32 P / r is 0 modulo the group length: it runs alone, and
            // the levels below it without the test
            const int below = top == a.H ? top - 1 : top;
            if (s <= below)
                run_segment<Sch, P, false, WALL, true, A, P0, false>(a, lane, 1, s, below, 0, r0, r1, hl, hr,
                                                                     nullptr, org, stage);
            if (below < top)
                run_segment<Sch, P, false, WALL, true, A, P0, true>(a, lane, 1, top, top, 0, r0, r1, hl, hr, nullptr,
                                                                    org, stage);
        } else {
            run_segment<Sch, P, false, WALL, true, A, P0>(a, lane, 1, s, top, 0, r0, r1, hl, hr, nullptr, org, stage);
        }
        const int mtop = 2 * a.H;
        int s_next = n_last + 1;   // first level of the class below
        if constexpr (P > kMinClass) s_next = narrow_switch<Sch, P0, P>(mtop);
        const int cap = n_last < s_next - 1 ? n_last : s_next - 1;
        if (top + 1 <= cap)
            run_segment<Sch, P, false, WALL, false, 1, P0, !peel_widest<Sch>()>(a, lane, 1, top + 1, cap, mtop, r0,
                                                                                r1, hl, hr, nullptr, org, stage);
        park_rows<Sch, P, P0>(a, stage, org, lane, top + 1 <= cap ? cap : top, r0, r1);
        if constexpr (P > kMinClass) {
            if (n_last >= s_next)
                wave_narrow<Sch, prev_class<Sch>(P0, P), P0, WALL>(a, lane, stage, s_next, n_last, mtop, hl, hr);
        }
    }
}

// Global loads and stores of a tile's rows.  COH: coherent at agent scope (relaxed
// agent-scope atomics, which bypass the XCD-private caches' stale copies), for tiles
// whose inputs another XCD may have just written within the same launch.
template <bool COH>
__device__ __forceinline__ double gload(const double *p)
{
    if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <bool COH>
__device__ __forceinline__ void gstore(double *p, double v)
{
    if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

// One tile of one phase on a one-wave work-group.  `stage` holds 2 NV wave_span(P0)
// doubles of LDS: both rows of the tile.
template <class Sch, int P0, bool COH = false>
__device__ __forceinline__ void wave_tile(const TileArgs &args, int64_t j, int lane, double *stage)
{
    constexpr int NV = Sch::NV, R = Sch::R, SPAN = wave_span(P0);
    TileArgs a = args;
    a.ends = tile_ends(args, j);
    const int half = a.w >> 1;
    double hl[NV][R], hr[NV][R];
    __syncthreads();   // the work-group's previous tile has finished with the stage
    if (a.kind == PH_UP) {
        const int64_t g0 = tile_start(a, j);
#pragma unroll
        for (int i = 0; i < P0; ++i) {
            const int x = 64 * i + lane;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                stage[(2 * v + 0) * SPAN + lds_pos(x)] = gload<COH>(a.state + (int64_t)v * a.n + g0 + x);
                stage[(2 * v + 1) * SPAN + lds_pos(x)] = 0.0;
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int i = 0; i < R; ++i) { hl[v][i] = 0.0; hr[v][i] = 0.0; }
    } else {
        // left half from slot a (an R slot: points [-r, w/2)), right half from slot b
        // (an L slot: points [w/2, w + r)); the previous triangles' tips beyond the
        // tile come with them, read once at the widest level
        const double *sa = a.edges + slot_base<Sch>(a, slot_a(a, j));
        const double *sb = a.edges + slot_base<Sch>(a, slot_b(a, j));
#pragma unroll
        for (int i = 0; i < P0; ++i) {
            const int x = 64 * i + lane;
            const double *src = x < half ? sa + x + R : sb + x - half;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                stage[(2 * v + 0) * SPAN + lds_pos(x)] = gload<COH>(src + (v * 2 + 0) * a.E);
                stage[(2 * v + 1) * SPAN + lds_pos(x)] = gload<COH>(src + (v * 2 + 1) * a.E);
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                hl[v][i] = gload<COH>(sa + (v * 2 + 1) * a.E + i);
                hr[v][i] = gload<COH>(sb + (v * 2 + 1) * a.E + half + i);
            }
        }
        if (a.bc == BC_DIRICHLET && a.offset == 0) {   // the unshifted tiles at the walls
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    if (j == 0) hl[v][i] = a.c.ghost_l[v];
                    if (j == a.K - 1) hr[v][i] = a.c.ghost_r[v];
                }
        }
    }
    __syncthreads();
    const int nlev = tile_levels(a);
    const bool wall = straddles_wall(a, j);
    if (a.kind == PH_UP) {
        if (wall) wave_narrow<Sch, P0, P0, true>(a, lane, stage, 1, nlev, a.H, hl, hr);
        else wave_narrow<Sch, P0, P0, false>(a, lane, stage, 1, nlev, a.H, hl, hr);
    } else {
        const int top = a.kind == PH_DOWN ? nlev : a.H;
        const int n_last = a.kind == PH_DIAMOND ? nlev : 0;
        if (wall) wave_widen<Sch, kMinClass, P0, true>(a, lane, stage, 1, top, n_last, hl, hr);
        else wave_widen<Sch, kMinClass, P0, false>(a, lane, stage, 1, top, n_last, hl, hr);
    }
    // every class parked its rows: the stage holds both final rows of the whole tile;
    // new L slot into a (points [0, w/2 + r)), new R slot into b (points [w/2 - r, w))
    if (a.kind != PH_DOWN) {
        double *sa = a.edges + slot_base<Sch>(a, slot_a(a, j));
        double *sb = a.edges + slot_base<Sch>(a, slot_b(a, j));
#pragma unroll
        for (int i = 0; i < P0; ++i) {
            const int x = 64 * i + lane;
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const double val = stage[(2 * v + q) * SPAN + lds_pos(x)];
                    if (x < half + R) gstore<COH>(sa + (v * 2 + q) * a.E + x, val);
                    if (x >= half - R) gstore<COH>(sb + (v * 2 + q) * a.E + x - (half - R), val);
                }
        }
    }
    int lo, hi;
    const int topl = store_top_level<Sch>(a, lo, hi);
    if (topl < 0) return;
    const int64_t g0 = tile_start(a, j);
#pragma unroll
    for (int i = 0; i < P0; ++i) {
        const int x = 64 * i + lane;
        if (x >= lo && x < hi) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                gstore<COH>(a.state + (int64_t)v * a.n + wrap_once(g0 + x, a.n),
                            stage[(2 * v + (topl & 1)) * SPAN + lds_pos(x)]);
        }
    }
}

// One tile of one phase on a multi-wave work-group: load the two rows, run the
// phase's levels with one barrier and LDS exchange per level, store.
template <class Sch, int P>
__device__ __forceinline__ void tile_body(const TileArgs &args, int64_t j, int g, int NW,
                                          double (*xch)[16][2][Sch::NV][Sch::R])
{
    constexpr int NV = Sch::NV, R = Sch::R;
    TileArgs a = args;
    a.ends = tile_ends(args, j);
    double r0[NV][P], r1[NV][P], hl[NV][R], hr[NV][R];
    lane_load<Sch, P>(a, j, g, r0, r1, hl, hr);
    if (straddles_wall(a, j)) run_levels<Sch, P, true, true>(a, g, NW, r0, r1, hl, hr, xch);
    else run_levels<Sch, P, true, false>(a, g, NW, r0, r1, hl, hr, xch);
    __syncthreads();  // every wave has read its inputs before any slot is rewritten
    lane_store<Sch, P>(a, j, g, r0, r1);
}

// MAXT bounds the work-group size the kernel is compiled for.  MAXT = 64 is the
// one-wave tile: the multi-wave path (LDS exchange, barriers) is compiled out and
// the register allocator is not held to a many-wave bound's share of the register
// file.
template <class Sch, int P, int MAXT>
__global__ __launch_bounds__(MAXT) void swept_tile(TileArgs a)
{
    if constexpr (MAXT == 64) {
        __shared__ double stage[2 * Sch::NV * wave_span(P)];
        wave_tile<Sch, P>(a, (int64_t)blockIdx.x, (int)threadIdx.x, stage);
    } else {
        __shared__ double xch[2][16][2][Sch::NV][Sch::R];
        tile_body<Sch, P>(a, (int64_t)blockIdx.x, (int)threadIdx.x, (int)(blockDim.x >> 6), xch);
    }
}

// Batched phase: every work item is (solve, tile) of one of many independent
// solves; one-wave work-groups stride over the items, so a launch covers the
// current phase of every solve in the batch.  `global_phase` >= 0 runs that
// phase for every solve; -1 takes each solve's own phase (served batches).
template <class Sch, int P>
__global__ __launch_bounds__(64) void batch_tiles(const SolveDesc *__restrict__ desc,
                                                  const int2 *__restrict__ items, int64_t nitems,
                                                  int global_phase)
{
    __shared__ double stage[2 * Sch::NV * wave_span(P)];
    for (int64_t i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        const SolveDesc &d = desc[it.x];
        const int p = global_phase >= 0 ? global_phase : d.phase;
        if (p >= d.nphases) continue;
        TileArgs a;
        a.state = d.state;
        a.edges = d.edges;
        a.n = d.n;
        a.K = d.K;
        a.w = d.w;
        a.H = d.H;
        a.E = d.E;
        a.bc = d.bc;
        a.ends = 0;
        a.c = d.c;
        phase_at(d.Q, d.rem, d.H, p, a.kind, a.levels, a.offset);
        wave_tile<Sch, P>(a, (int64_t)it.y, (int)threadIdx.x, stage);
    }
}

constexpr int kPersistChunk = 4;   // queue entries taken per counter update

// Persistent batched launch (ensemble): one-wave work-groups take entries from one
// counter in phase-major order -- every (solve, tile) of phase 0, then of phase 1,
// ... -- and run each as soon as the tiles of the previous phase whose outputs it
// reads (phase_deps) are done: no launch per phase and no grid-wide barrier, the
// GPU-side synchronisation the paper's Conclusions suggest in place of kernel
// launches.  The eight XCDs' L2 caches are not coherent with each other, so every
// global access of these tiles is a relaxed agent-scope atomic (coherent at the device
// level, no whole-cache write-back or invalidation), and a tile publishes its
// completion counter only after all its stores have completed; a dependent tile
// issues its loads only after it has read that counter.  Entry i of phase p is items[i - phase_start[p]]; its tile's
// counter is done[i - phase_start[p]].  Phase-major order makes every dependency an
// earlier entry, so the work-group holding the earliest unfinished entry can always
// proceed; a wait that runs past spin_limit polls (never in a correct run) sets
// *error, and every wait gives up once *error is set, so the launch always ends.
template <class Sch, int P>
__global__ __launch_bounds__(64) void batch_persistent(PersistArgs q)
{
    __shared__ double stage[2 * Sch::NV * wave_span(P)];
    __shared__ unsigned long long entry;
    const int lane = (int)threadIdx.x;
    const int64_t total = q.phase_start[q.max_phases];
    int p = 0;   // a work-group's entries only increase, so its phase only moves forward
    for (;;) {
        // a chunk of consecutive entries per counter update
        if (lane == 0) entry = atomicAdd(q.next, (unsigned long long)kPersistChunk);
        __syncthreads();
        const int64_t i0 = (int64_t)entry;
        __syncthreads();   // every lane has read `entry` before lane 0 takes the next chunk
        if (i0 >= total) break;
        const int64_t i1 = i0 + kPersistChunk < total ? i0 + kPersistChunk : total;
        for (int64_t i = i0; i < i1; ++i) {
            while (q.phase_start[p + 1] <= i) ++p;
            const int64_t r = i - q.phase_start[p];
            const int2 it = q.items[r];
            const SolveDesc &d = q.desc[it.x];
            const int64_t base = r - it.y;   // counter of the solve's tile 0
            if (p > 0) {
                // poll the counters with coherent loads; the tile's own loads are issued after
                int64_t deps[2];
                const int nd = phase_deps(d.Q, d.rem, d.H, d.K, p, it.y, deps);
                for (int k = 0; k < nd; ++k) {
                    int64_t spins = 0;
                    while (__hip_atomic_load(q.done + base + deps[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < p) {
                        if (++spins > q.spin_limit ||
                            __hip_atomic_load(q.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            if (lane == 0) atomicOr(q.error, 1);   // every later wait gives up at once
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
            }
            TileArgs a;
            a.state = d.state;
            a.edges = d.edges;
            a.n = d.n;
            a.K = d.K;
            a.w = d.w;
            a.H = d.H;
            a.E = d.E;
            a.bc = d.bc;
            a.ends = 0;
            a.c = d.c;
            phase_at(d.Q, d.rem, d.H, p, a.kind, a.levels, a.offset);
            wave_tile<Sch, P, true>(a, (int64_t)it.y, lane, stage);
            // every coherent store of this one-wave work-group has completed before the
            // counter is published (the wave's memory counter covers all its lanes)
            __builtin_amdgcn_s_waitcnt(0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (lane == 0) {
                __hip_atomic_store(q.done + r, p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (p + 1 == d.nphases && atomicAdd(q.finished + it.x, 1) + 1 == d.K)
                    q.stamps[it.x] = wall_clock64();   // the solve's last tile is done
            }
        }
    }
}

template <class Sch, int P>
hipError_t persistent_launch_t(const PersistArgs &q, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((batch_persistent<Sch, P>), dim3((unsigned)grid), dim3(64), 0, st, q);
    return hipGetLastError();
}

template <class Sch, int P>
int persistent_occupancy_t()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_persistent<Sch, P>, 64, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

template <class Sch, int P>
hipError_t launch_tile(const TileArgs &a, int threads, hipStream_t st, int64_t tiles)
{
    constexpr int MAXT = max_threads_for(Sch::NV, P);
    if (threads > MAXT) return hipErrorInvalidValue;
    if (threads == 64)
        hipLaunchKernelGGL((swept_tile<Sch, P, 64>), dim3((unsigned)tiles), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((swept_tile<Sch, P, MAXT>), dim3((unsigned)tiles), dim3(threads), 0, st, a);
    return hipGetLastError();
}

template <class Sch, int P>
hipError_t batch_launch_t(const SolveDesc *desc, const int2 *items, int64_t nitems, int global_phase,
                          int grid, hipStream_t st)
{
    hipLaunchKernelGGL((batch_tiles<Sch, P>), dim3((unsigned)grid), dim3(64), 0, st, desc, items, nitems,
                       global_phase);
    return hipGetLastError();
}

template <class Sch, int P>
int batch_occupancy_t()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_tiles<Sch, P>, 64, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

}  // namespace

template <class Sch>
hipError_t swept_phase_for(int P, int threads, const TileArgs &a, hipStream_t st, int64_t tiles)
{
    switch (P) {
    case 1: return launch_tile<Sch, 1>(a, threads, st, tiles);
    case 2: return launch_tile<Sch, 2>(a, threads, st, tiles);
    case 4: return launch_tile<Sch, 4>(a, threads, st, tiles);
    case 8: return launch_tile<Sch, 8>(a, threads, st, tiles);
    case 16: if constexpr (Sch::NV == 1) return launch_tile<Sch, 16>(a, threads, st, tiles); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <class Sch>
hipError_t batch_phase_for(int P, const SolveDesc *desc, const int2 *items, int64_t nitems, int global_phase,
                           int grid, hipStream_t st)
{
    switch (P) {
    case 1: return batch_launch_t<Sch, 1>(desc, items, nitems, global_phase, grid, st);
    case 2: return batch_launch_t<Sch, 2>(desc, items, nitems, global_phase, grid, st);
    case 4: return batch_launch_t<Sch, 4>(desc, items, nitems, global_phase, grid, st);
    case 8: return batch_launch_t<Sch, 8>(desc, items, nitems, global_phase, grid, st);
    default: return hipErrorInvalidValue;
    }
}

template <class Sch>
hipError_t persistent_phase_for(int P, const PersistArgs &q, int grid, hipStream_t st)
{
    switch (P) {
    case 1: return persistent_launch_t<Sch, 1>(q, grid, st);
    case 2: return persistent_launch_t<Sch, 2>(q, grid, st);
    case 4: return persistent_launch_t<Sch, 4>(q, grid, st);
    case 8: return persistent_launch_t<Sch, 8>(q, grid, st);
    default: return hipErrorInvalidValue;
    }
}

template <class Sch>
int persistent_blocks_for(int P)
{
    switch (P) {
    case 1: return persistent_occupancy_t<Sch, 1>();
    case 2: return persistent_occupancy_t<Sch, 2>();
    case 4: return persistent_occupancy_t<Sch, 4>();
    case 8: return persistent_occupancy_t<Sch, 8>();
    default: return 1;
    }
}

template <class Sch>
int batch_blocks_for(int P)
{
    switch (P) {
    case 1: return batch_occupancy_t<Sch, 1>();
    case 2: return batch_occupancy_t<Sch, 2>();
    case 4: return batch_occupancy_t<Sch, 4>();
    case 8: return batch_occupancy_t<Sch, 8>();
    default: return 1;
    }
}

}  // namespace sw
