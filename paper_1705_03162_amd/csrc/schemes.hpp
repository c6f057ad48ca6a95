// Per-point update rules of the three schemes, in one fixed binary64 operation
// order.  Every file is compiled with -ffp-contract=off, so the only fused
// multiply-adds are the explicit sw_fma calls (one rounding each, v_fma_f64).
//
// Each rule works on a lane-local run of P consecutive points: `ext` holds the
// source level on those points plus R halo points on each side, `dst` holds
// the destination row (which, for a final RK2 stage, still carries u^m / Q^m
// at the same points).  Only points k with in[k] set are written; the others
// keep their previous contents, which is what lets a tile keep its edges in place.
// With SEL every point is computed and the written ones are selected afterwards,
// so the P independent updates form one block the compiler can interleave (hides
// FP64 latency when few waves are resident); without it each point is a branch
// (exec-masked regions), which the host evaluation of single points uses.
// FREE_ONE_WAVE: one-wave tiles may update every point of a narrowing level (in[] all
// set) and store the few finished boundary points to LDS instead of selecting
// (swept_tile.hpp, free_class and level_step); on for heat, whose three-instruction
// update makes the selects its largest overhead.
// CLASS12: one-wave tiles of 16 points per lane add a 12-point class layout between the
// 8- and 16-point ones (swept_tile.hpp, next_class); on for KS, where it cuts the lane
// slots of the widest levels (heat's select-free 16-point levels already cost about as
// little as selecting 12-point ones, and a class change more).
//
//   Heat  (Appendix B, Eq. Heatdisc):  T' = Fo (T_{i+1} + T_{i-1}) + (1 - 2 Fo) T_i,
//         the Fo product fused with the addition
//   KS    (Appendix C, Eqs. KSDisc, RKm, RKf): 5-point central differences,
//         predictor u + dt/2 f(u), final u + dt f(u^{m+1/2}); f collected by
//         symmetric stencil pair (the advection term as the factored difference of
//         squares, sharing the factor v_{i+1} + v_{i-1} with the second and fourth
//         differences), products fused into the sums that consume them, every step
//         odd under the mirror v_j -> -v_{-j}
//   Euler (Appendix D): pressure-ratio limited reconstruction, Roe-averaged
//         spectral radius, interface flux, same RK2 stages; products fused into the
//         sums that consume them, each cell's pressure ratio computed once
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define SW_HD __host__ __device__ inline
#else
#include <cmath>
#define SW_HD inline
#endif

namespace sw {

// Canonical constants, computed once on the host in the order written here and
// passed by value to every kernel.
struct Consts {
    double fo, c0;                  // heat: Fo = (alpha*dt)/(dx*dx), 1 - 2 Fo
    double c1, c2, c4, hdt, dt;     // KS: 1/(4 dx), 1/dx^2, c2*c2, dt/2, dt
    double k1, k0;                  // KS: c2 - 4 c4 (pair i+-1), 6 c4 - 2 c2 (point i)
    double gm1, gamma, lam, hlam;   // Euler: gamma-1, gamma, dt/dx, lam/2
    int32_t limiter, pad;           // Euler: 0 ratio as printed, 1 reciprocal
    double ghost_l[3], ghost_r[3];  // Dirichlet ghost values per variable
};

SW_HD double sw_min(double a, double b) { return a < b ? a : b; }
SW_HD double sw_fma(double a, double b, double c) { return fma(a, b, c); }
SW_HD double sw_sqrt(double x) { return sqrt(x); }
SW_HD double sw_fabs(double x) { return fabs(x); }

struct Heat {
    static constexpr int R = 1, S = 1, NV = 1;
    static constexpr bool SELECT_ONE_WAVE = true;
    static constexpr bool FREE_ONE_WAVE = true;
    static constexpr bool CLASS12 = false;          // measured slower: 110.7 vs 109.3 us at 2^20
    static constexpr bool LANE_EXCHANGE = false;    // no per-cell quantity shared by neighbours
    template <int P, bool SEL = true>
    SW_HD static void level(double (&dst)[NV][P], const double (&ext)[NV][P + 2 * R],
                            bool /*predictor*/, const Consts &c, const bool (&in)[P])
    {
        double val[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double s = ext[0][k + 2] + ext[0][k];
            val[k] = sw_fma(c.fo, s, c.c0 * ext[0][k + 1]);
            // Most points of a level lie inside the computed set: the hint lets the
            // compiler drop the exec-zero skip branches around the masked updates.
            if (!SEL && __builtin_expect(in[k], 1)) dst[0][k] = val[k];
        }
        if (SEL) {
#pragma unroll
            for (int k = 0; k < P; ++k) dst[0][k] = in[k] ? val[k] : dst[0][k];
        }
    }
};

struct KS {
    static constexpr int R = 2, S = 2, NV = 1;
    static constexpr bool SELECT_ONE_WAVE = true;
    static constexpr bool FREE_ONE_WAVE = false;   // measured slower: 122.4 vs 121.6 us at 2^20, 895 vs 823 at 2^23
    static constexpr bool CLASS12 = true;
    static constexpr bool LANE_EXCHANGE = false;
    // g_i(v) = -f_i(v) = (v_{i+1}^2 - v_{i-1}^2)/(4dx) + (v_{i+1} + v_{i-1} - 2v_i)/dx^2
    //                   + (v_{i+2} + v_{i-2} - 4(v_{i+1} + v_{i-1}) + 6v_i)/dx^4,
    // collected by symmetric stencil pair (s1 = v_{i+1} + v_{i-1}, d1 = v_{i+1} - v_{i-1},
    // s2 = v_{i+2} + v_{i-2}), the advection term and the i+-1 pair sharing the factor s1:
    // g = s1 (c1 d1 + c2 - 4 c4) + c4 s2 + (6 c4 - 2 c2) v_i -- seven operations, the
    // pair factor one fused multiply-add
    SW_HD static double g(double vm2, double vm1, double v0, double vp1, double vp2,
                          const Consts &c)
    {
        const double s1 = vp1 + vm1, d1 = vp1 - vm1, s2 = vp2 + vm2;
        const double pair = sw_fma(c.c1, d1, c.k1);
        return sw_fma(s1, pair, sw_fma(c.c4, s2, c.k0 * v0));
    }
    template <int P, bool SEL = true>
    SW_HD static void level(double (&dst)[NV][P], const double (&ext)[NV][P + 2 * R],
                            bool predictor, const Consts &c, const bool (&in)[P])
    {
        double val[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double gk = g(ext[0][k], ext[0][k + 1], ext[0][k + 2], ext[0][k + 3], ext[0][k + 4], c);
            // u + coef f = u - coef g
            val[k] = predictor ? sw_fma(-c.hdt, gk, ext[0][k + 2]) : sw_fma(-c.dt, gk, dst[0][k]);
            if (!SEL && in[k]) dst[0][k] = val[k];
        }
        if (SEL) {
#pragma unroll
            for (int k = 0; k < P; ++k) dst[0][k] = in[k] ? val[k] : dst[0][k];
        }
    }
};

struct Euler {
    static constexpr int R = 2, S = 2, NV = 3;
    static constexpr bool SELECT_ONE_WAVE = true;
    static constexpr bool FREE_ONE_WAVE = false;   // not measured in a select-free class
    // Pressures, pressure ratios and interface fluxes belong to cells and interfaces, so
    // a lane may take its neighbours' values instead of evaluating them on its halo.
    static constexpr bool CLASS12 = false;   // its tuned tiles have at most 8 points per lane
    static constexpr bool LANE_EXCHANGE = true;

    // Eq. EulerP with E the total energy per volume: P = (gamma-1)(E - (m u)/2), u = m/rho.
    // Products that feed a sum are fused into it throughout (for this halving the
    // fusion is exact either way).
    SW_HD static double pressure(double rho, double m, double e, const Consts &c)
    {
        double u = m / rho;
        return c.gm1 * sw_fma(-0.5, m * u, e);
    }

    // Eq. Pratio at cell j from the pressures of cells j-1, j, j+1.
    SW_HD static double pratio(double pm, double p0, double pp) { return (pp - p0) / (p0 - pm); }

    // Flux through the interface between cells b and c, given both cells and the
    // pressure ratios at b and c (each ratio is shared by two interfaces).
    SW_HD static void flux(const double qb[3], const double qc[3], double pr_b, double pr_c,
                           const Consts &k, double out[3])
    {
        // Eqs. limitleft / limitright (tl: ratio used on the left state, tr: right).
        double tl = k.limiter ? 1.0 / pr_b : pr_b;
        double tr = k.limiter ? pr_c : 1.0 / pr_c;
        bool okl = tl > 0.0 && tl < INFINITY;
        bool okr = tr > 0.0 && tr < INFINITY;
        double sl = 0.5 * sw_min(tl, 1.0), sr = 0.5 * sw_min(tr, 1.0);
        double ql[3], qr[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            ql[v] = okl ? sw_fma(sl, qc[v] - qb[v], qb[v]) : qb[v];
            qr[v] = okr ? sw_fma(sr, qb[v] - qc[v], qc[v]) : qc[v];
        }
        // Eq. EulerF on both reconstructed states.
        double ul = ql[1] / ql[0], ur = qr[1] / qr[0];
        double pl = k.gm1 * sw_fma(-0.5, ql[1] * ul, ql[2]);
        double prr = k.gm1 * sw_fma(-0.5, qr[1] * ur, qr[2]);
        double fl[3] = {ql[1], sw_fma(ql[1], ul, pl), ul * (ql[2] + pl)};
        double fr[3] = {qr[1], sw_fma(qr[1], ur, prr), ur * (qr[2] + prr)};
        // Roe average and spectral radius.
        double sql = sw_sqrt(ql[0]), sqr = sw_sqrt(qr[0]);
        double rho_s = sw_sqrt(ql[0] * qr[0]);
        double den = sql + sqr;
        double u_s = sw_fma(sql, ul, sqr * ur) / den;
        double e_s = sw_fma(sql, ql[2], sqr * qr[2]) / den;
        double p_s = k.gm1 * sw_fma(-0.5, (rho_s * u_s) * u_s, e_s);
        double r_sp = sw_sqrt((k.gamma * p_s) / rho_s) + sw_fabs(u_s);
#pragma unroll
        for (int v = 0; v < 3; ++v) out[v] = 0.5 * sw_fma(r_sp, ql[v] - qr[v], fr[v] + fl[v]);
    }

    template <int P, bool SEL = true>
    SW_HD static void level(double (&dst)[NV][P], const double (&ext)[NV][P + 2 * R],
                            bool predictor, const Consts &c, const bool (&in)[P])
    {
        double val[NV][P];
        double pres[P + 2 * R];
#pragma unroll
        for (int j = 0; j < P + 2 * R; ++j) pres[j] = pressure(ext[0][j], ext[1][j], ext[2][j], c);
        // ratio at ext cells 1 .. P+2 (index j - 1)
        double pr[P + 2];
#pragma unroll
        for (int j = 1; j <= P + 2; ++j) pr[j - 1] = pratio(pres[j - 1], pres[j], pres[j + 1]);
        const double coef = predictor ? c.hlam : c.lam;
        // Interface j sits between ext cells j+1 and j+2 (point k has interfaces k, k+1).
        double fprev[3];
        {
            double qb[3] = {ext[0][1], ext[1][1], ext[2][1]};
            double qc[3] = {ext[0][2], ext[1][2], ext[2][2]};
            flux(qb, qc, pr[0], pr[1], c, fprev);
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double fnext[3];
            double qb[3] = {ext[0][k + 2], ext[1][k + 2], ext[2][k + 2]};
            double qc[3] = {ext[0][k + 3], ext[1][k + 3], ext[2][k + 3]};
            flux(qb, qc, pr[k + 1], pr[k + 2], c, fnext);
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                double base = predictor ? ext[v][k + 2] : dst[v][k];
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
};

}  // namespace sw
