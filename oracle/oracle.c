/*
 * CPU oracle: plain classic time-stepping, one level (sub-timestep) at a time,
 * reading the previous level from one buffer and writing the next into another.
 * Test infrastructure only -- see oracle.h.  OpenMP only splits the loop over
 * grid points (no reductions, so the result does not depend on the thread
 * count).  Build with -ffp-contract=off and no fast-math: the only fused
 * operations are the explicit fma() calls.
 *
 * Each scheme is written twice:
 *   literal form   -- the equation as the appendix prints it (after the
 *                     readings of its typos), evaluated left to right, every
 *                     product and quotient rounded on its own;
 *   canonical form -- the same polynomial or formula in one fixed rounding
 *                     order: products that feed a sum fused into it (C99 fma,
 *                     one rounding), the KS right-hand side collected by
 *                     symmetric stencil pair.  The paper fixes no rounding
 *                     order; this one is frozen, and the GPU library must
 *                     reproduce it bit for bit.
 * Exact-arithmetic tests (Fractions, 50-digit mpmath) evaluate one level of the
 * literal equations and bound both forms' deviation from it.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------------ */
/* Boundary handling                                                          */
/* ------------------------------------------------------------------------ */

/* Value of variable v at grid index j, which may lie outside [0, n).
 * Periodic: the stencil at point 0 reaches points n-1, n-2 (Appendix C).
 * Dirichlet: the end states are held at their ends for every (sub)level
 * (Appendix D, Eq. SodCond: the spatial boundary values are the two initial
 * states, each at its own end). */
static double at(const oracle_problem *p, const double *a, int64_t j, int v)
{
    const int64_t n = p->n;
    if (j >= 0 && j < n) return a[(int64_t)v * n + j];
    if (p->bc == ORACLE_PERIODIC) {
        int64_t k = j % n;
        if (k < 0) k += n;
        return a[(int64_t)v * n + k];
    }
    if (p->bc == ORACLE_REFLECTIVE) {
        /* insulated ends, Eq. heatcond: T_{-1} = T_1 and, for points 0..n-1, T_n = T_{n-2}
           (mirror images about the end points) */
        return j < 0 ? a[(int64_t)v * n - j] : a[(int64_t)v * n + 2 * (n - 1) - j];
    }
    return j < 0 ? p->bc_left[v] : p->bc_right[v];
}

/* ------------------------------------------------------------------------ */
/* Heat equation, Appendix B, Eq. Heatdisc:                                   */
/*   T_i^{m+1} = Fo (T_{i+1}^m + T_{i-1}^m) + (1 - 2 Fo) T_i^m,               */
/*   Fo = alpha dt / dx^2.                                                    */
/* The product Fo * (sum) and the addition of (1 - 2 Fo) T_i are one fused     */
/* multiply-add (C99 fma: a single rounding).                                 */
/* ------------------------------------------------------------------------ */

static void heat_level(const oracle_problem *p, const double *cur, double *nxt,
                       double fo, double c0)
{
    const int64_t n = p->n;
    if (p->form == ORACLE_FORM_LITERAL) {
        /* Fo (T_{i+1} + T_{i-1}) + (1 - 2 Fo) T_i, two products and a sum */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            nxt[i] = fo * (at(p, cur, i + 1, 0) + at(p, cur, i - 1, 0)) + c0 * cur[i];
        return;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = at(p, cur, i + 1, 0) + at(p, cur, i - 1, 0);
        nxt[i] = fma(fo, s, c0 * cur[i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Kuramoto-Sivashinsky, Appendix C.  Right-hand side of Eq. KSDisc           */
/*   f_i(v) = -( (v_{i+1}^2 - v_{i-1}^2)/(4 dx)                               */
/*              + (v_{i+1} + v_{i-1} - 2 v_i)/dx^2                            */
/*              + (v_{i+2} - 4 v_{i+1} + 6 v_i - 4 v_{i-1} + v_{i-2})/dx^4 )   */
/* (the central second difference carries -2 v_i).  Returned is g = -f, the   */
/* same polynomial collected by symmetric stencil pair: with                  */
/*   s1 = v_{i+1} + v_{i-1},  d1 = v_{i+1} - v_{i-1},  s2 = v_{i+2} + v_{i-2},  */
/*   c1 = 1/(4 dx), c2 = 1/dx^2, c4 = c2^2,                                   */
/*   g = c1 d1 s1 + (c2 - 4 c4) s1 + c4 s2 + (6 c4 - 2 c2) v_i,               */
/* the advection term being the factored difference of squares; the two      */
/* terms of the i+-1 pair share the factor s1,                                */
/*   g = s1 (c1 d1 + c2 - 4 c4) + c4 s2 + (6 c4 - 2 c2) v_i,                  */
/* evaluated as                                                               */
/*   g = fma(s1, fma(c1, d1, c2 - 4 c4), fma(c4, s2, (6 c4 - 2 c2) v_i))      */
/* (C99 fma, one rounding each).  Every step is odd under the mirror          */
/* v_j -> -v_{-j} (d1 is even there, s1, s2 and v_i odd), which keeps the     */
/* scheme's mirror antisymmetry exact in floating point; for a constant state */
/* d1 = 0 and the pair factor is exactly c2 - 4 c4.                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    double c1, c4, k1, k0;          /* canonical: 1/(4 dx), c2^2, c2 - 4 c4, 6 c4 - 2 c2 */
    double four_dx, dx2, dx4;       /* literal: 4 dx, dx^2, dx^4 */
    int literal;
} ks_consts;

/* Literal Eq. KSDisc (second difference with -2 v_i): f_i(v), three quotients
 * summed left to right and negated. */
static double ks_f_literal(const oracle_problem *p, const double *v, int64_t i, const ks_consts *k)
{
    double vm2 = at(p, v, i - 2, 0), vm1 = at(p, v, i - 1, 0), v0 = v[i];
    double vp1 = at(p, v, i + 1, 0), vp2 = at(p, v, i + 2, 0);
    double adv = (vp1 * vp1 - vm1 * vm1) / k->four_dx;
    double diff2 = (vp1 + vm1 - 2.0 * v0) / k->dx2;
    double diff4 = (vp2 - 4.0 * vp1 + 6.0 * v0 - 4.0 * vm1 + vm2) / k->dx4;
    return -(adv + diff2 + diff4);
}

static double ks_g(const oracle_problem *p, const double *v, int64_t i, const ks_consts *k)
{
    double vm2 = at(p, v, i - 2, 0), vm1 = at(p, v, i - 1, 0), v0 = v[i];
    double vp1 = at(p, v, i + 1, 0), vp2 = at(p, v, i + 2, 0);
    double s1 = vp1 + vm1, d1 = vp1 - vm1, s2 = vp2 + vm2;
    double pair = fma(k->c1, d1, k->k1);
    return fma(s1, pair, fma(k->c4, s2, k->k0 * v0));
}

/* One RK2 stage: out_i = base_i + coef f_i(src).  Predictor, Eq. RKm:
 * u^{m+1/2} = u^m + (dt/2) f(u^m); final, Eq. RKf: u^{m+1} = u^m + dt f(u^{m+1/2}).
 * Canonical: base - coef g with g = -f, one fused multiply-add. */
static void ks_stage(const oracle_problem *p, const double *src, const double *base, double *out,
                     const ks_consts *k, double coef)
{
    const int64_t n = p->n;
    if (k->literal) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            out[i] = base[i] + coef * ks_f_literal(p, src, i, k);
        return;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = fma(-coef, ks_g(p, src, i, k), base[i]);
}

/* ------------------------------------------------------------------------ */
/* Euler equations, Appendix D.  Q = (rho, rho u, E) with E the total energy   */
/* per volume; F(Q) = (rho u, rho u^2 + P, u (E + P)); P from Eq. EulerP.      */
/* ------------------------------------------------------------------------ */

typedef struct { double gm1, gamma; int limiter, literal; } euler_consts;

/* Eq. EulerP: P = (gamma - 1)(E - rho u^2 / 2), evaluated as (m u)/2 with u = m/rho.
 * Products that feed a sum are fused into it (C99 fma) throughout this scheme; for
 * the halving here the fusion is exact either way. */
static double pressure(const double q[3], const euler_consts *c)
{
    double u = q[1] / q[0];
    return c->gm1 * fma(-0.5, q[1] * u, q[2]);
}

static double min_d(double a, double b) { return a < b ? a : b; }

/* Flux through the interface between cells b and c = b + 1, from the four cells
 * a = b-1, b, c, d = c+1 (the interface flux of Appendix D). */
static void interface_flux(const double qa[3], const double qb[3], const double qc[3],
                           const double qd[3], const euler_consts *c, double flux[3])
{
    /* Eq. Pratio: P_{r,j} = (P_{j+1} - P_j) / (P_j - P_{j-1}) at j = b and j = c. */
    double pa = pressure(qa, c), pb = pressure(qb, c), pc = pressure(qc, c), pd = pressure(qd, c);
    double pr_b = (pc - pb) / (pb - pa);
    double pr_c = (pd - pc) / (pc - pb);
    double ql[3], qr[3];
    int v;

    if (c->limiter == 0) {
        /* Eq. limitleft: Q^L = Q_b + min(Pr_b, 1)/2 (Q_c - Q_b) if 0 < Pr_b < inf. */
        int okl = pr_b > 0.0 && pr_b < INFINITY;
        /* Eq. limitright: Q^R = Q_c + min(1/Pr_c, 1)/2 (Q_b - Q_c) if 0 < 1/Pr_c < inf. */
        double ir = 1.0 / pr_c;
        int okr = ir > 0.0 && ir < INFINITY;
        double sl = 0.5 * min_d(pr_b, 1.0), sr = 0.5 * min_d(ir, 1.0);
        for (v = 0; v < 3; ++v) {
            ql[v] = okl ? fma(sl, qc[v] - qb[v], qb[v]) : qb[v];
            qr[v] = okr ? fma(sr, qb[v] - qc[v], qc[v]) : qc[v];
        }
    } else {
        /* Reciprocal orientation: the ratio backward/forward on the left side. */
        double il = 1.0 / pr_b;
        int okl = il > 0.0 && il < INFINITY;
        int okr = pr_c > 0.0 && pr_c < INFINITY;
        double sl = 0.5 * min_d(il, 1.0), sr = 0.5 * min_d(pr_c, 1.0);
        for (v = 0; v < 3; ++v) {
            ql[v] = okl ? fma(sl, qc[v] - qb[v], qb[v]) : qb[v];
            qr[v] = okr ? fma(sr, qb[v] - qc[v], qc[v]) : qc[v];
        }
    }

    /* Physical fluxes of the two reconstructed states, Eq. EulerF. */
    double ul = ql[1] / ql[0], ur = qr[1] / qr[0];
    double pl = c->gm1 * fma(-0.5, ql[1] * ul, ql[2]);
    double prr = c->gm1 * fma(-0.5, qr[1] * ur, qr[2]);
    double fl[3] = { ql[1], fma(ql[1], ul, pl), ul * (ql[2] + pl) };
    double fr[3] = { qr[1], fma(qr[1], ur, prr), ur * (qr[2] + prr) };

    /* Roe-averaged state and spectral radius r_sp = sqrt(gamma P_sp/rho_sp) + |u_sp|. */
    double sql = sqrt(ql[0]), sqr = sqrt(qr[0]);
    double rho_s = sqrt(ql[0] * qr[0]);
    double den = sql + sqr;
    double u_s = fma(sql, ul, sqr * ur) / den;
    double e_s = fma(sql, ql[2], sqr * qr[2]) / den;
    double p_s = c->gm1 * fma(-0.5, (rho_s * u_s) * u_s, e_s);
    double r_sp = sqrt((c->gamma * p_s) / rho_s) + fabs(u_s);

    /* Flux = (F(Q^R) + F(Q^L) + r_sp (Q^L - Q^R)) / 2. */
    for (v = 0; v < 3; ++v)
        flux[v] = 0.5 * fma(r_sp, ql[v] - qr[v], fr[v] + fl[v]);
}

/* Literal form of the same interface flux: Eq. EulerP as P = (gamma-1)(E - rho u^2/2)
 * with u = m/rho, Eq. EulerF as (m, rho u^2 + P, u (E + P)), the Roe average and
 * spectral radius as printed, Flux = (F(Q^R) + F(Q^L) + r_sp (Q^L - Q^R)) / 2; every
 * product and quotient rounded on its own, sums left to right. */
static double pressure_literal(const double q[3], const euler_consts *c)
{
    double u = q[1] / q[0];
    return c->gm1 * (q[2] - q[0] * u * u / 2.0);
}

static void physical_flux_literal(const double q[3], const euler_consts *c, double f[3])
{
    double u = q[1] / q[0];
    double pr = pressure_literal(q, c);
    f[0] = q[1];
    f[1] = q[0] * u * u + pr;
    f[2] = u * (q[2] + pr);
}

static void interface_flux_literal(const double qa[3], const double qb[3], const double qc[3],
                                   const double qd[3], const euler_consts *c, double flux[3])
{
    double pa = pressure_literal(qa, c), pb = pressure_literal(qb, c);
    double pc = pressure_literal(qc, c), pd = pressure_literal(qd, c);
    double pr_b = (pc - pb) / (pb - pa);        /* Eq. Pratio at cell b */
    double pr_c = (pd - pc) / (pc - pb);        /* and at cell c */
    /* the ratio each side's limiter takes (reading of Eqs. limitleft/limitright) */
    double tl = c->limiter == 0 ? pr_b : 1.0 / pr_b;
    double tr = c->limiter == 0 ? 1.0 / pr_c : pr_c;
    double ql[3], qr[3];
    for (int v = 0; v < 3; ++v) {
        ql[v] = (tl > 0.0 && tl < INFINITY) ? qb[v] + min_d(tl, 1.0) / 2.0 * (qc[v] - qb[v]) : qb[v];
        qr[v] = (tr > 0.0 && tr < INFINITY) ? qc[v] + min_d(tr, 1.0) / 2.0 * (qb[v] - qc[v]) : qc[v];
    }
    double fl[3], fr[3];
    physical_flux_literal(ql, c, fl);
    physical_flux_literal(qr, c, fr);
    double ul = ql[1] / ql[0], ur = qr[1] / qr[0];
    double rho_sp = sqrt(ql[0] * qr[0]);
    double u_sp = (sqrt(ql[0]) * ul + sqrt(qr[0]) * ur) / (sqrt(ql[0]) + sqrt(qr[0]));
    double e_sp = (sqrt(ql[0]) * ql[2] + sqrt(qr[0]) * qr[2]) / (sqrt(ql[0]) + sqrt(qr[0]));
    double p_sp = c->gm1 * (e_sp - rho_sp * u_sp * u_sp / 2.0);
    double r_sp = sqrt(c->gamma * p_sp / rho_sp) + fabs(u_sp);
    for (int v = 0; v < 3; ++v)
        flux[v] = 0.5 * (fr[v] + fl[v] + r_sp * (ql[v] - qr[v]));
}

static void load_cell(const oracle_problem *p, const double *q, int64_t j, double out[3])
{
    for (int v = 0; v < 3; ++v) out[v] = at(p, q, j, v);
}

/* One RK2 stage of the finite-volume update: out_i = base_i + coef (F_{i-1/2} - F_{i+1/2}),
 * fluxes evaluated from `src`.  The conservation law (Eq. EulerGeneral) fixes the sign:
 * the flux leaving through i+1/2 is subtracted. */
static void euler_stage(const oracle_problem *p, const double *src, const double *base,
                        double *out, double coef, const euler_consts *c)
{
    const int64_t n = p->n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double q[5][3];
        for (int k = 0; k < 5; ++k) load_cell(p, src, i - 2 + k, q[k]);
        double fm[3], fp[3];
        if (c->literal) {
            interface_flux_literal(q[0], q[1], q[2], q[3], c, fm);   /* i - 1/2 */
            interface_flux_literal(q[1], q[2], q[3], q[4], c, fp);   /* i + 1/2 */
            for (int v = 0; v < 3; ++v)
                out[(int64_t)v * n + i] = base[(int64_t)v * n + i] + coef * (fm[v] - fp[v]);
            continue;
        }
        interface_flux(q[0], q[1], q[2], q[3], c, fm);   /* i - 1/2 */
        interface_flux(q[1], q[2], q[3], q[4], c, fp);   /* i + 1/2 */
        for (int v = 0; v < 3; ++v)
            out[(int64_t)v * n + i] = fma(coef, fm[v] - fp[v], base[(int64_t)v * n + i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Driver                                                                     */
/* ------------------------------------------------------------------------ */

static int nvars_of(int scheme) { return scheme == ORACLE_EULER ? 3 : 1; }

/* Constants of each scheme, computed once per solve in the order written here. */
static void heat_consts(const oracle_problem *p, double *fo, double *c0)
{
    *fo = (p->alpha * p->dt) / (p->dx * p->dx);
    *c0 = 1.0 - 2.0 * *fo;
}

static void make_ks_consts(const oracle_problem *p, ks_consts *k)
{
    double c2 = 1.0 / (p->dx * p->dx);
    k->c1 = 1.0 / (4.0 * p->dx);
    k->c4 = c2 * c2;
    k->k1 = c2 - 4.0 * k->c4;
    k->k0 = 6.0 * k->c4 - 2.0 * c2;
    k->four_dx = 4.0 * p->dx;
    k->dx2 = p->dx * p->dx;
    k->dx4 = k->dx2 * k->dx2;
    k->literal = p->form == ORACLE_FORM_LITERAL;
}

static void make_euler_consts(const oracle_problem *p, euler_consts *c)
{
    c->gm1 = p->gamma - 1.0;
    c->gamma = p->gamma;
    c->limiter = p->limiter;
    c->literal = p->form == ORACLE_FORM_LITERAL;
}

static int valid(const oracle_problem *p)
{
    if (!p) return 0;
    if (p->scheme < ORACLE_HEAT || p->scheme > ORACLE_EULER) return 0;
    if (p->bc != ORACLE_PERIODIC && p->bc != ORACLE_DIRICHLET && p->bc != ORACLE_REFLECTIVE) return 0;
    if (p->bc == ORACLE_REFLECTIVE && (p->scheme != ORACLE_HEAT || p->n < 2)) return 0;
    if (p->n < 1 || p->nsteps < 0) return 0;
    if (p->form != ORACLE_FORM_CANONICAL && p->form != ORACLE_FORM_LITERAL) return 0;
    if (!(p->dt > 0.0) || !(p->dx > 0.0)) return 0;
    return 1;
}

int oracle_threads(int nthreads)
{
    int t = 1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    else omp_set_num_threads(omp_get_num_procs());
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int oracle_solve_timed(const oracle_problem *p, double *state, int nthreads, double *seconds)
{
    if (!valid(p) || !state) return -1;
    const int64_t n = p->n;
    const int nv = nvars_of(p->scheme);
    const size_t bytes = (size_t)nv * (size_t)n * sizeof(double);
    double *a = state;
    double *b = (double *)malloc(bytes);
    double *h = (double *)malloc(bytes);
    if (!b || !h) { free(b); free(h); return -1; }
    oracle_threads(nthreads);

    double t0 = now_s();
    if (p->scheme == ORACLE_HEAT) {
        double fo, c0;
        heat_consts(p, &fo, &c0);
        for (int64_t m = 0; m < p->nsteps; ++m) {
            heat_level(p, a, b, fo, c0);
            double *t = a; a = b; b = t;
        }
    } else if (p->scheme == ORACLE_KS) {
        ks_consts k;
        make_ks_consts(p, &k);
        double hdt = 0.5 * p->dt;
        for (int64_t m = 0; m < p->nsteps; ++m) {
            ks_stage(p, a, a, h, &k, hdt);      /* predictor */
            ks_stage(p, h, a, b, &k, p->dt);    /* final */
            double *t = a; a = b; b = t;
        }
    } else {
        euler_consts c;
        make_euler_consts(p, &c);
        double lam = p->dt / p->dx;
        double hlam = 0.5 * lam;
        for (int64_t m = 0; m < p->nsteps; ++m) {
            euler_stage(p, a, a, h, hlam, &c);   /* predictor: Q^{m+1/2} */
            euler_stage(p, h, a, b, lam, &c);    /* final: Q^{m+1} */
            double *t = a; a = b; b = t;
        }
    }
    double t1 = now_s();
    if (seconds) *seconds = t1 - t0;

    if (a != state) {               /* odd number of swaps: result lives in the scratch buffer */
        memcpy(state, a, bytes);
        b = a;                      /* free the scratch buffer, never the caller's array */
    }
    free(b);
    free(h);
    return 0;
}

int oracle_solve(const oracle_problem *p, double *state, int nthreads)
{
    return oracle_solve_timed(p, state, nthreads, 0);
}

int oracle_stage(const oracle_problem *p, int final_stage, const double *src, const double *base,
                 double *out, int nthreads)
{
    if (!valid(p) || !src || !base || !out) return -1;
    if (final_stage != 0 && final_stage != 1) return -1;
    if (p->scheme == ORACLE_HEAT && final_stage) return -1;
    oracle_threads(nthreads);
    if (p->scheme == ORACLE_HEAT) {
        double fo, c0;
        heat_consts(p, &fo, &c0);
        heat_level(p, src, out, fo, c0);
    } else if (p->scheme == ORACLE_KS) {
        ks_consts k;
        make_ks_consts(p, &k);
        ks_stage(p, src, base, out, &k, final_stage ? p->dt : 0.5 * p->dt);
    } else {
        euler_consts c;
        make_euler_consts(p, &c);
        double lam = p->dt / p->dx;
        euler_stage(p, src, base, out, final_stage ? lam : 0.5 * lam, &c);
    }
    return 0;
}

void oracle_euler_flux(const double cells[4][3], double gamma, int limiter, double flux[3])
{
    euler_consts c;
    c.gm1 = gamma - 1.0;
    c.gamma = gamma;
    c.limiter = limiter;
    c.literal = 0;
    interface_flux(cells[0], cells[1], cells[2], cells[3], &c, flux);
}
