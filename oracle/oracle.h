/*
 * CPU oracle for explicit 1D stencil time-stepping (test infrastructure only).
 *
 * This library exists to check the GPU library, nothing else: only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU path.
 *
 * It computes the plain definition of what the swept decomposition must
 * reproduce: the swept rule performs the same operations as a classic
 * decomposition in a different order and place (Sec. 2, Related work), so the
 * reference result is classic level-by-level time-stepping of each scheme in
 * IEEE-754 binary64, round-to-nearest, no FMA contraction:
 *   heat equation, FTCS             Appendix B, Eq. Heatdisc
 *   Kuramoto-Sivashinsky, RK2       Appendix C, Eqs. KSDisc, RKm, RKf
 *   Euler equations, 2nd-order FV   Appendix D, Eqs. EulerQ-EulerP, Pratio,
 *                                   limitleft, limitright, flux, Roe average
 *
 * Two rounding orders of the same arithmetic (the paper fixes none):
 *   ORACLE_FORM_CANONICAL (default) -- one fixed order with products fused into
 *       the sums that consume them; frozen; the GPU library reproduces it bit for
 *       bit, which is what keeps long chaotic KS runs comparable at all;
 *   ORACLE_FORM_LITERAL -- each equation as printed, evaluated left to right with
 *       every operation rounded on its own.
 * Both are checked against one level of the printed equations in exact arithmetic
 * by the tests.
 */
#ifndef SWEPT_ORACLE_H
#define SWEPT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_HEAT = 0, ORACLE_KS = 1, ORACLE_EULER = 2 };
enum { ORACLE_PERIODIC = 0, ORACLE_DIRICHLET = 1, ORACLE_REFLECTIVE = 2 };
enum { ORACLE_FORM_CANONICAL = 0, ORACLE_FORM_LITERAL = 1 };

typedef struct {
    int32_t scheme;      /* ORACLE_HEAT, ORACLE_KS, ORACLE_EULER */
    int32_t bc;          /* ORACLE_PERIODIC, ORACLE_DIRICHLET, or ORACLE_REFLECTIVE (heat only:
                            the insulated ends of Appendix B, Eq. heatcond) */
    int64_t n;           /* grid points (heat, KS) or cells (Euler) */
    int64_t nsteps;      /* full timesteps */
    double dt, dx;
    double alpha;        /* heat diffusivity */
    double gamma;        /* Euler heat-capacity ratio */
    double bc_left[3];   /* Dirichlet ghost values (conserved variables for Euler) */
    double bc_right[3];
    int32_t limiter;     /* Euler: 0 = ratio as printed in Eqs. limitleft/limitright,
                            1 = reciprocal ratio (textbook minmod orientation) */
    int32_t form;        /* ORACLE_FORM_CANONICAL or ORACLE_FORM_LITERAL */
} oracle_problem;

/* Advance state[nv][n] (nv = 1, or 3 for Euler; SoA, in place) by p->nsteps
 * timesteps with nthreads OpenMP threads (<= 0: all).  Returns 0, or -1 for
 * an invalid problem (state untouched). */
int oracle_solve(const oracle_problem *p, double *state, int nthreads);

/* Same as oracle_solve; *seconds receives the wall time of the step loop. */
int oracle_solve_timed(const oracle_problem *p, double *state, int nthreads, double *seconds);

/* One sub-step from given arrays: out = base + coef * f(src), with coef = dt/2
 * (final_stage = 0: predictor, Eq. RKm) or dt (final_stage = 1: Eq. RKf); for the
 * heat equation (final_stage must be 0) out = the next FTCS level of src and base
 * is ignored.  Arrays are [nv][n]; nsteps is ignored.  Returns 0, or -1. */
int oracle_stage(const oracle_problem *p, int final_stage, const double *src, const double *base,
                 double *out, int nthreads);

/* Interface flux of Appendix D between cells[1] and cells[2] (conserved states of
 * the four cells i-1, i, i+1, i+2 around interface i+1/2). */
void oracle_euler_flux(const double cells[4][3], double gamma, int limiter, double flux[3]);

/* Number of threads an OpenMP parallel region with this request actually uses. */
int oracle_threads(int nthreads);

#ifdef __cplusplus
}
#endif
#endif
