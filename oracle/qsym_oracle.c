/*
 * qsym_oracle.c -- plain FP64 CPU oracle of the democratic-heliocentric (DH)
 * hybrid symplectic step of Moore & Quillen, "QYMSYM: A GPU-Accelerated Hybrid
 * Symplectic Integrator That Permits Close Encounters" (arXiv:1007.3458).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct checker
 * that the HIP library is compared against.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never calls it and shares no code, header, table or constant with it.
 *
 * Conventions (all FP64, no FMA contraction: built with -ffp-contract=off):
 *   n bodies, the central mass m0 is NOT stored in the arrays;
 *   q[3*i+k]  heliocentric position of body i, component k;
 *   v[3*i+k]  barycentric velocity (barycentric momentum / m_i, so massless
 *             bodies are allowed);
 *   m[i]      mass, h[i] = cbrt(m_i / (3 m0)) supplied by the caller
 *             (the Hill factor; computed once on the host for both sides).
 *   mu = G*m0 (the paper's appendix writes mu = sqrt(GM) but every formula
 *   uses sqrt(mu) as the square root of GM; we read mu = G m0).
 *
 * Every function below cites the passage of the paper it follows.  Where the
 * paper is silent or garbled the reading taken is stated at the function.
 *
 * Parity pins: every function is pinned by the CPU tests (closed forms,
 * invariants, brute force); see the tests for each.  Among them: r_crit of
 * each set against the r_crit equation of Sec. 2.2 evaluated with the
 * semi-major axes the orbits were drawn with; the angular-momentum checker
 * against hand values and the two-body closed form; the crude sweep against
 * a brute-force fine test of every pair.  The composite hybrid step
 * (orc_step) has no worked numeric example in the paper: its parity is
 * pinned through its pinned parts, through invariants (reversibility with
 * encounters off, exact Kepler for a test particle, angular-momentum
 * conservation, second-order energy scaling) and through convergence to an
 * independent integration of Newton's equations across an active set.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* parameter block (Sec. 2.5, list of parameters) */
typedef struct {
    double G, m0;        /* gravitational constant, central mass          */
    double aE;           /* Hill factor for encounter identification      */
    double aH;           /* Hill factor setting r_crit                    */
    double epsH;         /* Hermite smoothing length                      */
    double eta, eta_s;   /* Hermite accuracy parameters                   */
    double crude_safety; /* multiplicative slack of the crude sweep       */
    int32_t hill_mode;   /* 0: a_E x mutual Hill radius, 1: a_E x sum     */
    int32_t kepler_mode; /* 0: Laguerre from x=r0, 1: Newton, 2: Newton from a guess */
    int32_t max_substeps;/* Hermite substep cap per set per step          */
    int32_t pad;
    double planet_mass;  /* > 0: bodies this massive are planets, and a set
                            holding two of them makes the step integrate
                            the whole system with the Hermite (Sec. 2.3);
                            0: off                                         */
} orc_params;

typedef struct {
    int64_t n_candidates;  /* crude-sweep pairs                        */
    int64_t n_encounters;  /* fine-sweep pairs                         */
    int64_t n_sets;        /* non-intersecting encounter sets          */
    int64_t max_set;       /* members of the largest set               */
    int64_t substeps;      /* Hermite substeps summed over sets        */
    int64_t kepler_iters;  /* Kepler solver iterations summed          */
    int64_t kepler_max;    /* largest iteration count of one solve     */
    int64_t kepler_fail;   /* solves that hit the iteration cap        */
    int64_t hermite_fail;  /* sets that hit the substep cap            */
    int64_t cand_overflow; /* candidates beyond the caller's capacity  */
    int64_t whole_system;  /* 1 when the step ran the whole-system Hermite */
} orc_stats;

#define ORC_KEPLER_CAP 30
#define ORC_KEPLER_TOL 1e-14

/* ------------------------------------------------------------------ */
/* Appendix A: Stumpff functions C(y), S(y).  Series for |y| < 1       */
/* (the paper's "y ~ 0" branch, threshold not given: we take |y| < 1),  */
/* closed trigonometric / hyperbolic forms otherwise.                  */
/* ------------------------------------------------------------------ */
void orc_stumpff(double y, double *C, double *S)
{
    if (fabs(y) < 1.0) {
        /* C = sum_k (-y)^k/(2k+2)!,  S = sum_k (-y)^k/(2k+3)! */
        double tc = 0.5, ts = 1.0 / 6.0, c = 0.0, s = 0.0;
        for (int k = 0; k < 14; ++k) {
            c += tc;
            s += ts;
            tc *= -y / ((2.0 * k + 3.0) * (2.0 * k + 4.0));
            ts *= -y / ((2.0 * k + 4.0) * (2.0 * k + 5.0));
        }
        *C = c;
        *S = s;
    } else if (y > 0.0) {
        double sy = sqrt(y);
        *C = (1.0 - cos(sy)) / y;
        *S = (sy - sin(sy)) / (y * sy);
    } else {
        double sy = sqrt(-y);
        *C = (cosh(sy) - 1.0) / (-y);
        *S = (sinh(sy) - sy) / ((-y) * sy);
    }
}

/* ------------------------------------------------------------------ */
/* Appendix A: universal-variable Kepler advance of one body about mu. */
/*   F(x)  = -sqrt(mu) dt + (r0.v0) x^2 C / sqrt(mu) + (1 - r0 a) x^3 S + r0 x
 *   F'(x) = (r0.v0) x (1 - a x^2 S)/sqrt(mu) + (1 - r0 a) x^2 C + r0
 *   F''(x)= (r0.v0) (1 - a x^2 C)/sqrt(mu) + (1 - r0 a) x (1 - a x^2 S)
 * with a = alpha = 1/semi-major axis = 2/r0 - v0^2/mu, C,S at a x^2.
 * Laguerre iteration, n = 5, denominator sign = sign of F' (the printed
 * update lacks the "x_i -"; we read x_{i+1} = x_i - nF/(F' +- sqrt(...))).
 * Start x = r0 as the paper states (kepler_mode 0), or the first-order
 * guess sqrt(mu) dt / r0 with Newton steps (kepler_modes 1, 2; not in the
 * paper).  Stop when |dx| <= 1e-14 |x|, cap 30 iterations per start.
 * f = 1 - x^2 C/r0, g = dt - x^3 S/sqrt(mu), x = f x0 + g v0, r = |x|,
 * fdot = sqrt(mu) x (a x^2 S - 1)/(r r0)  (printed with a x^3 S, which is
 * dimensionally inconsistent; the Wronskian f gdot - fdot g = 1 fixes it),
 * gdot = 1 - x^2 C / r.                                               */
/* ------------------------------------------------------------------ */
int orc_kepler_root(double mu, const double *x0, const double *v0, double dt,
                    int32_t mode, double x_start, int32_t use_start, double *x_out,
                    int32_t *iters);

int orc_kepler_body(double mu, const double *x0, const double *v0, double dt,
                    int32_t mode, double *xo, double *vo, int32_t *iters)
{
    if (dt == 0.0) {
        for (int k = 0; k < 3; ++k) { xo[k] = x0[k]; vo[k] = v0[k]; }
        *iters = 0;
        return 0;
    }
    double x;
    int fail = orc_kepler_root(mu, x0, v0, dt, mode, 0.0, 0, &x, iters);
    double r0 = sqrt(x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2]);
    double vv = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    double smu = sqrt(mu);
    double alpha = 2.0 / r0 - vv / mu;
    double C, S;
    double z = alpha * x * x;
    orc_stumpff(z, &C, &S);
    double f = 1.0 - x * x * C / r0;
    double g = dt - x * x * x * S / smu;
    for (int k = 0; k < 3; ++k) xo[k] = f * x0[k] + g * v0[k];
    double r = sqrt(xo[0] * xo[0] + xo[1] * xo[1] + xo[2] * xo[2]);
    double fd = smu * x * (z * S - 1.0) / (r * r0);
    double gd = 1.0 - x * x * C / r;
    for (int k = 0; k < 3; ++k) vo[k] = fd * x0[k] + gd * v0[k];
    return fail;
}

/* Universal anomaly x solving F(x) = 0 (Appendix A).  x_start overrides the
 * starting value when use_start is set (used to count iterations from a
 * proposed guess). */
static int orc_kepler_iterate(double smu, double r0, double rv, double alpha, double dt,
                              int32_t laguerre, double *xio, int32_t *count)
{
    double b = 1.0 - r0 * alpha;
    double x = *xio, C, S;
    int it = 0;
    while (it < ORC_KEPLER_CAP) {
        ++it;
        double z = alpha * x * x;
        orc_stumpff(z, &C, &S);
        double F = rv * x * x * C / smu + b * x * x * x * S + r0 * x - smu * dt;
        double Fp = rv * x * (1.0 - z * S) / smu + b * x * x * C + r0;
        double dx;
        if (laguerre) {
            double Fpp = rv * (1.0 - z * C) / smu + b * x * (1.0 - z * S);
            const double nl = 5.0; /* Laguerre order */
            double rad = sqrt(fabs((nl - 1.0) * (nl - 1.0) * Fp * Fp - nl * (nl - 1.0) * F * Fpp));
            dx = nl * F / (Fp + (Fp >= 0.0 ? rad : -rad));
        } else {
            dx = F / Fp;
        }
        x = x - dx;
        if (fabs(dx) <= ORC_KEPLER_TOL * fabs(x)) {
            *xio = x;
            *count += it;
            return 1;
        }
    }
    *xio = x;
    *count += it;
    return 0;
}

/* Universal anomaly x solving F(x) = 0 (Appendix A).
 * mode 0: Laguerre (n = 5) from x = r0 as the paper states; starting there
 *         is not always convergent (rare high-eccentricity / large-r0 cases
 *         hit the cap), so on reaching the cap it restarts once from the
 *         first-order guess sqrt(mu) dt / r0 (a reading, see the tests).
 * mode 1: Newton from the first-order guess sqrt(mu) dt / r0.
 * mode 2: Newton from x_start (a proposed guess, e.g. a learned one) when
 *         it is admissible (orc_start_admissible), else from the
 *         first-order guess.
 * Modes 1 and 2 fall back to Laguerre from the first-order guess when
 * Newton reaches the cap (possible over many revolutions).
 * Returns 0 on convergence, 1 if the iteration cap was hit. */
/* Admissible starting values.  Along the orbit dx/dt = sqrt(mu)/r, so the
 * root over a step dt is x = sqrt(mu) dt <1/r> and its ratio to the
 * first-order guess sqrt(mu) dt / r0 lies between r0/r_max and r0/q, with q
 * the pericentre distance and r_max the apocentre (unbounded for e >= 1):
 * q = h^2 / (mu (1 + e)), r_max = h^2 / (mu (1 - e)), h = |x0 x v0|,
 * e^2 = 1 - alpha h^2 / mu.  A proposed start outside that range (or not
 * finite, or of the wrong sign) cannot be close to the root and is not
 * used; far outside it, the Stumpff functions of a huge argument can even
 * make Newton stop at a wrong value. */
int orc_start_admissible(double mu, const double *x0, const double *v0, double dt, double xs)
{
    if (!isfinite(xs) || dt == 0.0) return 0;
    double r0 = sqrt(x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2]);
    double vv = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    double alpha = 2.0 / r0 - vv / mu;
    double hx = x0[1] * v0[2] - x0[2] * v0[1];
    double hy = x0[2] * v0[0] - x0[0] * v0[2];
    double hz = x0[0] * v0[1] - x0[1] * v0[0];
    double h2 = hx * hx + hy * hy + hz * hz;
    double e2 = 1.0 - alpha * h2 / mu;
    double e = e2 > 0.0 ? sqrt(e2) : 0.0;
    double rho = xs / (sqrt(mu) * dt / r0);
    if (!(rho > 0.0)) return 0;
    if (h2 > 0.0 && rho > r0 * mu * (1.0 + e) / h2) return 0;
    if (alpha > 0.0 && e < 1.0 && h2 > 0.0 && rho < r0 * mu * (1.0 - e) / h2) return 0;
    return 1;
}

int orc_kepler_root(double mu, const double *x0, const double *v0, double dt,
                    int32_t mode, double x_start, int32_t use_start, double *x_out,
                    int32_t *iters)
{
    double r0 = sqrt(x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2]);
    double vv = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    double rv = x0[0] * v0[0] + x0[1] * v0[1] + x0[2] * v0[2];
    double smu = sqrt(mu);
    double alpha = 2.0 / r0 - vv / mu;
    int32_t count = 0;
    int ok;
    if (dt == 0.0) { *x_out = 0.0; *iters = 0; return 0; }
    double guess = smu * dt / r0;
    double x;
    if (mode == 0) {
        x = r0;
        ok = orc_kepler_iterate(smu, r0, rv, alpha, dt, 1, &x, &count);
        if (!ok) {
            x = guess;
            ok = orc_kepler_iterate(smu, r0, rv, alpha, dt, 1, &x, &count);
        }
    } else {
        x = (mode == 2 && use_start && orc_start_admissible(mu, x0, v0, dt, x_start)) ? x_start
                                                                                       : guess;
        ok = orc_kepler_iterate(smu, r0, rv, alpha, dt, 0, &x, &count);
        if (!ok) {
            x = guess;
            ok = orc_kepler_iterate(smu, r0, rv, alpha, dt, 1, &x, &count);
        }
    }
    *x_out = x;
    *iters = count;
    return ok ? 0 : 1;
}

/* Kepler advance of every body (Sec. 2, E_Kep; one independent solve per body). */
int64_t orc_kepler_all(int64_t n, double mu, const double *q, const double *v, double dt,
                       int32_t mode, double *q1, double *v1, int32_t *iters)
{
    int64_t fails = 0;
#pragma omp parallel for schedule(static) reduction(+ : fails)
    for (int64_t i = 0; i < n; ++i) {
        int32_t it;
        fails += orc_kepler_body(mu, q + 3 * i, v + 3 * i, dt, mode, q1 + 3 * i, v1 + 3 * i, &it);
        if (iters) iters[i] = it;
    }
    return fails;
}

/* ------------------------------------------------------------------ */
/* Sec. 2, E_Dft: H_Dft = |sum P_i|^2 / (2 m0).  Momenta are unchanged; */
/* every position moves by dt * (sum_j m_j v_j) / m0.                  */
/* ------------------------------------------------------------------ */
void orc_drift(int64_t n, double m0, const double *m, const double *v, double *q, double dt)
{
    double P[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) P[k] += m[i] * v[3 * i + k];
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) q[3 * i + k] += dt * (P[k] / m0);
}

/* ------------------------------------------------------------------ */
/* Per-body quantities used by encounter identification (Sec. 2.4) and  */
/* r_crit (Sec. 2.2): osculating semi-major axis A_i (r_i if unbound)   */
/* and escape speed ve_i = sqrt(2 mu / r_i).  Reading: taken from the   */
/* state after the first drift and before the first kick.              */
/* ------------------------------------------------------------------ */
void orc_prepass(int64_t n, double mu, const double *q, const double *v, double *A, double *ve)
{
    for (int64_t i = 0; i < n; ++i) {
        const double *x = q + 3 * i, *u = v + 3 * i;
        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        double inva = 2.0 / r - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / mu;
        A[i] = (inva > 0.0) ? 1.0 / inva : r;
        ve[i] = sqrt(2.0 * mu / r);
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 2, E_Int: acceleration from H_Int (all pairs, central mass     */
/* excluded): a_i = sum_{j != i} G m_j (Q_j - Q_i)/|Q_j - Q_i|^3.       */
/* A pair at zero separation contributes nothing (degenerate input).   */
/* ------------------------------------------------------------------ */
void orc_accel(int64_t n, double G, const double *m, const double *q, double *a)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = q[3 * j] - q[3 * i];
            double dy = q[3 * j + 1] - q[3 * i + 1];
            double dz = q[3 * j + 2] - q[3 * i + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double s = G * m[j] / (r2 * r);
            ax += s * dx;
            ay += s * dy;
            az += s * dz;
        }
        a[3 * i] = ax;
        a[3 * i + 1] = ay;
        a[3 * i + 2] = az;
    }
}

/* The same acceleration for a subset of bodies (rows), e.g. a sample of a
 * large system. */
void orc_accel_rows(int64_t n, double G, const double *m, const double *q, int64_t nrows,
                    const int64_t *rows, double *a)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = q[3 * j] - q[3 * i];
            double dy = q[3 * j + 1] - q[3 * i + 1];
            double dz = q[3 * j + 2] - q[3 * i + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double rr = sqrt(r2);
            double s = G * m[j] / (r2 * rr);
            ax += s * dx;
            ay += s * dy;
            az += s * dz;
        }
        a[3 * r] = ax;
        a[3 * r + 1] = ay;
        a[3 * r + 2] = az;
    }
}

/* E_Int(dt): v_i += dt * a_i */
void orc_kick(int64_t n, double G, const double *m, const double *q, double *v, double dt)
{
    double *a = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    orc_accel(n, G, m, q, a);
    for (int64_t i = 0; i < 3 * n; ++i) v[i] += dt * a[i];
    free(a);
}

/* ------------------------------------------------------------------ */
/* Sec. 2.4, crude sweep.  The printed predicate is garbled; the        */
/* reading taken is the symmetric conservative test                    */
/*   |Q_j - Q_i|^2 < ( c_s (R_up(i,j) + tau (ve_i + ve_j)) )^2           */
/* with R_up = a_E (h_i + h_j)(A_i + A_j)/2 (>= a_E x mutual Hill        */
/* radius because (x+y)^(1/3) <= x^(1/3) + y^(1/3)) in mutual mode and  */
/* R_up = a_E (h_i A_i + h_j A_j) in sum mode.  Candidates are the      */
/* unordered pairs (i < j) in lexicographic order.  Returns the count;  */
/* at most cap pairs are written.                                      */
/* ------------------------------------------------------------------ */
static int orc_crude_pair(const orc_params *p, double tau, const double *q, const double *h,
                          const double *A, const double *ve, int64_t i, int64_t j)
{
    double dx = q[3 * j] - q[3 * i];
    double dy = q[3 * j + 1] - q[3 * i + 1];
    double dz = q[3 * j + 2] - q[3 * i + 2];
    double r2 = dx * dx + dy * dy + dz * dz;
    double Rup;
    if (p->hill_mode == 0)
        Rup = p->aE * (h[i] + h[j]) * (A[i] + A[j]) / 2.0;
    else
        Rup = p->aE * (h[i] * A[i] + h[j] * A[j]);
    double lim = p->crude_safety * (Rup + fabs(tau) * (ve[i] + ve[j]));
    return r2 < lim * lim;
}

int64_t orc_crude(int64_t n, const orc_params *p, double tau, const double *q, const double *h,
                  const double *A, const double *ve, int32_t *pairs, int64_t cap)
{
    int64_t *cnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = i + 1; j < n; ++j) c += orc_crude_pair(p, tau, q, h, A, ve, i, j);
        cnt[i + 1] = c;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t total = cnt[n];
    if (pairs) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            int64_t o = cnt[i];
            if (o >= cap) continue;
            for (int64_t j = i + 1; j < n && o < cap; ++j) {
                if (orc_crude_pair(p, tau, q, h, A, ve, i, j)) {
                    pairs[2 * o] = (int32_t)i;
                    pairs[2 * o + 1] = (int32_t)j;
                    ++o;
                }
            }
        }
    }
    free(cnt);
    return total;
}

/* ------------------------------------------------------------------ */
/* Sec. 2.4, fine sweep.  The paper cites a third-order interpolation   */
/* of the separation over the step without spelling it out.  Reading:   */
/* the cubic Hermite interpolant of D(s) = |dq(s)|^2 on s in [0,1]      */
/* built from D and dD/ds at both ends:                                 */
/*   D(0) = |dq0|^2, D(1) = |dq1|^2, D'(0) = 2 tau dq0.dv0,             */
/*   D'(1) = 2 tau dq1.dv1,                                             */
/*   D(s) = c0 + c1 s + c2 s^2 + c3 s^3,                                */
/*   c0 = D(0), c1 = D'(0), c2 = 3(D(1)-D(0)) - 2D'(0) - D'(1),         */
/*   c3 = 2(D(0)-D(1)) + D'(0) + D'(1).                                 */
/* Its minimum over [0,1] is taken over the ends and the interior roots */
/* of D'(s) = c1 + 2 c2 s + 3 c3 s^2:                                   */
/*   disc = c2*c2 - 3*c3*c1, q = -(c2 + sign(c2) sqrt(disc)),           */
/*   s = q / (3 c3) and s = c1 / q  (stable for c3 -> 0, where the      */
/*   textbook (-c2 +- sqrt(disc))/(3 c3) cancels catastrophically).     */
/* Dm = max(0, min(...)).  A pair is marked (an encounter) when the     */
/* minimum separation is below a_E x (mutual Hill radius):              */
/*   mutual: Dm*Dm*Dm < (T*T)*(T*T)*(T*T)*M*M, T = a_E (A_i+A_j)/2,     */
/*           M = (m_i+m_j)/(3 m0)   (cube of the squared comparison,    */
/*           which avoids a cube root; evaluated left to right);        */
/*   sum:    Dm < R*R, R = a_E (h_i A_i + h_j A_j).                     */
/* lhs/rhs of that comparison are returned for the borderline rule.     */
/* ------------------------------------------------------------------ */
static double orc_cubic_at(double c0, double c1, double c2, double c3, double s)
{
    return c0 + s * (c1 + s * (c2 + s * c3));
}

int orc_fine_pair(const orc_params *p, double tau, const double *m, const double *h,
                  const double *A, const double *q0, const double *v0, const double *q1,
                  const double *v1, int64_t i, int64_t j, double *Dm_out, double *lhs_out,
                  double *rhs_out)
{
    double a0[3], b0[3], a1[3], b1[3];
    for (int k = 0; k < 3; ++k) {
        a0[k] = q0[3 * j + k] - q0[3 * i + k];
        b0[k] = v0[3 * j + k] - v0[3 * i + k];
        a1[k] = q1[3 * j + k] - q1[3 * i + k];
        b1[k] = v1[3 * j + k] - v1[3 * i + k];
    }
    double D0 = a0[0] * a0[0] + a0[1] * a0[1] + a0[2] * a0[2];
    double D1 = a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2];
    double d0 = 2.0 * tau * (a0[0] * b0[0] + a0[1] * b0[1] + a0[2] * b0[2]);
    double d1 = 2.0 * tau * (a1[0] * b1[0] + a1[1] * b1[1] + a1[2] * b1[2]);
    double c0 = D0, c1 = d0;
    double c2 = 3.0 * (D1 - D0) - 2.0 * d0 - d1;
    double c3 = 2.0 * (D0 - D1) + d0 + d1;
    double Dm = (D0 < D1) ? D0 : D1;
    /* stationary points: roots of 3 c3 s^2 + 2 c2 s + c1 = 0, in the
       cancellation-free form q = -(c2 + sign(c2) sqrt(disc)), s = q/(3 c3),
       s = c1/q (the second root also covers c3 -> 0, where D is quadratic) */
    double disc = c2 * c2 - 3.0 * c3 * c1;
    if (disc >= 0.0) {
        double sq = sqrt(disc);
        double qq = -(c2 + (c2 >= 0.0 ? sq : -sq));
        double sr[2];
        int nr = 0;
        if (c3 != 0.0) sr[nr++] = qq / (3.0 * c3);
        if (qq != 0.0) sr[nr++] = c1 / qq;
        for (int r = 0; r < nr; ++r) {
            if (sr[r] > 0.0 && sr[r] < 1.0) {
                double D = orc_cubic_at(c0, c1, c2, c3, sr[r]);
                if (D < Dm) Dm = D;
            }
        }
    }
    if (Dm < 0.0) Dm = 0.0;
    double lhs, rhs;
    if (p->hill_mode == 0) {
        double T = p->aE * (A[i] + A[j]) / 2.0;
        double M = (m[i] + m[j]) / (3.0 * p->m0);
        double T2 = T * T;
        lhs = Dm * Dm * Dm;
        rhs = T2 * T2 * T2 * M * M;
    } else {
        double R = p->aE * (h[i] * A[i] + h[j] * A[j]);
        lhs = Dm;
        rhs = R * R;
    }
    if (Dm_out) *Dm_out = Dm;
    if (lhs_out) *lhs_out = lhs;
    if (rhs_out) *rhs_out = rhs;
    return lhs < rhs;
}

int64_t orc_fine(int64_t npairs, const int32_t *pairs, const orc_params *p, double tau,
                 const double *m, const double *h, const double *A, const double *q0,
                 const double *v0, const double *q1, const double *v1, int32_t *flags,
                 double *lhs, double *rhs)
{
    int64_t c = 0;
    for (int64_t k = 0; k < npairs; ++k) {
        double l, r;
        int f = orc_fine_pair(p, tau, m, h, A, q0, v0, q1, v1, pairs[2 * k], pairs[2 * k + 1],
                              NULL, &l, &r);
        if (flags) flags[k] = f;
        if (lhs) lhs[k] = l;
        if (rhs) rhs[k] = r;
        c += f;
    }
    return c;
}

/* ------------------------------------------------------------------ */
/* Brute force of Sec. 2.4's identification without the crude sweep:    */
/* the fine test of every pair (i, j), j != i, for each i in rows[];    */
/* pairs (min, max) are written to pairs[] (capacity cap) grouped by    */
/* row in the order of rows[], j ascending.  Returns the count.  It is  */
/* the reference the two-stage sweep must reproduce.                    */
/* ------------------------------------------------------------------ */
int64_t orc_fine_brute(int64_t n, int64_t nrows, const int64_t *rows, const orc_params *p,
                       double tau, const double *m, const double *h, const double *A,
                       const double *q0, const double *v0, const double *q1, const double *v1,
                       int32_t *pairs, int64_t cap)
{
    int64_t *cnt = (int64_t *)calloc((size_t)(nrows + 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const int64_t a = i < j ? i : j, b = i < j ? j : i;
            c += orc_fine_pair(p, tau, m, h, A, q0, v0, q1, v1, a, b, NULL, NULL, NULL);
        }
        cnt[r + 1] = c;
    }
    for (int64_t r = 0; r < nrows; ++r) cnt[r + 1] += cnt[r];
    const int64_t total = cnt[nrows];
    if (pairs) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; ++r) {
            const int64_t i = rows[r];
            int64_t o = cnt[r];
            for (int64_t j = 0; j < n && o < cap; ++j) {
                if (j == i) continue;
                const int64_t a = i < j ? i : j, b = i < j ? j : i;
                if (orc_fine_pair(p, tau, m, h, A, q0, v0, q1, v1, a, b, NULL, NULL, NULL)) {
                    pairs[2 * o] = (int32_t)a;
                    pairs[2 * o + 1] = (int32_t)b;
                    ++o;
                }
            }
        }
    }
    free(cnt);
    return total;
}

/* ------------------------------------------------------------------ */
/* Sec. 2.3 step 4 / Sec. 2.4: division of the encounter pairs into     */
/* non-intersecting sets = connected components of the encounter graph. */
/* label[i] = smallest body index of i's component, -1 if i is in no    */
/* encounter.  Plain repeated relaxation until nothing changes.         */
/* ------------------------------------------------------------------ */
int64_t orc_sets(int64_t n, int64_t npairs, const int32_t *pairs, int32_t *label)
{
    for (int64_t i = 0; i < n; ++i) label[i] = -1;
    for (int64_t k = 0; k < npairs; ++k) {
        label[pairs[2 * k]] = pairs[2 * k];
        label[pairs[2 * k + 1]] = pairs[2 * k + 1];
    }
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int64_t k = 0; k < npairs; ++k) {
            int32_t a = pairs[2 * k], b = pairs[2 * k + 1];
            int32_t l = label[a] < label[b] ? label[a] : label[b];
            if (label[a] != l) { label[a] = l; changed = 1; }
            if (label[b] != l) { label[b] = l; changed = 1; }
        }
    }
    int64_t nsets = 0;
    for (int64_t i = 0; i < n; ++i) nsets += (label[i] == i);
    return nsets;
}

/* ------------------------------------------------------------------ */
/* Sec. 2.1: transition function K(y), y = 1.1 s / r_crit - 0.1,        */
/* K = 0 (y <= 0), sin(pi y / 2) (0 < y < 1), 1 (y >= 1); derivatives   */
/* with respect to the separation s: K' = (pi/2)(1.1/r_crit) cos(pi y/2),*/
/* K'' = -(pi/2)^2 (1.1/r_crit)^2 sin(pi y/2) inside, 0 outside.        */
/* W(s) = 1 - K + s K' is the weight of a full pair force that belongs  */
/* to H'_Kep (Sec. 2.2 acceleration; the correction of Sec. 2.3 steps   */
/* 5 and 7 subtracts the same weight from the kick).                    */
/* ------------------------------------------------------------------ */
void orc_transition(double s, double rcrit, double *K, double *Kp, double *Kpp)
{
    double y = 1.1 * s / rcrit - 0.1;
    if (y <= 0.0) {
        *K = 0.0; *Kp = 0.0; *Kpp = 0.0;
    } else if (y >= 1.0) {
        *K = 1.0; *Kp = 0.0; *Kpp = 0.0;
    } else {
        double w = M_PI / 2.0;
        double c = 1.1 / rcrit;
        *K = sin(w * y);
        *Kp = w * c * cos(w * y);
        *Kpp = -(w * c) * (w * c) * sin(w * y);
    }
}

/* Acceleration of member i of a set from the other members, weighted by
 * W at separation s = sqrt(q^2 + eps^2).  Used unsoftened (eps = 0) by the
 * corrections of Sec. 2.3 steps 5 and 7, softened by the Hermite. */
static void orc_set_pair_acc(int64_t nm, const int32_t *mem, const double *m, const double *q,
                             double G, double rcrit, double eps, int64_t a, double *acc)
{
    int64_t i = mem[a];
    acc[0] = acc[1] = acc[2] = 0.0;
    for (int64_t b = 0; b < nm; ++b) {
        if (b == a) continue;
        int64_t j = mem[b];
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = q[3 * j + k] - q[3 * i + k];
        double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
        if (s2 == 0.0) continue;
        double s = sqrt(s2);
        double K, Kp, Kpp;
        orc_transition(s, rcrit, &K, &Kp, &Kpp);
        double W = 1.0 - K + s * Kp;
        double f = G * m[j] * W / (s2 * s);
        for (int k = 0; k < 3; ++k) acc[k] += f * d[k];
    }
}

/* Sec. 2.3 steps 5 and 7: v_i -= dt * sum_{j in S, j != i} G m_j W(q_ij)
 * (Q_j - Q_i)/q_ij^3 for every member i of set S (members ascending). */
void orc_correct_set(int64_t nm, const int32_t *mem, const double *m, const double *q,
                     double *v, double G, double rcrit, double dt)
{
    double *acc = (double *)malloc(sizeof(double) * 3 * (size_t)(nm > 0 ? nm : 1));
    for (int64_t a = 0; a < nm; ++a) orc_set_pair_acc(nm, mem, m, q, G, rcrit, 0.0, a, acc + 3 * a);
    for (int64_t a = 0; a < nm; ++a)
        for (int k = 0; k < 3; ++k) v[3 * mem[a] + k] -= dt * acc[3 * a + k];
    free(acc);
}

/* ------------------------------------------------------------------ */
/* Sec. 2.2: acceleration and jerk of the H'_Kep flow of one set, star  */
/* fixed at the origin (sign written attractive, central jerk with      */
/* 1/r^3; the print divides the central jerk by s_i0 only):             */
/*  a_i = -mu Q_i/r_i^3 + sum_j G m_j W(s) q_ji / s^3                   */
/*  j_i = -mu [v_i/r_i^3 - 3 (Q_i.v_i) Q_i / r_i^5]                     */
/*        + sum_j G m_j / s^3 { (v_ji.q_ji) q_ji K''(s)                 */
/*                          + (v_ji - 3 (v_ji.q_ji) q_ji / s^2) W(s) }  */
/* q_ji = Q_j - Q_i, v_ji = v_j - v_i, s = sqrt(|q_ji|^2 + eps_H^2).    */
/* The smoothing applies to the in-set pairs only.                      */
/* x, u are the member states packed [3*a + k].                         */
/* ------------------------------------------------------------------ */
void orc_hermite_force(int64_t nm, const double *mm, const double *x, const double *u,
                       double G, double mu, double rcrit, double eps, double *acc, double *jrk)
{
    for (int64_t a = 0; a < nm; ++a) {
        const double *X = x + 3 * a, *U = u + 3 * a;
        double r2 = X[0] * X[0] + X[1] * X[1] + X[2] * X[2];
        double r = sqrt(r2);
        double r3 = r2 * r;
        double xv = X[0] * U[0] + X[1] * U[1] + X[2] * U[2];
        double A3[3], J3[3];
        for (int k = 0; k < 3; ++k) {
            A3[k] = -mu * X[k] / r3;
            J3[k] = -mu * (U[k] / r3 - 3.0 * xv * X[k] / (r3 * r2));
        }
        for (int64_t b = 0; b < nm; ++b) {
            if (b == a) continue;
            double d[3], w[3];
            for (int k = 0; k < 3; ++k) {
                d[k] = x[3 * b + k] - X[k];
                w[k] = u[3 * b + k] - U[k];
            }
            double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
            if (s2 == 0.0) continue;
            double s = sqrt(s2);
            double K, Kp, Kpp;
            orc_transition(s, rcrit, &K, &Kp, &Kpp);
            double W = 1.0 - K + s * Kp;
            double gm = G * mm[b] / (s2 * s);
            double dw = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
            for (int k = 0; k < 3; ++k) {
                A3[k] += gm * W * d[k];
                J3[k] += gm * (dw * d[k] * Kpp + (w[k] - 3.0 * dw * d[k] / s2) * W);
            }
        }
        for (int k = 0; k < 3; ++k) { acc[3 * a + k] = A3[k]; jrk[3 * a + k] = J3[k]; }
    }
}

static double norm3(const double *a) { return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

/* ------------------------------------------------------------------ */
/* Sec. 2.2: 4th-order Hermite integration of one set over dt, written  */
/* from the predictor-corrector scheme the paper cites (no Ahmad-Cohen):*/
/*  predict  x_p = x + v h + a h^2/2 + j h^3/6,  v_p = v + a h + j h^2/2 */
/*  evaluate a1, j1 at (x_p, v_p)                                       */
/*  a2 = (-6 (a - a1) - h (4 j + 2 j1)) / h^2                           */
/*  a3 = (12 (a - a1) + 6 h (j + j1)) / h^3                             */
/*  correct  x = x_p + a2 h^4/24 + a3 h^5/120, v = v_p + a2 h^3/6 + a3 h^4/24 */
/*  a <- a1, j <- j1 (one force evaluation per substep).                */
/* Steps: first h = eta_s |a|/|j|; afterwards                            */
/*  h = sqrt(eta (|a1||a2e| + |j1|^2) / (|j1||a3| + |a2e|^2)),          */
/*  a2e = a2 + h a3.  Reading: one shared step per set, the minimum over */
/*  members, clipped so that the last substep ends exactly at dt.        */
/* Returns the number of substeps (negative if the cap was hit).         */
/* ------------------------------------------------------------------ */
static double orc_step_of(const double *a1, const double *j1, const double *a2e,
                          const double *a3, double eta)
{
    double na = norm3(a1), nj = norm3(j1), n2 = norm3(a2e), n3 = norm3(a3);
    return sqrt(eta * (na * n2 + nj * nj) / (nj * n3 + n2 * n2));
}

int64_t orc_hermite_set(int64_t nm, const int32_t *mem, const double *m, double *q, double *v,
                        const orc_params *p, double rcrit, double dt)
{
    double mu = p->G * p->m0;
    size_t sz = sizeof(double) * 3 * (size_t)(nm > 0 ? nm : 1);
    double *x = malloc(sz), *u = malloc(sz), *a = malloc(sz), *jk = malloc(sz);
    double *xp = malloc(sz), *up = malloc(sz), *a1 = malloc(sz), *j1 = malloc(sz);
    double *mm = malloc(sizeof(double) * (size_t)(nm > 0 ? nm : 1));
    for (int64_t b = 0; b < nm; ++b) {
        mm[b] = m[mem[b]];
        for (int k = 0; k < 3; ++k) { x[3 * b + k] = q[3 * mem[b] + k]; u[3 * b + k] = v[3 * mem[b] + k]; }
    }
    orc_hermite_force(nm, mm, x, u, p->G, mu, rcrit, p->epsH, a, jk);
    double sgn = dt >= 0.0 ? 1.0 : -1.0;
    double T = fabs(dt);
    double h = INFINITY;
    for (int64_t b = 0; b < nm; ++b) {
        double hb = p->eta_s * norm3(a + 3 * b) / norm3(jk + 3 * b);
        if (hb > 0.0 && hb < h) h = hb;
    }
    double t = 0.0;
    int64_t nsub = 0;
    int last = (T == 0.0); /* a zero step leaves the set unchanged */
    while (!last) {
        if (nsub >= p->max_substeps) { nsub = -nsub - 1; break; }
        if (!(h > 0.0) || h >= T - t) { h = T - t; last = 1; }
        double hs = sgn * h;
        for (int64_t c = 0; c < 3 * nm; ++c) {
            xp[c] = x[c] + hs * u[c] + hs * hs * a[c] / 2.0 + hs * hs * hs * jk[c] / 6.0;
            up[c] = u[c] + hs * a[c] + hs * hs * jk[c] / 2.0;
        }
        orc_hermite_force(nm, mm, xp, up, p->G, mu, rcrit, p->epsH, a1, j1);
        double hn = INFINITY;
        for (int64_t b = 0; b < nm; ++b) {
            double A2[3], A3[3], A2e[3];
            for (int k = 0; k < 3; ++k) {
                int64_t c = 3 * b + k;
                A2[k] = (-6.0 * (a[c] - a1[c]) - hs * (4.0 * jk[c] + 2.0 * j1[c])) / (hs * hs);
                A3[k] = (12.0 * (a[c] - a1[c]) + 6.0 * hs * (jk[c] + j1[c])) / (hs * hs * hs);
                x[c] = xp[c] + A2[k] * hs * hs * hs * hs / 24.0 + A3[k] * hs * hs * hs * hs * hs / 120.0;
                u[c] = up[c] + A2[k] * hs * hs * hs / 6.0 + A3[k] * hs * hs * hs * hs / 24.0;
                A2e[k] = A2[k] + hs * A3[k];
            }
            double hb = orc_step_of(a1 + 3 * b, j1 + 3 * b, A2e, A3, p->eta);
            if (hb > 0.0 && hb < hn) hn = hb;
        }
        memcpy(a, a1, sz);
        memcpy(jk, j1, sz);
        t += h;
        ++nsub;
        h = hn;
    }
    for (int64_t b = 0; b < nm; ++b)
        for (int k = 0; k < 3; ++k) { q[3 * mem[b] + k] = x[3 * b + k]; v[3 * mem[b] + k] = u[3 * b + k]; }
    free(x); free(u); free(a); free(jk); free(xp); free(up); free(a1); free(j1); free(mm);
    return nsub;
}

/* H'_Kep of one set with the star fixed (Sec. 2.1, modified Keplerian
 * Hamiltonian; pair part uses the softened separation of the Hermite). */
double orc_hkep_set(int64_t nm, const int32_t *mem, const double *m, const double *q,
                    const double *v, const orc_params *p, double rcrit)
{
    double E = 0.0;
    double mu = p->G * p->m0;
    for (int64_t a = 0; a < nm; ++a) {
        int64_t i = mem[a];
        double vv = v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
        E += 0.5 * m[i] * vv - mu * m[i] / norm3(q + 3 * i);
        for (int64_t b = a + 1; b < nm; ++b) {
            int64_t j = mem[b];
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = q[3 * j + k] - q[3 * i + k];
            double s = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + p->epsH * p->epsH);
            double K, Kp, Kpp;
            orc_transition(s, rcrit, &K, &Kp, &Kpp);
            E -= p->G * m[i] * m[j] * (1.0 - K) / s;
        }
    }
    return E;
}

/* ------------------------------------------------------------------ */
/* Total energy, Sec. 2 eq. for H (H_Dft + H_Kep + H_Int):               */
/*  E = sum 1/2 m v^2 + |sum m v|^2/(2 m0) - sum G m0 m_i / r_i          */
/*      - sum_{i<j} G m_i m_j / q_ij                                    */
/* ------------------------------------------------------------------ */
double orc_energy(int64_t n, double G, double m0, const double *m, const double *q,
                  const double *v)
{
    double *row = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = i + 1; j < n; ++j) {
            double dx = q[3 * j] - q[3 * i], dy = q[3 * j + 1] - q[3 * i + 1], dz = q[3 * j + 2] - q[3 * i + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r > 0.0) s += m[j] / r;
        }
        row[i] = s;
    }
    double kin = 0.0, pot0 = 0.0, potp = 0.0, P[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        const double *x = q + 3 * i, *u = v + 3 * i;
        kin += 0.5 * m[i] * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int k = 0; k < 3; ++k) P[k] += m[i] * u[k];
        pot0 += G * m0 * m[i] / norm3(x);
        potp += G * m[i] * row[i];
    }
    free(row);
    return kin + (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]) / (2.0 * m0) - pot0 - potp;
}

/* Angular momentum L = sum m_i Q_i x v_i (DH coordinates are canonical). */
void orc_angmom(int64_t n, const double *m, const double *q, const double *v, double *L)
{
    L[0] = L[1] = L[2] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *x = q + 3 * i, *u = v + 3 * i;
        L[0] += m[i] * (x[1] * u[2] - x[2] * u[1]);
        L[1] += m[i] * (x[2] * u[0] - x[0] * u[2]);
        L[2] += m[i] * (x[0] * u[1] - x[1] * u[0]);
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 2.3: one hybrid step, procedure steps 1-10, with the sweeps of  */
/* Sec. 2.4.  In order:                                                 */
/*  1  drift tau/2;  per-body A_i, ve_i                                 */
/*  2  kick tau/2 with all pairs and no K; crude candidates at these Q  */
/*  3  Kepler tau from (q0, v0) = state after the kick -> (q1, v1)      */
/*  4  fine test on candidates -> encounter pairs -> sets -> r_crit(S)  */
/*     = a_H max_{i in S} h_i A_i (Hill radius h_i A_i)                 */
/*  5  correction at q0: v0_i -= tau/2 sum_S G m_j W (q0_j-q0_i)/q^3    */
/*  6  Hermite of each set from (q0, v0) over tau -> q1, v1 of members  */
/*  7  correction at q1 on v1 (anticipating the kick of step 9)         */
/*  8  state = (q1, v1)                                                 */
/*  9  kick tau/2 (all pairs, no K)                                     */
/* 10  drift tau/2                                                      */
/* Pairs in different sets, or with a non-member, keep K = 1.           */
/* enc_pairs (capacity enc_cap pairs) and label (n) receive the step's  */
/* encounter list (i<j, lexicographic) and component labels; rcrit_out  */
/* (n entries) receives r_crit of every set, sets numbered by their     */
/* smallest member.                                                     */
/* Returns 0, or a positive code: 1 Kepler cap hit, 2 Hermite cap hit,  */
/* 4 candidate capacity exceeded.                                       */
/* ------------------------------------------------------------------ */
int orc_step(int64_t n, const orc_params *p, double tau, const double *m, const double *h,
             double *q, double *v, int64_t cand_cap, int32_t *enc_pairs, int64_t enc_cap,
             int32_t *label_out, double *rcrit_out, orc_stats *st)
{
    int rc = 0;
    double mu = p->G * p->m0;
    size_t sz3 = sizeof(double) * 3 * (size_t)(n > 0 ? n : 1);
    size_t sz1 = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *A = malloc(sz1), *ve = malloc(sz1);
    double *q0 = malloc(sz3), *v0 = malloc(sz3);
    int32_t *iters = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *label = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cand = malloc(sizeof(int32_t) * 2 * (size_t)(cand_cap > 0 ? cand_cap : 1));
    orc_stats s;
    memset(&s, 0, sizeof s);

    /* 1 */
    orc_drift(n, p->m0, m, v, q, tau / 2.0);
    orc_prepass(n, mu, q, v, A, ve);
    /* 2 (crude sweep at the kick's positions) */
    int64_t nc = orc_crude(n, p, tau, q, h, A, ve, cand, cand_cap);
    s.n_candidates = nc;
    if (nc > cand_cap) { s.cand_overflow = nc - cand_cap; nc = cand_cap; rc |= 4; }
    orc_kick(n, p->G, m, q, v, tau / 2.0);
    /* 3 */
    memcpy(q0, q, sz3);
    memcpy(v0, v, sz3);
    s.kepler_fail = orc_kepler_all(n, mu, q0, v0, tau, p->kepler_mode, q, v, iters);
    if (s.kepler_fail) rc |= 1;
    for (int64_t i = 0; i < n; ++i) {
        s.kepler_iters += iters[i];
        if (iters[i] > s.kepler_max) s.kepler_max = iters[i];
    }
    /* 4 */
    int32_t *enc = malloc(sizeof(int32_t) * 2 * (size_t)(nc > 0 ? nc : 1));
    int64_t ne = 0;
    for (int64_t k = 0; k < nc; ++k) {
        int32_t i = cand[2 * k], j = cand[2 * k + 1];
        if (orc_fine_pair(p, tau, m, h, A, q0, v0, q, v, i, j, NULL, NULL, NULL)) {
            enc[2 * ne] = i;
            enc[2 * ne + 1] = j;
            ++ne;
        }
    }
    s.n_encounters = ne;
    s.n_sets = orc_sets(n, ne, enc, label);
    /* Sec. 2.3, after the steps: when a set holds more than one planet the
     * step may integrate every body with the Hermite.  Reading: all bodies
     * form one set whose r_crit is infinite, so K = 0 and W = 1 for every
     * pair; the corrections then take back both half kicks entirely and the
     * Hermite integrates H_Kep + H_Int of the whole system between the two
     * drifts. */
    double rc_whole = 0.0;
    if (p->planet_mass > 0.0 && s.n_sets > 0) {
        int32_t *np = calloc((size_t)n, sizeof(int32_t));
        int whole = 0;
        for (int64_t i = 0; i < n; ++i)
            if (label[i] >= 0 && m[i] >= p->planet_mass && ++np[label[i]] >= 2) whole = 1;
        free(np);
        if (whole) {
            for (int64_t i = 0; i < n; ++i) label[i] = 0;
            s.n_sets = 1;
            s.whole_system = 1;
            rc_whole = INFINITY;
        }
    }
    if (s.n_sets > 0) {
        /* members of each set, ascending, grouped by label ascending */
        int64_t nmem = 0;
        for (int64_t i = 0; i < n; ++i) nmem += (label[i] >= 0);
        int32_t *mem = malloc(sizeof(int32_t) * (size_t)nmem);
        int64_t *start = malloc(sizeof(int64_t) * (size_t)(s.n_sets + 1));
        int32_t *root = malloc(sizeof(int32_t) * (size_t)s.n_sets);
        int64_t ns = 0, o = 0;
        for (int64_t r = 0; r < n; ++r) {
            if (label[r] != r) continue;
            root[ns] = (int32_t)r;
            start[ns] = o;
            for (int64_t i = r; i < n; ++i)
                if (label[i] == r) mem[o++] = (int32_t)i;
            ++ns;
        }
        start[ns] = o;
        for (int64_t k = 0; k < ns; ++k) {
            int64_t nm = start[k + 1] - start[k];
            const int32_t *mk = mem + start[k];
            if (nm > s.max_set) s.max_set = nm;
            double hmax = 0.0;
            for (int64_t b = 0; b < nm; ++b) {
                double rh = h[mk[b]] * A[mk[b]];
                if (rh > hmax) hmax = rh;
            }
            double rcrit = s.whole_system ? rc_whole : p->aH * hmax;
            if (rcrit_out) rcrit_out[k] = rcrit;
            /* 5 */
            orc_correct_set(nm, mk, m, q0, v0, p->G, rcrit, tau / 2.0);
            /* 6: Hermite from (q0, v0) of the members, results into (q, v) */
            for (int64_t b = 0; b < nm; ++b)
                for (int c = 0; c < 3; ++c) {
                    q[3 * mk[b] + c] = q0[3 * mk[b] + c];
                    v[3 * mk[b] + c] = v0[3 * mk[b] + c];
                }
            int64_t ns_k = orc_hermite_set(nm, mk, m, q, v, p, rcrit, tau);
            if (ns_k < 0) { s.hermite_fail++; rc |= 2; ns_k = -ns_k - 1; }
            s.substeps += ns_k;
            /* 7 */
            orc_correct_set(nm, mk, m, q, v, p->G, rcrit, tau / 2.0);
        }
        free(mem); free(start); free(root);
    }
    if (enc_pairs) {
        int64_t c = ne < enc_cap ? ne : enc_cap;
        memcpy(enc_pairs, enc, sizeof(int32_t) * 2 * (size_t)c);
    }
    if (label_out) memcpy(label_out, label, sizeof(int32_t) * (size_t)n);
    /* 9, 10 */
    orc_kick(n, p->G, m, q, v, tau / 2.0);
    orc_drift(n, p->m0, m, v, q, tau / 2.0);
    if (st) *st = s;
    free(A); free(ve); free(q0); free(v0); free(iters); free(label); free(cand); free(enc);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Step without the close-encounter search (Sec. 2, after the second-   */
/* order composition): with no search the Keplerian and interaction     */
/* operators trade places, so one O(N^2) evaluation serves a step:      */
/*   E_Dft(tau/2) E_Kep(tau/2) E_Int(tau) E_Kep(tau/2) E_Dft(tau/2)     */
/* (the paper states the swap without writing the product out; this is */
/* the symmetric second-order arrangement of the same three operators). */
/* Returns the number of Kepler solves that hit the cap; iteration      */
/* counts summed into *kepler_iters when not NULL.                      */
/* ------------------------------------------------------------------ */
int64_t orc_step_swapped(int64_t n, const orc_params *p, double tau, const double *m, double *q,
                         double *v, int64_t *kepler_iters)
{
    double mu = p->G * p->m0;
    double *qt = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *vt = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int32_t *it = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t fails = 0, iters = 0;
    orc_drift(n, p->m0, m, v, q, tau / 2.0);
    fails += orc_kepler_all(n, mu, q, v, tau / 2.0, p->kepler_mode, qt, vt, it);
    for (int64_t i = 0; i < n; ++i) iters += it[i];
    orc_kick(n, p->G, m, qt, vt, tau);
    fails += orc_kepler_all(n, mu, qt, vt, tau / 2.0, p->kepler_mode, q, v, it);
    for (int64_t i = 0; i < n; ++i) iters += it[i];
    orc_drift(n, p->m0, m, v, q, tau / 2.0);
    if (kepler_iters) *kepler_iters += iters;
    free(qt); free(vt); free(it);
    return fails;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}
