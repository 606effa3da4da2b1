/*
 * lbm_ref.c -- CPU oracle for the D2Q37 thermal lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY (see lbm_ref.h): only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark load this library.  It shares no
 * code with the GPU library; the GPU side derives its constants by another
 * method and both are cross-checked by the tests.
 *
 * Plain serial FP64.  Built with -O2 -ffp-contract=off so that every product
 * and sum is rounded as written.  An OpenMP build of this same file (only the
 * outer x loops are annotated) gives bitwise the same results, because the
 * arithmetic of each site does not depend on the thread that runs it.
 *
 * Paper: arXiv:1703.04594, section 3 ("Lattice Boltzmann methods").
 *
 * Readings where the paper is silent (it defers these to its model papers):
 *  (R1) velocity set: the 37 integer hops e = (ex, ey) with |e|^2 in
 *       {0,1,2,4,5,8,9,10}; every hop is at most 3 lattice points long, as the
 *       section on the model states.  Canonical order: by |e|^2, then by the
 *       angle atan2(ey, ex) taken in [0, 2*pi).
 *  (R2) weights and scale: xi_l = c * e_l; the 8 shell weights and c solve the
 *       9 equations  sum_l w_l xi_x^(2i) xi_y^(2j) = (2i-1)!! (2j-1)!!,
 *       2i + 2j <= 8, i >= j  (unit-temperature Gaussian moments), solved here
 *       in quad precision and rounded once to double.
 *  (R3) equilibrium: the 4th-order Hermite expansion of the Maxwellian at
 *       (rho, u, T) in D = 2, written out term by term (ref_feq).
 *  (R4) gravity (the -rho g delta_{i,2} force of the continuum equations) by
 *       shifting the equilibrium: u* = u + tau g, T* = T + tau (1 - tau) g^2 / 2.
 *  (R5) walls: after propagate, every slot of the 3 bottom / 3 top rows whose
 *       pull source lies outside the lattice receives f^eq_l(1, 0, T_wall)
 *       times the density, in the pre-propagate state, of the fluid site that
 *       mirrors the source across the wall (rows -1-k <-> k).
 */
#include "lbm_ref.h"

#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q REF_NPOP
#define D 2

/* ------------------------------------------------------------------------ */
/* Velocity set (R1)                                                         */
/* ------------------------------------------------------------------------ */

static const int SHELL_R2[8] = {0, 1, 2, 4, 5, 8, 9, 10};

static int EX[Q], EY[Q];
static double WL[Q];     /* weight of each population */
static double XI_X[Q], XI_Y[Q];
static double C_SCALE;
static int tables_ready = 0;

static double hop_angle(int ex, int ey)
{
    double a = atan2((double)ey, (double)ex);
    if (a < 0.0) a += 2.0 * M_PI;
    return a;
}

static void build_velocity_set(void)
{
    int n = 0;
    for (int ex = -3; ex <= 3; ++ex)
        for (int ey = -3; ey <= 3; ++ey) {
            int r2 = ex * ex + ey * ey;
            for (int s = 0; s < 8; ++s)
                if (SHELL_R2[s] == r2) { EX[n] = ex; EY[n] = ey; ++n; }
        }
    /* insertion sort by (|e|^2, angle) */
    for (int i = 1; i < n; ++i) {
        int ex = EX[i], ey = EY[i], j = i - 1;
        int r2 = ex * ex + ey * ey;
        double an = hop_angle(ex, ey);
        while (j >= 0) {
            int r2j = EX[j] * EX[j] + EY[j] * EY[j];
            double anj = hop_angle(EX[j], EY[j]);
            if (r2j < r2 || (r2j == r2 && anj < an)) break;
            EX[j + 1] = EX[j]; EY[j + 1] = EY[j]; --j;
        }
        EX[j + 1] = ex; EY[j + 1] = ey;
    }
}

/* ------------------------------------------------------------------------ */
/* Quadrature (R2), in __float128                                            */
/* ------------------------------------------------------------------------ */

/* the 9 moment equations: (i, j) with 2i+2j <= 8, i >= j */
static const int MOM_I[9] = {0, 1, 1, 2, 2, 3, 2, 3, 4};
static const int MOM_J[9] = {0, 0, 1, 0, 1, 0, 2, 1, 0};

static __float128 double_factorial_odd(int i) /* (2i-1)!! */
{
    __float128 r = 1;
    for (int k = 2 * i - 1; k > 1; k -= 2) r *= k;
    return r;
}

/* S[k][s] = sum over hops of shell s of ex^(2i) ey^(2j), equation k. */
static void shell_sums(__float128 S[9][8])
{
    for (int k = 0; k < 9; ++k)
        for (int s = 0; s < 8; ++s) {
            __float128 acc = 0;
            for (int l = 0; l < Q; ++l) {
                if (EX[l] * EX[l] + EY[l] * EY[l] != SHELL_R2[s]) continue;
                __float128 t = 1;
                for (int p = 0; p < 2 * MOM_I[k]; ++p) t *= EX[l];
                for (int p = 0; p < 2 * MOM_J[k]; ++p) t *= EY[l];
                acc += t;
            }
            S[k][s] = acc;
        }
}

/* For a trial q = c^2, solve the first 8 equations for the 8 shell weights by
 * Gaussian elimination with partial pivoting and return the residual of the
 * ninth.  Returns 0 if the 8x8 system is singular. */
static int weights_for_q(const __float128 S[9][8], __float128 q,
                         __float128 w[8], __float128* resid)
{
    __float128 A[8][9];
    for (int k = 0; k < 8; ++k) {
        int d = MOM_I[k] + MOM_J[k];
        __float128 qd = powq(q, d);
        for (int s = 0; s < 8; ++s) A[k][s] = qd * S[k][s];
        A[k][8] = double_factorial_odd(MOM_I[k]) * double_factorial_odd(MOM_J[k]);
    }
    for (int col = 0; col < 8; ++col) {
        int piv = col;
        for (int r = col + 1; r < 8; ++r)
            if (fabsq(A[r][col]) > fabsq(A[piv][col])) piv = r;
        if (A[piv][col] == 0) return 0;
        if (piv != col)
            for (int c = 0; c < 9; ++c) { __float128 t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
        for (int r = col + 1; r < 8; ++r) {
            __float128 f = A[r][col] / A[col][col];
            for (int c = col; c < 9; ++c) A[r][c] -= f * A[col][c];
        }
    }
    for (int r = 7; r >= 0; --r) {
        __float128 acc = A[r][8];
        for (int c = r + 1; c < 8; ++c) acc -= A[r][c] * w[c];
        w[r] = acc / A[r][r];
    }
    int d8 = MOM_I[8] + MOM_J[8];
    __float128 lhs = 0;
    for (int s = 0; s < 8; ++s) lhs += powq(q, d8) * S[8][s] * w[s];
    *resid = lhs - double_factorial_odd(MOM_I[8]) * double_factorial_odd(MOM_J[8]);
    return 1;
}

static int all_positive(const __float128 w[8])
{
    for (int s = 0; s < 8; ++s) if (!(w[s] > 0)) return 0;
    return 1;
}

static __float128 Q_ROOT;        /* c^2 */
static __float128 W_SHELL_Q[8];  /* shell weights */

static void solve_quadrature(void)
{
    __float128 S[9][8];
    shell_sums(S);
    /* scan q for a sign change of the residual with positive weights */
    __float128 lo = 0, hi = 0, rlo = 0, w[8], r;
    int found = 0, have_prev = 0;
    __float128 qprev = 0, rprev = 0;
    for (int i = 1; i <= 6000 && !found; ++i) {
        __float128 q = (__float128)i * 1e-3Q;
        if (!weights_for_q(S, q, w, &r) || !all_positive(w)) { have_prev = 0; continue; }
        if (have_prev && ((rprev < 0) != (r < 0))) { lo = qprev; hi = q; rlo = rprev; found = 1; }
        qprev = q; rprev = r; have_prev = 1;
    }
    if (!found) abort();
    for (int it = 0; it < 400; ++it) {
        __float128 mid = 0.5Q * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (!weights_for_q(S, mid, w, &r)) abort();
        if ((r < 0) == (rlo < 0)) { lo = mid; rlo = r; } else { hi = mid; }
    }
    Q_ROOT = 0.5Q * (lo + hi);
    weights_for_q(S, Q_ROOT, W_SHELL_Q, &r);
}

static void ensure_tables(void)
{
    if (tables_ready) return;
    build_velocity_set();
    solve_quadrature();
    C_SCALE = (double)sqrtq(Q_ROOT);
    for (int l = 0; l < Q; ++l) {
        int r2 = EX[l] * EX[l] + EY[l] * EY[l];
        for (int s = 0; s < 8; ++s)
            if (SHELL_R2[s] == r2) WL[l] = (double)W_SHELL_Q[s];
        XI_X[l] = C_SCALE * EX[l];
        XI_Y[l] = C_SCALE * EY[l];
    }
    tables_ready = 1;
}

void ref_velocity_table(int32_t ex[Q], int32_t ey[Q])
{
    ensure_tables();
    for (int l = 0; l < Q; ++l) { ex[l] = EX[l]; ey[l] = EY[l]; }
}

double ref_scale_c(void) { ensure_tables(); return C_SCALE; }

void ref_weights(double w[Q])
{
    ensure_tables();
    for (int l = 0; l < Q; ++l) w[l] = WL[l];
}

void ref_quadrature_residuals(double res[9])
{
    ensure_tables();
    for (int k = 0; k < 9; ++k) {
        __float128 acc = 0;
        for (int l = 0; l < Q; ++l) {
            int r2 = EX[l] * EX[l] + EY[l] * EY[l];
            __float128 ws = 0;
            for (int s = 0; s < 8; ++s) if (SHELL_R2[s] == r2) ws = W_SHELL_Q[s];
            __float128 xx = sqrtq(Q_ROOT) * EX[l], yy = sqrtq(Q_ROOT) * EY[l];
            __float128 t = ws;
            for (int p = 0; p < 2 * MOM_I[k]; ++p) t *= xx;
            for (int p = 0; p < 2 * MOM_J[k]; ++p) t *= yy;
            acc += t;
        }
        res[k] = (double)(acc - double_factorial_odd(MOM_I[k]) * double_factorial_odd(MOM_J[k]));
    }
}

/* ------------------------------------------------------------------------ */
/* Equilibrium (R3): 4th-order Hermite expansion, D = 2, expanded form.      */
/* With a = xi.u, u2 = |u|^2, x2 = |xi|^2, th = T - 1:                        */
/*  f = w rho { 1 + a + [a^2 - u2 + th (x2 - 2)]/2                            */
/*            + a [a^2 - 3 u2 + 3 th (x2 - 4)]/6                              */
/*            + [a^4 - 6 a^2 u2 + 3 u2^2 + 6 th (a^2 (x2 - 6) + u2 (4 - x2))   */
/*               + 3 th^2 (x2^2 - 8 x2 + 8)]/24 }                             */
/* ------------------------------------------------------------------------ */

void ref_feq(double rho, double ux, double uy, double T, double out[Q])
{
    ensure_tables();
    double u2 = ux * ux + uy * uy;
    double th = T - 1.0;
    for (int l = 0; l < Q; ++l) {
        double a = XI_X[l] * ux + XI_Y[l] * uy;
        double x2 = XI_X[l] * XI_X[l] + XI_Y[l] * XI_Y[l];
        double h1 = a;
        double h2 = (a * a - u2 + th * (x2 - 2.0)) / 2.0;
        double h3 = a * (a * a - 3.0 * u2 + 3.0 * th * (x2 - 4.0)) / 6.0;
        double h4 = (a * a * a * a - 6.0 * a * a * u2 + 3.0 * u2 * u2
                     + 6.0 * th * (a * a * (x2 - 6.0) + u2 * (4.0 - x2))
                     + 3.0 * th * th * (x2 * x2 - 8.0 * x2 + 8.0)) / 24.0;
        out[l] = WL[l] * rho * (1.0 + h1 + h2 + h3 + h4);
    }
}

/* ------------------------------------------------------------------------ */
/* Lattice                                                                   */
/* ------------------------------------------------------------------------ */

struct ref_lattice {
    int lx, ly;
    int xbc, ybc_bottom, ybc_top;
    double tau, g_y, t_bottom, t_top;
    double* cur;   /* current state           [Q][lx][ly] */
    double* prev;  /* state before the last propagate      */
    int have_prev;
};

#define AT(buf, L, l, x, y) ((buf)[((size_t)(l) * (L)->lx + (size_t)(x)) * (L)->ly + (size_t)(y)])

ref_lattice* ref_create(int32_t lx, int32_t ly, int32_t xbc, int32_t ybc_bottom,
                        int32_t ybc_top, double tau, double g_y,
                        double t_bottom, double t_top)
{
    ensure_tables();
    if (lx < 1 || ly < 1 || !(tau > 0.5)) return NULL;
    if (xbc != REF_PERIODIC && xbc != REF_OPEN) return NULL;
    if ((ybc_bottom == REF_PERIODIC) != (ybc_top == REF_PERIODIC)) return NULL;
    if (ybc_bottom < 0 || ybc_bottom > 2 || ybc_top < 0 || ybc_top > 2) return NULL;
    if ((ybc_bottom == REF_WALL || ybc_top == REF_WALL) && ly < 7) return NULL;
    ref_lattice* L = (ref_lattice*)calloc(1, sizeof(ref_lattice));
    if (!L) return NULL;
    L->lx = lx; L->ly = ly; L->xbc = xbc;
    L->ybc_bottom = ybc_bottom; L->ybc_top = ybc_top;
    L->tau = tau; L->g_y = g_y; L->t_bottom = t_bottom; L->t_top = t_top;
    size_t n = (size_t)Q * lx * ly;
    L->cur = (double*)calloc(n, sizeof(double));
    L->prev = (double*)calloc(n, sizeof(double));
    if (!L->cur || !L->prev) { ref_destroy(L); return NULL; }
    return L;
}

void ref_destroy(ref_lattice* L)
{
    if (!L) return;
    free(L->cur); free(L->prev); free(L);
}

int ref_init(ref_lattice* L, const double* rho, const double* ux,
             const double* uy, const double* T)
{
    double feq[Q];
    for (int x = 0; x < L->lx; ++x)
        for (int y = 0; y < L->ly; ++y) {
            size_t s = (size_t)x * L->ly + y;
            ref_feq(rho[s], ux[s], uy[s], T[s], feq);
            for (int l = 0; l < Q; ++l) AT(L->cur, L, l, x, y) = feq[l];
        }
    L->have_prev = 0;
    return 0;
}

int ref_set_pops(ref_lattice* L, const double* src)
{
    memcpy(L->cur, src, sizeof(double) * (size_t)Q * L->lx * L->ly);
    L->have_prev = 0;
    return 0;
}

int ref_get_pops(const ref_lattice* L, double* dst)
{
    memcpy(dst, L->cur, sizeof(double) * (size_t)Q * L->lx * L->ly);
    return 0;
}

/* Pull propagate, eq. (4): f_l(y) <- f_l(y - c_l dt).  A source outside the
 * lattice wraps on a periodic side; otherwise it reads as NaN (a wall's bc
 * overwrites exactly those slots). */
int ref_propagate(ref_lattice* L)
{
    double* nxt = L->prev;   /* reuse the older buffer as the destination */
    const double* src = L->cur;
    #pragma omp parallel for schedule(static)
    for (int x = 0; x < L->lx; ++x)
        for (int l = 0; l < Q; ++l)
            for (int y = 0; y < L->ly; ++y) {
                int xs = x - EX[l], ys = y - EY[l];
                int ok = 1;
                if (xs < 0 || xs >= L->lx) {
                    if (L->xbc == REF_PERIODIC) xs = ((xs % L->lx) + L->lx) % L->lx;
                    else ok = 0;
                }
                if (ys < 0 || ys >= L->ly) {
                    if (L->ybc_bottom == REF_PERIODIC) ys = ((ys % L->ly) + L->ly) % L->ly;
                    else ok = 0;
                }
                AT(nxt, L, l, x, y) = ok ? AT(src, L, l, xs, ys) : NAN;
            }
    L->prev = L->cur;
    L->cur = nxt;
    L->have_prev = 1;
    return 0;
}

static double prev_density(const ref_lattice* L, int x, int y)
{
    if (x < 0 || x >= L->lx) {
        if (L->xbc != REF_PERIODIC) return NAN;
        x = ((x % L->lx) + L->lx) % L->lx;
    }
    double rho = 0.0;
    for (int l = 0; l < Q; ++l) rho += AT(L->prev, L, l, x, y);
    return rho;
}

/* Wall rule (R5).  Applied after propagate; reads the pre-propagate state. */
int ref_bc(ref_lattice* L)
{
    if (L->ybc_bottom != REF_WALL && L->ybc_top != REF_WALL) return 0;
    if (!L->have_prev) return 1;
    double ew_bot[Q], ew_top[Q];
    ref_feq(1.0, 0.0, 0.0, L->t_bottom, ew_bot);
    ref_feq(1.0, 0.0, 0.0, L->t_top, ew_top);
    for (int x = 0; x < L->lx; ++x)
        for (int l = 0; l < Q; ++l)
            for (int k = 0; k < 3; ++k) {
                if (L->ybc_bottom == REF_WALL) {
                    int y = k, ys = y - EY[l];
                    if (ys < 0) {
                        int ym = -ys - 1;
                        AT(L->cur, L, l, x, y) = ew_bot[l] * prev_density(L, x - EX[l], ym);
                    }
                }
                if (L->ybc_top == REF_WALL) {
                    int y = L->ly - 1 - k, ys = y - EY[l];
                    if (ys >= L->ly) {
                        int ym = 2 * L->ly - 1 - ys;
                        AT(L->cur, L, l, x, y) = ew_top[l] * prev_density(L, x - EX[l], ym);
                    }
                }
            }
    return 0;
}

/* Moments of eq. (2) at one site: rho = sum f, rho u = sum xi f,
 * D rho T = sum |xi - u|^2 f. */
static void site_moments(const double f[Q], double* rho, double* ux, double* uy, double* T)
{
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int l = 0; l < Q; ++l) { r += f[l]; jx += XI_X[l] * f[l]; jy += XI_Y[l] * f[l]; }
    double vx = jx / r, vy = jy / r;
    double e = 0.0;
    for (int l = 0; l < Q; ++l) {
        double dx = XI_X[l] - vx, dy = XI_Y[l] - vy;
        e += (dx * dx + dy * dy) * f[l];
    }
    *rho = r; *ux = vx; *uy = vy; *T = e / (D * r);
}

/* BGK collision, eq. (1) with dt = 1: f <- f - (f - f^eq)/tau, with the
 * gravity shift (R4) of the equilibrium's velocity and temperature. */
int ref_collide(ref_lattice* L)
{
    const double tau = L->tau, g = L->g_y;
    #pragma omp parallel for schedule(static)
    for (int x = 0; x < L->lx; ++x) {
        double f[Q], feq[Q];
        for (int y = 0; y < L->ly; ++y) {
            for (int l = 0; l < Q; ++l) f[l] = AT(L->cur, L, l, x, y);
            double rho, ux, uy, T;
            site_moments(f, &rho, &ux, &uy, &T);
            double uys = uy + tau * g;
            double Ts = T + tau * (1.0 - tau) * g * g / D;
            ref_feq(rho, ux, uys, Ts, feq);
            for (int l = 0; l < Q; ++l)
                AT(L->cur, L, l, x, y) = f[l] - (f[l] - feq[l]) / tau;
        }
    }
    return 0;
}

int ref_step(ref_lattice* L, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        ref_propagate(L);
        ref_bc(L);
        ref_collide(L);
    }
    return 0;
}

int ref_get_macros(const ref_lattice* L, double* rho, double* ux, double* uy, double* T)
{
    #pragma omp parallel for schedule(static)
    for (int x = 0; x < L->lx; ++x) {
        double f[Q];
        for (int y = 0; y < L->ly; ++y) {
            for (int l = 0; l < Q; ++l) f[l] = AT(L->cur, L, l, x, y);
            size_t s = (size_t)x * L->ly + y;
            site_moments(f, &rho[s], &ux[s], &uy[s], &T[s]);
        }
    }
    return 0;
}

/* Lattice totals of the collision invariants: sum rho, sum j_x, sum j_y,
 * sum E with E = sum_l |xi_l|^2 f_l (eq. (2) summed over the lattice).
 * Serial, fixed order, accumulated in quad precision: a double accumulator
 * adding 10^5 values whose low-order bits all agree (FP32 deviations widened
 * onto the fixed FP64 weights) rounds the same way at every addition, and
 * its error grows like n ulp/2 (1e-8 of a 3000-site total), far above the
 * error of the sums it is meant to check. */
int ref_conservation(const ref_lattice* L, double out[4])
{
    __float128 a = 0, b = 0, c = 0, d = 0;
    for (int l = 0; l < Q; ++l) {
        double x2 = XI_X[l] * XI_X[l] + XI_Y[l] * XI_Y[l];
        for (int x = 0; x < L->lx; ++x)
            for (int y = 0; y < L->ly; ++y) {
                double v = AT(L->cur, L, l, x, y);
                a += v;
                b += (__float128)XI_X[l] * v;
                c += (__float128)XI_Y[l] * v;
                d += (__float128)x2 * v;
            }
    }
    out[0] = (double)a; out[1] = (double)b; out[2] = (double)c; out[3] = (double)d;
    return 0;
}

int ref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
