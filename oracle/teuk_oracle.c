/*
 * Teukolsky Lax-Wendroff ORACLE -- test infrastructure only.
 *
 * A plain, slow, deliberately unfused CPU implementation (IEEE binary64) of
 * the time evolution in Choudhary, Navada, Ginjupalli & Khanna, "An
 * exploration of OpenCL on multiple hardware platforms for a numerical
 * relativity application" (arXiv:1010.3816), Section 3:
 *   - the Teukolsky master equation, Eq. (1), Boyer-Lindquist coordinates,
 *     M = 1;
 *   - the azimuthal decomposition Psi = sum_m exp(i m phi) r^3 Phi_m (Sec. 3.2);
 *   - the first-order system in Phi and an auxiliary "momentum" Pi (Sec. 3.2);
 *   - the two-step Lax-Wendroff scheme, Eqs. (lw1) and (lw2), with angular
 *     derivatives by 2nd-order centred differences;
 *   - the angular boundary conditions (d_theta Phi = 0 at the poles for even
 *     |m|, Phi = 0 for odd |m|) and Phi = Pi = 0 on both radial boundaries.
 * The averaging step follows the printed kernel_average1 (Sec. 4): the value
 * between radial points i and i+1 is the arithmetic mean of the two.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no source, header, table or helper with
 * the GPU library; the two are compared on identical inputs.
 *
 * Where the paper is silent (definition of Pi, the matrices D and S, the
 * tortoise coordinate, grid placement, the argument of S in each stage,
 * extraction) the reading used is stated at the code that implements it.
 *
 * Parity pins (tests that tie this code to the paper and to mathematics
 * rather than to itself):
 *   coefficients      -> symbolic re-derivation from Eq. (1)
 *   tortoise          -> round trip and d(r*)/dr = (r^2+a^2)/Delta
 *   LW structure      -> exact d'Alembert translation at Courant 1, 2nd-order
 *                        convergence to the closed form otherwise
 *   theta stencil     -> exact discrete eigenmode, amplification 1+z+z^2/2
 *   Kerr operator     -> static solution of Eq. (1) for s = m = 0,
 *                        m <-> -m conjugate mirror symmetry,
 *                        Schwarzschild l = 2 ringdown frequency
 *   adjoint           -> dot-product identity, finite differences,
 *                        forward-mode tangent for d/da
 * The size of the a*m terms is pinned only by the symbolic derivation.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Real coefficients of the first-order system, in this order. */
enum { K_B, K_CRE, K_CIM, K_CTRE, K_CTIM, K_A2, K_A1, K_V0RE, K_V0IM, NCOEF };

/* Complex-step size for d/da (Squire & Trapp 1998): f(a + i h) = f(a) + i h f'(a) + O(h^2). */
#define CSTEP 1e-20

/* ------------------------------------------------------------------------ */
/* Kerr geometry, M = 1.  All routines take a complexified spin so that the  */
/* same code yields the value (real part) and, by the complex step, d/da.     */
/* ------------------------------------------------------------------------ */

static cplx r_plus(cplx a) { return 1.0 + csqrt(1.0 - a * a); }
static cplx r_minus(cplx a) { return 1.0 - csqrt(1.0 - a * a); }

/* Tortoise coordinate as a function of x = r - r_+ (reading: the standard
 * Kerr form with integration constants ln((r - r_pm)/2M); the paper only
 * uses r* through its grid spacing delta r*):
 *   r* = r + 2 r+/(r+ - r-) ln((r - r+)/2) - 2 r-/(r+ - r-) ln((r - r-)/2).
 * It satisfies d(r*)/dr = (r^2 + a^2)/Delta. */
static cplx rstar_of_x(cplx a, cplx x)
{
    cplx rp = r_plus(a), rm = r_minus(a), d = rp - rm;
    return rp + x + (2.0 * rp / d) * clog(x / 2.0) - (2.0 * rm / d) * clog((x + d) / 2.0);
}

/* d(r*)/d(ln x) = x (r^2 + a^2) / Delta with Delta = x (x + r+ - r-). */
static cplx drstar_dlnx(cplx a, cplx x)
{
    cplx rp = r_plus(a), rm = r_minus(a);
    cplx r = rp + x;
    return (r * r + a * a) / (x + rp - rm);
}

/* Solve r*(x) = target for x = r - r_+ > 0.  The unknown is y = ln x, so that
 * points a few hundred M inside (x ~ 1e-19) are resolved.  Bracketed Newton
 * on the real problem, then three complex Newton steps to carry the complex
 * step of a into x.  Returns 0 on success. */
static int solve_x(cplx a, double target, cplx* x_out)
{
    double ar = creal(a);
    double ylo = -60.0, yhi = 8.0;
    while (creal(rstar_of_x(ar, exp(ylo))) > target) { ylo *= 2.0; if (ylo < -4000.0) return -1; }
    while (creal(rstar_of_x(ar, exp(yhi))) < target) { yhi += 8.0; if (yhi > 80.0) return -1; }
    double y = 0.5 * (ylo + yhi);
    for (int it = 0; it < 400; ++it) {
        double x = exp(y);
        double f = creal(rstar_of_x(ar, x)) - target;
        if (f > 0) yhi = y; else ylo = y;
        double ynew = y - f / creal(drstar_dlnx(ar, x));
        if (!(ynew > ylo && ynew < yhi)) ynew = 0.5 * (ylo + yhi);
        if (fabs(ynew - y) <= 4.0 * 2.220446049250313e-16 * fmax(1.0, fabs(y))) { y = ynew; break; }
        y = ynew;
        if (yhi - ylo <= 2.220446049250313e-16 * fmax(1.0, fabs(y))) break;
    }
    /* Polish in x itself: a representable y = ln x only fixes x to about
     * |y| ulp relative, which is too coarse far from the horizon. */
    double xr = exp(y);
    double fr = fabs(creal(rstar_of_x(ar, xr)) - target);
    for (int it = 0; it < 4; ++it) {
        double f = creal(rstar_of_x(ar, xr)) - target;
        double xn = xr - f * xr / creal(drstar_dlnx(ar, xr));
        double fn = fabs(creal(rstar_of_x(ar, xn)) - target);
        if (!(xn > 0.0) || !(fn < fr)) break;
        xr = xn;
        fr = fn;
    }
    cplx yc = log(xr);
    for (int it = 0; it < 3; ++it) {
        cplx xc = cexp(yc);
        yc = yc - (rstar_of_x(a, xc) - target) / drstar_dlnx(a, xc);
    }
    /* keep the converged real part; take only the complex-step part from the complex refinement */
    *x_out = xr * cexp(I * cimag(yc));
    return 0;
}

/* The nine real coefficients of the first-order system at (r = r_+ + x, theta).
 *
 * Derivation (reading of the auxiliary field and of D and S, which the paper
 * defers to its reference for the scheme): substitute
 * Psi = exp(i m phi) r^3 Phi into Eq. (1), use d/dr = (rho/Delta) d/dr*
 * (rho = r^2 + a^2) and multiply by -Delta / (Sigma^2 r^3), where
 * Sigma^2 = rho^2 - a^2 Delta sin^2(theta).  This gives
 *   Phi_tt - b^2 Phi'' - B1 Phi' + Ct Phi_t - A2 Phi_thth - A1 Phi_th + V0 Phi = 0
 * (' = d/dr*) with b = rho/Sigma and
 *   Ct = [2s(r Delta - (r^2 - a^2)) + i(4 a m r + 2 s a Delta cos th)] / Sigma^2
 *   B1 = (rho/Sigma^2) [6 Delta/r + 2 s (r - 1) + 2 r Delta/rho]
 *   A2 = Delta/Sigma^2,  A1 = (Delta/Sigma^2) cot th
 *   V0 = (Delta/Sigma^2)[(m + s cos th)^2/sin^2 th - s]
 *        - [m^2 a^2 + 2 i s m a (r - 1)]/Sigma^2
 *        - 6 Delta [(s+2) r^2 - (s+3) r + a^2] / (r^2 Sigma^2).
 * With Pi = Phi_t + b Phi' the system is
 *   d_t Phi + b Phi'          = Pi
 *   d_t Pi  - b Pi' + c Phi'  = -Ct Pi + A2 Phi_thth + A1 Phi_th - V0 Phi
 * with c = b b' - b Ct - B1, i.e. d_t u + D d_r* u = S with
 * D = [[b, 0], [c, -b]] acting on the complex pair (Phi, Pi).
 * Delta is formed as x (x + r+ - r-) so that it keeps its relative precision
 * close to the horizon. */
static void coefficients_cs(cplx a, int s, int m, cplx x, double th, cplx out[NCOEF])
{
    cplx rp = r_plus(a), rm = r_minus(a);
    cplx r = rp + x;
    cplx Delta = x * (x + rp - rm);
    cplx rho = r * r + a * a;
    double sn = sin(th), cs = cos(th);
    cplx Sig2 = rho * rho - a * a * Delta * sn * sn;
    cplx Sig = csqrt(Sig2);
    cplx b = rho / Sig;
    cplx dSig2_dr = 4.0 * r * rho - 2.0 * a * a * (r - 1.0) * sn * sn;
    cplx db_dr = 2.0 * r / Sig - rho * dSig2_dr / (2.0 * Sig * Sig2);
    cplx bprime = (Delta / rho) * db_dr;
    cplx Ct_re = 2.0 * s * (r * Delta - (r * r - a * a)) / Sig2;
    cplx Ct_im = (4.0 * a * m * r + 2.0 * s * a * Delta * cs) / Sig2;
    cplx B1 = (rho / Sig2) * (6.0 * Delta / r + 2.0 * s * (r - 1.0) + 2.0 * r * Delta / rho);
    cplx A2 = Delta / Sig2;
    cplx A1 = (Delta / Sig2) * (cs / sn);
    cplx mc = m + s * cs;
    cplx V0_re = (Delta / Sig2) * (mc * mc / (sn * sn) - s) - (double)(m * m) * a * a / Sig2
               - 6.0 * Delta * ((s + 2.0) * r * r - (s + 3.0) * r + a * a) / (r * r * Sig2);
    cplx V0_im = -2.0 * s * m * a * (r - 1.0) / Sig2;
    out[K_B] = b;
    out[K_CRE] = b * bprime - b * Ct_re - B1;
    out[K_CIM] = -b * Ct_im;
    out[K_CTRE] = Ct_re;
    out[K_CTIM] = Ct_im;
    out[K_A2] = A2;
    out[K_A1] = A1;
    out[K_V0RE] = V0_re;
    out[K_V0IM] = V0_im;
}

/* ------------------------------------------------------------------------ */
/* Grid                                                                       */
/* ------------------------------------------------------------------------ */

/* Grid reading: r*_i = rmin + i dr (i = 0..nr-1, both ends on the grid,
 * dr = (rmax - rmin)/(nr - 1)); the value "between grid points" of Eq. (lw1)
 * sits at r*_{i+1/2} = rmin + (i + 1/2) dr, i = 0..nr-2.  theta is
 * cell-centred: theta_j = (j + 1/2) dth, dth = pi/nth, so the poles are not
 * grid points.  Storage is [theta][r*] with r* fastest, as in the paper's
 * idx(b, a) = N b + a. */
typedef struct {
    double a;
    int s, m, nr, nth;
    double rmin, rmax, dt, dr, dth;
    int sigma;      /* ghost-row parity: +1 for even |m|, -1 for odd |m| */
    int kerr;       /* 1: coefficients from Eq. (1); 0: caller-supplied tables */
    double* ci;     /* [NCOEF][nth][nr]   coefficients at r*_i            */
    double* ch;     /* [NCOEF][nth][nr-1] coefficients at r*_{i+1/2}      */
    double* dci;    /* d/da of ci (Kerr mode)                             */
    double* dch;    /* d/da of ch (Kerr mode)                             */
    double* xi;     /* r - r_+ at r*_i      */
    double* xh;     /* r - r_+ at r*_{i+1/2} */
} orc_grid;

static size_t tab_i(const orc_grid* g, int c, int j, int i) { return ((size_t)c * g->nth + j) * g->nr + i; }
static size_t tab_h(const orc_grid* g, int c, int j, int i) { return ((size_t)c * g->nth + j) * (g->nr - 1) + i; }

void orc_destroy(orc_grid* g)
{
    if (!g) return;
    free(g->ci); free(g->ch); free(g->dci); free(g->dch); free(g->xi); free(g->xh);
    free(g);
}

/* Create a grid.  kerr = 1 fills the coefficient tables (and their d/da) from
 * Eq. (1); kerr = 0 leaves them zero for orc_set_coefficients.  Returns NULL
 * on invalid arguments or on a failed tortoise inversion. */
orc_grid* orc_create(double a, int s, int m, int nr, int nth, double rmin, double rmax, double dt, int kerr)
{
    if (nr < 3 || nth < 2 || !(rmax > rmin) || !(a >= 0.0 && a < 1.0)) return NULL;
    orc_grid* g = (orc_grid*)calloc(1, sizeof(orc_grid));
    g->a = a; g->s = s; g->m = m; g->nr = nr; g->nth = nth;
    g->rmin = rmin; g->rmax = rmax; g->dt = dt;
    g->dr = (rmax - rmin) / (nr - 1);
    g->dth = M_PI / nth;
    g->sigma = (abs(m) % 2 == 0) ? 1 : -1;
    g->kerr = kerr;
    size_t ni = (size_t)NCOEF * nth * nr, nh = (size_t)NCOEF * nth * (nr - 1);
    g->ci = (double*)calloc(ni, sizeof(double));
    g->ch = (double*)calloc(nh, sizeof(double));
    g->dci = (double*)calloc(ni, sizeof(double));
    g->dch = (double*)calloc(nh, sizeof(double));
    g->xi = (double*)calloc(nr, sizeof(double));
    g->xh = (double*)calloc(nr - 1, sizeof(double));
    if (!kerr) return g;

    cplx acs = a + I * CSTEP;
    cplx* xci = (cplx*)malloc(sizeof(cplx) * nr);
    cplx* xch = (cplx*)malloc(sizeof(cplx) * (nr - 1));
    int bad = 0;
    for (int i = 0; i < nr; ++i) {
        bad |= solve_x(acs, rmin + i * g->dr, &xci[i]);
        g->xi[i] = creal(xci[i]);
    }
    for (int i = 0; i < nr - 1; ++i) {
        bad |= solve_x(acs, rmin + (i + 0.5) * g->dr, &xch[i]);
        g->xh[i] = creal(xch[i]);
    }
    if (bad) { free(xci); free(xch); orc_destroy(g); return NULL; }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nth; ++j) {
        double th = (j + 0.5) * g->dth;
        cplx out[NCOEF];
        for (int i = 0; i < nr; ++i) {
            coefficients_cs(acs, s, m, xci[i], th, out);
            for (int c = 0; c < NCOEF; ++c) {
                g->ci[tab_i(g, c, j, i)] = creal(out[c]);
                g->dci[tab_i(g, c, j, i)] = cimag(out[c]) / CSTEP;
            }
        }
        for (int i = 0; i < nr - 1; ++i) {
            coefficients_cs(acs, s, m, xch[i], th, out);
            for (int c = 0; c < NCOEF; ++c) {
                g->ch[tab_h(g, c, j, i)] = creal(out[c]);
                g->dch[tab_h(g, c, j, i)] = cimag(out[c]) / CSTEP;
            }
        }
    }
    free(xci); free(xch);
    return g;
}

/* Caller-supplied coefficient tables (layouts as ci and ch above). */
void orc_set_coefficients(orc_grid* g, const double* ci, const double* ch)
{
    memcpy(g->ci, ci, sizeof(double) * NCOEF * g->nth * g->nr);
    memcpy(g->ch, ch, sizeof(double) * NCOEF * g->nth * (g->nr - 1));
}

void orc_get_coefficients(const orc_grid* g, double* ci, double* ch, double* dci, double* dch)
{
    size_t ni = (size_t)NCOEF * g->nth * g->nr, nh = (size_t)NCOEF * g->nth * (g->nr - 1);
    if (ci) memcpy(ci, g->ci, sizeof(double) * ni);
    if (ch) memcpy(ch, g->ch, sizeof(double) * nh);
    if (dci) memcpy(dci, g->dci, sizeof(double) * ni);
    if (dch) memcpy(dch, g->dch, sizeof(double) * nh);
}

void orc_get_x(const orc_grid* g, double* xi, double* xh)
{
    memcpy(xi, g->xi, sizeof(double) * g->nr);
    memcpy(xh, g->xh, sizeof(double) * (g->nr - 1));
}

double orc_dr(const orc_grid* g) { return g->dr; }
double orc_dth(const orc_grid* g) { return g->dth; }
void orc_set_dt(orc_grid* g, double dt) { g->dt = dt; }

/* Point-wise access for tests: tortoise inversion and coefficients. */
int orc_tortoise_x(double a, double rstar, double* x)
{
    cplx xc;
    int rc = solve_x(a, rstar, &xc);
    *x = creal(xc);
    return rc;
}

double orc_rstar_of_x(double a, double x) { return creal(rstar_of_x(a, x)); }

/* value[9] and d/da[9] at (r*, theta); returns the tortoise status. */
int orc_coefficients(double a, int s, int m, double rstar, double th, double* val, double* dval)
{
    cplx acs = a + I * CSTEP, x, out[NCOEF];
    int rc = solve_x(acs, rstar, &x);
    if (rc) return rc;
    coefficients_cs(acs, s, m, x, th, out);
    for (int c = 0; c < NCOEF; ++c) {
        val[c] = creal(out[c]);
        if (dval) dval[c] = cimag(out[c]) / CSTEP;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The Lax-Wendroff step                                                      */
/* ------------------------------------------------------------------------ */

/* S applied to a field pair (fP, fQ) laid out [nth][ncol] with coefficient
 * table `coef` of the same shape:
 *   S_Phi = fQ
 *   S_Pi  = -Ct fQ + A2 (f_{j+1} - 2 f_j + f_{j-1})/dth^2
 *                  + A1 (f_{j+1} - f_{j-1})/(2 dth) - V0 f_j,  f = fP,
 * i.e. 2nd-order centred angular differences.  The angular boundary
 * condition enters through ghost rows f_{-1} = sigma f_0 and
 * f_{nth} = sigma f_{nth-1}: a mirror (zero derivative at the pole) for even
 * |m| and an anti-mirror (zero value at the pole) for odd |m|.  Only Phi is
 * differentiated in theta, so only Phi needs ghosts. */
static void apply_S(const orc_grid* g, const double* coef, int ncol,
                    const cplx* fP, const cplx* fQ, cplx* oP, cplx* oQ)
{
    const int nth = g->nth;
    const double dth = g->dth, sg = g->sigma;
    const size_t plane = (size_t)nth * ncol;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nth; ++j) {
        for (int i = 0; i < ncol; ++i) {
            size_t k = (size_t)j * ncol + i;
            cplx f0 = fP[k];
            cplx fm = (j > 0) ? fP[k - ncol] : sg * f0;
            cplx fp = (j < nth - 1) ? fP[k + ncol] : sg * f0;
            cplx Ct = coef[K_CTRE * plane + k] + I * coef[K_CTIM * plane + k];
            cplx V0 = coef[K_V0RE * plane + k] + I * coef[K_V0IM * plane + k];
            double A2 = coef[K_A2 * plane + k], A1 = coef[K_A1 * plane + k];
            oP[k] = fQ[k];
            oQ[k] = -Ct * fQ[k] + A2 * (fp - 2.0 * f0 + fm) / (dth * dth)
                  + A1 * (fp - fm) / (2.0 * dth) - V0 * f0;
        }
    }
}

/* Working arrays of one step. */
typedef struct {
    cplx *ubP, *ubQ, *dP, *dQ, *sP, *sQ, *hP, *hQ;   /* half points [nth][nr-1] */
    cplx *hbP, *hbQ, *dhP, *dhQ, *tP, *tQ;           /* integer points [nth][nr] */
} work;

static void work_alloc(const orc_grid* g, work* w)
{
    size_t nh = (size_t)g->nth * (g->nr - 1), ni = (size_t)g->nth * g->nr;
    cplx** half[] = {&w->ubP, &w->ubQ, &w->dP, &w->dQ, &w->sP, &w->sQ, &w->hP, &w->hQ};
    cplx** full[] = {&w->hbP, &w->hbQ, &w->dhP, &w->dhQ, &w->tP, &w->tQ};
    for (int k = 0; k < 8; ++k) *half[k] = (cplx*)calloc(nh, sizeof(cplx));
    for (int k = 0; k < 6; ++k) *full[k] = (cplx*)calloc(ni, sizeof(cplx));
}

static void work_free(work* w)
{
    cplx* all[] = {w->ubP, w->ubQ, w->dP, w->dQ, w->sP, w->sQ, w->hP, w->hQ,
                   w->hbP, w->hbQ, w->dhP, w->dhQ, w->tP, w->tQ};
    for (int k = 0; k < 14; ++k) free(all[k]);
}

/* Stage 1, Eq. (lw1): for i = 0..nr-2 and every j
 *   ubar  = (u_{i+1} + u_i)/2                 (kernel_average1)
 *   delta = u_{i+1} - u_i
 *   h_{i+1/2} = ubar - (dt/2) [ D_{i+1/2} delta / dr - S_{i+1/2}(ubar) ].
 * Reading: D and S are evaluated with the coefficients at r*_{i+1/2} itself,
 * and S acts on the averaged state (average first, then the right-hand
 * side, as the printed kernel order implies). */
static void stage1(const orc_grid* g, const cplx* phi, const cplx* pi, work* w)
{
    const int nr = g->nr, nth = g->nth, nh = nr - 1;
    const size_t plane = (size_t)nth * nh;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nth; ++j)
        for (int i = 0; i < nh; ++i) {
            size_t k = (size_t)j * nh + i, u = (size_t)j * nr + i;
            w->ubP[k] = 0.5 * (phi[u + 1] + phi[u]);
            w->ubQ[k] = 0.5 * (pi[u + 1] + pi[u]);
            w->dP[k] = phi[u + 1] - phi[u];
            w->dQ[k] = pi[u + 1] - pi[u];
        }
    apply_S(g, g->ch, nh, w->ubP, w->ubQ, w->sP, w->sQ);
    const double dt = g->dt, dr = g->dr;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nth; ++j)
        for (int i = 0; i < nh; ++i) {
            size_t k = (size_t)j * nh + i;
            double b = g->ch[K_B * plane + k];
            cplx c = g->ch[K_CRE * plane + k] + I * g->ch[K_CIM * plane + k];
            cplx DP = b * w->dP[k] / dr;
            cplx DQ = (c * w->dP[k] - b * w->dQ[k]) / dr;
            w->hP[k] = w->ubP[k] - 0.5 * dt * (DP - w->sP[k]);
            w->hQ[k] = w->ubQ[k] - 0.5 * dt * (DQ - w->sQ[k]);
        }
}

/* Stage 2, Eq. (lw2): for i = 1..nr-2
 *   u^{n+1}_i = u_i - dt [ D_i (h_{i+1/2} - h_{i-1/2}) / dr - S_i(hbar_i) ],
 *   hbar_i = (h_{i+1/2} + h_{i-1/2})/2.
 * Reading: the half-time state at the integer point, needed by S_i, is the
 * average of the two neighbouring stage-1 values (a second averaging pass).
 * Radial boundary condition: Phi = Pi = 0 at i = 0 and i = nr-1. */
static void stage2(const orc_grid* g, cplx* phi, cplx* pi, work* w)
{
    const int nr = g->nr, nth = g->nth, nh = nr - 1;
    const size_t plane = (size_t)nth * nr;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nth; ++j)
        for (int i = 0; i < nr; ++i) {
            size_t u = (size_t)j * nr + i;
            if (i == 0 || i == nr - 1) {
                w->hbP[u] = w->hbQ[u] = w->dhP[u] = w->dhQ[u] = 0.0;
                continue;
            }
            size_t kr = (size_t)j * nh + i, kl = kr - 1;   /* halves i+1/2 and i-1/2 */
            w->hbP[u] = 0.5 * (w->hP[kr] + w->hP[kl]);
            w->hbQ[u] = 0.5 * (w->hQ[kr] + w->hQ[kl]);
            w->dhP[u] = w->hP[kr] - w->hP[kl];
            w->dhQ[u] = w->hQ[kr] - w->hQ[kl];
        }
    apply_S(g, g->ci, nr, w->hbP, w->hbQ, w->tP, w->tQ);
    const double dt = g->dt, dr = g->dr;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nth; ++j)
        for (int i = 0; i < nr; ++i) {
            size_t u = (size_t)j * nr + i;
            if (i == 0 || i == nr - 1) { phi[u] = 0.0; pi[u] = 0.0; continue; }
            double b = g->ci[K_B * plane + u];
            cplx c = g->ci[K_CRE * plane + u] + I * g->ci[K_CIM * plane + u];
            cplx DP = b * w->dhP[u] / dr;
            cplx DQ = (c * w->dhP[u] - b * w->dhQ[u]) / dr;
            phi[u] = phi[u] - dt * (DP - w->tP[u]);
            pi[u] = pi[u] - dt * (DQ - w->tQ[u]);
        }
}

/* Radial boundary condition applied to initial data: Phi = Pi = 0 at i = 0
 * and i = nr-1. */
void orc_project(const orc_grid* g, cplx* phi, cplx* pi)
{
    for (int j = 0; j < g->nth; ++j) {
        size_t r0 = (size_t)j * g->nr;
        phi[r0] = pi[r0] = 0.0;
        phi[r0 + g->nr - 1] = pi[r0 + g->nr - 1] = 0.0;
    }
}

/* Bilinear interpolation of Phi at (r*, theta) between the bracketing
 * integer columns and cell-centre rows; outside the first/last row centre
 * the ghost row (sigma times the mirrored row) is used.  Reading of the
 * paper's waveform extraction, which it does not spell out. */
static cplx extract(const orc_grid* g, const cplx* phi, double rs, double th)
{
    double p = (rs - g->rmin) / g->dr;
    int i0 = (int)floor(p);
    if (i0 < 0) i0 = 0;
    if (i0 > g->nr - 2) i0 = g->nr - 2;
    double wr = p - i0;
    double q = th / g->dth - 0.5;
    int j0 = (int)floor(q);
    if (j0 < -1) j0 = -1;
    if (j0 > g->nth - 1) j0 = g->nth - 1;
    double wt = q - j0;
    cplx row[2];
    for (int t = 0; t < 2; ++t) {
        int j = j0 + t;
        double sgn = 1.0;
        if (j < 0) { j = 0; sgn = g->sigma; }
        if (j > g->nth - 1) { j = g->nth - 1; sgn = g->sigma; }
        size_t u = (size_t)j * g->nr + i0;
        row[t] = sgn * ((1.0 - wr) * phi[u] + wr * phi[u + 1]);
    }
    return (1.0 - wt) * row[0] + wt * row[1];
}

void orc_extract(const orc_grid* g, const cplx* phi, double rs, double th, cplx* out)
{
    *out = extract(g, phi, rs, th);
}

/* One full Lax-Wendroff step in place. */
void orc_step(const orc_grid* g, cplx* phi, cplx* pi)
{
    work w;
    work_alloc(g, &w);
    stage1(g, phi, pi, &w);
    stage2(g, phi, pi, &w);
    work_free(&w);
}

/* n steps; after step k (k = 1..n) the n_ext extraction samples of Phi are
 * written to series[(k-1) n_ext + e]. series may be NULL. */
void orc_evolve(const orc_grid* g, cplx* phi, cplx* pi, int64_t n, int n_ext,
                const double* ext_r, const double* ext_th, cplx* series)
{
    work w;
    work_alloc(g, &w);
    for (int64_t k = 0; k < n; ++k) {
        stage1(g, phi, pi, &w);
        stage2(g, phi, pi, &w);
        if (series)
            for (int e = 0; e < n_ext; ++e)
                series[k * n_ext + e] = extract(g, phi, ext_r[e], ext_th[e]);
    }
    work_free(&w);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
