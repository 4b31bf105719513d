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
 *   mode sum          -> discrete Fourier transform over equally spaced
 *                        azimuths recovers r^3 Phi_m (numpy's FFT); a
 *                        single m = 0 mode gives r^3 with r from the
 *                        closed-form tortoise coordinate
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
    cplx* gsi;      /* source profile g at r*_i      [nth][nr]   (NULL: none) */
    cplx* gsh;      /* source profile g at r*_{i+1/2} [nth][nr-1] (NULL: none) */
} orc_grid;

static size_t tab_i(const orc_grid* g, int c, int j, int i) { return ((size_t)c * g->nth + j) * g->nr + i; }
static size_t tab_h(const orc_grid* g, int c, int j, int i) { return ((size_t)c * g->nth + j) * (g->nr - 1) + i; }

void orc_destroy(orc_grid* g)
{
    if (!g) return;
    free(g->ci); free(g->ch); free(g->dci); free(g->dch); free(g->xi); free(g->xh);
    free(g->gsi); free(g->gsh);
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

/* The field at observers from its azimuthal modes (Sec. 3.2): the solution
 * is Psi = sum over m of exp(i m phi) r^3 Phi_m, so for sample k and observer
 * o, at Boyer-Lindquist radius r_o = r_+ + x(r*_o) and azimuth phi_o,
 *   psi[k][o] = sum_j exp(i m_j phi_o) r_o^3 samples[k][j][o].
 * samples: [n_samples][n_modes][n_obs], psi: [n_samples][n_obs].  Returns
 * nonzero if a tortoise inversion fails. */
int orc_mode_sum(double a, int64_t n_samples, int n_modes, const int* m, int n_obs, const double* rstar,
                 const double* phi, const cplx* samples, cplx* psi)
{
    for (int o = 0; o < n_obs; ++o) {
        cplx x;
        if (solve_x(a, rstar[o], &x)) return 1;
        double r = creal(r_plus(a) + x);
        for (int64_t k = 0; k < n_samples; ++k) {
            cplx sum = 0.0;
            for (int j = 0; j < n_modes; ++j)
                sum += cexp(I * (double)m[j] * phi[o]) * (r * r * r) * samples[((size_t)k * n_modes + j) * n_obs + o];
            psi[(size_t)k * n_obs + o] = sum;
        }
    }
    return 0;
}

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
static void stage1(const orc_grid* g, const cplx* phi, const cplx* pi, work* w, const cplx* J)
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
    if (J)  /* inhomogeneous variant: the source is part of S's Pi row */
        for (size_t k = 0; k < (size_t)nth * nh; ++k) w->sQ[k] += J[k];
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
static void stage2(const orc_grid* g, cplx* phi, cplx* pi, work* w, const cplx* J)
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
    if (J)
        for (size_t u = 0; u < (size_t)nth * nr; ++u) w->tQ[u] += J[u];
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
    stage1(g, phi, pi, &w, NULL);
    stage2(g, phi, pi, &w, NULL);
    work_free(&w);
}

/* Inhomogeneous variant (a source term J in the Pi equation, as the
 * particle-driven form of Eq. (1) has; the paper does not give the source
 * model, so J(t, r*, theta) = f(t) g(r*, theta) is supplied by the caller).
 * Reading: J is part of S's Pi row and is evaluated where and when S is in
 * each stage: at (t_n, r*_{i+1/2}) in Eq. (lw1) and at (t_n + dt/2, r*_i) in
 * Eq. (lw2).  g is given at both positions: gi [nth][nr], gh [nth][nr-1]
 * (NULL pointers remove the source). */
void orc_set_source(orc_grid* g, const cplx* gi, const cplx* gh)
{
    free(g->gsi);
    free(g->gsh);
    g->gsi = g->gsh = NULL;
    if (!gi || !gh) return;
    size_t ni = (size_t)g->nth * g->nr, nh = (size_t)g->nth * (g->nr - 1);
    g->gsi = malloc(ni * sizeof(cplx));
    g->gsh = malloc(nh * sizeof(cplx));
    memcpy(g->gsi, gi, ni * sizeof(cplx));
    memcpy(g->gsh, gh, nh * sizeof(cplx));
}

/* n steps of the inhomogeneous variant: f[2k] = f(t_k) and f[2k+1] =
 * f(t_k + dt/2) for step k of the call (t_k its start).  Samples as
 * orc_evolve. */
void orc_evolve_source(const orc_grid* g, cplx* phi, cplx* pi, int64_t n, const cplx* f, int n_ext,
                       const double* ext_r, const double* ext_th, cplx* series)
{
    size_t ni = (size_t)g->nth * g->nr, nh = (size_t)g->nth * (g->nr - 1);
    cplx* J1 = malloc(nh * sizeof(cplx));
    cplx* J2 = malloc(ni * sizeof(cplx));
    work w;
    work_alloc(g, &w);
    for (int64_t k = 0; k < n; ++k) {
        for (size_t u = 0; u < nh; ++u) J1[u] = g->gsh ? f[2 * k] * g->gsh[u] : 0.0;
        for (size_t u = 0; u < ni; ++u) J2[u] = g->gsi ? f[2 * k + 1] * g->gsi[u] : 0.0;
        stage1(g, phi, pi, &w, J1);
        stage2(g, phi, pi, &w, J2);
        if (series)
            for (int e = 0; e < n_ext; ++e)
                series[k * n_ext + e] = extract(g, phi, ext_r[e], ext_th[e]);
    }
    work_free(&w);
    free(J1);
    free(J2);
}

/* n steps; after step k (k = 1..n) the n_ext extraction samples of Phi are
 * written to series[(k-1) n_ext + e]. series may be NULL. */
void orc_evolve(const orc_grid* g, cplx* phi, cplx* pi, int64_t n, int n_ext,
                const double* ext_r, const double* ext_th, cplx* series)
{
    work w;
    work_alloc(g, &w);
    for (int64_t k = 0; k < n; ++k) {
        stage1(g, phi, pi, &w, NULL);
        stage2(g, phi, pi, &w, NULL);
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

/* Threads used by later calls (timing only; results do not depend on it:
   every output point is written by one thread). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Adjoint (conjugate transpose) of the step and its spin derivative          */
/* ------------------------------------------------------------------------ */
/* The step u -> u' is complex-linear in u.  For a real loss L and the
 * gradient convention dL/dRe + i dL/dIm, the cotangent of u is A^H applied
 * to the cotangent of u'.  Each sub-operation of the step is transposed
 * separately below, in scatter form (every forward read becomes an
 * accumulation into the location that was read), in the reverse order of
 * the forward step. */

/* Transpose of apply_S: (oP, oQ) is the cotangent of S's output; the
 * cotangent of its input is ADDED to (fP, fQ).  The theta stencil scatters
 * into rows j-1, j, j+1; a contribution to a ghost row lands on the row it
 * mirrors, times sigma. */
static void apply_S_adj(const orc_grid* g, const double* coef, int ncol,
                        const cplx* oP, const cplx* oQ, cplx* fP, cplx* fQ)
{
    const int nth = g->nth;
    const double dth = g->dth, sg = g->sigma;
    const size_t plane = (size_t)nth * ncol;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < ncol; ++i) {          /* columns are independent */
        for (int j = 0; j < nth; ++j) {
            size_t k = (size_t)j * ncol + i;
            cplx Ct = coef[K_CTRE * plane + k] + I * coef[K_CTIM * plane + k];
            cplx V0 = coef[K_V0RE * plane + k] + I * coef[K_V0IM * plane + k];
            double A2 = coef[K_A2 * plane + k] / (dth * dth), A1 = coef[K_A1 * plane + k] / (2.0 * dth);
            cplx w = oQ[k];
            fQ[k] += oP[k] + conj(-Ct) * w;
            fP[k] += (-2.0 * A2 - conj(V0)) * w;
            /* f_{j+1} with weight A2 + A1, f_{j-1} with weight A2 - A1 */
            if (j < nth - 1) fP[k + ncol] += (A2 + A1) * w; else fP[k] += sg * (A2 + A1) * w;
            if (j > 0) fP[k - ncol] += (A2 - A1) * w; else fP[k] += sg * (A2 - A1) * w;
        }
    }
}

/* In place: (lp, lq) = cotangent of u^{n+1}  ->  cotangent of u^n. */
void orc_adjoint_step(const orc_grid* g, cplx* lp, cplx* lq)
{
    const int nr = g->nr, nth = g->nth, nh = nr - 1;
    const size_t ni = (size_t)nth * nr, nhs = (size_t)nth * nh;
    const size_t pi_ = ni, ph = nhs;
    const double dt = g->dt, dr = g->dr, hdt = 0.5 * g->dt;
    cplx *nuP = calloc(ni, sizeof(cplx)), *nuQ = calloc(ni, sizeof(cplx));
    cplx *sP = calloc(ni, sizeof(cplx)), *sQ = calloc(ni, sizeof(cplx));
    cplx *hbP = calloc(ni, sizeof(cplx)), *hbQ = calloc(ni, sizeof(cplx));
    cplx *dhP = calloc(ni, sizeof(cplx)), *dhQ = calloc(ni, sizeof(cplx));
    cplx *hP = calloc(nhs, sizeof(cplx)), *hQ = calloc(nhs, sizeof(cplx));
    cplx *s1P = calloc(nhs, sizeof(cplx)), *s1Q = calloc(nhs, sizeof(cplx));
    cplx *ubP = calloc(nhs, sizeof(cplx)), *ubQ = calloc(nhs, sizeof(cplx));
    cplx *dP = calloc(nhs, sizeof(cplx)), *dQ = calloc(nhs, sizeof(cplx));

    /* radial boundary condition of the output: those entries are constants */
    for (int j = 0; j < nth; ++j)
        for (int i = 1; i < nr - 1; ++i) {
            size_t u = (size_t)j * nr + i;
            nuP[u] = lp[u];
            nuQ[u] = lq[u];
        }
    /* stage 2: Phi' = Phi - dt [ b dhP/dr - S_P ],  Pi' = Pi - dt [ (c dhP - b dhQ)/dr - S_Q ] */
    for (int j = 0; j < nth; ++j)
        for (int i = 1; i < nr - 1; ++i) {
            size_t u = (size_t)j * nr + i;
            double b = g->ci[K_B * pi_ + u];
            cplx c = g->ci[K_CRE * pi_ + u] + I * g->ci[K_CIM * pi_ + u];
            dhP[u] = -(dt / dr) * (b * nuP[u] + conj(c) * nuQ[u]);
            dhQ[u] = (dt / dr) * b * nuQ[u];
            sP[u] = dt * nuP[u];
            sQ[u] = dt * nuQ[u];
        }
    apply_S_adj(g, g->ci, nr, sP, sQ, hbP, hbQ);
    /* hbar_i = (h_{i+1/2} + h_{i-1/2})/2, dh_i = h_{i+1/2} - h_{i-1/2} */
    for (int j = 0; j < nth; ++j)
        for (int i = 1; i < nr - 1; ++i) {
            size_t u = (size_t)j * nr + i, kr = (size_t)j * nh + i, kl = kr - 1;
            hP[kr] += 0.5 * hbP[u] + dhP[u];
            hP[kl] += 0.5 * hbP[u] - dhP[u];
            hQ[kr] += 0.5 * hbQ[u] + dhQ[u];
            hQ[kl] += 0.5 * hbQ[u] - dhQ[u];
        }
    /* stage 1: hP = ubP - dt/2 [ b dP/dr - S_P ],  hQ = ubQ - dt/2 [ (c dP - b dQ)/dr - S_Q ] */
    for (int j = 0; j < nth; ++j)
        for (int i = 0; i < nh; ++i) {
            size_t k = (size_t)j * nh + i;
            double b = g->ch[K_B * ph + k];
            cplx c = g->ch[K_CRE * ph + k] + I * g->ch[K_CIM * ph + k];
            ubP[k] = hP[k];
            ubQ[k] = hQ[k];
            dP[k] = -(hdt / dr) * (b * hP[k] + conj(c) * hQ[k]);
            dQ[k] = (hdt / dr) * b * hQ[k];
            s1P[k] = hdt * hP[k];
            s1Q[k] = hdt * hQ[k];
        }
    apply_S_adj(g, g->ch, nh, s1P, s1Q, ubP, ubQ);
    /* ubar = (u_{i+1} + u_i)/2, delta = u_{i+1} - u_i; plus the direct term u of stage 2 */
    for (int j = 0; j < nth; ++j) {
        for (int i = 0; i < nr; ++i) {
            size_t u = (size_t)j * nr + i;
            lp[u] = nuP[u];
            lq[u] = nuQ[u];
        }
        for (int i = 0; i < nh; ++i) {
            size_t k = (size_t)j * nh + i, u = (size_t)j * nr + i;
            lp[u] += 0.5 * ubP[k] - dP[k];
            lp[u + 1] += 0.5 * ubP[k] + dP[k];
            lq[u] += 0.5 * ubQ[k] - dQ[k];
            lq[u + 1] += 0.5 * ubQ[k] + dQ[k];
        }
    }
    cplx* all[] = {nuP, nuQ, sP, sQ, hbP, hbQ, dhP, dhQ, hP, hQ, s1P, s1Q, ubP, ubQ, dP, dQ};
    for (int k = 0; k < 16; ++k) free(all[k]);
}

/* d/da of one step at a fixed state: the step with every coefficient
 * replaced, where it appears, by its derivative (forward-mode tangent;
 * the state does not depend on a).  Output (tp, tq) = (dA/da) u. */
void orc_tangent_a(const orc_grid* g, const cplx* phi, const cplx* pi, cplx* tp, cplx* tq)
{
    const int nr = g->nr, nth = g->nth, nh = nr - 1;
    const size_t ni = (size_t)nth * nr, nhs = (size_t)nth * nh;
    const double dt = g->dt, dr = g->dr, hdt = 0.5 * g->dt;
    work w;
    work_alloc(g, &w);
    cplx *dsP = calloc(nhs, sizeof(cplx)), *dsQ = calloc(nhs, sizeof(cplx));
    cplx *thP = calloc(nhs, sizeof(cplx)), *thQ = calloc(nhs, sizeof(cplx));
    cplx *tbP = calloc(ni, sizeof(cplx)), *tbQ = calloc(ni, sizeof(cplx));
    cplx *tdP = calloc(ni, sizeof(cplx)), *tdQ = calloc(ni, sizeof(cplx));
    cplx *s2P = calloc(ni, sizeof(cplx)), *s2Q = calloc(ni, sizeof(cplx));
    cplx *d2P = calloc(ni, sizeof(cplx)), *d2Q = calloc(ni, sizeof(cplx));
    /* values of stage 1 (h) and its tangent th = -dt/2 [ dD delta/dr - dS(ubar) ] */
    stage1(g, phi, pi, &w, NULL);
    apply_S(g, g->dch, nh, w.ubP, w.ubQ, dsP, dsQ);   /* coefficient part only: */
    for (size_t k = 0; k < nhs; ++k) dsP[k] = 0.0;    /* the Phi row of S has no coefficient */
    for (int j = 0; j < nth; ++j)
        for (int i = 0; i < nh; ++i) {
            size_t k = (size_t)j * nh + i;
            double db = g->dch[K_B * nhs + k];
            cplx dc = g->dch[K_CRE * nhs + k] + I * g->dch[K_CIM * nhs + k];
            thP[k] = -hdt * (db * w.dP[k] / dr - dsP[k]);
            thQ[k] = -hdt * ((dc * w.dP[k] - db * w.dQ[k]) / dr - dsQ[k]);
        }
    /* stage 2 values (hbar, dh) and tangents (tbar, td) at interior points */
    for (int j = 0; j < nth; ++j)
        for (int i = 1; i < nr - 1; ++i) {
            size_t u = (size_t)j * nr + i, kr = (size_t)j * nh + i, kl = kr - 1;
            w.hbP[u] = 0.5 * (w.hP[kr] + w.hP[kl]);
            w.hbQ[u] = 0.5 * (w.hQ[kr] + w.hQ[kl]);
            w.dhP[u] = w.hP[kr] - w.hP[kl];
            w.dhQ[u] = w.hQ[kr] - w.hQ[kl];
            tbP[u] = 0.5 * (thP[kr] + thP[kl]);
            tbQ[u] = 0.5 * (thQ[kr] + thQ[kl]);
            tdP[u] = thP[kr] - thP[kl];
            tdQ[u] = thQ[kr] - thQ[kl];
        }
    /* d/da [ -dt (D_i dh/dr - S_i(hbar)) ] = -dt (dD dh/dr + D td/dr - dS(hbar) - S(tbar)) */
    apply_S(g, g->dci, nr, w.hbP, w.hbQ, s2P, s2Q);
    for (size_t u = 0; u < ni; ++u) s2P[u] = 0.0;
    apply_S(g, g->ci, nr, tbP, tbQ, d2P, d2Q);
    for (int j = 0; j < nth; ++j)
        for (int i = 0; i < nr; ++i) {
            size_t u = (size_t)j * nr + i;
            if (i == 0 || i == nr - 1) { tp[u] = 0.0; tq[u] = 0.0; continue; }
            double b = g->ci[K_B * ni + u], db = g->dci[K_B * ni + u];
            cplx c = g->ci[K_CRE * ni + u] + I * g->ci[K_CIM * ni + u];
            cplx dc = g->dci[K_CRE * ni + u] + I * g->dci[K_CIM * ni + u];
            tp[u] = -dt * ((db * w.dhP[u] + b * tdP[u]) / dr - s2P[u] - d2P[u]);
            tq[u] = -dt * ((dc * w.dhP[u] - db * w.dhQ[u] + c * tdP[u] - b * tdQ[u]) / dr - s2Q[u] - d2Q[u]);
        }
    cplx* all[] = {dsP, dsQ, thP, thQ, tbP, tbQ, tdP, tdQ, s2P, s2Q, d2P, d2Q};
    for (int k = 0; k < 12; ++k) free(all[k]);
    work_free(&w);
}

/* Transpose of the bilinear extraction: lam_phi += E^T gval. */
void orc_extract_adjoint(const orc_grid* g, cplx* lam_phi, double rs, double th, const cplx* gval)
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
    for (int t = 0; t < 2; ++t) {
        int j = j0 + t;
        double sgn = 1.0;
        if (j < 0) { j = 0; sgn = g->sigma; }
        if (j > g->nth - 1) { j = g->nth - 1; sgn = g->sigma; }
        double wrow = (t == 0 ? 1.0 - wt : wt) * sgn;
        size_t u = (size_t)j * g->nr + i0;
        lam_phi[u] += wrow * (1.0 - wr) * (*gval);
        lam_phi[u + 1] += wrow * wr * (*gval);
    }
}

/* Reverse pass of n steps from (phi0, pi0) for a loss whose gradient with
 * respect to the extraction series (n x n_ext, sample k taken after step
 * k+1) is gser.  Returns the cotangent of the initial data (projected by
 * the radial boundary condition of the initial data) and dL/da.  Keeps all
 * n states in memory: small grids only. */
void orc_adjoint_evolve(const orc_grid* g, const cplx* phi0, const cplx* pi0, int64_t n, int n_ext,
                        const double* ext_r, const double* ext_th, const cplx* gser,
                        cplx* lam_phi, cplx* lam_pi, double* dLda)
{
    const size_t ni = (size_t)g->nth * g->nr;
    cplx* states = malloc(sizeof(cplx) * 2 * ni * (size_t)(n > 0 ? n : 1));
    cplx *p = malloc(sizeof(cplx) * ni), *q = malloc(sizeof(cplx) * ni);
    cplx *tp = malloc(sizeof(cplx) * ni), *tq = malloc(sizeof(cplx) * ni);
    memcpy(p, phi0, sizeof(cplx) * ni);
    memcpy(q, pi0, sizeof(cplx) * ni);
    orc_project(g, p, q);
    for (int64_t k = 0; k < n; ++k) {
        memcpy(states + 2 * ni * k, p, sizeof(cplx) * ni);
        memcpy(states + 2 * ni * k + ni, q, sizeof(cplx) * ni);
        orc_step(g, p, q);
    }
    memset(lam_phi, 0, sizeof(cplx) * ni);
    memset(lam_pi, 0, sizeof(cplx) * ni);
    double acc = 0.0;
    if (n > 0)
        for (int e = 0; e < n_ext; ++e) orc_extract_adjoint(g, lam_phi, ext_r[e], ext_th[e], &gser[(n - 1) * n_ext + e]);
    for (int64_t m = n - 1; m >= 0; --m) {
        orc_tangent_a(g, states + 2 * ni * m, states + 2 * ni * m + ni, tp, tq);
        for (size_t u = 0; u < ni; ++u) acc += creal(conj(lam_phi[u]) * tp[u] + conj(lam_pi[u]) * tq[u]);
        orc_adjoint_step(g, lam_phi, lam_pi);
        if (m >= 1)
            for (int e = 0; e < n_ext; ++e)
                orc_extract_adjoint(g, lam_phi, ext_r[e], ext_th[e], &gser[(m - 1) * n_ext + e]);
    }
    orc_project(g, lam_phi, lam_pi);
    *dLda = acc;
    free(states); free(p); free(q); free(tp); free(tq);
}
