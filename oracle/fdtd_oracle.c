/*
 * Plain, slow CPU oracle for the FDTD march of the 1+1D delay PDE of
 * Fang, "FDTD: solving 1+1D delay PDE in parallel" (arXiv:1707.05943).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header or table with the GPU path.
 *
 * Everything is double precision, single-threaded, in the paper's serial
 * space-then-time order (Sec. 2: the solver sweeps x left to right, then
 * advances t by one step).  Where the paper fixes a formula it is written out
 * as printed (Eqs. 1-13, App. C); where it is silent the reading used is
 * stated at the point of use.
 *
 * Contents
 *   1. P(n,z) = gamma(n,z)/(n-1)!   (App. C, four regimes (a)-(d))
 *   2. one-excitation amplitude E(t): closed forms Eqs. (6), (9), (13), and
 *      the delay series evaluated by direct Gauss-Legendre quadrature
 *   3. the march, Eq. (1) discretised with squares (Eq. 3) and bars (Eq. 4)
 *   4. readouts: int |psi|^2 dx (trapezoid) and chi at the detectors (Eq. 2)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The complex type of the arithmetic.  Built with -DORC_LONG_DOUBLE it is
 * long double (an extended-precision build that pins the rounding of the
 * FP64 march); the arrays a caller passes are double complex either way. */
#ifdef ORC_LONG_DOUBLE
typedef long double complex cplx;
#else
typedef double complex cplx;
#endif
typedef double complex dcplx;

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ======================================================================
 * 1.  P(n, z) for integer n >= 1 and complex z  (App. C)
 * ====================================================================== */

/* status of the last call: regime used (1..4 = a..d), and convergence */
static int g_regime = 0;
static int g_converged = 1;

int orc_gamma_last_regime(void) { return g_regime; }
int orc_gamma_last_converged(void) { return g_converged; }

/* (a) continued fraction for Q = 1 - P (Eq. C.2), modified Lentz evaluation */
static cplx gamma_Q_cf(int n, cplx z)
{
    const double tiny = 1e-300, eps = 1e-16;
    cplx b = z + 1.0 - n;
    cplx c = 1.0 / tiny;
    cplx d = 1.0 / b;
    cplx h = d;
    g_converged = 0;
    for (int i = 1; i < 2000000; ++i) {
        double an = -(double)i * (double)(i - n);
        b += 2.0;
        d = an * d + b;
        if (cabs(d) < tiny) d = tiny;
        c = b + an / c;
        if (cabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        cplx del = d * c;
        h *= del;
        if (cabs(del - 1.0) < eps) { g_converged = 1; break; }
    }
    /* e^{-z} z^n / Gamma(n) * CF */
    return cexp(-z + n * clog(z) - lgamma((double)n)) * h;
}

/* (b) series P = e^{-z} z^n sum_i z^i / Gamma(n+i+1)   (Eq. C.3) */
static cplx gamma_P_series(int n, cplx z)
{
    cplx del = 1.0 / (double)n;       /* Gamma(n) z^0 / Gamma(n+1) */
    cplx sum = del;
    double ap = n;
    g_converged = 0;
    for (int i = 1; i < 2000000; ++i) {
        ap += 1.0;
        del *= z / ap;
        sum += del;
        if (cabs(del) < cabs(sum) * 1e-17) { g_converged = 1; break; }
    }
    /* sum holds Gamma(n) * sum_i z^i/Gamma(n+i+1) */
    return sum * cexp(-z + n * clog(z) - lgamma((double)n));
}

/* (c) gamma-star series P = z^n/Gamma(n) sum_i (-z)^i / (i! (i+n))   (Eq. C.4) */
static cplx gamma_P_gstar(int n, cplx z)
{
    cplx t = 1.0;          /* (-z)^i / i! */
    cplx sum = 1.0 / (double)n;
    g_converged = 0;
    for (int i = 1; i < 2000000; ++i) {
        t *= -z / (double)i;
        cplx term = t / (double)(i + n);
        sum += term;
        if (cabs(term) < cabs(sum) * 1e-17) { g_converged = 1; break; }
    }
    return sum * cexp(n * clog(z) - lgamma((double)n));
}

/* (d) Poincare-type expansion for the argument -zeta, zeta = -z on (or next
 * to) the positive real axis (Eq. C.5):
 *   P(n,-zeta) ~ (-1)^n e^{zeta}/Gamma(n) sum_i (1-n)_i zeta^{n-i-1}.
 * For integer n the Pochhammer symbol (1-n)_i vanishes for i >= n, so the sum
 * is finite; it then equals -Q(n,-zeta) exactly and P = 1 + (that sum). */
static cplx gamma_P_poincare(int n, cplx z)
{
    cplx zeta = -z;
    cplx lz = clog(zeta);
    cplx sum = 0.0;
    /* (1-n)_i / Gamma(n) = (-1)^i / (n-1-i)!  */
    for (int i = 0; i < n; ++i) {
        double sgn = (i & 1) ? -1.0 : 1.0;
        sum += sgn * cexp(zeta + (double)(n - 1 - i) * lz - lgamma((double)(n - i)));
    }
    g_converged = 1;
    double sn = (n & 1) ? -1.0 : 1.0;
    return 1.0 + sn * sum;
}

/* Regime map.  The paper's map (its Fig. 9) is not available; the split used
 * here: near the negative real axis (Re z < 0, |Im z| <= 1e-12 |z|) use (c)
 * for moderate |z| and (d) beyond; elsewhere use the series (b) for
 * |z| < n + 1 and the continued fraction (a) otherwise, as for real z. */
cplx orc_gamma_P(int n, cplx z)
{
    if (n < 1) { g_regime = 0; g_converged = 0; return NAN; }
    double az = cabs(z);
    if (az == 0.0) { g_regime = 2; g_converged = 1; return 0.0; }
    if (creal(z) < 0.0 && fabs(cimag(z)) <= 1e-12 * az) {
        if (az <= 2.0 * n + 60.0) { g_regime = 3; return gamma_P_gstar(n, z); }
        g_regime = 4; return gamma_P_poincare(n, z);
    }
    if (az < n + 1.0) { g_regime = 2; return gamma_P_series(n, z); }
    g_regime = 1;
    return 1.0 - gamma_Q_cf(n, z);
}

/* exported pieces for tests: each regime on its own */
cplx orc_gamma_P_regime(int n, cplx z, int regime)
{
    switch (regime) {
    case 1: return 1.0 - gamma_Q_cf(n, z);
    case 2: return gamma_P_series(n, z);
    case 3: return gamma_P_gstar(n, z);
    case 4: return gamma_P_poincare(n, z);
    default: return NAN;
    }
}

/* ======================================================================
 * 2.  One-excitation amplitude E(t)
 * ====================================================================== */

enum { INC_PLANE = 1, INC_EXP1 = 2, INC_EXP2 = 3, INC_GAUSS2 = 4 };

typedef struct {
    int64_t Nx, D, Nt;
    double Delta, omega0, Gamma;
    int32_t incident;
    int32_t pad0;
    double k, alpha;        /* carrier; exponential width in units of Gamma */
    double x0, width;       /* Gaussian centre and std of |phi|^2 */
    double phase;           /* global phase of the two-photon state */
    int32_t identical;      /* 0: two different exponential photons (Sec. 2 case (c), Table 1) */
    int32_t pad1;
    double k1, k2, alpha1, alpha2;   /* photon 1 and photon 2 when identical = 0 */
} orc_params;

static double half_a(const orc_params *p) { return 0.5 * (double)p->D * p->Delta; }

/* the single-photon packet phi(x) of each family, support x <= -a
 * (theta(0) = 1: the point x = -a belongs to the packet).  Arguments are
 * grid coordinates computed in floating point, so the support test allows
 * a rounding slack of 1e-9 Delta. */
cplx orc_phi(const orc_params *p, double x)
{
    double a = half_a(p);
    if (x > -a + 1e-9 * p->Delta) return 0.0;
    switch (p->incident) {
    case INC_PLANE:                                   /* Eq. (5): A = 1 */
        return cexp(I * p->k * x);
    case INC_EXP1:
    case INC_EXP2:                                    /* Eq. (7) */
        return I * sqrt(p->alpha * p->Gamma) * cexp(I * p->k * x + p->alpha * p->Gamma * (x + a) / 2.0);
    case INC_GAUSS2: {                                /* Gaussian, |phi|^2 has std `width` */
        double w = p->width, u = x - p->x0;
        double nrm = pow(2.0 * M_PI * w * w, -0.25);
        return nrm * cexp(-u * u / (4.0 * w * w) + I * p->k * u);
    }
    }
    return NAN;
}

/* ---- two different photons (Sec. 2 case (c)) ----
 * chi(x1, x2, 0) = (A/sqrt 2) [phi1(x1) phi2(x2) + phi1(x2) phi2(x1)] (Eq. 10),
 * phi_i the packet of Eq. (7) with (k_i, alpha_i), A of Eq. (11); in x <= -a
 * psi(x, t) = A [phi1(x-t) e0^(2)(t) + phi2(x-t) e0^(1)(t)] (Eq. 12), e0^(i)
 * the one-excitation amplitude driven by phi_i (Eq. 13).  A global phase
 * e^{i theta} multiplies the whole state, as for the other families. */
static int two_photons(const orc_params *p) { return p->incident == INC_EXP2 && !p->identical; }

/* photon i (1 or 2) as a one-packet parameter set */
static orc_params photon(const orc_params *p, int i)
{
    orc_params q = *p;
    q.identical = 1;
    q.k = (i == 1) ? p->k1 : p->k2;
    q.alpha = (i == 1) ? p->alpha1 : p->alpha2;
    return q;
}

/* Eq. (11) */
static double two_photon_A(const orc_params *p)
{
    double dk = p->k1 - p->k2, s = (p->alpha1 + p->alpha2) * p->Gamma;
    double num = 4.0 * dk * dk + s * s;
    return sqrt(num / (num + 4.0 * p->alpha1 * p->alpha2 * p->Gamma * p->Gamma));
}

/* the initial two-photon state chi(x1, x2, 0) of every two-photon family,
 * global phase included (zero for stimulated emission) */
cplx orc_chi0(const orc_params *p, double x1, double x2)
{
    cplx eth = cexp(I * p->phase);
    if (p->incident == INC_EXP1) return 0.0;
    if (two_photons(p)) {
        orc_params a = photon(p, 1), b = photon(p, 2);
        return eth * two_photon_A(p) / sqrt(2.0) *
               (orc_phi(&a, x1) * orc_phi(&b, x2) + orc_phi(&a, x2) * orc_phi(&b, x1));
    }
    return eth * orc_phi(p, x1) * orc_phi(p, x2);
}

/* closed form Eq. (6): plane wave, A = 1 */
static cplx E_plane_closed(const orc_params *p, double t)
{
    double a = half_a(p), G = p->Gamma, k = p->k, w0 = p->omega0;
    cplx W = I * w0 + G / 2.0;
    cplx pp = k - w0 + I * G / 2.0;
    if (t <= 0.0) return 0.0;
    cplx e = I * sqrt(G / 2.0) * cexp(-I * k * a) * (cexp(-I * k * t) - cexp(-W * t)) / pp;
    for (int n = 1; t - 2.0 * n * a > 0.0; ++n) {
        double T = t - 2.0 * n * a;
        cplx in = cpow(I, n);
        /* (G/2)^{n-1/2}/n! [T^n e^{-W T} + i^n (k-w0)/p^{n+1} gamma(n+1, -i p T) e^{-ikT}],
         * with gamma(n+1,z)/n! = P(n+1,z) */
        cplx t1 = cexp(n * log(T) - W * T - lgamma(n + 1.0));
        cplx t2 = in * (k - w0) * orc_gamma_P(n + 1, -I * pp * T) / cpow(pp, n + 1) * cexp(-I * k * T);
        e -= cexp(-I * k * a) * pow(G / 2.0, n - 0.5) * (t1 + t2);
    }
    return e;
}

/* closed form Eq. (9): emitter excited at t = 0, no photon */
static cplx E_exp1_closed(const orc_params *p, double t)
{
    double a = half_a(p), G = p->Gamma;
    cplx W = I * p->omega0 + G / 2.0;
    if (t < 0.0) return 0.0;
    cplx s = 0.0;
    for (int n = 0; t - 2.0 * n * a >= 0.0; ++n) {
        double T = t - 2.0 * n * a;
        cplx base = (G / 2.0) * cexp(W * 2.0 * a) * T;
        s += (n == 0) ? 1.0 : cpow(base, n) / tgamma(n + 1.0);
    }
    return cexp(-W * t) * s;
}

/* Eq. (13) where its p = k - w0 + i (G/2)(1 - alpha) vanishes (k = w0 and
 * alpha = 1: the packet decays at the emitter's rate, lambda = W), a removable
 * 0/0 of the closed form.  Then phi(-a-s) = A e^{-ika} e^{-W s},
 * A = i sqrt(alpha G), and the integrals of the delay series are elementary:
 * J_n(T) = int_0^T (T-s)^n/n! e^{-W(T-s)} A e^{-ika} e^{-W s} ds
 *        = A e^{-ika} e^{-W T} T^{n+1}/(n+1)!, so
 * E(t) = sqrt(G/2) sum_n (G/2)^n [J_n(t - 2na) - J_n(t - 2(n+1)a)]. */
static cplx E_exp2_resonant(const orc_params *p, double t)
{
    double a = half_a(p), G = p->Gamma;
    cplx W = I * p->omega0 + G / 2.0;
    cplx A = I * sqrt(p->alpha * G) * cexp(-I * p->k * a);
    cplx s = 0.0;
    for (int n = 0; t - 2.0 * n * a > 0.0; ++n) {
        double T1 = t - 2.0 * n * a, T2 = t - 2.0 * (n + 1) * a;
        cplx j = cexp((n + 1) * log(T1) - W * T1 - lgamma(n + 2.0));
        if (T2 > 0.0) j -= cexp((n + 1) * log(T2) - W * T2 - lgamma(n + 2.0));
        s += pow(G / 2.0, n) * j;
    }
    return sqrt(G / 2.0) * A * s;
}

/* closed form Eq. (13), multiplied by e^{-ika} so that phi's phase is the
 * one of Eq. (7) (the two must use the same packet).  Near p = 0 its two
 * terms cancel (relative rounding ~ 1e-16/|p|); at p = 0 exactly the limit
 * above is taken. */
static cplx E_exp2_closed(const orc_params *p, double t)
{
    double a = half_a(p), G = p->Gamma, k = p->k, w0 = p->omega0, al = p->alpha;
    cplx W = I * w0 + G / 2.0;
    cplx lam = I * k + al * G / 2.0;
    cplx pp = k - w0 + I * G / 2.0 * (1.0 - al);
    if (t <= 0.0) return 0.0;
    if (creal(pp) == 0.0 && cimag(pp) == 0.0) return E_exp2_resonant(p, t);
    cplx e = sqrt(al * G * G / 2.0) * (cexp(-W * t) - cexp(-lam * t)) / pp;
    for (int n = 1; t - 2.0 * n * a > 0.0; ++n) {
        double T = t - 2.0 * n * a;
        cplx in = cpow(I, n);
        cplx t1 = cexp(n * log(T) - W * T - lgamma(n + 1.0));
        cplx t2 = in * (k - w0 - I * al * G / 2.0) * orc_gamma_P(n + 1, -I * pp * T) / cpow(pp, n + 1)
                  * cexp(-lam * T);
        e -= I * sqrt(al * G) * pow(G / 2.0, n - 0.5) * (t1 + t2);
    }
    return cexp(-I * k * a) * e;
}

cplx orc_E_closed(const orc_params *p, double t)
{
    switch (p->incident) {
    case INC_PLANE: return E_plane_closed(p, t);
    case INC_EXP1: return E_exp1_closed(p, t);
    case INC_EXP2: return E_exp2_closed(p, t);
    }
    return NAN;
}

/* ---- Gauss-Legendre nodes on [-1, 1] (Newton on P_m) ---- */
#define GL_M 24
static double gl_x[GL_M], gl_w[GL_M];
static int gl_ready = 0;

static void gl_init(void)
{
    if (gl_ready) return;
    const int m = GL_M;
    for (int i = 0; i < m; ++i) {
        double x = cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int l = 2; l <= m; ++l) {
                double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
                p0 = p1; p1 = p2;
            }
            dp = m * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int l = 2; l <= m; ++l) {
                double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
                p0 = p1; p1 = p2;
            }
            dp = m * (x * p1 - p0) / (x * x - 1.0);
        }
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

/* upper end of the packet's support seen from x = -a: phi(-a-s) is below
 * 1e-20 of its peak for s beyond this (only the Gaussian is bounded). */
static double s_support(const orc_params *p, double T)
{
    if (p->incident == INC_GAUSS2) {
        double a = half_a(p);
        double hi = (-a - p->x0) + 20.0 * p->width;
        return hi < T ? hi : T;
    }
    return T;
}

/* panel width for the composite rule: short against the packet's width,
 * its decay length and the fastest phase of the integrand */
static double panel_width(const orc_params *p)
{
    double h = 1.0;
    double freq = fabs(p->k) + fabs(p->omega0) + p->Gamma + 1.0;
    if (3.0 / freq < h) h = 3.0 / freq;
    if (p->incident == INC_GAUSS2 && 0.5 * p->width < h) h = 0.5 * p->width;
    if (p->incident == INC_EXP1 || p->incident == INC_EXP2) {
        double dec = 0.5 * p->alpha * p->Gamma;
        if (dec > 0.0 && 1.0 / dec < h) h = 1.0 / dec;
    }
    return h;
}

/* one Gauss-Legendre panel [lo, hi] of
 * int (T-s)^n/n! e^{-W (T-s)} phi(-a-s) ds; phi_nodes may hold phi at the
 * panel's nodes (else they are evaluated here) */
static cplx jn_panel(const orc_params *p, int n, double T, double lo, double hi, const cplx *phi_nodes)
{
    double a = half_a(p);
    cplx W = I * p->omega0 + p->Gamma / 2.0;
    double lnf = lgamma(n + 1.0);
    double c = 0.5 * (lo + hi), hw = 0.5 * (hi - lo);
    cplx sum = 0.0;
    for (int i = 0; i < GL_M; ++i) {
        double s = c + hw * gl_x[i];
        double u = T - s;
        cplx ker = (n == 0) ? cexp(-W * u) : cexp(n * log(u) - lnf - W * u);
        cplx ph = phi_nodes ? phi_nodes[i] : orc_phi(p, -a - s);
        sum += gl_w[i] * ker * ph;
    }
    return hw * sum;
}

/* J_n(T) = int_0^T (T-s)^n/n! e^{-W (T-s)} phi(-a-s) ds, composite 24-point
 * Gauss-Legendre over panels [qh, (q+1)h] and a last partial panel */
cplx orc_Jn_quad(const orc_params *p, int n, double T)
{
    if (T <= 0.0) return 0.0;
    gl_init();
    double hi = s_support(p, T);
    double h = panel_width(p);
    if (n > 0 && hi / (n + 1.0) < h) h = hi / (n + 1.0);
    long nfull = (long)floor(hi / h);
    cplx sum = 0.0;
    for (long q = 0; q < nfull; ++q) sum += jn_panel(p, n, T, q * h, (q + 1) * h, NULL);
    if (hi > nfull * h) sum += jn_panel(p, n, T, nfull * h, hi, NULL);
    return sum;
}

/* E(t) = sqrt(G/2) sum_{n>=0} (G/2)^n [J_n(t - 2na) - J_n(t - 2(n+1)a)]
 * (solution of the one-excitation delay equation driven by phi).  For the
 * stimulated-emission family E is Eq. (9) instead. */
cplx orc_E_quad(const orc_params *p, double t)
{
    if (p->incident == INC_EXP1) return E_exp1_closed(p, t);
    double a = half_a(p), G = p->Gamma;
    cplx s = 0.0;
    for (int n = 0; t - 2.0 * n * a > 0.0; ++n) {
        s += pow(G / 2.0, n) * (orc_Jn_quad(p, n, t - 2.0 * n * a) - orc_Jn_quad(p, n, t - 2.0 * (n + 1) * a));
    }
    return sqrt(G / 2.0) * s;
}

/* The same series on the grid t_r = r Delta: with 2a = D Delta, the shifted
 * times are T = (r - nD) Delta, so J_n is needed at T = q Delta only and each
 * value serves two rows (r = q + nD and r = q + (n+1)D). */
static void E_table_quad(const orc_params *p, dcplx *E)
{
    const int64_t Nt = p->Nt, D = p->D;
    const double G = p->Gamma, dl = p->Delta;
    gl_init();
    for (int64_t r = 0; r <= Nt; ++r) E[r] = 0.0;
    if (p->incident == INC_EXP1) { for (int64_t r = 0; r <= Nt; ++r) E[r] = E_exp1_closed(p, r * dl); return; }
    cplx *J = (cplx *)malloc(sizeof(cplx) * (size_t)(Nt + 1));
    for (int n = 0; (int64_t)n * D <= Nt; ++n) {
        int64_t qmax = Nt - (int64_t)n * D;
        for (int64_t q = 0; q <= qmax; ++q) {
            double T = q * dl;
            J[q] = orc_Jn_quad(p, n, T);
        }
        double gn = pow(G / 2.0, n);
        for (int64_t r = (int64_t)n * D; r <= Nt; ++r) {
            cplx v = J[r - (int64_t)n * D];
            if (r - (int64_t)(n + 1) * D >= 0) v -= J[r - (int64_t)(n + 1) * D];
            E[r] += gn * v;
        }
    }
    for (int64_t r = 0; r <= Nt; ++r) E[r] *= sqrt(G / 2.0);
    free(J);
}

/* E(t_r), r = 0..Nt: the closed form where the paper gives one, else the
 * quadrature of the delay series.  mode 0: default, 1: force quadrature (on
 * the grid), 2: quadrature row by row.  Two different photons: e0^(1) in
 * E[0..Nt], then e0^(2) in E[Nt+1..2Nt+1]. */
void orc_E_table(const orc_params *p, int mode, dcplx *E)
{
    if (two_photons(p)) {
        orc_params a = photon(p, 1), b = photon(p, 2);
        orc_E_table(&a, mode, E);
        orc_E_table(&b, mode, E + (p->Nt + 1));
        return;
    }
    for (int64_t r = 0; r <= p->Nt; ++r) {
        double t = (double)r * p->Delta;
        if (mode == 0 && p->incident != INC_GAUSS2) E[r] = orc_E_closed(p, t);
        else if (mode == 2) E[r] = orc_E_quad(p, t);
        else { E_table_quad(p, E); return; }
    }
}

/* ======================================================================
 * 3.  The march (Eq. 1 with squares, Eq. 3, and bars, Eq. 4)
 * ====================================================================== */

typedef struct {
    const orc_params *p;
    const dcplx *E;          /* E(t_r), r = 0..Nt (two different photons: e0^(1)) */
    const cplx *phig;        /* phi(-a - q Delta), q = 0..Nt: phi at the grid points x - t of x <= -a
                                (two different photons: phi1) */
    const dcplx *E2;         /* two different photons: e0^(2)(t_r); else NULL */
    const cplx *phig2;       /* two different photons: phi2(-a - q Delta); else NULL */
    cplx c_ex;               /* psi = c_ex phi(x-t) E(t) in x <= -a (two photons: c_ex [phi1 e0^(2) + phi2 e0^(1)]) */
    cplx *ring;              /* (D+2) rows of Nx+1 columns; row rho in slot rho mod (D+2) */
    int64_t cur;             /* row being solved */
    int fault;               /* set when a read violates the ring's lag bound */
    /* the paper's own reads (orc_march_diag): columns lo..Nx (lo <= 0) are
     * marched and kept for every row; only columns left of lo are read from
     * the exact solution.  NULL in the hybrid march. */
    cplx *hist;              /* (Nt+1) rows of Nx - lo + 1 columns */
    int64_t lo;
    int64_t cur_col;         /* column being solved in row cur */
} orc_state;

/* exact solution in x <= -a (Eq. 12 for identical photons, Eq. 8 for
 * stimulated emission): psi(x,t) = c phi(x-t) E(t); on the grid
 * x_i - t_rho = -a - (rho - i) Delta */
static cplx psi_exact(const orc_state *s, int64_t i, int64_t rho)
{
    if (s->E2) return s->c_ex * (s->phig[rho - i] * s->E2[rho] + s->phig2[rho - i] * s->E[rho]);
    return s->c_ex * s->phig[rho - i] * s->E[rho];
}

/* psi at grid column i (x_i = -a + i Delta) and row rho: zero before t = 0;
 * the exact solution at x <= -a; the marched values elsewhere. */
static cplx psi_at(orc_state *s, int64_t i, int64_t rho)
{
    const orc_params *p = s->p;
    if (rho < 0) return 0.0;
    if (s->hist) {
        if (i < s->lo) return psi_exact(s, i, rho);
        if (i > p->Nx || rho > s->cur || (rho == s->cur && i >= s->cur_col)) { s->fault = 1; return NAN; }
        return s->hist[rho * (p->Nx - s->lo + 1) + (i - s->lo)];
    }
    if (i <= 0) return psi_exact(s, i, rho);
    if (i > p->Nx) { s->fault = 1; return NAN; }
    int64_t lag = s->cur - rho;
    if (lag < 0 || lag > p->D + 1) { s->fault = 1; return NAN; }
    return s->ring[(rho % (p->D + 2)) * (p->Nx + 1) + i];
}

/* the bar of Eq. (4): f at the midpoint of columns i and i+1 */
static cplx bar(orc_state *s, int64_t i, int64_t rho)
{
    return 0.5 * (psi_at(s, i, rho) + psi_at(s, i + 1, rho));
}

/* Solve psi(j, r) from the square whose corners are (j-1, r-1), (j, r-1),
 * (j-1, r), (j, r); its centre is (x_c, t_c) = (x_j - Delta/2, t_r - Delta/2).
 *
 * Terms of Eq. (1) at the centre:
 *   d/dt + d/dx + W  -> Eq. (3a-c) over the four corners
 *   (G/2) psi(x-2a, t-2a) theta(t-2a)  -> square average (line-1 term) of the
 *       square shifted by D columns and D rows; active when t_c > 2a
 *   source terms (lines 2-3) -> bars: their time argument falls on a grid row
 *       and their space argument midway between two columns
 *   drive (line 4) -> chi(x-t, -/+a - t, 0) evaluated at the centre.  */
static cplx solve_cell(orc_state *s, int64_t j, int64_t r, cplx left /* psi(j-1, r) */,
                       cplx drive_row /* phi(-a - t_c) - phi(a - t_c) */,
                       cplx drive_row2 /* two photons: the same for phi2 (drive_row is phi1's) */)
{
    const orc_params *p = s->p;
    const int64_t D = p->D;
    const double dl = p->Delta, G = p->Gamma, a = half_a(p);
    const cplx W = I * p->omega0 + G / 2.0;

    cplx bl = psi_at(s, j - 1, r - 1);     /* bottom left  */
    cplx br = psi_at(s, j, r - 1);         /* bottom right */
    cplx tl = left;                        /* top left     */

    cplx rhs = 0.0;
    /* delay: active iff t_c = (r - 1/2) Delta > 2a = D Delta, i.e. r - 1 >= D */
    if (r - 1 >= D) {
        rhs += (G / 2.0) * 0.25 * (psi_at(s, j - 1 - D, r - 1 - D) + psi_at(s, j - D, r - 1 - D)
                                   + psi_at(s, j - 1 - D, r - D) + psi_at(s, j - D, r - D));
    }
    /* source 1: [psi(-x-2a, t-x-a) - psi(-x, t-x-a)] theta(x+a) theta(t-x-a).
     * At the centre t - x - a = (r - j) Delta; -x - 2a is midway between
     * columns -j and -j+1; -x is midway between D-j and D-j+1.
     * theta(x_c + a) holds for every j >= 1; theta(0) = 1 at r = j. */
    cplx src = 0.0;
    if (j >= 1 && r - j >= 0) src += bar(s, -j, r - j) - bar(s, D - j, r - j);
    /* source 2: [psi(2a-x, t-x+a) - psi(-x, t-x+a)] theta(x-a) theta(t-x+a).
     * t - x + a = (r - j + D) Delta; 2a - x is midway between 2D-j and
     * 2D-j+1; theta(x_c - a) holds iff j >= D+1. */
    if (j >= D + 1 && r - j + D >= 0) src += bar(s, 2 * D - j, r - j + D) - bar(s, D - j, r - j + D);
    rhs -= (G / 2.0) * src;
    /* drive: sqrt(G) [chi0(x-t, -a-t) - chi0(x-t, a-t)] at the centre, where
     * x_c - t_c = x_j - t_r lies on the grid (phi there is phig[r - j]) and
     * phi(-a - t_c), phi(a - t_c) are the same for the whole row */
    if (s->E2 && r - j >= 0)
        /* chi0(xi, y) = e^{i theta} (A/sqrt 2) [phi1(xi) phi2(y) + phi2(xi) phi1(y)] */
        rhs += sqrt(G) * cexp(I * p->phase) * two_photon_A(p) / sqrt(2.0) *
               (s->phig[r - j] * drive_row2 + s->phig2[r - j] * drive_row);
    else if (p->incident != INC_EXP1 && r - j >= 0)
        rhs += sqrt(G) * cexp(I * p->phase) * s->phig[r - j] * drive_row;
    (void)a; (void)dl;
    /* (U - bl)/Delta + (W/4)(bl + br + tl + U) = rhs, solved for the
     * increment U - bl: (U - bl)(1/Delta + W/4) = rhs - (W/4)(2 bl + br + tl).
     * (Solved for U instead, the rounded divisor would scale psi once per row
     * along every characteristic and bias the march by about one rounding per
     * row; here it scales only the increment.) */
    return bl + (rhs - (W / 4.0) * (2.0 * bl + br + tl)) / (1.0 / dl + W / 4.0);
}

/* chi(x1, x2, t_r) at x1 = a + Delta (column D+1), x2 = x1 + k Delta
 * (column D+1+k), from Eq. (2); reads rows r-1 .. r-D-1 and the exact
 * solution.  theta(x2 + a), theta(x2 - a) and theta(x1 - a) all hold. */
static cplx chi_detector(orc_state *s, int64_t r, int64_t kk)
{
    const orc_params *p = s->p;
    const int64_t D = p->D;
    const double dl = p->Delta, a = half_a(p), G = p->Gamma;
    const int64_t j1 = D + 1, j2 = D + 1 + kk;
    /* chi(x1 - t, x2 - t, 0) = e^{i theta} phi(x1 - t) phi(x2 - t); x_j - t_r = -a - (r - j) Delta */
    cplx c0 = 0.0;
    if (s->E2 && r - j1 >= 0 && r - j2 >= 0)
        c0 = cexp(I * p->phase) * two_photon_A(p) / sqrt(2.0) *
             (s->phig[r - j1] * s->phig2[r - j2] + s->phig[r - j2] * s->phig2[r - j1]);
    else if (p->incident != INC_EXP1 && r - j1 >= 0 && r - j2 >= 0)
        c0 = cexp(I * p->phase) * s->phig[r - j1] * s->phig[r - j2];
    (void)a; (void)dl;
    cplx acc = 0.0;
    /* psi(x1 - x2 - a, t - x2 - a): column j1 - j2, row r - j2 */
    acc += psi_at(s, j1 - j2, r - j2);
    /* - psi(x1 - x2 + a, t - x2 + a): column j1 - j2 + D, row r - j2 + D */
    acc -= psi_at(s, j1 - j2 + D, r - j2 + D);
    /* the same with x1 <-> x2 */
    acc += psi_at(s, j2 - j1, r - j1);
    acc -= psi_at(s, j2 - j1 + D, r - j1 + D);
    return c0 - sqrt(G) / 2.0 * acc;
}

/* probability that the emitter is excited, P_e(t_r) = int |psi(x,t_r)|^2 dx:
 * the exact part x <= -a in closed form, plus the trapezoid rule over the
 * marched columns 0..Nx.  int_{-inf}^{-a} |psi|^2 = |c|^2 |E|^2 int_{-inf}^{-a-t}|phi|^2. */
static double phi_mass_below(const orc_params *p, double y)
{
    double a = half_a(p);
    if (y > -a) y = -a;
    switch (p->incident) {
    case INC_GAUSS2:
        return 0.5 * erfc((p->x0 - y) / (sqrt(2.0) * p->width));
    case INC_EXP1:
    case INC_EXP2:
        return exp(p->alpha * p->Gamma * (y + a));
    }
    return NAN;   /* plane wave: not normalisable */
}

/* two exponential photons: int_{-inf}^{y} conj(phi1) phi2 for y <= -a.  With
 * v = u + a the integrand is sqrt(alpha1 alpha2) G e^{-i(k2-k1)a} e^{c v},
 * c = i(k2 - k1) + (alpha1 + alpha2) G/2 (Eq. 7 for both photons). */
static cplx phi_cross_below(const orc_params *p, double y)
{
    double a = half_a(p), G = p->Gamma;
    if (y > -a) y = -a;
    cplx c = I * (p->k2 - p->k1) + 0.5 * (p->alpha1 + p->alpha2) * G;
    return sqrt(p->alpha1 * p->alpha2) * G * cexp(-I * (p->k2 - p->k1) * a) * cexp(c * (y + a)) / c;
}

/* int_{-inf}^{-a} |psi(x, t_r)|^2 dx from the exact solution: |c E|^2 times
 * the packet's mass below -a - t, and for two different photons
 * A^2 [|e2|^2 m11 + |e1|^2 m22 + 2 Re(conj(e2) e1 m12)] with m_ij the mass of
 * conj(phi_i) phi_j below -a - t */
static double exact_part(const orc_state *s, int64_t r)
{
    const orc_params *p = s->p;
    double y = -half_a(p) - r * p->Delta;
    if (s->E2) {
        orc_params a = photon(p, 1), b = photon(p, 2);
        double A = two_photon_A(p);
        cplx e1 = s->E[r], e2 = s->E2[r];
        return A * A * (creal(e2 * conj(e2)) * phi_mass_below(&a, y) + creal(e1 * conj(e1)) * phi_mass_below(&b, y)
                        + 2.0 * creal(conj(e2) * e1 * phi_cross_below(p, y)));
    }
    double cc = (p->incident == INC_EXP1) ? 1.0 : 2.0;
    return cc * creal(s->E[r] * conj(s->E[r])) * phi_mass_below(p, y);
}

static double pe_row(orc_state *s, int64_t r)
{
    const orc_params *p = s->p;
    double ex = exact_part(s, r);
    double acc = 0.0;
    for (int64_t j = 0; j <= p->Nx; ++j) {
        cplx v = psi_at(s, j, r);
        double m2 = creal(v * conj(v));
        acc += (j == 0 || j == p->Nx) ? 0.5 * m2 : m2;
    }
    return ex + p->Delta * acc;
}

/*
 * Run the march over rows 1..Nt.
 *   E        : E(t_r), r = 0..Nt
 *   pe       : out, P_e(t_r) for r = 0..Nt (may be NULL)
 *   ring_out : out, rows Nt-D-1..Nt (oldest first), each Nx+1 columns; rows
 *              before 0 are zero (may be NULL)
 *   chi_rows/n_chi_rows, n_tau, chi : chi at detectors (k = 0..n_tau-1) at the
 *              listed rows, written row after row (may be NULL)
 *   snap_rows/n_snap, snaps : full rows (Nx+1 values) at the listed rows
 * Returns 0, or -1 when a read broke the lag bound (an oracle bug).
 */
int orc_march(const orc_params *p, const dcplx *E, double *pe, dcplx *ring_out,
              const int64_t *chi_rows, int64_t n_chi_rows, int64_t n_tau, dcplx *chi,
              const int64_t *snap_rows, int64_t n_snap, dcplx *snaps)
{
    const int64_t D = p->D, Nx = p->Nx, Nt = p->Nt, R = D + 2, C = Nx + 1;
    const int two = two_photons(p);
    orc_params ph1 = two ? photon(p, 1) : *p, ph2 = two ? photon(p, 2) : *p;
    orc_state s = { p, E, NULL, NULL, NULL, 0.0, NULL, 0, 0, NULL, 0, 0 };
    s.ring = (cplx *)calloc((size_t)(R * C), sizeof(cplx));
    cplx *phig = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * (Nt + 1)));
    if (!s.ring || !phig) { free(s.ring); free(phig); return -2; }
    for (int64_t q = 0; q <= Nt; ++q) {
        phig[q] = orc_phi(&ph1, -half_a(p) - (double)q * p->Delta);
        phig[Nt + 1 + q] = orc_phi(&ph2, -half_a(p) - (double)q * p->Delta);
    }
    s.phig = phig;
    s.c_ex = (p->incident == INC_EXP1) ? 1.0 : sqrt(2.0) * cexp(I * p->phase);
    if (two) {
        s.phig2 = phig + (Nt + 1);
        s.E2 = E + (Nt + 1);
        s.c_ex = two_photon_A(p) * cexp(I * p->phase);
    }

    /* row 0: psi(x, 0) = 0 for x > -a in every family */
    s.cur = 0;
    if (pe) pe[0] = pe_row(&s, 0);
    for (int64_t q = 0; q < n_chi_rows; ++q)
        if (chi_rows[q] == 0)
            for (int64_t kk = 0; kk < n_tau; ++kk) chi[q * n_tau + kk] = chi_detector(&s, 0, kk);
    for (int64_t q = 0; q < n_snap; ++q)
        if (snap_rows[q] == 0)
            for (int64_t j = 0; j <= Nx; ++j) snaps[q * C + j] = psi_at(&s, j, 0);

    for (int64_t r = 1; r <= Nt; ++r) {
        s.cur = r;
        cplx *row = s.ring + (r % R) * C;
        row[0] = 0.0;              /* column 0 is read from the exact solution */
        cplx left = psi_at(&s, 0, r);
        double tc = ((double)r - 0.5) * p->Delta;
        cplx drive_row = orc_phi(&ph1, -half_a(p) - tc) - orc_phi(&ph1, half_a(p) - tc);
        cplx drive_row2 = orc_phi(&ph2, -half_a(p) - tc) - orc_phi(&ph2, half_a(p) - tc);
        for (int64_t j = 1; j <= Nx; ++j) {
            cplx u = solve_cell(&s, j, r, left, drive_row, drive_row2);
            row[j] = u;
            left = u;
        }
        if (pe) pe[r] = pe_row(&s, r);
        for (int64_t q = 0; q < n_chi_rows; ++q)
            if (chi_rows[q] == r)
                for (int64_t kk = 0; kk < n_tau; ++kk) chi[q * n_tau + kk] = chi_detector(&s, r, kk);
        for (int64_t q = 0; q < n_snap; ++q)
            if (snap_rows[q] == r)
                for (int64_t j = 0; j <= Nx; ++j) snaps[q * C + j] = psi_at(&s, j, r);
        if (s.fault) break;
    }
    if (ring_out && !s.fault) {
        s.cur = Nt;
        for (int64_t q = 0; q < R; ++q) {
            int64_t rho = Nt - (R - 1) + q;
            for (int64_t j = 0; j <= Nx; ++j)
                ring_out[q * C + j] = (rho < 0) ? 0.0 : (j == 0 ? psi_exact(&s, 0, rho) : s.ring[(rho % R) * C + j]);
        }
    }
    free(s.ring);
    free(phig);
    return s.fault ? -1 : 0;
}

/*
 * The march with the paper's own reads (Sec. 3; its test 1 in Sec. 4): the
 * diag_cols columns 1-diag_cols .. 0 (x <= -a) are marched too, with the
 * same square of Eq. (1) (no source terms there: theta(x + a) = 0), and every
 * read of a marched point takes the marched value; only points left of
 * column 1-diag_cols take the exact solution (the region the paper fills
 * with its boundary condition).  Row 0 is the initial condition (the exact
 * solution in x <= -a, zero right of it).  Every row is kept.
 *   pe    : out, P_e(t_r) (exact part below -a plus the trapezoid over
 *           columns 0..Nx, column 0 marched) (may be NULL)
 *   snaps : out, columns 1-diag_cols .. Nx of each listed row
 * Returns 0, -1 when a read reached a point not yet solved, -2 when out of
 * memory.
 */
int orc_march_diag(const orc_params *p, const dcplx *E, int64_t diag_cols, double *pe,
                   const int64_t *snap_rows, int64_t n_snap, cplx *snaps)
{
    const int64_t D = p->D, Nx = p->Nx, Nt = p->Nt;
    const int64_t lo = 1 - diag_cols, W = Nx - lo + 1;
    if (diag_cols < 1 || two_photons(p)) return -3;
    /* exact reads reach x - t = -a - q Delta with q up to Nt - lo + D + 1 */
    const int64_t nq = Nt - lo + D + 2;
    orc_state s = { p, E, NULL, NULL, NULL, 0.0, NULL, 0, 0, NULL, lo, 0 };
    s.hist = (cplx *)calloc((size_t)((Nt + 1) * W), sizeof(cplx));
    cplx *phig = (cplx *)malloc(sizeof(cplx) * (size_t)nq);
    if (!s.hist || !phig) { free(s.hist); free(phig); return -2; }
    for (int64_t q = 0; q < nq; ++q) phig[q] = orc_phi(p, -half_a(p) - (double)q * p->Delta);
    s.phig = phig;
    s.c_ex = (p->incident == INC_EXP1) ? 1.0 : sqrt(2.0) * cexp(I * p->phase);

    /* row 0: the exact solution at x <= -a, zero right of it */
    for (int64_t i = lo; i <= 0; ++i) s.hist[i - lo] = psi_exact(&s, i, 0);
    s.cur = 1;
    for (int64_t r = 1; r <= Nt; ++r) {
        s.cur = r;
        s.cur_col = lo;
        cplx *row = s.hist + r * W;
        cplx left = psi_at(&s, lo - 1, r);
        double tc = ((double)r - 0.5) * p->Delta;
        cplx drive_row = orc_phi(p, -half_a(p) - tc) - orc_phi(p, half_a(p) - tc);
        for (int64_t j = lo; j <= Nx; ++j) {
            s.cur_col = j;
            cplx u = solve_cell(&s, j, r, left, drive_row, 0.0);
            row[j - lo] = u;
            left = u;
        }
        if (s.fault) break;
    }
    if (!s.fault) {
        s.cur = Nt + 1;
        s.cur_col = lo;
        for (int64_t r = 0; pe && r <= Nt; ++r) pe[r] = pe_row(&s, r);
        for (int64_t q = 0; q < n_snap; ++q)
            for (int64_t j = lo; j <= Nx; ++j) snaps[q * W + (j - lo)] = s.hist[snap_rows[q] * W + (j - lo)];
    }
    free(s.hist);
    free(phig);
    return s.fault ? -1 : 0;
}

/* thin exports used by the tests */
cplx orc_phi_at(const orc_params *p, double x) { return orc_phi(p, x); }
double orc_two_photon_A(const orc_params *p) { return two_photon_A(p); }
double orc_phi_mass_below(const orc_params *p, double y) { return phi_mass_below(p, y); }

/* ======================================================================
 * pointer-based entry points for the Python test harness (ctypes cannot
 * pass C99 complex values): complex arrays are interleaved (re, im) pairs
 * ====================================================================== */
void orc_gamma_P_arr(int64_t m, const int32_t *n, const dcplx *z, dcplx *out, int32_t *regime, int32_t *ok)
{
    for (int64_t i = 0; i < m; ++i) {
        out[i] = orc_gamma_P(n[i], z[i]);
        if (regime) regime[i] = g_regime;
        if (ok) ok[i] = g_converged;
    }
}

void orc_gamma_P_regime_arr(int64_t m, const int32_t *n, const dcplx *z, int32_t regime, dcplx *out)
{
    for (int64_t i = 0; i < m; ++i) out[i] = orc_gamma_P_regime(n[i], z[i], regime);
}

void orc_E_closed_arr(const orc_params *p, int64_t m, const double *t, dcplx *out)
{
    for (int64_t i = 0; i < m; ++i) out[i] = orc_E_closed(p, t[i]);
}

void orc_E_quad_arr(const orc_params *p, int64_t m, const double *t, dcplx *out)
{
    for (int64_t i = 0; i < m; ++i) out[i] = orc_E_quad(p, t[i]);
}

void orc_Jn_quad_arr(const orc_params *p, int n, int64_t m, const double *T, dcplx *out)
{
    for (int64_t i = 0; i < m; ++i) out[i] = orc_Jn_quad(p, n, T[i]);
}

void orc_phi_arr(const orc_params *p, int64_t m, const double *x, dcplx *out)
{
    for (int64_t i = 0; i < m; ++i) out[i] = orc_phi(p, x[i]);
}

void orc_phi_mass_below_arr(const orc_params *p, int64_t m, const double *y, double *out)
{
    for (int64_t i = 0; i < m; ++i) out[i] = phi_mass_below(p, y[i]);
}

void orc_chi0_arr(const orc_params *p, int64_t m, const double *x1, const double *x2, dcplx *out)
{
    for (int64_t i = 0; i < m; ++i) out[i] = orc_chi0(p, x1[i], x2[i]);
}

/* int_{-inf}^{-a} |psi(x, t_r)|^2 dx of the exact solution for rows r = 0..Nt
 * (E as for orc_march) */
void orc_exact_part_arr(const orc_params *p, const dcplx *E, double *out)
{
    const int64_t Nt = p->Nt;
    orc_state s = { p, E, NULL, NULL, NULL, 0.0, NULL, 0, 0, NULL, 0, 0 };
    if (two_photons(p)) s.E2 = E + (Nt + 1);
    for (int64_t r = 0; r <= Nt; ++r) out[r] = exact_part(&s, r);
}
