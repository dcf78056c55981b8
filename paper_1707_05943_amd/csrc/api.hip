// Host side of the C ABI declared in include/fdtd.h.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fdtd_common.h"
#include "nm.h"

static char g_err[512];

static int fail(fdtd_ctx* c, int code, const char* fmt, ...)
{
    char* dst = c ? c->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return code;
}

static int64_t align256(int64_t n) { return (n + 255) & ~(int64_t)255; }

// Scheme coefficients of the solved square (Eq. 3): with
// d = 1/Delta + W/4, psi(j,r) = alpha psi(j-1,r) + cA psi(j-1,r-1) + cB psi(j,r-1) + S/d.
static void coefficients(const fdtd_params* p, Geom* g)
{
    const cd W = mk(0.5 * p->Gamma, p->omega0);
    const cd d = mk(1.0 / p->Delta, 0.0) + 0.25 * W;
    g->W = W;
    g->cinv = cdiv(mk(1.0, 0.0), d);
    g->alpha = (-0.25 * W) * g->cinv;
    g->cB = g->alpha;
    g->cA = (mk(1.0 / p->Delta, 0.0) - 0.25 * W) * g->cinv;
    g->cAm1 = (-0.5 * W) * g->cinv;
}

// columns recomputed left of a block so that the dropped term alpha^halo U is
// below 2^-60 relative
static int halo_for(cd alpha)
{
    const double m = cabs_(alpha);
    if (m == 0.0) return 1;
    const double h = ceil(log(ldexp(1.0, -60)) / log(m));
    return h < 1.0 ? 1 : (int)h;
}

static int plan_for(const fdtd_params* p, const PlanKnobs& kn, Plan* P, char* why, size_t n);

int ctx_validate(const fdtd_params* p, const PlanKnobs& kn, char* why, size_t n)
{
    if (!p) { snprintf(why, n, "params is NULL"); return FDTD_EINVAL; }
    if (p->abi_version != FDTD_ABI_VERSION || p->struct_size != sizeof(fdtd_params)) {
        snprintf(why, n, "abi_version/struct_size mismatch (%u/%u, expected %u/%zu)", p->abi_version,
                 p->struct_size, FDTD_ABI_VERSION, sizeof(fdtd_params));
        return FDTD_EINVAL;
    }
    if (p->D < 2 || (p->D & 1)) { snprintf(why, n, "D = %lld must be even and >= 2", (long long)p->D); return FDTD_EINVAL; }
    if (p->Nx < p->D + 1) { snprintf(why, n, "Nx = %lld must be >= D+1", (long long)p->Nx); return FDTD_EINVAL; }
    if (p->Nt < 1) { snprintf(why, n, "Nt must be >= 1"); return FDTD_EINVAL; }
    if (!(p->Delta > 0.0) || !(p->Gamma > 0.0) || !isfinite(p->Delta) || !isfinite(p->Gamma) ||
        !isfinite(p->omega0) || !isfinite(p->k) || !isfinite(p->alpha) || !isfinite(p->x0) ||
        !isfinite(p->width) || !isfinite(p->phase)) {
        snprintf(why, n, "Delta and Gamma must be > 0 and every parameter finite");
        return FDTD_EINVAL;
    }
    if (p->boundary != FDTD_E_SERIES && p->boundary != FDTD_E_DELAY_ODE) {
        snprintf(why, n, "unknown boundary method %d", p->boundary);
        return FDTD_EINVAL;
    }
    if (p->incident < FDTD_INC_PLANE || p->incident > FDTD_INC_GAUSS2) {
        snprintf(why, n, "unknown incident family %d", p->incident);
        return FDTD_EINVAL;
    }
    if (p->identical_photons != 0 && p->identical_photons != 1) {
        snprintf(why, n, "identical_photons must be 0 or 1");
        return FDTD_EINVAL;
    }
    if (p->read_mode != FDTD_READ_EXACT && p->read_mode != FDTD_READ_PAPER_DIAG) {
        snprintf(why, n, "unknown read mode %d", p->read_mode);
        return FDTD_EINVAL;
    }
    if (p->read_mode == FDTD_READ_EXACT && p->diag_cols != 0) {
        snprintf(why, n, "diag_cols must be 0 unless read_mode is FDTD_READ_PAPER_DIAG");
        return FDTD_EINVAL;
    }
    if (p->read_mode == FDTD_READ_PAPER_DIAG) {
        if (p->diag_cols < 1 || p->diag_cols > ((int64_t)1 << 26)) {
            snprintf(why, n, "FDTD_READ_PAPER_DIAG needs 1 <= diag_cols <= 2^26");
            return FDTD_EINVAL;
        }
        if (p->identical_photons == 0) {
            snprintf(why, n, "FDTD_READ_PAPER_DIAG is for the one-packet families");
            return FDTD_EINVAL;
        }
        // every row of Nx + diag_cols columns is kept
        if ((double)(p->Nt + 1) * (double)(p->Nx + p->diag_cols) * 16.0 > 9.0e18) {
            snprintf(why, n, "FDTD_READ_PAPER_DIAG keeps every row: (Nt+1)(Nx+diag_cols) is too large");
            return FDTD_EINVAL;
        }
    }
    if (p->identical_photons == 0) {
        if (p->incident != FDTD_INC_EXP2) {
            snprintf(why, n, "two different photons are defined for the exponential family (FDTD_INC_EXP2) only");
            return FDTD_EINVAL;
        }
        if (!isfinite(p->k1) || !isfinite(p->k2) || !(p->alpha1 > 0.0) || !(p->alpha2 > 0.0) ||
            !isfinite(p->alpha1) || !isfinite(p->alpha2)) {
            snprintf(why, n, "two different photons need finite k1, k2 and alpha1, alpha2 > 0");
            return FDTD_EINVAL;
        }
    } else if ((p->incident == FDTD_INC_EXP1 || p->incident == FDTD_INC_EXP2) && !(p->alpha > 0.0)) {
        snprintf(why, n, "exponential packets need alpha > 0");
        return FDTD_EINVAL;
    }
    if (p->incident == FDTD_INC_GAUSS2 && (!(p->width > 0.0) || p->x0 > -0.5 * p->D * p->Delta)) {
        snprintf(why, n, "Gaussian packets need width > 0 and x0 <= -a");
        return FDTD_EINVAL;
    }
    Geom g;
    coefficients(p, &g);
    if (halo_for(g.alpha) > MAX_HALO) {
        snprintf(why, n, "|alpha| = %.3g needs a halo of more than %d columns: Delta too coarse for |W|",
                 cabs_(g.alpha), MAX_HALO);
        return FDTD_EINVAL;
    }
    Plan P;
    return plan_for(p, kn, &P, why, n);
}

static int validate(const fdtd_params* p, char* why, size_t n) { return ctx_validate(p, SOLO_KNOBS, why, n); }

struct Layout {
    int64_t ring, Md, Et, Phi, Drv, Pex, Ppart, Pe, chi, Ebuf, status, Gn, ode, odeinst, Epart, E0, Mu, mupart, hist,
        stage, total;
};

// ring rows: the delay reaches D+1 rows back; the strip runs one block of T
// rows ahead of the outgoing region and a launch may write up to 2T rows
// past the oldest row it still reads
static int64_t ring_rows(const fdtd_params* p, const Plan& P) { return p->D + 2 * (int64_t)P.T + 2; }

static Layout layout(const fdtd_params* p, const Plan& P)
{
    Layout L;
    const int64_t C = p->Nx + 1, R = ring_rows(p, P), n = p->Nt + 1, nblk = P.nwg;
    int64_t off = 0;
    L.ring = off; off += align256(R * C * 16);
    L.Md = off; off += align256(R * (p->D + 1) * 16);
    // the paper's own reads reach phi(-a - q Delta) for q up to Nt + diag_cols + D
    const int64_t n_phi = p->read_mode == FDTD_READ_PAPER_DIAG ? n + p->diag_cols + p->D : n;
    L.Et = off; off += align256(n * 16);
    L.Phi = off; off += align256(n_phi * 16);
    L.Drv = off; off += align256(n * 16);
    L.Pex = off; off += align256(n * 8);
    L.Ppart = off; off += align256(n * nblk * 8);
    L.Pe = off; off += align256(n * 8);
    L.chi = off; off += align256(C * 16);
    L.Ebuf = off; off += align256(n * 16);
    L.status = off; off += 256;
    L.Gn = off; off += align256((p->D + 1) * ODE_P * 16);
    L.ode = off; off += align256((int64_t)sizeof(OdeTab));
    L.odeinst = off; off += align256((int64_t)sizeof(OdeInst));
    L.Epart = -1;
    if (p->incident == FDTD_INC_GAUSS2 && p->boundary == FDTD_E_SERIES) {
        L.Epart = off;
        off += align256((int64_t)EPART_CHUNKS * n * 16);
    }
    // stimulated emission: e0, mu and mu's per-row partial sums (App. D)
    L.E0 = L.Mu = L.mupart = -1;
    if (p->incident == FDTD_INC_EXP1) {
        L.E0 = off; off += align256(n * 16);
        L.Mu = off; off += align256(n * 16);
        L.mupart = off; off += align256(n * NM_BLOCKS * 16);
    }
    L.hist = L.stage = -1;
    if (p->read_mode == FDTD_READ_PAPER_DIAG) {
        L.hist = off; off += align256(n * (p->Nx + p->diag_cols) * 16);
        L.stage = off; off += align256(p->diag_cols * 16);
    }
    L.total = off;
    return L;
}

// Gauss-Legendre rule on [-1, 1] (Newton on the Legendre recurrence)
static void gl_rule(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// What the collocation weights of one step of the delay equation (OdeTab)
// need that does not depend on the instance, in units of Delta: the nodes
// s_i = tau_i / Delta (Gauss-Legendre on (0, 1), then s_P = 1), and for the
// integral over (0, s_i) of row i its NQ Gauss-Legendre nodes u, their
// weights and the Lagrange basis of the nodes s_0..s_{P-1} at them.
constexpr int ODE_NQ = 48;
struct OdeUnit {
    double s[ODE_P + 1];
    double u[ODE_P + 1][ODE_NQ];
    double wq[ODE_P + 1][ODE_NQ];
    double l[ODE_P + 1][ODE_NQ][ODE_P];
};

static OdeUnit make_ode_unit()
{
    OdeUnit U;
    double x[ODE_P], w[ODE_P], xq[ODE_NQ], wq[ODE_NQ];
    gl_rule(ODE_P, x, w);
    gl_rule(ODE_NQ, xq, wq);
    for (int i = 0; i < ODE_P; ++i) U.s[i] = 0.5 * (1.0 + x[i]);
    U.s[ODE_P] = 1.0;
    for (int i = 0; i <= ODE_P; ++i) {
        for (int q = 0; q < ODE_NQ; ++q) {
            const double u = 0.5 * U.s[i] * (1.0 + xq[q]);
            U.u[i][q] = u;
            U.wq[i][q] = 0.5 * U.s[i] * wq[q];
            for (int j = 0; j < ODE_P; ++j) {
                double lj = 1.0;
                for (int k = 0; k < ODE_P; ++k)
                    if (k != j) lj *= (u - U.s[k]) / (U.s[j] - U.s[k]);
                U.l[i][q][j] = lj;
            }
        }
    }
    return U;
}

static const OdeUnit& ode_unit()
{
    static const OdeUnit U = make_ode_unit();
    return U;
}

// collocation weights of one step of the delay equation (OdeTab): tau_i =
// Delta s_i, ew_i = e^{-W tau_i} and M_ij = int_0^{tau_i} l_j(u) e^{-W (tau_i
// - u)} du by the quadrature of OdeUnit
static void ode_table(const Geom& g, OdeTab* T)
{
    const OdeUnit& U = ode_unit();
    const double h = g.Delta;
    for (int i = 0; i <= ODE_P; ++i) {
        const double ti = h * U.s[i];
        T->tau[i] = ti;
        T->ew[i] = cexp_(-(g.W * ti));
        cd acc[ODE_P];
        for (int j = 0; j < ODE_P; ++j) acc[j] = mk(0.0, 0.0);
        for (int q = 0; q < ODE_NQ; ++q) {
            const cd e = cexp_(-(g.W * (h * (U.s[i] - U.u[i][q]))));
            const double wt = h * U.wq[i][q];
            for (int j = 0; j < ODE_P; ++j) acc[j] += (wt * U.l[i][q][j]) * e;
        }
        for (int j = 0; j < ODE_P; ++j) T->M[i][j] = acc[j];
    }
}

static int plan_for(const fdtd_params* p, const PlanKnobs& kn, Plan* P, char* why, size_t n)
{
    Geom g;
    coefficients(p, &g);
    return make_plan(p, halo_for(g.alpha), kn, P, why, n);
}

static int two_photons(const fdtd_params* p) { return p->incident == FDTD_INC_EXP2 && p->identical_photons == 0; }

// a context's workspace: one march, or for two different photons two marches
// and the row sums of |psi_a + psi_b|^2
static int64_t ctx_total(const fdtd_params* p, const Plan& P)
{
    const int64_t one = layout(p, P).total;
    if (!two_photons(p)) return one;
    return 2 * one + align256((p->Nt + 1) * PAIR_CHUNKS * 8);
}

int64_t ctx_bytes(const fdtd_params* p, const PlanKnobs& kn)
{
    char why[256];
    Plan P;
    if (plan_for(p, kn, &P, why, sizeof why)) return -1;
    return ctx_total(p, P);
}

// A of Eq. (11): chi(x1, x2, 0) = (A/sqrt 2)[phi1(x1) phi2(x2) + phi1(x2) phi2(x1)] has unit norm
static double two_photon_A(const fdtd_params* p)
{
    const double dk = p->k1 - p->k2, s = (p->alpha1 + p->alpha2) * p->Gamma;
    const double num = 4.0 * dk * dk + s * s;
    return sqrt(num / (num + 4.0 * p->alpha1 * p->alpha2 * p->Gamma * p->Gamma));
}

// One march in *c over the workspace at `base` (layout L): photon 0 for the
// one-packet families; for two different photons 2 (march a: photon 2's e0
// and drive) or 1 (march b: photon 1's).  Enqueues the clearing of the ring
// and the copies of the boundary's step weights and waits for them; with
// `defer` it does neither and hands the step weights and the launch record
// to the caller (see CtxDefer).
static int march_setup(fdtd_ctx* c, const fdtd_params* p, const Plan& P, const Layout& L, char* base, int photon,
                       hipStream_t stream, char* why, size_t nwhy, const CtxDefer* defer)
{
    const int64_t nblk = P.nwg;
    int rc = FDTD_OK;
    memset(c, 0, sizeof *c);
    c->p = *p;
    c->stream = stream;
    c->nblk = nblk;
    c->plan = P;
    Geom& g = c->g;
    g.Nx = p->Nx; g.D = p->D; g.Nt = p->Nt; g.C = p->Nx + 1; g.R = ring_rows(p, P); g.Mc = p->D + 1;
    g.Delta = p->Delta; g.a = 0.5 * (double)p->D * p->Delta; g.Gamma = p->Gamma;
    coefficients(p, &g);
    g.halo = halo_for(g.alpha);

    Packet& pk = c->pk;
    pk.incident = p->incident; pk.k = p->k; pk.alpha = p->alpha; pk.x0 = p->x0; pk.width = p->width;
    pk.phase = p->phase; pk.Gamma = p->Gamma; pk.a = g.a;
    const cd eth = mk(cos(p->phase), sin(p->phase));
    if (p->incident == FDTD_INC_EXP1) {
        pk.c_ex = mk(1.0, 0.0);      // Eq. (8): psi = phi(x-t) e1(t)
        pk.c_drive = mk(0.0, 0.0);   // no two-photon component
    } else if (photon) {
        // Eq. (12): psi = A e^{i theta} [phi1(x-t) e0^(2)(t) + phi2(x-t) e0^(1)(t)]; this march takes one
        // packet's e0 and drive (Eq. 10's chi0 in line 4 of Eq. 1), the other packet's phi on the x - t grid
        const double A = two_photon_A(p);
        pk.k = photon == 1 ? p->k1 : p->k2;
        pk.alpha = photon == 1 ? p->alpha1 : p->alpha2;
        pk.c_ex = A * eth;
        pk.c_drive = (sqrt(p->Gamma) * A / sqrt(2.0)) * eth;
    } else {
        pk.c_ex = sqrt(2.0) * eth;   // Eq. (12), identical photons: sqrt(2) phi(x-t) E(t)
        pk.c_drive = sqrt(p->Gamma) * eth;
    }

    Bufs& b = c->b;
    b.ring = (cd*)(base + L.ring);
    b.Md = (cd*)(base + L.Md);
    b.Et = (cd*)(base + L.Et);
    b.Phi = (cd*)(base + L.Phi);
    b.Drv = (cd*)(base + L.Drv);
    b.Pex = (double*)(base + L.Pex);
    b.Ppart = (double*)(base + L.Ppart);
    b.Pe = (double*)(base + L.Pe);
    b.chi = (cd*)(base + L.chi);
    b.Ebuf = (cd*)(base + L.Ebuf);
    b.status = (int*)(base + L.status);
    b.Gn = (cd*)(base + L.Gn);
    b.ode = (OdeTab*)(base + L.ode);
    b.Epart = L.Epart >= 0 ? (cd*)(base + L.Epart) : nullptr;
    c->d_ode = (OdeInst*)(base + L.odeinst);
    c->E0 = L.E0 >= 0 ? (cd*)(base + L.E0) : nullptr;
    c->Mu = L.Mu >= 0 ? (cd*)(base + L.Mu) : nullptr;
    c->mupart = L.mupart >= 0 ? (cd*)(base + L.mupart) : nullptr;
    b.hist = L.hist >= 0 ? (cd*)(base + L.hist) : nullptr;
    c->stage = L.stage >= 0 ? (cd*)(base + L.stage) : nullptr;
    c->dc = p->read_mode == FDTD_READ_PAPER_DIAG ? p->diag_cols : 0;
    c->mu_row = -1;
    c->row = -1;
    c->strip_row = -1;
    c->boundary_ready = 0;
    if (defer) {
        b.ode = defer->d_tab;
        c->d_ode = nullptr;
    } else {
        rc = launch_clear(c);
        if (rc) {
            snprintf(why, nwhy, "clearing the ring failed: %s", hipGetErrorString(hipGetLastError()));
            return rc;
        }
    }
    // the delay-equation boundary's step weights and launch record
    OdeTab tab;
    ode_table(g, &tab);
    OdeInst oi;
    memset(&oi, 0, sizeof oi);
    oi.g = g;
    oi.pk = pk;
    oi.b = b;
    oi.nblk = nblk;
    if (defer) {
        *defer->h_tab = tab;
        *defer->h_inst = oi;
        return FDTD_OK;
    }
    hipError_t e = hipMemcpyAsync(b.ode, &tab, sizeof tab, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->d_ode, &oi, sizeof oi, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        snprintf(why, nwhy, "copy of the boundary tables failed: %s", hipGetErrorString(e));
        return FDTD_EDEVICE;
    }
    return FDTD_OK;
}

// Fill the context *c (caller's storage; for two different photons also
// *pair, march b) for parameters p over the caller's workspace.  Allocates
// nothing.
static int ctx_setup(fdtd_ctx* c, fdtd_ctx* pair, const fdtd_params* p, const PlanKnobs& kn, void* d_workspace,
                     size_t bytes, hipStream_t stream, char* why, size_t nwhy, const CtxDefer* defer = nullptr)
{
    int rc = ctx_validate(p, kn, why, nwhy);
    if (rc) return rc;
    Plan P;
    plan_for(p, kn, &P, why, nwhy);
    const Layout L = layout(p, P);
    const int64_t total = ctx_total(p, P);
    if (!d_workspace || bytes < (size_t)total) {
        snprintf(why, nwhy, "workspace of %zu bytes is smaller than the %lld needed", bytes, (long long)total);
        return FDTD_ESIZE;
    }
    if (((uintptr_t)d_workspace) & 255) { snprintf(why, nwhy, "workspace must be 256-byte aligned"); return FDTD_EINVAL; }
    const int two = two_photons(p);
    if (two && !pair) { snprintf(why, nwhy, "two different photons need the second march's context"); return FDTD_EINVAL; }
    if (two && defer) { snprintf(why, nwhy, "two different photons are set up one instance at a time"); return FDTD_EINVAL; }
    char* base = (char*)d_workspace;
    rc = march_setup(c, p, P, L, base, two ? 2 : 0, stream, why, nwhy, defer);
    if (rc || !two) return rc;
    rc = march_setup(pair, p, P, L, base + L.total, 1, stream, why, nwhy, nullptr);
    if (rc) return rc;
    c->pair = pair;
    c->xpart = (double*)(base + 2 * L.total);
    c->c0_pair = (two_photon_A(p) / sqrt(2.0)) * mk(cos(p->phase), sin(p->phase));
    return FDTD_OK;
}

int ctx_create(const fdtd_params* p, const PlanKnobs& kn, void* d_workspace, size_t bytes, hipStream_t stream,
               fdtd_ctx** out, char* why, size_t nwhy, const CtxDefer* defer)
{
    int rc = ctx_validate(p, kn, why, nwhy);
    if (rc) return rc;
    if (!out) { snprintf(why, nwhy, "out is NULL"); return FDTD_EINVAL; }
    *out = nullptr;
    fdtd_ctx* c = (fdtd_ctx*)calloc(1, sizeof(fdtd_ctx));
    fdtd_ctx* pair = two_photons(p) ? (fdtd_ctx*)calloc(1, sizeof(fdtd_ctx)) : nullptr;
    if (!c || (two_photons(p) && !pair)) {
        free(c);
        free(pair);
        snprintf(why, nwhy, "out of host memory");
        return FDTD_EDEVICE;
    }
    rc = ctx_setup(c, pair, p, kn, d_workspace, bytes, stream, why, nwhy, defer);
    if (rc) {
        free(pair);
        free(c);
        return rc;
    }
    *out = c;
    return FDTD_OK;
}

int ctx_boundary_enqueue(fdtd_ctx* c)
{
    c->boundary_ready = 0;
    int rc = launch_boundary(c, 0);
    if (rc) return fail(c, rc, "boundary launch failed: %s", hipGetErrorString(hipGetLastError()));
    return FDTD_OK;
}

int ctx_boundary_status(fdtd_ctx* c, int st)
{
    if (st & STATUS_GAMMA_RANGE) return fail(c, FDTD_ERANGE, "gamma(n,z) series out of range");
    if (st & STATUS_NONFINITE) return fail(c, FDTD_ERANGE, "non-finite boundary value");
    c->row = 0;
    c->strip_row = 0;
    c->mu_row = c->mupart ? 0 : -1;
    c->boundary_ready = 1;
    return FDTD_OK;
}

extern "C" {

int fdtd_workspace_size(const fdtd_params* p, size_t* bytes)
{
    char why[256];
    int rc = validate(p, why, sizeof why);
    if (rc) return fail(nullptr, rc, "%s", why);
    if (!bytes) return fail(nullptr, FDTD_EINVAL, "bytes is NULL");
    *bytes = (size_t)ctx_bytes(p, SOLO_KNOBS);
    return FDTD_OK;
}

int fdtd_init(const fdtd_params* p, void* d_workspace, size_t bytes, void* hip_stream, fdtd_ctx** out)
{
    char why[256];
    int rc = ctx_create(p, SOLO_KNOBS, d_workspace, bytes, (hipStream_t)hip_stream, out, why, sizeof why);
    if (rc) return fail(nullptr, rc, "%s", why);
    return FDTD_OK;
}

// enqueue the copy of the status word(s) into st[0..1] (the second march's
// for two different photons, else 0); the caller waits for the stream
static hipError_t status_copy(fdtd_ctx* c, int* st)
{
    st[0] = st[1] = 0;
    hipError_t e = hipMemcpyAsync(&st[0], c->b.status, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && c->pair)
        e = hipMemcpyAsync(&st[1], c->pair->b.status, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    return e;
}

// the boundary of one march, or of both marches of two different photons:
// march a takes photon 2's e0 and drive but photon 1's packet on the x - t
// grid, march b the reverse, so each march's boundary kernels write their phi
// table into the other march's; then the exact part of P_e (with the
// packets' cross term) and row 0's sum of |psi_a + psi_b|^2
static int boundary_enqueue(fdtd_ctx* c, int from_host)
{
    if (!c->pair) return launch_boundary(c, from_host);
    fdtd_ctx* m[2] = {c, c->pair};
    for (int i = 0; i < 2; ++i) {
        fdtd_ctx t = *m[i];
        t.b.Phi = m[1 - i]->b.Phi;
        int rc = launch_boundary(&t, from_host);
        if (rc) return rc;
    }
    int rc = launch_pex_pair(c);
    if (!rc) rc = launch_pair_rows(c, 0, 0);
    return rc;
}

static void boundary_done(fdtd_ctx* c)
{
    for (fdtd_ctx* m = c; m; m = (m == c) ? c->pair : nullptr) {
        m->row = 0;
        m->strip_row = 0;
        m->mu_row = m->mupart ? 0 : -1;
        m->boundary_ready = 1;
    }
}

static int check_status(fdtd_ctx* c)
{
    int sts[2];
    hipError_t e = status_copy(c, sts);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, FDTD_EDEVICE, "HIP error: %s", hipGetErrorString(e));
    const int st = sts[0] | sts[1];
    if (st & STATUS_GAMMA_RANGE) return fail(c, FDTD_ERANGE, "gamma(n,z) series out of range");
    if (st & STATUS_NONFINITE) return fail(c, FDTD_ERANGE, "non-finite boundary value");
    return FDTD_OK;
}

// the march's part of the status word
static int march_status(fdtd_ctx* c, int st)
{
    if (st & STATUS_MARCH_NONFINITE)
        return fail(c, FDTD_ERANGE, "non-finite value (NaN or infinity) in the march, rows 1..%lld",
                    (long long)c->row);
    return FDTD_OK;
}

int fdtd_set_boundary(fdtd_ctx* c)
{
    if (!c) return fail(nullptr, FDTD_EINVAL, "ctx is NULL");
    int rc = boundary_enqueue(c, 0);
    if (rc) return fail(c, rc, "boundary launch failed: %s", hipGetErrorString(hipGetLastError()));
    rc = check_status(c);
    if (rc) return rc;
    boundary_done(c);
    return FDTD_OK;
}

int fdtd_set_boundary_tables(fdtd_ctx* c, const double* h_E, int64_t n)
{
    if (!c) return fail(nullptr, FDTD_EINVAL, "ctx is NULL");
    const int64_t n1 = c->p.Nt + 1;
    if (!h_E || n != (c->pair ? 2 : 1) * n1)
        return fail(c, FDTD_ESIZE, "expected %s%lld values", c->pair ? "2 (Nt+1) = " : "Nt+1 = ",
                    (long long)((c->pair ? 2 : 1) * n1));
    // two different photons: e0^(1) then e0^(2); march a takes e0^(2), march b e0^(1)
    hipError_t e = hipMemcpyAsync(c->b.Ebuf, h_E + (c->pair ? 2 * n1 : 0), (size_t)n1 * 16, hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess && c->pair)
        e = hipMemcpyAsync(c->pair->b.Ebuf, h_E, (size_t)n1 * 16, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return fail(c, FDTD_EDEVICE, "copy of E failed: %s", hipGetErrorString(e));
    int rc = boundary_enqueue(c, 1);
    if (rc) return fail(c, rc, "boundary launch failed: %s", hipGetErrorString(hipGetLastError()));
    rc = check_status(c);
    if (rc) return rc;
    boundary_done(c);
    return FDTD_OK;
}

// Launch schedule.  Rows are grouped in blocks [1 + kT, (k+1)T].  A launch
// marches the outgoing region over (a prefix of) one block and the strip
// over the next block.  A march that stopped inside a block resumes from the
// block's first row, so every row is computed from the same block start
// whatever the call boundaries (the results are bitwise the same).
// mu's row sums (stimulated emission) are taken of complete rows while the
// ring still holds them.  Rows wait for several launches and go in one
// launch of up to MU_ROWS rows: before a launch that would overwrite the
// oldest waiting row (it writes rows up to w; the slot of row p comes back
// at p + R), once MU_ROWS rows wait, and at the end of the call.  (On a
// second stream beside the march these sums would take CUs the next march
// launch needs whole, and delay it more than they save.)
constexpr int64_t MU_ROWS = 256;

static int march_to(fdtd_ctx* c, int64_t target)
{
    if (c->dc) {
        // the paper's own reads: one launch per row over every marched column
        const int64_t first = c->row + 1;
        for (int64_t r = first; r <= target; ++r) {
            int rc = launch_diag_row(c, r);
            if (rc) return rc;
        }
        c->row = c->strip_row = target;
        return launch_check_rows(c, first, target);
    }
    const int64_t T = c->plan.T, Nt = c->p.Nt, R = c->g.R;
    const int64_t first = c->row + 1;                 // rows this call completes: first..target
    int64_t p0 = -1, p1 = -1;     // complete rows waiting for their row sums (mu; |psi_a + psi_b|^2)
    auto flush = [&]() -> int {
        if (p0 < 0) return FDTD_OK;
        int rc = FDTD_OK;
        if (c->mupart) rc = launch_mu_rows(c, p0, p1, c->stream);
        if (!rc && c->pair) rc = launch_pair_rows(c, p0, p1);
        if (rc) return rc;
        if (c->mupart) c->mu_row = p1;
        p0 = p1 = -1;
        return FDTD_OK;
    };
    // a launch of the march, and of the second march of two different photons
    // (the same plan: the two advance in lock step)
    auto block = [&](int64_t a0, int64_t a1, int64_t b0, int64_t b1) -> int {
        int rc = launch_block(c, a0, a1, b0, b1);
        if (!rc && c->pair) rc = launch_block(c->pair, a0, a1, b0, b1);
        return rc;
    };
    while (c->row < target) {
        const int64_t m0 = 1 + T * (c->row / T);
        const int64_t m1 = (m0 + T - 1 < target) ? m0 + T - 1 : target;
        int64_t s0 = c->strip_row + 1, s1 = -1;
        if (s0 <= Nt && s0 <= m0 + T) s1 = (s0 + T - 1 < Nt) ? s0 + T - 1 : Nt;
        const bool strip_only = c->strip_row < m1;
        const int64_t w = strip_only ? s1 : (s1 > m1 ? s1 : m1);
        if (p0 >= 0 && w - p0 >= R) {
            int rc = flush();
            if (rc) return rc;
        }
        if (strip_only) {
            // the strip must hold every row this block reads: march it alone first
            int rc = block(1, 0, s0, s1);
            if (rc) return rc;
            c->strip_row = s1;
            continue;
        }
        int rc = block(m0, m1, s1 >= s0 ? s0 : 1, s1 >= s0 ? s1 : 0);
        if (rc) return rc;
        if (c->mupart || c->pair) {
            if (p0 < 0) p0 = m0;
            p1 = m1;
            if (p1 - p0 + 1 >= MU_ROWS && (rc = flush())) return rc;
        }
        c->row = m1;
        if (s1 >= s0) c->strip_row = s1;
    }
    int rc = flush();
    if (rc) return rc;
    // a NaN or infinity anywhere in the rows just marched sets the status word
    // (reported by fdtd_sync and by readouts into host memory)
    rc = launch_check_rows(c, first, target);
    if (!rc && c->pair) {
        c->pair->row = c->row;
        c->pair->strip_row = c->strip_row;
        rc = launch_check_rows(c->pair, first, target);
    }
    return rc;
}

int fdtd_march(fdtd_ctx* c, int64_t n_rows)
{
    if (!c) return fail(nullptr, FDTD_EINVAL, "ctx is NULL");
    if (!c->boundary_ready) return fail(c, FDTD_ESTATE, "march before set_boundary");
    if (n_rows < 0) return fail(c, FDTD_EINVAL, "n_rows < 0");
    if (c->row + n_rows > c->p.Nt) return fail(c, FDTD_ESTATE, "march past Nt = %lld", (long long)c->p.Nt);
    if (n_rows == 0) return FDTD_OK;
    int rc = march_to(c, c->row + n_rows);
    if (rc) return fail(c, rc, "march launch failed: %s", hipGetErrorString(hipGetLastError()));
    return FDTD_OK;
}

int fdtd_current_row(const fdtd_ctx* c, int64_t* row)
{
    if (!c || !row) return FDTD_EINVAL;
    *row = c->row;
    return FDTD_OK;
}

int fdtd_readout(fdtd_ctx* c, int32_t what, int64_t arg, void* dst, int64_t count, int32_t dst_on_device)
{
    if (!c) return fail(nullptr, FDTD_EINVAL, "ctx is NULL");
    if (!dst || count < 0) return fail(c, FDTD_EINVAL, "bad destination");
    if (!c->boundary_ready) return fail(c, FDTD_ESTATE, "readout before set_boundary");
    size_t esz = 16;
    void* src = nullptr;
    int rc = FDTD_OK;
    switch (what) {
    case FDTD_RO_ROW:
        if (count != c->p.Nx + 1) return fail(c, FDTD_ESIZE, "a row has Nx+1 = %lld values", (long long)(c->p.Nx + 1));
        if (arg < 0 || arg > c->row || (!c->dc && arg < c->row - (c->p.D + 1)))
            return fail(c, FDTD_ESTATE, "row %lld is not held (current %lld)", (long long)arg, (long long)c->row);
        // stage through the chi scratch (it holds Nx+1 values)
        rc = c->pair ? launch_row_pair(c, arg, dst_on_device ? (cd*)dst : c->b.chi)
                     : launch_row_readout(c, arg, dst_on_device ? (cd*)dst : c->b.chi);
        if (dst_on_device) return rc ? fail(c, FDTD_EDEVICE, "launch failed") : FDTD_OK;
        src = c->b.chi;
        break;
    case FDTD_RO_PE:
        esz = 8;
        if (count > c->row + 1) return fail(c, FDTD_ESTATE, "only %lld rows marched", (long long)(c->row + 1));
        rc = c->pair ? launch_pe_pair(c, count, dst_on_device ? (double*)dst : c->b.Pe)
                     : launch_pe_final(c, count, dst_on_device ? (double*)dst : c->b.Pe);
        if (dst_on_device) return rc ? fail(c, rc, "launch failed") : FDTD_OK;
        src = c->b.Pe;
        break;
    case FDTD_RO_LEFT:
        if (!c->dc) return fail(c, FDTD_EINVAL, "the left columns are marched with FDTD_READ_PAPER_DIAG only");
        if (count != c->dc) return fail(c, FDTD_ESIZE, "the left columns are diag_cols = %lld values", (long long)c->dc);
        if (arg < 0 || arg > c->row)
            return fail(c, FDTD_ESTATE, "row %lld is not marched (current %lld)", (long long)arg, (long long)c->row);
        rc = launch_diag_copy(c, arg, 1 - c->dc, c->dc, dst_on_device ? (cd*)dst : c->stage);
        if (dst_on_device) return rc ? fail(c, FDTD_EDEVICE, "launch failed") : FDTD_OK;
        src = c->stage;
        break;
    case FDTD_RO_CHI:
        if (c->dc) return fail(c, FDTD_EINVAL, "chi is not read out with FDTD_READ_PAPER_DIAG");
        if (count > c->p.Nx - c->p.D) return fail(c, FDTD_ESIZE, "at most Nx-D = %lld detector separations",
                                                  (long long)(c->p.Nx - c->p.D));
        rc = c->pair ? launch_chi_pair(c, c->row, count, dst_on_device ? (cd*)dst : c->b.chi)
                     : launch_chi(c, c->row, count, dst_on_device ? (cd*)dst : c->b.chi);
        if (dst_on_device) return rc ? fail(c, rc, "launch failed") : FDTD_OK;
        src = c->b.chi;
        break;
    case FDTD_RO_MU:
        if (c->dc) return fail(c, FDTD_EINVAL, "the measures of App. D are not read out with FDTD_READ_PAPER_DIAG");
        if (!c->mupart) return fail(c, FDTD_EINVAL, "mu is defined for stimulated emission (FDTD_INC_EXP1) only");
        if (count > c->mu_row + 1)
            return fail(c, FDTD_ESTATE, "mu holds %lld rows (fdtd_march accumulates it, batches do not)",
                        (long long)(c->mu_row + 1));
        rc = launch_mu_final(c, count, dst_on_device ? (cd*)dst : c->Mu);
        if (dst_on_device) return rc ? fail(c, rc, "launch failed") : FDTD_OK;
        src = c->Mu;
        break;
    case FDTD_RO_LAMBDA:
        if (c->dc) return fail(c, FDTD_EINVAL, "the measures of App. D are not read out with FDTD_READ_PAPER_DIAG");
        esz = 8;
        if (!c->E0) return fail(c, FDTD_EINVAL, "lambda is defined for stimulated emission (FDTD_INC_EXP1) only");
        if (count > c->row + 1) return fail(c, FDTD_ESTATE, "only %lld rows marched", (long long)(c->row + 1));
        rc = launch_lambda_final(c, count, dst_on_device ? (double*)dst : c->b.Pe);
        if (dst_on_device) return rc ? fail(c, rc, "launch failed") : FDTD_OK;
        src = c->b.Pe;
        break;
    case FDTD_RO_NGEO:
        if (c->dc) return fail(c, FDTD_EINVAL, "the measures of App. D are not read out with FDTD_READ_PAPER_DIAG");
        esz = 8;
        if (!c->mupart) return fail(c, FDTD_EINVAL, "N_geo is defined for stimulated emission (FDTD_INC_EXP1) only");
        if (count != 1) return fail(c, FDTD_ESIZE, "N_geo is one value");
        if (arg < 0 || arg > c->mu_row)
            return fail(c, FDTD_ESTATE, "mu holds rows 0..%lld", (long long)c->mu_row);
        rc = launch_ngeo(c, arg, dst_on_device ? (double*)dst : (double*)c->b.chi);
        if (dst_on_device) return rc ? fail(c, rc, "launch failed") : FDTD_OK;
        src = c->b.chi;
        break;
    case FDTD_RO_E: {
        if (count > c->p.Nt + 1) return fail(c, FDTD_ESIZE, "E has Nt+1 values");
        if (arg != 0 && !(c->pair && arg == 1))
            return fail(c, FDTD_EINVAL, "E: arg selects the photon (0, or 1 for the second of two different photons)");
        // two different photons: march b carries photon 1's e0, march a photon 2's
        const cd* Et = c->pair ? (arg == 0 ? c->pair->b.Et : c->b.Et) : c->b.Et;
        if (dst_on_device) {
            hipError_t e = hipMemcpyAsync(dst, Et, (size_t)count * 16, hipMemcpyDeviceToDevice, c->stream);
            return e == hipSuccess ? FDTD_OK : fail(c, FDTD_EDEVICE, "%s", hipGetErrorString(e));
        }
        src = (void*)Et;
        break;
    }
    default:
        return fail(c, FDTD_EINVAL, "unknown readout %d", what);
    }
    if (rc) return fail(c, rc, "readout launch failed");
    int st[2];
    hipError_t e = hipMemcpyAsync(dst, src, (size_t)count * esz, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = status_copy(c, st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, FDTD_EDEVICE, "readout copy failed: %s", hipGetErrorString(e));
    return march_status(c, st[0] | st[1]);
}

// checkpoint: a header, then the context's workspace (ring, diagonal copy,
// tables, partial sums) byte for byte
static int64_t ws_bytes(const fdtd_ctx* c) { return ctx_total(&c->p, c->plan); }
struct CkptHeader {
    char magic[8];
    uint32_t version, header_bytes;
    fdtd_params p;
    int64_t row, strip_row, boundary_ready, ws_bytes, mu_row;
};
static const char CKPT_MAGIC[8] = {'F', 'D', 'T', 'D', 'C', 'K', 'P', '1'};
static const uint32_t CKPT_VERSION = 2;

int fdtd_checkpoint_size(const fdtd_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return FDTD_EINVAL;
    *bytes = sizeof(CkptHeader) + (size_t)ws_bytes(c);
    return FDTD_OK;
}

int fdtd_checkpoint(fdtd_ctx* c, void* h_dst, size_t bytes)
{
    if (!c) return fail(nullptr, FDTD_EINVAL, "ctx is NULL");
    if (!h_dst) return fail(c, FDTD_EINVAL, "destination is NULL");
    const size_t need = sizeof(CkptHeader) + (size_t)ws_bytes(c);
    if (bytes < need) return fail(c, FDTD_ESIZE, "checkpoint needs %zu bytes", need);
    CkptHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, CKPT_MAGIC, sizeof h.magic);
    h.version = CKPT_VERSION;
    h.header_bytes = (uint32_t)sizeof h;
    h.p = c->p;
    h.row = c->row;
    h.strip_row = c->strip_row;
    h.boundary_ready = c->boundary_ready;
    h.ws_bytes = ws_bytes(c);
    h.mu_row = c->mu_row;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((char*)h_dst + sizeof h, c->b.ring, (size_t)ws_bytes(c), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, FDTD_EDEVICE, "checkpoint copy failed: %s", hipGetErrorString(e));
    memcpy(h_dst, &h, sizeof h);
    return FDTD_OK;
}

int fdtd_restore(fdtd_ctx* c, const void* h_src, size_t bytes)
{
    if (!c) return fail(nullptr, FDTD_EINVAL, "ctx is NULL");
    if (!h_src || bytes < sizeof(CkptHeader)) return fail(c, FDTD_EINVAL, "not a checkpoint");
    CkptHeader h;
    memcpy(&h, h_src, sizeof h);
    if (memcmp(h.magic, CKPT_MAGIC, sizeof h.magic) || h.version != CKPT_VERSION || h.header_bytes != sizeof h)
        return fail(c, FDTD_EINVAL, "not a checkpoint of this library");
    if (memcmp(&h.p, &c->p, sizeof h.p) || h.ws_bytes != ws_bytes(c))
        return fail(c, FDTD_EINVAL, "checkpoint of other parameters");
    if (bytes < sizeof h + (size_t)h.ws_bytes) return fail(c, FDTD_ESIZE, "checkpoint is truncated");
    hipError_t e = hipMemcpyAsync(c->b.ring, (const char*)h_src + sizeof h, (size_t)h.ws_bytes,
                                  hipMemcpyHostToDevice, c->stream);
    // the delay-equation launch records hold this context's device pointers
    OdeInst oi[2];
    memset(oi, 0, sizeof oi);
    fdtd_ctx* m[2] = {c, c->pair};
    for (int i = 0; i < 2 && m[i] && e == hipSuccess; ++i) {
        oi[i].g = m[i]->g;
        oi[i].pk = m[i]->pk;
        oi[i].b = m[i]->b;
        oi[i].nblk = m[i]->nblk;
        e = hipMemcpyAsync(m[i]->d_ode, &oi[i], sizeof oi[i], hipMemcpyHostToDevice, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, FDTD_EDEVICE, "restore copy failed: %s", hipGetErrorString(e));
    for (int i = 0; i < 2 && m[i]; ++i) {
        m[i]->row = h.row;
        m[i]->strip_row = h.strip_row;
        m[i]->boundary_ready = (int)h.boundary_ready;
        m[i]->mu_row = h.mu_row;
    }
    return FDTD_OK;
}

int fdtd_sync(fdtd_ctx* c)
{
    if (!c) return fail(nullptr, FDTD_EINVAL, "ctx is NULL");
    int st[2];
    hipError_t e = status_copy(c, st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, FDTD_EDEVICE, "%s", hipGetErrorString(e));
    return march_status(c, st[0] | st[1]);
}

int fdtd_destroy(fdtd_ctx* c)
{
    if (c) free(c->pair);
    free(c);
    return FDTD_OK;
}

int fdtd_describe(const fdtd_params* p, char* buf, size_t n)
{
    char why[256];
    int rc = validate(p, why, sizeof why);
    if (rc) return fail(nullptr, rc, "%s", why);
    if (!buf || n == 0) return fail(nullptr, FDTD_EINVAL, "buf is NULL");
    Plan P;
    plan_for(p, SOLO_KNOBS, &P, why, sizeof why);
    Geom g;
    coefficients(p, &g);
    snprintf(buf, n,
             "{\"T\": %d, \"H\": %d, \"hmax\": %d, \"cone_mode\": %d, \"Gs\": %d, \"Gm\": %d, \"Gn\": %d, "
             "\"strip_w\": %lld, \"near_w\": %lld, \"far_w\": %lld, \"near_end\": %lld, \"cone_L0\": %lld, "
             "\"nwg\": %d, \"nb\": %d, \"scan_stages\": %d, "
             "\"ring_rows\": %lld, \"alpha_abs\": %.6g, \"threads\": %d, \"cols_per_thread\": %d, "
             "\"stream_stores\": %d}",
             P.T, P.H, P.hmax, P.cone_mode, P.Gs, P.Gm, P.Gn, (long long)P.strip_w, (long long)P.near_w,
             (long long)P.far_w, (long long)P.near_end,
             (long long)P.cone_L0, P.nwg, P.nb, P.nst, (long long)ring_rows(p, P), cabs_(g.alpha), BM_THREADS, BM_K, P.stream);
    return FDTD_OK;
}

const char* fdtd_strerror(int s)
{
    switch (s) {
    case FDTD_OK: return "ok";
    case FDTD_EINVAL: return "invalid argument";
    case FDTD_ESIZE: return "buffer too small";
    case FDTD_ESTATE: return "call out of order";
    case FDTD_EDEVICE: return "HIP device error";
    case FDTD_ERANGE: return "value out of range";
    }
    return "unknown status";
}

const char* fdtd_last_error(const fdtd_ctx* c) { return c ? c->err : g_err; }

}  // extern "C"

// ---------------------------------------------------------------------------
// The allocation-free solve.  Its workspace is this file-scope array: each
// GPU the library runs on holds one copy (at its own address) from the
// library's load until the process ends.  In host code the array's name is
// not a device address: the address is taken once per device with
// hipGetSymbolAddress and only that address is handed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[FDTD_NOALLOC_MAX_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];   // device address of `scratch` per device ordinal

static int scratch_address(void** ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, FDTD_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(nullptr, FDTD_EDEVICE, "device ordinal %d beyond the %d this entry point serves", dev,
                    NOALLOC_MAX_DEVICES);
    if (!g_scratch_ptr[dev]) {
        void* a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !a)
            return fail(nullptr, FDTD_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = a;
    }
    *ptr = g_scratch_ptr[dev];
    return FDTD_OK;
}

extern "C" int fdtd_solve_noalloc(const fdtd_params* p, int64_t n_rows, double* d_pe, void* d_row, void* hip_stream)
{
    char why[256];
    int rc = validate(p, why, sizeof why);
    if (rc) return fail(nullptr, rc, "%s", why);
    if (n_rows < 0 || n_rows > p->Nt)
        return fail(nullptr, FDTD_EINVAL, "n_rows = %lld outside 0..Nt = %lld", (long long)n_rows, (long long)p->Nt);
    const int64_t need = ctx_bytes(p, SOLO_KNOBS);
    if (need < 0 || need > (int64_t)FDTD_NOALLOC_MAX_BYTES)
        return fail(nullptr, FDTD_ESIZE, "these parameters need %lld bytes of workspace, more than the %lld the "
                    "allocation-free entry point holds (use fdtd_init with a workspace of your own)",
                    (long long)need, (long long)FDTD_NOALLOC_MAX_BYTES);
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    // the context lives on this stack frame; its work is enqueued on the
    // caller's stream and needs no host state after the return
    fdtd_ctx c, c2;                 // c2: the second march of two different photons
    rc = ctx_setup(&c, &c2, p, SOLO_KNOBS, ws, (size_t)FDTD_NOALLOC_MAX_BYTES, (hipStream_t)hip_stream, why,
                   sizeof why);
    if (rc) return fail(nullptr, rc, "%s", why);
    rc = boundary_enqueue(&c, 0);
    if (rc) return fail(nullptr, rc, "boundary launch failed: %s", hipGetErrorString(hipGetLastError()));
    rc = check_status(&c);
    if (rc) return fail(nullptr, rc, "%s", c.err);
    boundary_done(&c);
    if (n_rows > 0 && (rc = march_to(&c, n_rows)))
        return fail(nullptr, rc, "march launch failed: %s", hipGetErrorString(hipGetLastError()));
    if (d_pe && (rc = c.pair ? launch_pe_pair(&c, n_rows + 1, d_pe) : launch_pe_final(&c, n_rows + 1, d_pe)))
        return fail(nullptr, rc, "P_e readout launch failed");
    if (d_row && (rc = c.pair ? launch_row_pair(&c, n_rows, (cd*)d_row) : launch_row_readout(&c, n_rows, (cd*)d_row)))
        return fail(nullptr, rc, "row readout launch failed");
    return FDTD_OK;
}
