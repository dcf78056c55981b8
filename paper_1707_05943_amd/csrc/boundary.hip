// Boundary tables of the march: the exact solution in x <= -a.
//
// In x <= -a the two-excitation amplitude is psi(x,t) = c phi(x-t) E(t)
// (Eqs. 5, 8, 12 for identical photons), where E(t) is the one-excitation
// emitter amplitude driven by the packet phi.  E solves a linear delay
// equation whose solution is a series over round trips 2a (Eqs. 6, 9, 13):
//
//   E(t) = sqrt(G/2) sum_{m>=0} (G/2)^m [J_m(t - 2ma) - J_m(t - 2(m+1)a)],
//   J_m(T) = int_0^T (T-s)^m/m! e^{-W(T-s)} phi(-a-s) ds.
//
// For phi(-a-s) = A e^{-ika} e^{-lambda s} (plane wave: lambda = ik; the
// exponential packet of Eq. 7: lambda = ik + alpha G/2) this integral is an
// incomplete Gamma function, J_m(T) = A e^{-ika} e^{-lambda T} T^{m+1}
// gamma*(m+1, bT) with b = W - lambda and gamma*(n,z) = z^{-n} gamma(n,z)/(n-1)!.
// Grouping the two J's that share T_m = t - 2ma and using
// gamma*(m,z) = z gamma*(m+1,z) + e^{-z}/m! gives one gamma* per term:
//
//   term_0 = e^{-lambda T} T gamma*(1, bT)
//   term_m = e^{-lambda T} (G/2)^{m-1} T^m [(G/2 - b) T gamma*(m+1, bT)] - (G/2)^{m-1} T^m e^{-W T}/m!
//
// which is Eq. (6) (and Eq. 13 times e^{-ika}) rearranged.  The Gaussian
// packet has no closed form; it is a superposition of plane waves,
// phi(x) = int dk c(k) e^{ikx}, and since the truncation x <= -a is common to
// every plane wave, E is the same superposition of plane-wave solutions.  The
// k-integral is a trapezoid sum whose spacing h puts the periodic images of
// the packet (at x0 +- 2 pi/h) outside the part of x <= -a that reaches the
// emitter before the last row.
//
// gamma*(n, z) for integer n >= 1 (App. C): for |z| <= n the series
// e^{-z} sum_k z^k/Gamma(n+k+1), whose terms decrease from the first; beyond,
// the terminating form z^{-n} - e^{-z} sum_{k<n} z^{k-n}/k! (exact for integer
// n), whose terms grow towards the last one.

#include "fdtd_common.h"

namespace {

// e^L gamma*(n, z): the scale factor enters the exponent, so that products
// like T^m gamma*(m+1, bT) that are moderate while their factors are not stay
// representable.  lf_n = log n! and lf_n1 = log (n-1)! come from the caller,
// which steps them along its sum.
__device__ inline cd gamma_star_x(int n, cd z, cd L, double lf_n, double lf_n1, int* range_flag)
{
    const double az = cabs_(z);
    if (az <= (double)n + 0.5) {
        // e^{-z}/n! sum_k z^k n!/(n+k)!
        cd term = mk(1.0, 0.0);
        cd sum = term;
        for (int k = 1; k < 20000; ++k) {
            term = term * z * (1.0 / (double)(n + k));
            sum += term;
            if (norm2(term) <= 1e-36 * norm2(sum)) break;
            if (k == 19999) *range_flag = 1;
        }
        return cexp_(L - z - mk(lf_n, 0.0)) * sum;
    }
    // z^{-n} - e^{-z} z^{-1}/(n-1)! sum_{i=0}^{n-1} (n-1)!/(n-1-i)! z^{-i}
    const cd zi = cdiv(mk(1.0, 0.0), z);
    cd t = mk(1.0, 0.0), s = mk(1.0, 0.0);
    for (int i = 0; i < n - 1; ++i) {
        t = t * zi * (double)(n - 1 - i);
        s += t;
    }
    const cd lz = clog_(z);
    return cexp_(L - (double)n * lz) - cexp_(L - z - lz - mk(lf_n1, 0.0)) * s;
}

// log m! stepped along a loop over m as a compensated (Kahan) sum of log k:
// a plain running sum drifts from log m! by ~1e-10 over thousands of round
// trips; the compensated one stays within a few rounding steps of it
struct LogFact {
    double s = 0.0, c = 0.0;
    __device__ void add(double v)
    {
        const double y = v - c;
        const double t = s + y;
        c = (t - s) - y;
        s = t;
    }
};

// sum over round trips for phi(-a-s) = e^{-lambda s} (the factor A e^{-ika}
// is applied by the caller); row r, T_m = (r - mD) Delta
__device__ cd delay_series(const Geom& g, cd lam, int64_t r, int* range_flag)
{
    const cd b = g.W - lam;
    const double hg = 0.5 * g.Gamma;
    const cd gmb = mk(hg, 0.0) - b;           // G/2 - b
    const double lhg = log(hg);
    cd sum = mk(0.0, 0.0);
    double lf_m = 0.0, lf_m1 = 0.0;                // log m!, log (m+1)!
    LogFact lfs;
    for (int64_t m = 0; m * g.D < r; ++m) {
        lf_m = lf_m1;
        lfs.add(log((double)m + 1.0));
        lf_m1 = lfs.s;
        const int64_t q = r - m * g.D;
        const double T = (double)q * g.Delta;
        const double lT = log(T);
        const cd z = b * T;
        const cd mlT = -(lam * T);
        if (m == 0) {
            sum += gamma_star_x(1, z, mlT + mk(lT, 0.0), 0.0, 0.0, range_flag);   // e^{-lam T} T gamma*(1, z)
        } else {
            const double lp = (double)(m - 1) * lhg + (double)m * lT;         // log (G/2)^{m-1} T^m
            sum += gmb * gamma_star_x((int)m + 1, z, mlT + mk(lp + lT, 0.0), lf_m1, lf_m, range_flag);
            sum -= cexp_(mk(lp - lf_m, 0.0) - g.W * T);
        }
    }
    return sqrt(hg) * sum;
}

// Eq. (9): emitter excited at t = 0, no incident photon
__device__ cd stimulated(const Geom& g, int64_t r)
{
    const double hg = 0.5 * g.Gamma;
    const cd w2a = cexp_(g.W * (2.0 * g.a));
    cd s = mk(0.0, 0.0);
    LogFact lfs;                                    // log n!
    for (int64_t n = 0; n * g.D <= r; ++n) {
        const double T = (double)(r - n * g.D) * g.Delta;
        if (n == 0) { s += mk(1.0, 0.0); continue; }
        lfs.add(log((double)n));
        const double lf = lfs.s;
        // [(G/2) e^{2aW} T]^n / n!
        const cd base = (hg * T) * w2a;
        const cd lb = clog_(base);
        s += cexp_((double)n * lb - mk(lf, 0.0));
    }
    return cexp_(-(g.W * ((double)r * g.Delta))) * s;
}

// phi inside its support (x <= -a)
__device__ inline cd phi_in(const Packet& pk, double x)
{
    switch (pk.incident) {
    case FDTD_INC_PLANE: {
        double s, c;
        sincos(pk.k * x, &s, &c);
        return mk(c, s);
    }
    case FDTD_INC_EXP1:
    case FDTD_INC_EXP2: {
        double amp = sqrt(pk.alpha * pk.Gamma) * exp(0.5 * pk.alpha * pk.Gamma * (x + pk.a));
        double s, c;
        sincos(pk.k * x, &s, &c);
        return mk(-amp * s, amp * c);          // i amp e^{ikx}
    }
    default: {
        double u = x - pk.x0, w = pk.width;
        double amp = pow(2.0 * M_PI * w * w, -0.25) * exp(-u * u / (4.0 * w * w));
        double s, c;
        sincos(pk.k * u, &s, &c);
        return mk(amp * c, amp * s);
    }
    }
}

// mass of |phi|^2 below y (y <= -a)
__device__ inline double phi_mass_below(const Packet& pk, double y)
{
    switch (pk.incident) {
    case FDTD_INC_GAUSS2: return 0.5 * erfc((pk.x0 - y) / (sqrt(2.0) * pk.width));
    case FDTD_INC_EXP1:
    case FDTD_INC_EXP2: return exp(pk.alpha * pk.Gamma * (y + pk.a));
    default: return __builtin_nan("");
    }
}

// phi on the grid, the drive per row, and row 0's share of int |psi|^2
__device__ inline void tables_row(const Geom& g, const Packet& pk, const Bufs& b, int64_t nblk, int64_t q)
{
    b.Phi[q] = phi_in(pk, -g.a - (double)q * g.Delta);
    cd d = mk(0.0, 0.0);
    if (q >= 1) {
        // t_c = (q - 1/2) Delta; phi(-a - t_c) - phi(a - t_c), the second
        // inside the support only once t_c > 2a, i.e. q >= D + 1
        d = phi_in(pk, -g.a - ((double)q - 0.5) * g.Delta);
        if (q >= g.D + 1) d -= phi_in(pk, -g.a - ((double)(q - g.D) - 0.5) * g.Delta);
        d = pk.c_drive * d;
    }
    b.Drv[q] = d;
    // partial sums of row 0 (only column 0 can be non-zero there)
    if (q < nblk) b.Ppart[q] = 0.0;
}

// phi(-a - q Delta) for q0 <= q <= q1 (the paper's own reads reach x - t
// beyond -a - Nt Delta)
__global__ void k_phi_tail(Geom g, Packet pk, Bufs b, int64_t q0, int64_t q1)
{
    const int64_t q = q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q <= q1) b.Phi[q] = phi_in(pk, -g.a - (double)q * g.Delta);
}

__global__ void k_tables(Geom g, Packet pk, Bufs b, int64_t nblk)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > g.Nt) return;
    tables_row(g, pk, b, nblk, q);
}

// source of E in k_E: computed here, copied from Ebuf, or formed from the
// delay equation's G in Ebuf
enum { E_COMPUTE = 0, E_COPY = 1, E_FROM_G = 2, E_SUM_PARTS = 3 };

// the Gaussian's plane-wave superposition, split over chunks of Fourier
// nodes (blockIdx.y) so that short windows still fill the chip; the chunks'
// partial sums are added in a fixed order by k_E
__global__ __launch_bounds__(64) void k_E_part(Geom g, Packet pk, Bufs b, int nk, double k_lo, double hk, int chunks)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > g.Nt) return;
    const int c = blockIdx.y;
    const int i0 = (int)(((int64_t)nk * c) / chunks), i1 = (int)(((int64_t)nk * (c + 1)) / chunks);
    int range_flag = 0;
    // c(k) = (N w / sqrt(pi)) e^{-i k x0} e^{-w^2 (k-k0)^2}; each plane wave
    // e^{ikx} (x <= -a) contributes e^{-ika} times its delay series
    const double w = pk.width;
    const double nrm = pow(2.0 * M_PI * w * w, -0.25) * w / sqrt(M_PI);
    cd acc = mk(0.0, 0.0);
    for (int i = i0; i < i1; ++i) {
        const double kk = k_lo + (double)i * hk;
        const double dk = kk - pk.k;
        const double wt = hk * nrm * exp(-(w * dk) * (w * dk));
        double s, co;
        sincos(-kk * (pk.x0 + g.a), &s, &co);
        const cd ser = delay_series(g, mk(0.0, kk), r, &range_flag);
        acc += (wt * mk(co, s)) * ser;
    }
    b.Epart[(int64_t)c * (g.Nt + 1) + r] = acc;
    if (range_flag) atomicOr(b.status, STATUS_GAMMA_RANGE);
}

__device__ inline void e_row(const Geom& g, const Packet& pk, const Bufs& b, int from_host, int nk, double k_lo,
                             double hk, int64_t r)
{
    int range_flag = 0;
    cd E;
    if (from_host == E_COPY) {
        E = b.Ebuf[r];
    } else if (from_host == E_SUM_PARTS) {
        E = mk(0.0, 0.0);
        for (int c = 0; c < nk; ++c) E += b.Epart[(int64_t)c * (g.Nt + 1) + r];
    } else if (from_host == E_FROM_G) {
        // E = sqrt(Gamma/2) [G(t) - G(t - 2a)]
        E = b.Ebuf[r];
        if (r >= g.D) E -= b.Ebuf[r - g.D];
        E = sqrt(0.5 * g.Gamma) * E;
    } else if (pk.incident == FDTD_INC_EXP1) {
        E = stimulated(g, r);
    } else {
        // plane wave (A = 1) or exponential packet (A = i sqrt(alpha G))
        cd lam = mk(0.0, pk.k);
        cd A = mk(1.0, 0.0);
        if (pk.incident == FDTD_INC_EXP2) {
            lam = mk(0.5 * pk.alpha * pk.Gamma, pk.k);
            A = mk(0.0, sqrt(pk.alpha * pk.Gamma));
        }
        double s, c;
        sincos(-pk.k * g.a, &s, &c);
        E = A * mk(c, s) * delay_series(g, lam, r, &range_flag);
    }
    cd Et = pk.c_ex * E;
    b.Et[r] = Et;
    const double t = (double)r * g.Delta;
    b.Pex[r] = norm2(Et) * phi_mass_below(pk, -g.a - t);
    if (range_flag) atomicOr(b.status, STATUS_GAMMA_RANGE);
    if (!isfinite(Et.re) || !isfinite(Et.im)) atomicOr(b.status, STATUS_NONFINITE);
    if (r == 0) {
        // row 0: psi(x,0) = 0 for x > -a; column 0 carries c phi(-a) E(0)
        cd v = b.Phi[0] * Et;
        b.Ppart[0] = 0.5 * norm2(v);
    }
    (void)k_lo;
    (void)hk;
}

__global__ __launch_bounds__(64) void k_E(Geom g, Packet pk, Bufs b, int from_host, int64_t nblk,
                    int nk, double k_lo, double hk)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > g.Nt) return;
    e_row(g, pk, b, from_host, nk, k_lo, hk, r);
    (void)nblk;
}

// The delay-equation boundary of a whole batch, one instance per blockIdx.y
// (tab holds the instances in any order), BB_X workgroups per instance
// striding over its rows: the status word and the tables (k_tables), E from
// G (k_E's E_FROM_G, or E_COPY for the stimulated family), then row 0 of the
// ring and of the diagonal copy (launch_boundary_post).
constexpr int BB_X = 8;
constexpr int BB_THREADS = 128;

__global__ __launch_bounds__(BB_THREADS) void k_tables_batch(const OdeInst* __restrict__ tab)
{
    const OdeInst& e = tab[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) *e.b.status = 0;
    for (int64_t q = (int64_t)blockIdx.x * BB_THREADS + threadIdx.x; q <= e.g.Nt; q += (int64_t)BB_X * BB_THREADS)
        tables_row(e.g, e.pk, e.b, e.nblk, q);
}

__global__ __launch_bounds__(BB_THREADS) void k_E_batch(const OdeInst* __restrict__ tab)
{
    const OdeInst& e = tab[blockIdx.y];
    const int mode = e.pk.incident == FDTD_INC_EXP1 ? E_COPY : E_FROM_G;
    for (int64_t r = (int64_t)blockIdx.x * BB_THREADS + threadIdx.x; r <= e.g.Nt; r += (int64_t)BB_X * BB_THREADS)
        e_row(e.g, e.pk, e.b, mode, 0, 0.0, 0.0, r);
}

__global__ __launch_bounds__(BB_THREADS) void k_post_batch(const OdeInst* __restrict__ tab)
{
    const OdeInst& e = tab[blockIdx.y];
    for (int64_t j = (int64_t)blockIdx.x * BB_THREADS + threadIdx.x; j < e.g.C; j += (int64_t)BB_X * BB_THREADS) {
        e.b.ring[j] = mk(0.0, 0.0);
        if (j >= 1 && j <= e.g.D) e.b.Md[(e.g.D - j) * e.g.Mc + j] = mk(0.0, 0.0);
    }
}

// the ring and the diagonal copy of every instance of a batch to zero
// (launch_clear), CLR_X workgroups per instance
constexpr int CLR_X = 16;

__global__ __launch_bounds__(256) void k_clear_batch(const BInst* __restrict__ tab)
{
    const BInst& e = tab[blockIdx.y];
    const int64_t n = e.g.R * e.g.C, nm = e.g.R * e.g.Mc;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)CLR_X * 256)
        e.b.ring[i] = mk(0.0, 0.0);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nm; i += (int64_t)CLR_X * 256)
        e.b.Md[i] = mk(0.0, 0.0);
}

// every instance's status word into out[e.index]
__global__ void k_gather_status(const BInst* __restrict__ tab, int n, int* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[tab[i].index] = *tab[i].b.status;
}

// The delay equation G' = -W G + (Gamma/2) G(t - 2a) + phi(-a - t), G = 0
// for t <= 0 (stimulated emission: no phi, G(0) = 1), stepped over t_rho =
// rho Delta with the collocation weights of OdeTab: with the forcing f_j of
// step rho at its nodes tau_j,
//   G(t_rho + tau_i) = ew_i G(t_rho) + sum_j M_ij f_j   (i < P: the nodes,
//   i = P: the end of the step, G(t_{rho+1})),
// and f_j = (Gamma/2) G(t_rho - 2a + tau_j) + phi(-a - t_rho - tau_j), the
// node values of step rho - D.  The forcing of K <= D consecutive steps
// needs only node values of earlier rounds, so one round of K steps forms
// the K P forcing values and the K (P + 1) sums S_i = sum_j M_ij f_j in
// parallel; only G(t_{rho+1}) = ew_P G(t_rho) + S_P is serial, and then the
// node values ew_i G(t_rho) + S_i of the K steps again in parallel.  One
// workgroup per instance; node values of the last D + 1 steps in Gn
// (row rho mod (D + 1)); G(t_r) goes to Ebuf[r].
constexpr int ODE_THREADS = 256;
constexpr int ODE_K = ODE_THREADS / ODE_P;          // steps per round (at most D)

__global__ __launch_bounds__(ODE_THREADS) void k_E_ode(const OdeInst* __restrict__ tab)
{
    const OdeInst& e = tab[blockIdx.x];
    const Geom& g = e.g;
    const Packet& pk = e.pk;
    const Bufs& b = e.b;
    const OdeTab* T = b.ode;
    __shared__ cd M[ODE_P + 1][ODE_P];
    __shared__ cd ew[ODE_P + 1];
    __shared__ double tau[ODE_P];
    __shared__ cd f[ODE_K][ODE_P];
    __shared__ cd S[ODE_K][ODE_P + 1];
    __shared__ cd Gs[ODE_K + 1];
    const int t = threadIdx.x;
    const int64_t D = g.D, Nt = g.Nt, R = D + 1;
    const double hg = 0.5 * g.Gamma;
    const int stim = pk.incident == FDTD_INC_EXP1;
    for (int q = t; q < (ODE_P + 1) * ODE_P; q += ODE_THREADS) M[q / ODE_P][q % ODE_P] = T->M[q / ODE_P][q % ODE_P];
    if (t <= ODE_P) ew[t] = T->ew[t];
    if (t < ODE_P) tau[t] = T->tau[t];
    if (t == 0) {
        Gs[0] = stim ? mk(1.0, 0.0) : mk(0.0, 0.0);
        b.Ebuf[0] = Gs[0];
    }
    const int K = D < ODE_K ? (int)D : ODE_K;
    __syncthreads();
    for (int64_t r0 = 0; r0 < Nt; r0 += K) {
        const int kn = Nt - r0 < K ? (int)(Nt - r0) : K;
        // forcing of steps r0..r0+kn-1 (node values of steps <= r0 - 1)
        if (t < kn * ODE_P) {
            const int k = t / ODE_P, j = t % ODE_P;
            const int64_t rho = r0 + k;
            cd fo = mk(0.0, 0.0);
            if (rho >= D) fo = hg * b.Gn[((rho - D) % R) * ODE_P + j];
            if (!stim) fo += phi_in(pk, -g.a - (double)rho * g.Delta - tau[j]);
            f[k][j] = fo;
        }
        __syncthreads();
        for (int q = t; q < kn * (ODE_P + 1); q += ODE_THREADS) {
            const int k = q / (ODE_P + 1), i = q % (ODE_P + 1);
            cd acc = mk(0.0, 0.0);
            #pragma unroll
            for (int j = 0; j < ODE_P; ++j) acc += M[i][j] * f[k][j];
            S[k][i] = acc;
        }
        __syncthreads();
        if (t == 0) {
            cd G = Gs[0];
            for (int k = 0; k < kn; ++k) {
                G = ew[ODE_P] * G + S[k][ODE_P];
                Gs[k + 1] = G;
                b.Ebuf[r0 + k + 1] = G;
            }
        }
        __syncthreads();
        if (t < kn * ODE_P) {
            const int k = t / ODE_P, i = t % ODE_P;
            b.Gn[((r0 + k) % R) * ODE_P + i] = ew[i] * Gs[k] + S[k][i];
        }
        __syncthreads();
        if (t == 0) Gs[0] = Gs[kn];
        __syncthreads();
    }
}

// e0(t_r) of App. D: the emitter amplitude of the one-excitation problem
// with the exponential packet of Eq. (7) and the emitter in its ground state
// at t = 0, i.e. the delay series of the exponential packet (A = i sqrt(alpha
// G), lambda = ik + alpha G/2) without the two-photon prefactor
__global__ __launch_bounds__(64) void k_E0(Geom g, Packet pk, cd* __restrict__ E0, int* status)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > g.Nt) return;
    int range_flag = 0;
    const cd lam = mk(0.5 * pk.alpha * pk.Gamma, pk.k);
    const cd A = mk(0.0, sqrt(pk.alpha * pk.Gamma));
    double s, c;
    sincos(-pk.k * g.a, &s, &c);
    const cd e = A * mk(c, s) * delay_series(g, lam, r, &range_flag);
    E0[r] = e;
    if (range_flag) atomicOr(status, STATUS_GAMMA_RANGE);
    if (!isfinite(e.re) || !isfinite(e.im)) atomicOr(status, STATUS_NONFINITE);
}

__global__ void k_clear_status(int* st)
{
    if (threadIdx.x == 0) *st = 0;
}

// row 0 of the strip in its diagonal copy: psi(c, 0) = 0 sits at row D - c
__global__ void k_md_row0(Geom g, Bufs b)
{
    int64_t c = 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > g.D) return;
    b.Md[(g.D - c) * g.Mc + c] = mk(0.0, 0.0);
}

__global__ void k_zero(cd* p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = mk(0.0, 0.0);
}

}  // namespace

// Node set of the plane-wave superposition for the Gaussian packet: range
// k0 +- 6.5/w (weights below e^{-42}) and spacing h with 2 pi/h beyond both
// the distance from the packet to -a and the distance a periodic image must
// keep to the left of -a - T, each with a 13 w margin.
static void gauss_nodes(const fdtd_ctx* c, int* nk, double* k_lo, double* hk)
{
    const double w = c->p.width;
    const double T = (double)c->p.Nt * c->p.Delta;
    const double d0 = -c->g.a - c->p.x0;
    double L = d0 + 13.0 * w;
    if (T - d0 + 13.0 * w > L) L = T - d0 + 13.0 * w;
    const double h = 2.0 * M_PI / L;
    const int half = (int)ceil(6.5 / w / h);
    *nk = 2 * half + 1;
    *k_lo = c->p.k - half * h;
    *hk = h;
}

int launch_boundary_pre(fdtd_ctx* c)
{
    const int64_t n = c->g.Nt + 1;
    const int th = 128;
    const int64_t blocks = (n + th - 1) / th;
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, c->stream, c->b.status);
    hipLaunchKernelGGL(k_tables, dim3((unsigned)blocks), dim3(th), 0, c->stream, c->g, c->pk, c->b, c->nblk);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_boundary_E(fdtd_ctx* c, int mode)
{
    const int64_t n = c->g.Nt + 1;
    int nk = 0;
    double k_lo = 0.0, hk = 0.0;
    if (mode == E_COMPUTE && c->p.incident == FDTD_INC_GAUSS2) {
        gauss_nodes(c, &nk, &k_lo, &hk);
        if (!c->b.Epart) return FDTD_EINVAL;
        const int chunks = nk < EPART_CHUNKS ? nk : EPART_CHUNKS;
        hipLaunchKernelGGL(k_E_part, dim3((unsigned)((n + 63) / 64), (unsigned)chunks), dim3(64), 0, c->stream, c->g,
                           c->pk, c->b, nk, k_lo, hk, chunks);
        mode = E_SUM_PARTS;
        nk = chunks;
    }
    // small E-threads blocks: the work per row grows with r, so spread rows
    hipLaunchKernelGGL(k_E, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, c->stream, c->g, c->pk, c->b,
                       mode, c->nblk, nk, k_lo, hk);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_E_from_G(fdtd_ctx* c)
{
    return launch_boundary_E(c, c->p.incident == FDTD_INC_EXP1 ? E_COPY : E_FROM_G);
}

int launch_boundary_post(fdtd_ctx* c)
{
    // row 0 of the ring is the initial condition (zero for x > -a)
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((c->g.C + 255) / 256)), dim3(256), 0, c->stream, c->b.ring, c->g.C);
    hipLaunchKernelGGL(k_md_row0, dim3((unsigned)((c->g.D + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b);
    if (hipGetLastError() != hipSuccess) return FDTD_EDEVICE;
    // stimulated emission: e0 and row 0 of mu
    if (c->E0) {
        int rc = launch_e0(c);
        if (!rc) rc = launch_mu_rows(c, 0, 0, c->stream);
        if (rc) return rc;
    }
    return FDTD_OK;
}

int launch_e0(fdtd_ctx* c)
{
    hipLaunchKernelGGL(k_E0, dim3((unsigned)((c->g.Nt + 64) / 64)), dim3(64), 0, c->stream, c->g, c->pk, c->E0,
                       c->b.status);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_boundary_batch(const OdeInst* d_tab, int n, hipStream_t s)
{
    if (n <= 0) return FDTD_OK;
    hipLaunchKernelGGL(k_tables_batch, dim3(BB_X, (unsigned)n), dim3(BB_THREADS), 0, s, d_tab);
    hipLaunchKernelGGL(k_E_ode, dim3((unsigned)n), dim3(ODE_THREADS), 0, s, d_tab);
    hipLaunchKernelGGL(k_E_batch, dim3(BB_X, (unsigned)n), dim3(BB_THREADS), 0, s, d_tab);
    hipLaunchKernelGGL(k_post_batch, dim3(BB_X, (unsigned)n), dim3(BB_THREADS), 0, s, d_tab);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_clear_batch(const BInst* d_tab, int n, hipStream_t s)
{
    if (n <= 0) return FDTD_OK;
    hipLaunchKernelGGL(k_clear_batch, dim3(CLR_X, (unsigned)n), dim3(256), 0, s, d_tab);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_gather_status(const BInst* d_tab, int n, int* d_out, hipStream_t s)
{
    if (n <= 0) return FDTD_OK;
    hipLaunchKernelGGL(k_gather_status, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_tab, n, d_out);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_E_ode(const OdeInst* d_tab, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_E_ode, dim3((unsigned)n), dim3(ODE_THREADS), 0, s, d_tab);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_phi_tail(fdtd_ctx* c, int64_t q0, int64_t q1)
{
    if (q1 < q0) return FDTD_OK;
    hipLaunchKernelGGL(k_phi_tail, dim3((unsigned)((q1 - q0 + 256) / 256)), dim3(256), 0, c->stream, c->g, c->pk, c->b,
                       q0, q1);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_boundary(fdtd_ctx* c, int from_host_E)
{
    int rc = launch_boundary_pre(c);
    if (rc) return rc;
    if (from_host_E) {
        rc = launch_boundary_E(c, E_COPY);
    } else if (c->p.boundary == FDTD_E_DELAY_ODE) {
        rc = launch_E_ode(c->d_ode, 1, c->stream);
        if (!rc) rc = launch_E_from_G(c);
    } else {
        rc = launch_boundary_E(c, E_COMPUTE);
    }
    if (rc) return rc;
    rc = launch_boundary_post(c);
    // the paper's own reads: phi further out and row 0 of every kept column
    if (!rc && c->dc) rc = launch_diag_setup(c);
    return rc;
}

int launch_clear(fdtd_ctx* c)
{
    // the ring and the diagonal copy start at zero: rows before t = 0 are
    // read (and their terms dropped) before they are first written
    const int64_t n = c->g.R * c->g.C;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->b.ring, n);
    const int64_t nm = c->g.R * c->g.Mc;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, c->stream, c->b.Md, nm);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}
