// Internal declarations shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdtd.h"

// ---------------------------------------------------------------------------
// complex double arithmetic (explicit, so the order of operations is ours)
// ---------------------------------------------------------------------------
struct __align__(16) cd {
    double re, im;
};

__host__ __device__ inline cd mk(double re, double im) { return cd{re, im}; }
__host__ __device__ inline cd operator+(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cd operator-(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cd operator-(cd a) { return cd{-a.re, -a.im}; }
__host__ __device__ inline cd operator*(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__host__ __device__ inline cd operator*(double s, cd a) { return cd{s * a.re, s * a.im}; }
__host__ __device__ inline cd operator*(cd a, double s) { return cd{s * a.re, s * a.im}; }
__host__ __device__ inline cd& operator+=(cd& a, cd b) { a.re += b.re; a.im += b.im; return a; }
__host__ __device__ inline cd& operator-=(cd& a, cd b) { a.re -= b.re; a.im -= b.im; return a; }
__host__ __device__ inline double norm2(cd a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ inline double cabs_(cd a) { return hypot(a.re, a.im); }
__host__ __device__ inline cd conj_(cd a) { return cd{a.re, -a.im}; }
__host__ __device__ inline cd cdiv(cd a, cd b)
{
    // Smith's algorithm
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, den = b.re + b.im * r;
        return cd{(a.re + a.im * r) / den, (a.im - a.re * r) / den};
    } else {
        double r = b.re / b.im, den = b.re * r + b.im;
        return cd{(a.re * r + a.im) / den, (a.im * r - a.re) / den};
    }
}
__host__ __device__ inline cd cexp_(cd z)
{
    double m = exp(z.re), s, c;
    sincos(z.im, &s, &c);
    return cd{m * c, m * s};
}
__host__ __device__ inline cd clog_(cd z) { return cd{log(hypot(z.re, z.im)), atan2(z.im, z.re)}; }

// ---------------------------------------------------------------------------
// per-instance constants, passed to kernels by value
// ---------------------------------------------------------------------------
struct Geom {
    int64_t Nx, D, Nt;
    int64_t C;          // columns per ring row = Nx + 1 (row pitch in elements)
    int64_t R;          // ring rows (also the rows of the diagonal copy of the strip)
    int64_t Mc;         // row pitch of the diagonal copy of the strip = D + 1
    double Delta, a, Gamma;
    cd W;               // i omega0 + Gamma/2
    cd alpha;           // coefficient of psi(j-1, r) in the solved square
    cd cA;              // coefficient of psi(j-1, r-1)
    cd cAm1;            // cA - 1 = -(W/2) cinv, formed directly: the march adds psi(j-1, r-1) + cAm1 psi(j-1, r-1),
                        // so the rounding of cA ~ 1 is not applied anew at every step of a characteristic
    cd cB;              // coefficient of psi(j, r-1)
    cd cinv;            // 1/(1/Delta + W/4)
    int halo;           // columns recomputed left of a block for the within-row recurrence
};

struct Packet {           // incident packet phi and the exact-solution prefactor
    int32_t incident;
    double k, alpha, x0, width, phase, Gamma, a;
    cd c_ex;              // psi(x<=-a, t) = c_ex phi(x - t) E(t)
    cd c_drive;           // drive = c_drive phi(xi) [phi(-a - t_c) - phi(a - t_c)]
};

// Delay-equation boundary (FDTD_E_DELAY_ODE): per step of width Delta, the
// values of G at ODE_P Gauss-Legendre nodes tau_i in (0, Delta) and at tau_P =
// Delta are  G(t + tau_i) = ew[i] G(t) + sum_j M[i][j] f(t + tau_j), with
// ew[i] = e^{-W tau_i} and M[i][j] = int_0^{tau_i} e^{-W(tau_i - u)} l_j(u) du
// (l_j the Lagrange basis on the nodes): exact when the forcing
// f = (Gamma/2) G(. - 2a) + phi(-a - .) is a polynomial of degree < ODE_P on
// the step.
constexpr int ODE_P = 16;
constexpr int EPART_CHUNKS = 16;
struct OdeTab {
    double tau[ODE_P + 1];
    cd ew[ODE_P + 1];
    cd M[ODE_P + 1][ODE_P];
};

// device pointers carved from the caller's workspace
struct Bufs {
    cd* ring;        // R x C
    cd* Md;          // the strip along anti-diagonals: psi(c, rho) at row (rho - c + D) mod R, column c (R x Mc)
    cd* Et;          // c_ex E(t_r), r = 0..Nt
    cd* Phi;         // phi(-a - q Delta), q = 0..Nt
    cd* Drv;         // drive per row, r = 0..Nt (r = 0 unused)
    double* Pex;     // exact part of P_e per row
    double* Ppart;   // per-row per-block partial sums of |psi|^2
    double* Pe;      // P_e per row
    cd* chi;         // chi readout scratch
    cd* Ebuf;        // host-supplied E staging (Nt+1); G(t_r) of the delay-equation boundary
    int* status;     // device error flags
    cd* Gn;          // delay-equation boundary: G at the nodes of the last D+1 steps ((D+1) x ODE_P)
    cd* Epart;       // series boundary of the Gaussian: partial sums over chunks of Fourier nodes
                     // (EPART_CHUNKS x (Nt+1)); NULL for the other boundaries
    OdeTab* ode;     // its step weights
    cd* hist;        // FDTD_READ_PAPER_DIAG: every row of columns 1-dc..Nx ((Nt+1) x (Nx+dc)); else NULL
};

// one instance of a (batched) delay-equation boundary launch
struct OdeInst {
    Geom g;
    Packet pk;
    Bufs b;
    int64_t nblk;        // the march's workgroups per row (row 0's partial sums)
};

// Work decomposition of the blocked march (fixed per context).
// Rows are marched in blocks of T; one launch computes one block of the
// outgoing region (columns D+1..Nx) and, one block ahead, the next block of
// the mirror strip (columns 1..D).  Every workgroup computes its columns for
// T rows from data of earlier launches only: a workgroup whose left
// neighbour is marched in the same launch recomputes a trapezoidal halo
// that starts (H+1)T-1 columns to its left and shrinks by H+1 per row.
struct Plan {
    int T;               // rows per block
    int H;               // columns of the within-row recurrence kept (|alpha|^H < 2^-60)
    int hmax;            // halo at a block's first row: (H+1)T - 1
    int cone_mode;       // 0: one strip workgroup marches the whole strip exactly;
                         // 1: several strip workgroups, the first also computes a cone at the strip's right end
    int Gs, Gm;          // strip and outgoing-region workgroups
    int Gn;              // of the Gm, those of the near part D+1..near_end (mirror reads)
    int64_t strip_w;     // strip columns per strip workgroup (the last one takes the rest)
    int64_t near_w;      // columns per near workgroup (the last one takes the rest)
    int64_t far_w;       // columns per far workgroup (the last one takes the rest)
    int64_t near_end;    // last column of the near part (>= 2D + hmax, so far halos hold no mirror reads)
    int64_t cone_L0;     // cone width at a block's first row
    int64_t win_lo;      // first strip column kept in the LDS window of the current block
    int nwg;             // Gs + Gm
    int nb;              // launched blocks (a multiple of 8, >= nwg)
    int nst;             // doubling stages of the within-row scan inside 16-lane rows (2^nst K > H, <= 4)
    int stream;          // ring rows leave as streaming stores (see make_plan)
};

struct fdtd_ctx {
    fdtd_params p;
    OdeInst* d_ode;       // this instance's delay-equation launch record (in the workspace)
    Geom g;
    Packet pk;
    Bufs b;
    Plan plan;
    hipStream_t stream;
    int64_t row;          // last solved row of the whole grid
    int64_t strip_row;    // last strip row marched (>= row)
    int boundary_ready;
    int64_t nblk;         // per-row partial sums of |psi|^2 (one per workgroup)
    // stimulated emission only (NULL / -1 otherwise): the one-excitation
    // emitter amplitude e0(t_r), per-row partial sums of mu(t_r), and the
    // last row whose partial sums are complete
    cd* E0;
    cd* Mu;               // mu(t_r) readout staging (Nt+1)
    cd* mupart;           // (Nt+1) x NM_BLOCKS
    int64_t mu_row;
    // two different photons (Sec. 2 case (c)): this context is march a (phi1 on
    // the x - t grid, photon 2's e0 and drive), `pair` march b (the photons
    // exchanged), psi = psi_a + psi_b; xpart holds the row sums of
    // |psi_a + psi_b|^2 ((Nt+1) x PAIR_CHUNKS) and c0_pair the coefficient
    // e^{i theta} A/sqrt 2 of chi's free term.  NULL for the other families.
    fdtd_ctx* pair;
    double* xpart;
    cd c0_pair;
    // FDTD_READ_PAPER_DIAG (Sec. 3's own reads): dc marched columns at x <=
    // -a, every row in b.hist, one launch per row; 0 otherwise.  stage holds
    // dc values for readouts of the left columns into host memory.
    int64_t dc;
    cd* stage;
    char err[512];
};

// device status word of a context (cleared with the boundary): gamma series
// out of range, a non-finite boundary value, a non-finite value in the march
enum { STATUS_GAMMA_RANGE = 1, STATUS_NONFINITE = 2, STATUS_MARCH_NONFINITE = 4 };

// launch helpers implemented in the .hip files
int launch_boundary(fdtd_ctx* c, int from_host_E);
// the pieces of launch_boundary, for batches: status and tables; E; the rest
int launch_boundary_pre(fdtd_ctx* c);
int launch_boundary_E(fdtd_ctx* c, int from_host_E);
int launch_boundary_post(fdtd_ctx* c);
int launch_E_ode(const OdeInst* d_tab, int n, hipStream_t s);
int launch_E_from_G(fdtd_ctx* c);
int launch_pe_final(fdtd_ctx* c, int64_t nrows, double* dst);
int launch_chi(fdtd_ctx* c, int64_t r, int64_t count, cd* dst);
int launch_row_readout(fdtd_ctx* c, int64_t rho, cd* dst);
// the march with the paper's own reads (diag.hip): the phi table beyond row
// Nt and row 0 of every kept column (after the boundary); row r; a copy of
// `count` columns from column j0 of row rho
int launch_diag_setup(fdtd_ctx* c);
int launch_phi_tail(fdtd_ctx* c, int64_t q0, int64_t q1);
int launch_diag_row(fdtd_ctx* c, int64_t r);
int launch_diag_copy(fdtd_ctx* c, int64_t rho, int64_t j0, int64_t count, cd* dst);
int launch_clear(fdtd_ctx* c);
// non-finite detection over the per-row partial sums of |psi|^2 of rows
// r0..r1 (every marched value enters them): sets STATUS_MARCH_NONFINITE
int launch_check_rows(fdtd_ctx* c, int64_t r0, int64_t r1);
int launch_clear_status(int* st, hipStream_t s);
// non-Markovian measures of stimulated emission: e0(t_r) into c->E0; the
// partial sums of mu over rows r0..r1 (complete rows of the ring); the
// readouts mu(t_r) and lambda(t_r) for r < nrows
constexpr int NM_BLOCKS = 256;
int launch_e0(fdtd_ctx* c);
int launch_mu_rows(fdtd_ctx* c, int64_t r0, int64_t r1, hipStream_t s);
int launch_mu_final(fdtd_ctx* c, int64_t nrows, cd* dst);
int launch_lambda_final(fdtd_ctx* c, int64_t nrows, double* dst);

constexpr int MAX_HALO = 64;

// two different photons: the exact part of P_e (into march a's Pex), the row
// sums of |psi_a + psi_b|^2 over rows r0..r1 (PAIR_CHUNKS per row), P_e, a
// row and chi of the sum
constexpr int PAIR_CHUNKS = 64;
int launch_pex_pair(fdtd_ctx* c);
int launch_pair_rows(fdtd_ctx* c, int64_t r0, int64_t r1);
int launch_pe_pair(fdtd_ctx* c, int64_t nrows, double* dst);
int launch_row_pair(fdtd_ctx* c, int64_t rho, cd* dst);
int launch_chi_pair(fdtd_ctx* c, int64_t r, int64_t count, cd* dst);

// blocked march: threads per workgroup and columns per thread
constexpr int BM_THREADS = 512;
constexpr int BM_K = 3;
constexpr int BM_CAP = BM_THREADS * BM_K;      // columns a workgroup can hold in one row
constexpr int BM_TMAX = 32;                    // largest block of rows (LDS window is BM_TMAX x BM_TMAX)
constexpr int BM_NEAR_CAP = 1024;              // columns a near workgroup may span (three tables, four row stages in LDS)

// Planner knobs: workgroups the instance should spread over (about one per
// compute unit when it runs alone), the largest block of rows, and the widest
// column range of one workgroup.
struct PlanKnobs {
    int ncu;
    int tmax;
    int64_t wmax;
    int stream_ok;       // streaming ring stores allowed (one instance per launch)
};
constexpr PlanKnobs SOLO_KNOBS = {256, BM_TMAX, BM_CAP, 1};

int make_plan(const fdtd_params* p, int H, const PlanKnobs& kn, Plan* out, char* why, size_t n);
int launch_block(fdtd_ctx* c, int64_t m0, int64_t m1, int64_t s0, int64_t s1);

// Rows of launch k of a march that starts at row 0, blocks being rows
// [1 + iT, (i+1)T]: launch 0 marches the strip's first block alone, launch
// k >= 1 the outgoing region over block k-1 and the strip over block k.  A
// march of Nt rows takes 1 + ceil(Nt / T) launches.  Empty ranges have
// m1 < m0 or s1 < s0.
__host__ __device__ inline void block_rows(int64_t T, int64_t Nt, int64_t k, int64_t* m0, int64_t* m1, int64_t* s0,
                                           int64_t* s1)
{
    if (k == 0) {
        *m0 = 1;
        *m1 = 0;
    } else {
        *m0 = 1 + (k - 1) * T;
        *m1 = (k * T < Nt) ? k * T : Nt;
    }
    *s0 = 1 + k * T;
    *s1 = ((k + 1) * T < Nt) ? (k + 1) * T : Nt;
}

// One instance of a batched launch (device table, sorted by `launches`,
// largest first).
struct BInst {
    Geom g;
    Bufs b;
    Plan P;
    int64_t wg_begin;    // first workgroup of this instance in a launch
    int64_t launches;    // 1 + ceil(Nt / T)
    int64_t index;       // the instance's position in the caller's order
};

int launch_block_batch(const BInst* d_tab, int n_active, int64_t k, int nb, hipStream_t s);
// a batch's set-up in bulk: the rings and diagonal copies to zero; the whole
// delay-equation boundary of the instances in d_ode (status, tables, G, E,
// row 0; not e0 and mu of stimulated emission); every status word into
// d_out[index]
int launch_clear_batch(const BInst* d_tab, int n, hipStream_t s);
int launch_boundary_batch(const OdeInst* d_ode, int n, hipStream_t s);
int launch_gather_status(const BInst* d_tab, int n, int* d_out, hipStream_t s);
// the same check over every row of every instance of a batch (each
// instance's status word, and `batch_status` for the whole batch)
int launch_check_batch(const BInst* d_tab, int n, int* batch_status, hipStream_t s);

// A chi snapshot of one instance at row `row`, detector separations
// k * stride * Delta for k < n_tau (zero beyond the last column).
struct ChiJob {
    Geom g;
    Bufs b;
    cd c0;               // coefficient of the free two-photon term of Eq. (2)
    int64_t row, stride, n_tau;
    cd* dst;
};
int launch_chi_batch(const ChiJob* d_jobs, int n, int64_t n_tau, hipStream_t s);
int launch_pe_sample_batch(const BInst* d_tab, int n, int64_t n_samples, const double* d_tend, double* dst,
                           hipStream_t s);
cd chi0_coefficient(const fdtd_params* p);

// Internal context life cycle, shared by the one-instance and batched ABIs.
// With a CtxDefer (one-packet families only) ctx_create enqueues nothing:
// the caller clears the ring and the diagonal copy, uploads the boundary's
// step weights (*h_tab) to d_tab, which the context's tables point at, and
// keeps the launch record (*h_inst) for its own delay-equation launches.
struct CtxDefer {
    OdeTab* d_tab;
    OdeTab* h_tab;
    OdeInst* h_inst;
};
int64_t ctx_bytes(const fdtd_params* p, const PlanKnobs& kn);
int ctx_validate(const fdtd_params* p, const PlanKnobs& kn, char* why, size_t n);
int ctx_create(const fdtd_params* p, const PlanKnobs& kn, void* d_ws, size_t bytes, hipStream_t s, fdtd_ctx** out,
               char* why, size_t n, const CtxDefer* defer = nullptr);
int ctx_boundary_enqueue(fdtd_ctx* c);          // boundary kernels without waiting
int ctx_boundary_status(fdtd_ctx* c, int st);    // turn the device status word into an error (sets c->err)
