/*
 * fdtd.h -- C ABI of the MI355X (gfx950) FDTD solver for the 1+1D delay PDE
 * of waveguide QED (Fang, "FDTD: solving 1+1D delay PDE in parallel",
 * arXiv:1707.05943).
 *
 * The library marches Eq. (1) of the paper on a square grid dx = dt = Delta
 * (Sec. 2), with the line-1 terms (time and space derivatives, W psi and the
 * delay term) discretised by "squares" (Eq. 3) and the source terms of lines
 * 2-3 by "bars" (Eq. 4).  The region x <= -a is not marched: its values are
 * the exact solution psi(x,t) = c phi(x-t) E(t) (Eqs. 5, 8, 12), with E(t)
 * the one-excitation amplitude (Eqs. 6, 9, 13), which involves the lower
 * incomplete Gamma function gamma(n, z) of App. C.
 *
 * Grid.  Columns j = 0..Nx sit at x_j = -a + j*Delta (j = 0 is x = -a);
 * rows r = 0..Nt at t_r = r*Delta.  D = 2a/Delta (the paper's n_x, Table 1)
 * is an even integer; columns 1..D are the mirror strip -a < x <= a, columns
 * beyond D the outgoing region.  Row 0 is the initial condition psi(x,0) = 0
 * for x > -a.  All values are complex double, stored as (re, im) pairs.
 *
 * Memory.  The caller allocates and owns every device buffer: it passes one
 * device workspace of at least fdtd_workspace_size() bytes, which must stay
 * alive and untouched until fdtd_destroy().  The context holds views only.
 * Inside, the march keeps a ring of D+2T+2 rows (the delay term reaches back
 * D+1 rows, every older value it needs lies in x <= -a and comes from the
 * exact solution; T <= 32 is the block of rows one launch marches, and the
 * strip -a < x <= a runs one block ahead), plus a copy of the strip stored
 * along anti-diagonals, so memory does not grow with Nt.
 *
 * Streams.  Every call enqueues its work on the HIP stream given to
 * fdtd_init and returns without waiting, except where stated.  A context is
 * not thread-safe; distinct contexts are independent.
 *
 * Errors.  Every call returns FDTD_OK (0) or a negative code; the text of the
 * last failure of a context is available from fdtd_last_error().
 */
#ifndef FDTD_H
#define FDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDTD_ABI_VERSION 3u

enum fdtd_status {
    FDTD_OK = 0,
    FDTD_EINVAL = -1,   /* invalid parameters (D odd or < 2, Nx < D+1, Delta <= 0, Gamma <= 0, non-finite) */
    FDTD_ESIZE = -2,    /* workspace too small, or an output buffer too short */
    FDTD_ESTATE = -3,   /* call out of order (march before boundary), or a row no longer held */
    FDTD_EDEVICE = -4,  /* a HIP runtime error */
    FDTD_ERANGE = -5    /* gamma(n,z) series out of range, a non-finite boundary value, or a non-finite
                           value (NaN or infinity) in the march */
};

/* Incident states (Table 1 "init_cond" 1-3, plus a Gaussian two-photon packet). */
enum fdtd_incident {
    FDTD_INC_PLANE = 1,  /* two-photon plane wave e^{ik(x1+x2)}, Eqs. (5)-(6), A = 1 */
    FDTD_INC_EXP1 = 2,   /* stimulated emission: one exponential photon, emitter excited, Eqs. (7)-(9) */
    FDTD_INC_EXP2 = 3,   /* two exponential photons, Eqs. (10)-(13): identical (k, alpha), or with
                            identical_photons = 0 two different ones (k1, alpha1), (k2, alpha2) */
    FDTD_INC_GAUSS2 = 4  /* two identical Gaussian photons, phi ~ exp(-(x-x0)^2/(4 w^2) + i k (x-x0)) for x <= -a */
};

/* How fdtd_set_boundary computes E(t_r).  Both give E to FP64 rounding.
 * FDTD_E_SERIES: the delay series of Eqs. (6), (9), (13), term by term with
 *   gamma(n+1, z) (App. C); the Gaussian as a superposition of plane-wave
 *   series over its Fourier components.  Work grows as Nt^2 / D per node.
 * FDTD_E_DELAY_ODE: the generating sum G(t) = sum_m (G/2)^m J_m(t - 2ma) of
 *   that series obeys G' = -W G + (Gamma/2) G(t - 2a) + phi(-a - t) exactly,
 *   and E = sqrt(Gamma/2) [G(t) - G(t - 2a)] (for stimulated emission E = G
 *   with G(0) = 1 and no drive).  The library integrates it step by step,
 *   exactly for a forcing that is a polynomial of degree 15 on each step
 *   (16 Gauss-Legendre collocation nodes, exponential weights), so the work is
 *   linear in Nt.  Meant for long windows and small D (parameter sweeps). */
enum fdtd_boundary_method {
    FDTD_E_SERIES = 0,
    FDTD_E_DELAY_ODE = 1
};

/* Where the march reads the solution at x <= -a.
 * FDTD_READ_EXACT: from the partial exact solution c phi(x - t) E(t) (Eqs. 8,
 *   12); column 0 (x = -a) included.  The marched columns are 1..Nx.
 * FDTD_READ_PAPER_DIAG: as the paper's program does (Sec. 3): diag_cols
 *   columns left of and at x = -a (columns 1-diag_cols..0) are marched with
 *   the same square of Eq. (1), and every read of a marched point, also from
 *   the source terms of x > -a, which reach x <= -a along diagonals x - t =
 *   const, takes the marched value; only points left of column 1-diag_cols
 *   take the exact solution (the region the paper fills with its boundary
 *   condition).  Every row is kept ((Nt+1) (Nx+diag_cols) complex values), and
 *   the march advances one row per launch: a test mode (the paper's test 1,
 *   Sec. 4: the marched x <= -a against the exact solution), not a fast path.
 *   Rows, the left columns (FDTD_RO_LEFT), P_e and E can be read out; chi and
 *   the measures of App. D cannot (FDTD_EINVAL).  One-packet families only. */
enum fdtd_read_mode {
    FDTD_READ_EXACT = 0,
    FDTD_READ_PAPER_DIAG = 1
};

typedef struct fdtd_params {
    uint32_t abi_version;   /* FDTD_ABI_VERSION */
    uint32_t struct_size;   /* sizeof(fdtd_params) */
    int64_t Nx;             /* last column; columns 0..Nx; Nx >= D+1 */
    int64_t D;              /* 2a/Delta, even, >= 2 (Table 1 n_x) */
    int64_t Nt;             /* last row; rows 0..Nt (Table 1 N_y = Nt+1) */
    double Delta;           /* grid step in x and t (absolute units, hbar = c = 1) */
    double omega0;          /* emitter frequency */
    double Gamma;           /* emitter decay rate */
    int32_t incident;       /* enum fdtd_incident */
    int32_t boundary;       /* enum fdtd_boundary_method: how E(t_r) is computed */
    double k;               /* carrier wavenumber of the incident packet */
    double alpha;           /* exponential packet width, units of Gamma (Eq. 7) */
    double x0;              /* Gaussian centre (x0 <= -a) */
    double width;           /* Gaussian: standard deviation of |phi|^2 */
    double phase;           /* global phase theta of the incident two-photon state */
    int32_t identical_photons; /* Table 1: 1 (the usual case) for identical photons; 0 for two different
                                  exponential photons (FDTD_INC_EXP2 only): then the incident state is
                                  (A/sqrt 2)[phi1(x1) phi2(x2) + phi1(x2) phi2(x1)] (Eq. 10, A of Eq. 11),
                                  phi_i of Eq. (7) with (k_i, alpha_i), and k, alpha are not used */
    int32_t read_mode;      /* enum fdtd_read_mode */
    double k1, k2;          /* carriers of photon 1 and photon 2 (identical_photons = 0) */
    double alpha1, alpha2;  /* widths of photon 1 and photon 2, units of Gamma (identical_photons = 0) */
    int64_t diag_cols;      /* FDTD_READ_PAPER_DIAG: marched columns at x <= -a (>= 1); else 0 */
} fdtd_params;

typedef struct fdtd_ctx fdtd_ctx;

/* Bytes of device workspace needed for these parameters (ring, boundary
 * tables, per-row reductions).  Returns FDTD_EINVAL on bad parameters. */
int fdtd_workspace_size(const fdtd_params *p, size_t *bytes);

/* Validate parameters, carve the caller's workspace (device pointer, at
 * least fdtd_workspace_size bytes, 256-byte aligned) and bind the HIP stream
 * (a hipStream_t; NULL is the default stream).  On success *out receives a
 * new context; free it with fdtd_destroy.  Enqueues the clearing of the ring. */
int fdtd_init(const fdtd_params *p, void *d_workspace, size_t bytes, void *hip_stream, fdtd_ctx **out);

/* Compute the boundary tables on the device (Sec. 2, Eqs. 5-13, App. C):
 * E(t_r) for r = 0..Nt from the delay series of the one-excitation problem
 * -- the closed forms with gamma(n+1, z) for the plane-wave and exponential
 * families, and for the Gaussian a superposition of plane-wave solutions
 * over the packet's Fourier components -- plus phi on the grid, the drive
 * and the exact part of int |psi|^2.  Resets the march to row 0. */
int fdtd_set_boundary(fdtd_ctx *ctx);

/* Test hook: as fdtd_set_boundary, but E(t_r) (r = 0..n-1, n = Nt+1) is
 * copied from the caller's host array of complex doubles (n pairs); for two
 * different photons n = 2 (Nt+1): e0^(1)(t_r) followed by e0^(2)(t_r). */
int fdtd_set_boundary_tables(fdtd_ctx *ctx, const double *h_E, int64_t n);

/* Advance the march by n_rows rows (resumable: the row counter lives in the
 * context).  Rows past Nt are not marched (FDTD_ESTATE).  Returns after
 * enqueueing the work, which ends with a check of the rows just marched for
 * non-finite values: every value the march writes enters the per-row sums of
 * |psi|^2, and a NaN or infinity there sets the context's status, which
 * fdtd_sync and readouts into host memory report as FDTD_ERANGE (until the
 * next fdtd_set_boundary). */
int fdtd_march(fdtd_ctx *ctx, int64_t n_rows);

/* Current row (the last row solved; 0 right after set_boundary). */
int fdtd_current_row(const fdtd_ctx *ctx, int64_t *row);

enum fdtd_readout_kind {
    FDTD_RO_ROW = 1,   /* arg = row rho (current-D-1 <= rho <= current); count = Nx+1 values psi(j, rho),
                          column 0 from the exact solution (FDTD_READ_PAPER_DIAG: any row 0..current,
                          column 0 marched) */
    FDTD_RO_PE = 2,    /* P_e(t_r) = int |psi(x,t_r)|^2 dx for r = 0..count-1 (count <= current+1), doubles:
                          the exact part x <= -a plus the trapezoid rule over columns 0..Nx */
    FDTD_RO_CHI = 3,   /* chi(x1, x2, t) of Eq. (2) at the current row, detectors x1 = a + Delta,
                          x2 = x1 + k Delta for k = 0..count-1 (count <= Nx-D) */
    FDTD_RO_E = 4,     /* the boundary table c E(t_r), r = 0..count-1 (count <= Nt+1); c = sqrt(2) e^{i theta}
                          for two identical photons, 1 for stimulated emission; two different photons:
                          A e^{i theta} e0^(1) (arg = 0) or A e^{i theta} e0^(2) (arg = 1) */
    /* Non-Markovian measures of stimulated emission (App. D; FDTD_INC_EXP1 contexts only, else
       FDTD_EINVAL).  e0(t) is the emitter amplitude of the one-excitation problem with the same
       packet and the emitter initially in its ground state, phi(x,t) = phi_in(x-t)
       - sqrt(G/2) e0(t-(x+a)) [x > -a] + sqrt(G/2) e0(t-(x-a)) [x > a] its photon field.
       Quadrature as for FDTD_RO_PE. */
    FDTD_RO_MU = 5,    /* mu(t_r) = int phi*(x,t_r) psi(x,t_r) dx for r = 0..count-1, complex; accumulated row
                          by row by fdtd_march (count <= current+1; instances of a batch hold row 0 only,
                          FDTD_ESTATE beyond) */
    FDTD_RO_LAMBDA = 6,/* lambda(t_r) = int |psi(x,t_r)|^2 dx - |e0(t_r)|^2 for r = 0..count-1 (count <= current+1),
                          doubles; the determinant of the dynamical map is |mu|^2 lambda */
    FDTD_RO_NGEO = 7,  /* the geometric measure N_geo (App. D) over [0, t_arg], 0 <= arg <= current (as mu):
                          the integral of d|det M_t|/dt where it is positive, |det M_t| = |mu|^2 |lambda|
                          taken linear between rows (the sum of its positive increments); count = 1 double */
    FDTD_RO_LEFT = 8   /* FDTD_READ_PAPER_DIAG only: arg = row rho (0..current); count = diag_cols values
                          psi(j, rho) for j = 1-diag_cols..0, the marched columns at x <= -a */
};

/* Copy a readout into dst: a device pointer (dst_on_device = 1, enqueued on
 * the context's stream) or a host pointer (dst_on_device = 0; the call then
 * waits for the stream, and returns FDTD_ERANGE, with the values copied, if
 * the march met a non-finite value).  Complex outputs are (re, im) pairs. */
int fdtd_readout(fdtd_ctx *ctx, int32_t what, int64_t arg, void *dst, int64_t count, int32_t dst_on_device);

/* Checkpoint and restore of a march (its state is the workspace: the ring
 * of the last D+2T+2 rows, the diagonal copy of the strip, the boundary
 * tables and the per-row sums of |psi|^2, plus the row counters).
 * fdtd_checkpoint_size gives the bytes a checkpoint takes; fdtd_checkpoint
 * waits for the context's stream and copies the state into the caller's
 * host buffer h_dst (at least that many bytes); fdtd_restore copies a
 * checkpoint into a context made with the same parameters (another
 * workspace is fine) and sets its rows, so that marching on gives the same
 * values bit for bit.  Errors: FDTD_EINVAL (NULL, not a checkpoint, other
 * parameters), FDTD_ESIZE (buffer too small or truncated), FDTD_EDEVICE. */
int fdtd_checkpoint_size(const fdtd_ctx *ctx, size_t *bytes);
int fdtd_checkpoint(fdtd_ctx *ctx, void *h_dst, size_t bytes);
int fdtd_restore(fdtd_ctx *ctx, const void *h_src, size_t bytes);

/* Wait for all work of this context; FDTD_ERANGE if the march met a
 * non-finite value. */
int fdtd_sync(fdtd_ctx *ctx);

/* Free the context (not the workspace).  Accepts NULL. */
int fdtd_destroy(fdtd_ctx *ctx);

/* Text description (a JSON object) of the work decomposition the library
 * would use for these parameters (rows per launch, halo, workgroups of the
 * strip and of the outgoing region, ring rows, and whether ring rows leave
 * as streaming stores: stream_stores = 1 when D (Nx + 1) 16 bytes, what the
 * grid writes between a row's store and its re-read, exceed the 256 MB
 * last-level cache), written into buf (at most n bytes, NUL-terminated).
 * Host only; no device work. */
int fdtd_describe(const fdtd_params *p, char *buf, size_t n);

/* Measurement aid, not part of the method: copy `bytes` (a multiple of 16,
 * both pointers 16-byte aligned device memory, not overlapping) from d_src
 * to d_dst with the library's streaming-copy kernel, enqueued on hip_stream.
 * The HBM bandwidth a plain copy attains is the practical ceiling of the
 * march's traffic; the benchmark reports the march against it as well as
 * against the vendor peak.  FDTD_EINVAL on misaligned or NULL arguments. */
int fdtd_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *hip_stream);

/* Static text for a status code; text of the last failure of ctx (or of the
 * last failed fdtd_init / fdtd_workspace_size / fdtd_solve_noalloc when ctx
 * is NULL). */
const char *fdtd_strerror(int status);
const char *fdtd_last_error(const fdtd_ctx *ctx);

/* ------------------------------------------------------------------------
 * Allocation-free solve, for callers that cannot allocate device memory
 * (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc).  It does what fdtd_init + fdtd_set_boundary + fdtd_march(n_rows)
 * + the P_e and row readouts into device memory do, with the same kernels and
 * the same results bit for bit, but its workspace is a device array inside
 * the library of FDTD_NOALLOC_MAX_BYTES, one per GPU, held from the library's
 * load until the process ends.  It calls no hipMalloc, hipFree or other
 * allocating routine, and needs no context.
 *   p       instance parameters (as fdtd_init); their workspace
 *           (fdtd_workspace_size) must fit in FDTD_NOALLOC_MAX_BYTES, else
 *           FDTD_ESIZE and nothing is enqueued
 *   n_rows  rows to march, 0..Nt
 *   d_pe    device array of n_rows+1 doubles: P_e(t_r), r = 0..n_rows (as
 *           FDTD_RO_PE), or NULL
 *   d_row   device array of Nx+1 complex doubles: row n_rows (as FDTD_RO_ROW),
 *           or NULL
 *   hip_stream  the stream everything is enqueued on (NULL: default stream)
 * The call waits for the boundary kernels (to report a gamma-series range
 * error, FDTD_ERANGE), then enqueues the march and the readouts and returns;
 * the outputs are complete when the stream is.  Every call on one GPU shares
 * that GPU's array and overwrites it: calls that overlap in time on one GPU
 * (other streams, other host threads) race and must be serialised by the
 * caller.  Errors: as fdtd_init and fdtd_march; the text is in
 * fdtd_last_error(NULL). */
#define FDTD_NOALLOC_MAX_BYTES (64ull << 20)
int fdtd_solve_noalloc(const fdtd_params *p, int64_t n_rows, double *d_pe, void *d_row, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batches: n independent instances (each with its own grid, emitter and
 * packet) marched together from row 0 to their own Nt.  Every kernel launch
 * advances each instance that is not finished by one block of rows, so one
 * launch carries the whole batch; the launch sequence is captured in a HIP
 * graph at the first fdtd_batch_march and replayed afterwards.  Results per
 * instance match the one-instance march to rounding (the batch uses wider
 * workgroups, which changes only the truncation of the within-row recurrence
 * below 2^-60 relative).
 * ------------------------------------------------------------------------ */
typedef struct fdtd_batch fdtd_batch;

typedef struct fdtd_batch_opts {
    uint32_t struct_size;   /* sizeof(fdtd_batch_opts) */
    int32_t tmax;           /* largest block of rows per launch, 1..32 (0: 32) */
    int64_t wmax;           /* widest column range of one workgroup (0: the most one holds, 1536) */
    int32_t use_graph;      /* 1: capture the launch sequence in a HIP graph and replay it; 0: plain launches */
    int32_t groups;         /* 0 or 1: one launch sequence; 2..4: the instances dealt in turn (by launch count)
                               to that many groups, each its own launch sequence (and graph) on its own stream,
                               the others private streams forked from and joined back into the batch's stream */
} fdtd_batch_opts;

/* Device workspace for the batch p[0..n-1] with these options (NULL: the
 * defaults, tmax 32, widest workgroups, graph on, one group).  Batches hold one-packet
 * instances (identical_photons = 1) with read_mode FDTD_READ_EXACT;
 * FDTD_EINVAL otherwise. */
int fdtd_batch_workspace_size(const fdtd_params *p, int32_t n, const fdtd_batch_opts *opts, size_t *bytes);

/* Set up the batch in the caller's workspace (device pointer, 256-byte
 * aligned, at least fdtd_batch_workspace_size bytes, owned by the caller and
 * untouched until fdtd_batch_destroy) on the given HIP stream.  Every
 * instance is validated as by fdtd_init; the first failure is reported with
 * its index.  Enqueues the clearing of every ring and waits for it. */
int fdtd_batch_init(const fdtd_params *p, int32_t n, const fdtd_batch_opts *opts, void *d_workspace, size_t bytes,
                    void *hip_stream, fdtd_batch **out);

/* Boundary tables of every instance (as fdtd_set_boundary); waits for them
 * and reports the first instance whose gamma series failed. */
int fdtd_batch_set_boundary(fdtd_batch *b);

/* March every instance from row 0 to its Nt (FDTD_ESTATE unless the boundary
 * was set since the last march).  Returns after enqueueing. */
int fdtd_batch_march(fdtd_batch *b);

/* fdtd_readout for instance i (0-based, the caller's order). */
int fdtd_batch_readout(fdtd_batch *b, int32_t i, int32_t what, int64_t arg, void *dst, int64_t count,
                       int32_t dst_on_device);

/* chi snapshots taken during the next marches: for instance i with
 * rows[i] >= 0, chi of Eq. (2) at row rows[i], detectors x1 = a + Delta and
 * x2 = x1 + k strides[i] Delta for k < n_tau (zero where x2 is beyond the
 * last column), into d_out[i n_tau + k] (device, complex doubles).  rows[i] < 0
 * takes none for that instance; rows = NULL switches snapshots off.  The
 * snapshot is taken right after the launch that completes its row, while the
 * ring still holds every row Eq. (2) reads.  Re-captures the graph. */
int fdtd_batch_set_chi(fdtd_batch *b, const int64_t *rows, const int64_t *strides, int64_t n_tau, void *d_out);

/* P_e(t_k) of every instance after a march at t_k = k t_end[i] / (n_samples - 1),
 * linear between rows, into d_out[i n_samples + k] (device doubles, the
 * caller's instance order); enqueued on the batch's stream.  d_t_end is a
 * device array of n window ends (at most Nt Delta; 0 or a NULL array means
 * Nt Delta). */
int fdtd_batch_sample_pe(fdtd_batch *b, int64_t n_samples, const double *d_t_end, double *d_out);

/* Launches of one march, and workgroups of the first (largest) launch. */
int fdtd_batch_info(const fdtd_batch *b, int64_t *launches, int64_t *max_workgroups);

int fdtd_batch_sync(fdtd_batch *b);      /* FDTD_ERANGE if any instance's march met a non-finite value */
int fdtd_batch_destroy(fdtd_batch *b);   /* frees host state and the graph, not the workspace; accepts NULL */
const char *fdtd_batch_last_error(const fdtd_batch *b);

/* Autotuner: try each candidate (tmax in {32, 16, 8}, wmax in {1536, 768}, groups in {1, 2})
 * whose workspace fits in `bytes`, march the first probe_rows rows of every
 * instance with plain launches, time them with HIP events on the stream, and
 * return the fastest candidate in *best (graph on) and its cell updates per
 * second in *best_rate.  Uses and overwrites the workspace; synchronous. */
int fdtd_batch_autotune(const fdtd_params *p, int32_t n, void *d_workspace, size_t bytes, void *hip_stream,
                        int64_t probe_rows, fdtd_batch_opts *best, double *best_rate);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_H */
