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
    int64_t R;          // ring rows
    double Delta, a, Gamma;
    cd W;               // i omega0 + Gamma/2
    cd alpha;           // coefficient of psi(j-1, r) in the solved square
    cd cA;              // coefficient of psi(j-1, r-1)
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

// device pointers carved from the caller's workspace
struct Bufs {
    cd* ring;        // R x C
    cd* Et;          // c_ex E(t_r), r = 0..Nt
    cd* Phi;         // phi(-a - q Delta), q = 0..Nt
    cd* Drv;         // drive per row, r = 0..Nt (r = 0 unused)
    double* Pex;     // exact part of P_e per row
    double* Ppart;   // per-row per-block partial sums of |psi|^2
    double* Pe;      // P_e per row
    cd* chi;         // chi readout scratch
    cd* Ebuf;        // host-supplied E staging (Nt+1)
    int* status;     // device error flags
};

struct fdtd_ctx {
    fdtd_params p;
    Geom g;
    Packet pk;
    Bufs b;
    hipStream_t stream;
    int64_t row;          // last solved row
    int boundary_ready;
    int64_t nblk;         // blocks per row of the march kernel
    char err[512];
};

enum { STATUS_GAMMA_RANGE = 1, STATUS_NONFINITE = 2 };

// launch helpers implemented in the .hip files
int launch_boundary(fdtd_ctx* c, int from_host_E);
int launch_march_rows(fdtd_ctx* c, int64_t r0, int64_t r1);
int launch_pe_final(fdtd_ctx* c, int64_t nrows, double* dst);
int launch_chi(fdtd_ctx* c, int64_t r, int64_t count, cd* dst);
int launch_row_readout(fdtd_ctx* c, int64_t rho, cd* dst);
int launch_clear(fdtd_ctx* c);

constexpr int MARCH_THREADS = 256;
constexpr int MARCH_COLS_PER_THREAD = 4;
constexpr int MARCH_TX = MARCH_THREADS * MARCH_COLS_PER_THREAD;   // columns per block
constexpr int MAX_HALO = 64;
