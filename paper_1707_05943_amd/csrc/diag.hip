// The march with the paper's own reads (Sec. 3; its test 1, Sec. 4): dc
// columns at x <= -a (columns lo = 1-dc .. 0) are marched with the same
// square of Eq. (1) as the rest, and every read of a marched point takes the
// marched value; only points left of column lo take the exact solution
// c phi(x - t) E(t) = Phi[rho - i] Et[rho].  The source terms of x > -a read
// x <= -a at lags up to the row itself (along diagonals x - t = const), so
// every row is kept: hist holds rows 0..Nt of columns lo..Nx.
//
// One launch per row, one workgroup: each thread forms beta_j = cA psi(j-1,
// r-1) + cB psi(j, r-1) + cinv S_j for DG_CPT consecutive columns (S: the
// delay square, the two source bars, the drive), runs the recurrence psi_j =
// alpha psi_{j-1} + beta_j over them from zero, and a scan of the threads'
// last values (each thread's map is c -> alpha^DG_CPT c + u) hands every
// thread its carry; rows wider than one pass go in passes, the carry of one
// pass entering the next.  The row's trapezoid of |psi|^2 over columns 0..Nx
// goes into the per-row partial sums as the march's does.  A test mode: the
// one-workgroup launches leave the chip mostly idle.

#include "fdtd_common.h"

namespace {

constexpr int DG_THREADS = 1024;
constexpr int DG_CPT = 8;

struct Diag {
    Geom g;
    Bufs b;
    int64_t lo, Wd;     // first marched column, row pitch of hist (Nx - lo + 1)
};

__device__ __forceinline__ void cmac(cd& acc, const cd a, const cd b)
{
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}

__device__ inline cd val(const Diag& d, int64_t i, int64_t rho)
{
    if (rho < 0) return mk(0.0, 0.0);
    if (i < d.lo) return d.b.Phi[rho - i] * d.b.Et[rho];
    return d.b.hist[rho * d.Wd + (i - d.lo)];
}

__device__ inline cd bar(const Diag& d, int64_t i, int64_t rho)
{
    return 0.5 * (val(d, i, rho) + val(d, i + 1, rho));
}

// everything of psi(j, r) but alpha psi(j-1, r)
__device__ inline cd beta(const Diag& d, int64_t j, int64_t r, cd drv)
{
    const Geom& g = d.g;
    const int64_t D = g.D;
    const double hg = 0.5 * g.Gamma;
    cd S = mk(0.0, 0.0);
    // delay: the square shifted by D columns and D rows, active iff t_c > 2a
    if (r - 1 >= D)
        S += (0.25 * hg) * (val(d, j - 1 - D, r - 1 - D) + val(d, j - D, r - 1 - D) + val(d, j - 1 - D, r - D) +
                            val(d, j - D, r - D));
    // sources (only x_c > -a): at t - x - a = (r - j) Delta, columns -j, -j+1
    // and D-j, D-j+1; for x_c > a also at t - x + a = (r - j + D) Delta,
    // columns 2D-j, 2D-j+1 and D-j, D-j+1
    cd src = mk(0.0, 0.0);
    if (j >= 1 && r - j >= 0) src += bar(d, -j, r - j) - bar(d, D - j, r - j);
    if (j >= D + 1 && r - j + D >= 0) src += bar(d, 2 * D - j, r - j + D) - bar(d, D - j, r - j + D);
    S -= hg * src;
    // drive: c_drive phi(x_c - t_c) [phi(-a - t_c) - phi(a - t_c)], x_c - t_c on the grid
    if (r - j >= 0) S += d.b.Phi[r - j] * drv;
    const cd bl = val(d, j - 1, r - 1), br = val(d, j, r - 1);
    cd v = bl;
    cmac(v, g.cAm1, bl);
    cmac(v, g.cB, br);
    cmac(v, g.cinv, S);
    return v;
}

__global__ __launch_bounds__(DG_THREADS) void k_diag_row(Diag d, int64_t r, int64_t nblk)
{
    __shared__ cd B[DG_THREADS];
    __shared__ double red[DG_THREADS / 64];
    const int t = threadIdx.x;
    const Geom& g = d.g;
    const cd al = g.alpha;
    cd apow[DG_CPT + 1];
    apow[0] = mk(1.0, 0.0);
    for (int k = 1; k <= DG_CPT; ++k) apow[k] = apow[k - 1] * al;
    const cd drv = d.b.Drv[r];
    cd carry = val(d, d.lo - 1, r);          // the exact solution left of the marched columns
    double psum = 0.0;
    cd* row = d.b.hist + r * d.Wd;
    for (int64_t c0 = d.lo; c0 <= g.Nx; c0 += (int64_t)DG_THREADS * DG_CPT) {
        const int64_t j0 = c0 + (int64_t)t * DG_CPT;
        cd u[DG_CPT];
        cd acc = mk(0.0, 0.0);
        #pragma unroll
        for (int k = 0; k < DG_CPT; ++k) {
            const int64_t j = j0 + k;
            acc = al * acc;
            if (j <= g.Nx) acc += beta(d, j, r, drv);
            u[k] = acc;
        }
        // thread t's last value given its carry c: alpha^CPT c + u[CPT-1];
        // thread 0 takes the pass's carry in, then an inclusive scan
        B[t] = (t == 0) ? apow[DG_CPT] * carry + u[DG_CPT - 1] : u[DG_CPT - 1];
        cd step = apow[DG_CPT];
        for (int off = 1; off < DG_THREADS; off <<= 1) {
            __syncthreads();
            const cd prev = t >= off ? B[t - off] : mk(0.0, 0.0);
            __syncthreads();
            if (t >= off) B[t] += step * prev;
            step = step * step;
        }
        __syncthreads();
        const cd cin = (t == 0) ? carry : B[t - 1];
        #pragma unroll
        for (int k = 0; k < DG_CPT; ++k) {
            const int64_t j = j0 + k;
            if (j > g.Nx) break;
            const cd v = apow[k + 1] * cin + u[k];
            row[j - d.lo] = v;
            if (j >= 0) psum += (j == 0 || j == g.Nx) ? 0.5 * norm2(v) : norm2(v);
        }
        carry = B[DG_THREADS - 1];
        __syncthreads();
    }
    // the row's trapezoid over columns 0..Nx, in a fixed order
    #pragma unroll
    for (int o = 32; o >= 1; o >>= 1) psum += __shfl_xor(psum, o, 64);
    if ((t & 63) == 0) red[t >> 6] = psum;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int w = 0; w < DG_THREADS / 64; ++w) s += red[w];
        d.b.Ppart[r * nblk] = s;
    }
    for (int64_t w = 1 + t; w < nblk; w += DG_THREADS) d.b.Ppart[r * nblk + w] = 0.0;
}

// row 0: the initial condition, the exact solution at x <= -a, zero right of it
__global__ void k_diag_row0(Diag d)
{
    const int64_t i = d.lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > d.g.Nx) return;
    d.b.hist[i - d.lo] = (i <= 0) ? d.b.Phi[-i] * d.b.Et[0] : mk(0.0, 0.0);
}

__global__ void k_diag_copy(Diag d, int64_t rho, int64_t j0, int64_t count, cd* __restrict__ dst)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) dst[k] = d.b.hist[rho * d.Wd + (j0 + k - d.lo)];
}

Diag diag_of(const fdtd_ctx* c)
{
    Diag d;
    d.g = c->g;
    d.b = c->b;
    d.lo = 1 - c->dc;
    d.Wd = c->g.Nx - d.lo + 1;
    return d;
}

}  // namespace

int launch_diag_setup(fdtd_ctx* c)
{
    int rc = launch_phi_tail(c, c->g.Nt + 1, c->g.Nt + c->dc + c->g.D);
    if (rc) return rc;
    const Diag d = diag_of(c);
    hipLaunchKernelGGL(k_diag_row0, dim3((unsigned)((d.Wd + 255) / 256)), dim3(256), 0, c->stream, d);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_diag_row(fdtd_ctx* c, int64_t r)
{
    hipLaunchKernelGGL(k_diag_row, dim3(1), dim3(DG_THREADS), 0, c->stream, diag_of(c), r, c->nblk);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_diag_copy(fdtd_ctx* c, int64_t rho, int64_t j0, int64_t count, cd* dst)
{
    if (count <= 0) return FDTD_OK;
    hipLaunchKernelGGL(k_diag_copy, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, c->stream, diag_of(c), rho,
                       j0, count, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}
