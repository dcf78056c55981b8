// Readouts of the march: P_e(t_r), the two-photon amplitude chi at the
// detectors (Eq. 2), and rows of the ring.

#include "fdtd_common.h"

namespace {

__device__ inline cd ring_rd(const Geom& g, const cd* __restrict__ ring, int64_t i, int64_t rho)
{
    return ring[(rho % g.R) * g.C + i];
}

__device__ inline cd psi_rd(const Geom& g, const Bufs& b, int64_t i, int64_t rho)
{
    if (rho < 0) return mk(0.0, 0.0);
    if (i <= 0) return b.Phi[rho - i] * b.Et[rho];
    return ring_rd(g, b.ring, i, rho);
}

__global__ void k_pe_final(Geom g, Bufs b, int64_t nrows, int64_t nblk, double* dst)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int64_t k = 0; k < nblk; ++k) s += b.Ppart[r * nblk + k];
    dst[r] = b.Pex[r] + g.Delta * s;
}

// chi(x1, x2, t_r) of Eq. (2) with x1 = a + Delta (column D+1) and
// x2 = x1 + k Delta (column D+1+k):
//   chi0(x1 - t, x2 - t) - (sqrt(G)/2) [psi(-k, r-D-1-k) - psi(D-k, r-1-k)
//                                       + psi(k, r-D-1) - psi(D+k, r-1)]
__device__ cd chi_at(const Geom& g, const Bufs& b, cd c_chi0, int64_t r, int64_t k)
{
    const int64_t D = g.D;
    cd c0 = mk(0.0, 0.0);
    const int64_t q1 = r - D - 1, q2 = r - D - 1 - k;
    if (q1 >= 0 && q2 >= 0) c0 = c_chi0 * (b.Phi[q1] * b.Phi[q2]);
    cd acc = psi_rd(g, b, -k, r - D - 1 - k) - psi_rd(g, b, D - k, r - 1 - k)
           + psi_rd(g, b, k, r - D - 1) - psi_rd(g, b, D + k, r - 1);
    return c0 - (0.5 * sqrt(g.Gamma)) * acc;
}

__global__ void k_chi(Geom g, Bufs b, cd c_chi0, int64_t r, int64_t count, cd* dst)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    dst[k] = chi_at(g, b, c_chi0, r, k);
}

// snapshots of several instances (one per blockIdx.y)
__global__ void k_chi_batch(const ChiJob* __restrict__ jobs)
{
    const ChiJob& j = jobs[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= j.n_tau) return;
    const int64_t kk = k * j.stride;
    j.dst[k] = (kk < j.g.Nx - j.g.D) ? chi_at(j.g, j.b, j.c0, j.row, kk) : mk(0.0, 0.0);
}

// P_e(t) of several instances (one per blockIdx.y) at t_k = k T / (n - 1),
// T = Nt Delta, linear in t between rows
__global__ void k_pe_sample(const BInst* __restrict__ tab, int64_t ns, const double* __restrict__ t_end,
                            double* dst)
{
    const BInst& e = tab[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns) return;
    const int64_t Nt = e.g.Nt, nw = e.P.nwg;
    // rows of t_k = k t_end / (ns - 1), t_end = Nt Delta unless given
    const double rows_end = (t_end && t_end[e.index] > 0.0) ? t_end[e.index] / e.g.Delta : (double)Nt;
    const double pos = ns > 1 ? (double)k * rows_end / (double)(ns - 1) : 0.0;
    int64_t r0 = (int64_t)floor(pos);
    if (r0 > Nt) r0 = Nt;
    const int64_t r1 = r0 < Nt ? r0 + 1 : Nt;
    const double f = pos - (double)r0;
    double p[2];
    const int64_t rr[2] = {r0, r1};
    for (int q = 0; q < 2; ++q) {
        double s = 0.0;
        for (int64_t w = 0; w < nw; ++w) s += e.b.Ppart[rr[q] * nw + w];
        p[q] = e.b.Pex[rr[q]] + e.g.Delta * s;
    }
    dst[e.index * ns + k] = (1.0 - f) * p[0] + f * p[1];
}

// Non-finite detection.  Every value the march writes enters the per-row,
// per-workgroup partial sums of |psi|^2, so a NaN or an infinity anywhere in
// a row makes one of that row's sums non-finite.  Entries lo..hi-1 of Ppart.
__device__ inline int nonfinite_in(const double* __restrict__ Ppart, int64_t lo, int64_t hi, int64_t i0,
                                   int64_t stride)
{
    int bad = 0;
    for (int64_t i = lo + i0; i < hi; i += stride) bad |= !isfinite(Ppart[i]);
    return bad;
}

__global__ void k_check_rows(const double* __restrict__ Ppart, int64_t lo, int64_t hi, int* status)
{
    const int bad = __syncthreads_or(nonfinite_in(Ppart, lo, hi, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                                                  (int64_t)gridDim.x * blockDim.x));
    if (bad && threadIdx.x == 0) atomicOr(status, STATUS_MARCH_NONFINITE);
}

// every row of instance blockIdx.y of a batch
__global__ void k_check_batch(const BInst* __restrict__ tab, int* batch_status)
{
    const BInst& e = tab[blockIdx.y];
    const int64_t hi = (e.g.Nt + 1) * (int64_t)e.P.nwg;
    const int bad = __syncthreads_or(nonfinite_in(e.b.Ppart, 0, hi, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                                                  (int64_t)gridDim.x * blockDim.x));
    if (bad && threadIdx.x == 0) {
        atomicOr(e.b.status, STATUS_MARCH_NONFINITE);
        atomicOr(batch_status, STATUS_MARCH_NONFINITE);
    }
}

__global__ void k_clear_word(int* st)
{
    if (threadIdx.x == 0) *st = 0;
}

__global__ void k_row_copy(Geom g, Bufs b, int64_t rho, cd* dst)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > g.Nx) return;
    dst[j] = (j == 0) ? b.Phi[rho] * b.Et[rho] : ring_rd(g, b.ring, j, rho);
}

}  // namespace

int launch_pe_final(fdtd_ctx* c, int64_t nrows, double* dst)
{
    hipLaunchKernelGGL(k_pe_final, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b,
                       nrows, c->nblk, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

cd chi0_coefficient(const fdtd_params* p)
{
    return (p->incident == FDTD_INC_EXP1) ? mk(0.0, 0.0) : mk(cos(p->phase), sin(p->phase));
}

int launch_chi_batch(const ChiJob* d_jobs, int n, int64_t n_tau, hipStream_t s)
{
    if (n <= 0) return FDTD_OK;
    hipLaunchKernelGGL(k_chi_batch, dim3((unsigned)((n_tau + 255) / 256), (unsigned)n), dim3(256), 0, s, d_jobs);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_pe_sample_batch(const BInst* d_tab, int n, int64_t ns, const double* d_tend, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_pe_sample, dim3((unsigned)((ns + 255) / 256), (unsigned)n), dim3(256), 0, s, d_tab, ns,
                       d_tend, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_chi(fdtd_ctx* c, int64_t r, int64_t count, cd* dst)
{
    cd c_chi0 = chi0_coefficient(&c->p);
    hipLaunchKernelGGL(k_chi, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b, c_chi0,
                       r, count, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_row_readout(fdtd_ctx* c, int64_t rho, cd* dst)
{
    if (c->dc) return launch_diag_copy(c, rho, 0, c->g.Nx + 1, dst);    // column 0 marched, every row kept
    hipLaunchKernelGGL(k_row_copy, dim3((unsigned)((c->g.C + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b,
                       rho, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_check_rows(fdtd_ctx* c, int64_t r0, int64_t r1)
{
    if (r1 < r0) return FDTD_OK;
    const int64_t lo = r0 * c->nblk, hi = (r1 + 1) * c->nblk;
    int64_t blocks = (hi - lo + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_check_rows, dim3((unsigned)blocks), dim3(256), 0, c->stream, c->b.Ppart, lo, hi,
                       c->b.status);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_check_batch(const BInst* d_tab, int n, int* batch_status, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_batch, dim3(16, (unsigned)n), dim3(256), 0, s, d_tab, batch_status);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_clear_status(int* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}
