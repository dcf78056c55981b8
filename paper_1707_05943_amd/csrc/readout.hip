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
__global__ void k_chi(Geom g, Bufs b, cd c_chi0, int64_t r, int64_t count, cd* dst)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int64_t D = g.D;
    cd c0 = mk(0.0, 0.0);
    const int64_t q1 = r - D - 1, q2 = r - D - 1 - k;
    if (q1 >= 0 && q2 >= 0) c0 = c_chi0 * (b.Phi[q1] * b.Phi[q2]);
    cd acc = psi_rd(g, b, -k, r - D - 1 - k) - psi_rd(g, b, D - k, r - 1 - k)
           + psi_rd(g, b, k, r - D - 1) - psi_rd(g, b, D + k, r - 1);
    dst[k] = c0 - (0.5 * sqrt(g.Gamma)) * acc;
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

int launch_chi(fdtd_ctx* c, int64_t r, int64_t count, cd* dst)
{
    cd c_chi0 = (c->p.incident == FDTD_INC_EXP1) ? mk(0.0, 0.0) : mk(cos(c->p.phase), sin(c->p.phase));
    hipLaunchKernelGGL(k_chi, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b, c_chi0,
                       r, count, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_row_readout(fdtd_ctx* c, int64_t rho, cd* dst)
{
    hipLaunchKernelGGL(k_row_copy, dim3((unsigned)((c->g.C + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b,
                       rho, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}
