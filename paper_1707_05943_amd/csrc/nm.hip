// Non-Markovian measures of stimulated emission (App. D).
//
// The emitter starts excited and an exponential packet (Eq. 7) comes in;
// psi(x,t) is the march's two-excitation amplitude (Eq. 8: psi = phi(x-t)
// e1(t) in x <= -a).  The one-excitation problem with the same packet and
// the emitter in its ground state has the emitter amplitude e0(t) and the
// photon field
//
//   phi(x,t) = phi_in(x-t) - sqrt(G/2) e0(t - (x+a)) [x > -a]
//                          + sqrt(G/2) e0(t - (x-a)) [x > +a]
//
// (emission at the emitter, and its mirror image of opposite sign), e0 = 0 at
// negative times.  The measures are the overlap mu(t) = int phi*(x,t)
// psi(x,t) dx and lambda(t) = int |psi|^2 dx - |e0(t)|^2 (the determinant of
// the dynamical map's matrix is |mu|^2 lambda).
//
// Quadrature as for P_e: x <= -a exactly (there phi = phi_in(x-t), psi =
// phi_in(x-t) e1(t), and int |phi_in(x-t)|^2 dx over x <= -a is
// e^{-alpha G t}), then the trapezoid rule over the columns j = 0..Nx,
// column 0 taken from the left of x = -a.
//
// On the grid x_j = -a + j Delta, t_r = r Delta: phi_in(x_j - t_r) =
// Phi[r - j] for j <= r (zero beyond), e0(t_r - (x_j + a)) = e0[r - j] and
// e0(t_r - (x_j - a)) = e0[r - j + D].
//
// k_mu_rows reduces rows right after the launch that completed them, while
// the ring holds them: each row is read once more (16 B per cell; the
// tables Phi and e0 are reused from L2), split over NM_BLOCKS workgroups
// whose partial sums k_mu_final adds in a fixed order.

#include "fdtd_common.h"

namespace {

constexpr int NM_THREADS = 256;

__device__ inline cd photon_conj(const Geom& g, const cd* __restrict__ Phi, const cd* __restrict__ E0, double s,
                                 int64_t j, int64_t r)
{
    cd v = mk(0.0, 0.0);
    if (j <= r) {
        v = Phi[r - j];
        if (j >= 1) v -= s * E0[r - j];
    }
    if (j > g.D && j <= r + g.D) v += s * E0[r - j + g.D];
    return conj_(v);
}

__device__ inline double wave_sum(double v)
{
    #pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// grid (NM_BLOCKS, rows): workgroup x sums columns [x per, (x+1) per) of row r0 + y
__global__ __launch_bounds__(NM_THREADS) void k_mu_rows(Geom g, Bufs b, const cd* __restrict__ E0,
                                                         cd* __restrict__ mupart, int64_t r0)
{
    __shared__ double red[2][NM_THREADS / 64];
    const int64_t r = r0 + blockIdx.y;
    const int64_t per = (g.C + NM_BLOCKS - 1) / NM_BLOCKS;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < g.C ? lo + per : g.C;
    const double s = sqrt(0.5 * g.Gamma);
    const cd* __restrict__ row = b.ring + (r % g.R) * g.C;
    cd acc = mk(0.0, 0.0);
    for (int64_t j = lo + threadIdx.x; j < hi; j += NM_THREADS) {
        const cd psi = (j == 0) ? b.Phi[r] * b.Et[r] : row[j];
        cd v = photon_conj(g, b.Phi, E0, s, j, r) * psi;
        if (j == 0 || j == g.Nx) v = 0.5 * v;
        acc += v;
    }
    const double re = wave_sum(acc.re), im = wave_sum(acc.im);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = re;
        red[1][w] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cd t = mk(0.0, 0.0);
        for (int k = 0; k < NM_THREADS / 64; ++k) t += mk(red[0][k], red[1][k]);
        mupart[r * NM_BLOCKS + blockIdx.x] = t;
    }
}

__global__ void k_mu_final(Geom g, const cd* __restrict__ Et, const cd* __restrict__ mupart, double aG,
                           int64_t nrows, cd* __restrict__ dst)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    cd s = mk(0.0, 0.0);
    for (int k = 0; k < NM_BLOCKS; ++k) s += mupart[r * NM_BLOCKS + k];
    const double t = (double)r * g.Delta;
    dst[r] = Et[r] * exp(-aG * t) + g.Delta * s;
}

__global__ void k_lambda_final(Geom g, Bufs b, const cd* __restrict__ E0, int64_t nrows, int64_t nblk,
                               double* __restrict__ dst)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int64_t k = 0; k < nblk; ++k) s += b.Ppart[r * nblk + k];
    dst[r] = (b.Pex[r] + g.Delta * s) - norm2(E0[r]);
}

}  // namespace

int launch_mu_rows(fdtd_ctx* c, int64_t r0, int64_t r1)
{
    if (!c->mupart || r0 < 0 || r1 < r0 || r1 > c->g.Nt) return FDTD_EINVAL;
    hipLaunchKernelGGL(k_mu_rows, dim3(NM_BLOCKS, (unsigned)(r1 - r0 + 1)), dim3(NM_THREADS), 0, c->stream, c->g,
                       c->b, c->E0, c->mupart, r0);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_mu_final(fdtd_ctx* c, int64_t nrows, cd* dst)
{
    if (!c->mupart || nrows <= 0) return nrows == 0 ? FDTD_OK : FDTD_EINVAL;
    hipLaunchKernelGGL(k_mu_final, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b.Et,
                       c->mupart, c->p.alpha * c->p.Gamma, nrows, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_lambda_final(fdtd_ctx* c, int64_t nrows, double* dst)
{
    if (!c->E0 || nrows <= 0) return nrows == 0 ? FDTD_OK : FDTD_EINVAL;
    hipLaunchKernelGGL(k_lambda_final, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b,
                       c->E0, nrows, c->nblk, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}
