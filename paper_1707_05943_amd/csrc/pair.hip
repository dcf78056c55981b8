// Two different photons (Sec. 2 case (c)).
//
// The incident state is chi(x1, x2, 0) = e^{i theta} (A/sqrt 2) [phi1(x1)
// phi2(x2) + phi1(x2) phi2(x1)] (Eq. 10, A of Eq. 11), phi_i the packet of
// Eq. (7) with (k_i, alpha_i); in x <= -a the solution is psi = A e^{i theta}
// [phi1(x-t) e0^(2)(t) + phi2(x-t) e0^(1)(t)] (Eq. 12).  The march is linear
// in its boundary data and its drive, so psi = psi_a + psi_b where march a
// has phi1 on the x - t grid with e0^(2) and phi2's drive, and march b the
// same with the photons exchanged: each is the one-packet march of
// march_block.hip with its own tables.  What is not linear in psi -- P_e --
// and what couples the two -- the free term of chi, Eq. (2) -- are formed
// here from both:
//   * the exact part of P_e, int_{x<=-a} |psi|^2 = |Ea|^2 m11 + |Eb|^2 m22 +
//     2 Re(conj(Ea) Eb m12), Ea = A e^{i theta} e0^(2), Eb = A e^{i theta}
//     e0^(1), m_ij(y) = int_{-inf}^{y} conj(phi_i) phi_j at y = -a - t;
//   * the trapezoid over columns 0..Nx of |psi_a + psi_b|^2, row by row from
//     both rings while they hold the row;
//   * rows and chi of the sum.

#include "fdtd_common.h"

namespace {

constexpr int PR_THREADS = 256;

// exact part of P_e per row (into Pex of march a).  pa, pb: the packets of
// the two marches (march a carries photon 2's e0, so pa.k = k2)
__global__ void k_pex_pair(Geom g, Packet pa, Packet pb, const cd* __restrict__ Ea, const cd* __restrict__ Eb,
                           double* __restrict__ Pex)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > g.Nt) return;
    const double G = g.Gamma;
    const double k1 = pb.k, a1 = pb.alpha, k2 = pa.k, a2 = pa.alpha;
    const double v = -(double)r * g.Delta;          // y + a, y = -a - t
    const double m11 = exp(a1 * G * v), m22 = exp(a2 * G * v);
    // conj(phi1) phi2 = sqrt(a1 a2) G e^{i (k2 - k1) u} e^{(a1 + a2) G (u + a)/2}
    const cd c = mk(0.5 * (a1 + a2) * G, k2 - k1);
    double s, co;
    sincos(-(k2 - k1) * g.a, &s, &co);
    const cd m12 = (sqrt(a1 * a2) * G) * (mk(co, s) * cdiv(cexp_(c * v), c));
    const cd ea = Ea[r], eb = Eb[r];
    const cd cross = conj_(ea) * eb * m12;
    Pex[r] = norm2(ea) * m11 + norm2(eb) * m22 + 2.0 * cross.re;
}

// sum over a workgroup in a fixed order (wave shuffles, then the waves)
__device__ inline double block_sum(double v, double* red)
{
    #pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < PR_THREADS / 64; ++i) t += red[i];
    return t;
}

// grid (nchunks, rows): chunk x of row r0 + y, trapezoid weights of
// |psi_a + psi_b|^2 over columns 0..Nx (column 0 from the exact solution)
__global__ __launch_bounds__(PR_THREADS) void k_pair_rows(Geom g, Bufs ba, Bufs bb, int64_t r0, int nchunks,
                                                          double* __restrict__ xpart)
{
    __shared__ double red[PR_THREADS / 64];
    const int64_t r = r0 + blockIdx.y;
    const int64_t per = (g.C + nchunks - 1) / nchunks;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < g.C ? lo + per : g.C;
    const int64_t off = (r % g.R) * g.C;
    double s = 0.0;
    for (int64_t j = lo + threadIdx.x; j < hi; j += PR_THREADS) {
        const cd v = (j == 0) ? ba.Phi[r] * ba.Et[r] + bb.Phi[r] * bb.Et[r] : ba.ring[off + j] + bb.ring[off + j];
        const double m2 = norm2(v);
        s += (j == 0 || j == g.Nx) ? 0.5 * m2 : m2;
    }
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) xpart[r * nchunks + blockIdx.x] = t;
}

__global__ void k_pe_pair(Geom g, const double* __restrict__ Pex, const double* __restrict__ xpart, int nchunks,
                          int64_t nrows, double* dst)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += xpart[r * nchunks + c];
    dst[r] = Pex[r] + g.Delta * s;
}

__global__ void k_row_pair(Geom g, Bufs ba, Bufs bb, int64_t rho, cd* dst)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > g.Nx) return;
    const int64_t off = (rho % g.R) * g.C;
    dst[j] = (j == 0) ? ba.Phi[rho] * ba.Et[rho] + bb.Phi[rho] * bb.Et[rho] : ba.ring[off + j] + bb.ring[off + j];
}

__device__ inline cd psi_of(const Geom& g, const Bufs& b, int64_t i, int64_t rho)
{
    if (rho < 0) return mk(0.0, 0.0);
    if (i <= 0) return b.Phi[rho - i] * b.Et[rho];
    return b.ring[(rho % g.R) * g.C + i];
}

// chi(x1, x2, t_r) of Eq. (2) at x1 = a + Delta, x2 = x1 + k Delta: the free
// term from both packets, the psi terms from both marches
__global__ void k_chi_pair(Geom g, Bufs ba, Bufs bb, cd c0, int64_t r, int64_t count, cd* dst)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int64_t D = g.D, q1 = r - D - 1, q2 = r - D - 1 - k;
    cd free_ = mk(0.0, 0.0);
    if (q1 >= 0 && q2 >= 0) free_ = c0 * (ba.Phi[q1] * bb.Phi[q2] + ba.Phi[q2] * bb.Phi[q1]);
    cd acc = mk(0.0, 0.0);
    const Bufs* bs[2] = {&ba, &bb};
    for (int m = 0; m < 2; ++m) {
        const Bufs& b = *bs[m];
        acc += psi_of(g, b, -k, r - D - 1 - k) - psi_of(g, b, D - k, r - 1 - k) + psi_of(g, b, k, r - D - 1) -
               psi_of(g, b, D + k, r - 1);
    }
    dst[k] = free_ - (0.5 * sqrt(g.Gamma)) * acc;
}

}  // namespace

int launch_pex_pair(fdtd_ctx* c)
{
    const fdtd_ctx* p = c->pair;
    const int64_t n = c->g.Nt + 1;
    hipLaunchKernelGGL(k_pex_pair, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->g, c->pk, p->pk,
                       c->b.Et, p->b.Et, c->b.Pex);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_pair_rows(fdtd_ctx* c, int64_t r0, int64_t r1)
{
    if (r1 < r0) return FDTD_OK;
    hipLaunchKernelGGL(k_pair_rows, dim3(PAIR_CHUNKS, (unsigned)(r1 - r0 + 1)), dim3(PR_THREADS), 0, c->stream,
                       c->g, c->b, c->pair->b, r0, PAIR_CHUNKS, c->xpart);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_pe_pair(fdtd_ctx* c, int64_t nrows, double* dst)
{
    hipLaunchKernelGGL(k_pe_pair, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b.Pex,
                       c->xpart, PAIR_CHUNKS, nrows, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_row_pair(fdtd_ctx* c, int64_t rho, cd* dst)
{
    hipLaunchKernelGGL(k_row_pair, dim3((unsigned)((c->g.C + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b,
                       c->pair->b, rho, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_chi_pair(fdtd_ctx* c, int64_t r, int64_t count, cd* dst)
{
    hipLaunchKernelGGL(k_chi_pair, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, c->stream, c->g, c->b,
                       c->pair->b, c->c0_pair, r, count, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}
