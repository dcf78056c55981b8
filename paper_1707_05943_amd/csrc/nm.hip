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
// the ring holds them: the columns j <= r + D of row r are read once more
// (16 B per cell; the tables Phi and e0 are reused from L2), split over
// NM_BLOCKS workgroups whose partial sums k_mu_final adds in a fixed order.

#include "fdtd_common.h"
#include "nm.h"

namespace {

constexpr int NM_THREADS = 256;
typedef double v2d __attribute__((ext_vector_type(2)));

// conj(phi(x_j, t_r)) from the table values at q = r - j (Phi, e0) and
// q + D (e0), loaded beforehand with clamped indices
__device__ inline cd photon_conj(const Geom& g, cd ph, cd e1, cd e2, double s, int64_t j, int64_t r)
{
    cd v = mk(0.0, 0.0);
    if (j <= r) {
        v = ph;
        if (j >= 1) v -= s * e1;
    }
    if (j > g.D && j <= r + g.D) v += s * e2;
    return conj_(v);
}

__device__ inline double wave_sum(double v)
{
    #pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// grid (nb <= NM_BLOCKS, rows): workgroup x sums columns [x per, (x+1) per)
// of row r0 + y that lie inside the photon field's support j <= r + D
// (beyond it phi = 0 and so is the integrand; the packet and both emission
// fronts move at speed 1).  Each thread issues the loads of NM_U columns (the
// row value and three table values each, indices clamped into range) before
// it uses any of them.  (Dealing a chunk's rows to one XCD cuts the tables'
// re-reads from 1.66x to 1.09x of the row bytes, but the launch got slower.)
constexpr int NM_U = 4;
__global__ __launch_bounds__(NM_THREADS) void k_mu_rows(Geom g, Bufs b, const cd* __restrict__ E0,
                                                         cd* __restrict__ mupart, int64_t r0)
{
    __shared__ double red[2][NM_THREADS / 64];
    const int64_t r = r0 + blockIdx.y;
    const int64_t chunk = blockIdx.x;
    const int64_t per = (g.C + NM_BLOCKS - 1) / NM_BLOCKS;
    const int64_t lo = chunk * per;
    int64_t hi = lo + per < g.C ? lo + per : g.C;
    if (hi > r + g.D + 1) hi = r + g.D + 1;
    const double s = sqrt(0.5 * g.Gamma);
    const cd* __restrict__ row = b.ring + (r % g.R) * g.C;
    const cd* __restrict__ Phi = b.Phi;
    const int64_t Nt = g.Nt, D = g.D;
    cd acc = mk(0.0, 0.0);
    for (int64_t j0 = lo + threadIdx.x; j0 < hi; j0 += NM_U * NM_THREADS) {
        cd psi[NM_U], ph[NM_U], e1[NM_U], e2[NM_U];
        #pragma unroll
        for (int u = 0; u < NM_U; ++u) {
            int64_t j = j0 + (int64_t)u * NM_THREADS;
            j = j < hi ? j : hi - 1;
            int64_t q = r - j;
            q = q < 0 ? 0 : q;
            int64_t q2 = r - j + D;
            q2 = q2 < 0 ? 0 : (q2 > Nt ? Nt : q2);
            // the row is streamed once: a non-temporal load keeps the tables in L2
            const v2d pv = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(row + j));
            psi[u] = mk(pv.x, pv.y);
            ph[u] = Phi[q];
            e1[u] = E0[q];
            e2[u] = E0[q2];
        }
        #pragma unroll
        for (int u = 0; u < NM_U; ++u) {
            const int64_t j = j0 + (int64_t)u * NM_THREADS;
            if (j < hi) {
                // column 0 from the left of x = -a
                const cd p = (j == 0) ? Phi[r] * b.Et[r] : psi[u];
                cd v = photon_conj(g, ph[u], e1[u], e2[u], s, j, r) * p;
                if (j == 0 || j == g.Nx) v = 0.5 * v;
                acc += v;
            }
        }
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
        mupart[r * NM_BLOCKS + chunk] = t;
    }
}

__global__ void k_mu_final(Geom g, const cd* __restrict__ Et, const cd* __restrict__ mupart, double aG,
                           int64_t nrows, cd* __restrict__ dst)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    // the workgroups that covered columns of the support j <= r + D
    const int64_t per = (g.C + NM_BLOCKS - 1) / NM_BLOCKS;
    const int64_t act = r + g.D + 1 < g.C ? r + g.D + 1 : g.C;
    const int64_t nb = (act + per - 1) / per;
    cd s = mk(0.0, 0.0);
    for (int64_t k = 0; k < nb; ++k) s += mupart[r * NM_BLOCKS + k];
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

// N_geo over rows 0..R: the sum of the positive increments of
// |det M| = |mu|^2 |lambda| between consecutive rows (|det M| linear in t
// between rows).  One workgroup; thread t takes r = t, t + NG, ...; the
// waves' sums are added in a fixed order.
constexpr int NG_THREADS = 1024;
__global__ __launch_bounds__(NG_THREADS) void k_ngeo(const cd* __restrict__ mu, const double* __restrict__ lam,
                                                      int64_t R, double* __restrict__ dst)
{
    __shared__ double red[NG_THREADS / 64];
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < R; r += NG_THREADS) {
        const double d0 = fabs(norm2(mu[r]) * lam[r]);
        const double d1 = fabs(norm2(mu[r + 1]) * lam[r + 1]);
        const double inc = d1 - d0;
        if (inc > 0.0) acc += inc;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NG_THREADS / 64; ++k) t += red[k];
        dst[0] = t;
    }
}

}  // namespace

int launch_ngeo(fdtd_ctx* c, int64_t R, double* dst)
{
    if (!c->mupart || R < 0) return FDTD_EINVAL;
    int rc = launch_mu_final(c, R + 1, c->Mu);
    if (!rc) rc = launch_lambda_final(c, R + 1, c->b.Pe);
    if (rc) return rc;
    hipLaunchKernelGGL(k_ngeo, dim3(1), dim3(NG_THREADS), 0, c->stream, c->Mu, c->b.Pe, R, dst);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

int launch_mu_rows(fdtd_ctx* c, int64_t r0, int64_t r1, hipStream_t s)
{
    if (!c->mupart || r0 < 0 || r1 < r0 || r1 > c->g.Nt) return FDTD_EINVAL;
    // only the workgroups whose columns meet the support of the last row
    const int64_t per = (c->g.C + NM_BLOCKS - 1) / NM_BLOCKS;
    const int64_t act = r1 + c->g.D + 1 < c->g.C ? r1 + c->g.D + 1 : c->g.C;
    const int64_t nb = (act + per - 1) / per;
    hipLaunchKernelGGL(k_mu_rows, dim3((unsigned)nb, (unsigned)(r1 - r0 + 1)), dim3(NM_THREADS), 0, s, c->g, c->b,
                       c->E0, c->mupart, r0);
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
