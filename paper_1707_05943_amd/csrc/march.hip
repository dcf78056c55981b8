// The march: one row of Eq. (1) per launch (row-synchronous version).
//
// The square with corners (j-1, r-1), (j, r-1), (j-1, r), (j, r) -- Eq. (3)
// for the line-1 terms -- gives, with the source terms of lines 2-3 as bars
// (Eq. 4) and the drive of line 4 at the square's centre,
//
//   (1/Delta + W/4) U = (1/Delta - W/4) psi(j-1, r-1) - (W/4) [psi(j, r-1) + psi(j-1, r)] + S
//   U = psi(j, r) = alpha psi(j-1, r) + beta_j,
//   beta_j = cA psi(j-1, r-1) + cB psi(j, r-1) + cinv S,
//
// S = delay + sources + drive evaluated at the centre (x_j - Delta/2, t_r - Delta/2):
//   delay   (G/8) [psi(j-1-D, r-1-D) + psi(j-D, r-1-D) + psi(j-1-D, r-D) + psi(j-D, r-D)]  when r-1 >= D
//   source1 -(G/2) [bar(-j, r-j) - bar(D-j, r-j)]                  when r-j >= 0
//   source2 -(G/2) [bar(2D-j, r-j+D) - bar(D-j, r-j+D)]            when j >= D+1, r-j+D >= 0
//   drive   c_drive phi(x_j - t_r) [phi(-a - t_c) - phi(a - t_c)]
// with bar(i, rho) = [psi(i, rho) + psi(i+1, rho)]/2.  Reads at columns i <= 0
// come from the exact solution psi(i, rho) = Phi[rho - i] Et[rho]; reads at
// i >= 1 from the ring, whose D+2 rows hold every lag the update needs
// (the delay reaches lag D+1, the sources lag <= D).
//
// Within a row, U_j = alpha U_{j-1} + beta_j is a first-order linear
// recurrence.  Each block of MARCH_TX columns evaluates all beta's in
// parallel and scans the recurrence exactly over its columns; the value
// entering the block is rebuilt from `halo` extra beta's to its left,
// sum_k alpha^k beta_{c0-1-k}, dropping alpha^halo U (|alpha|^halo < 2^-60).

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

__device__ inline cd bar_rd(const Geom& g, const Bufs& b, int64_t i, int64_t rho)
{
    return 0.5 * (psi_rd(g, b, i, rho) + psi_rd(g, b, i + 1, rho));
}

__device__ cd beta_at(const Geom& g, const Bufs& b, int64_t j, int64_t r)
{
    const int64_t D = g.D;
    cd S = mk(0.0, 0.0);
    if (r - 1 >= D) {
        cd s4 = psi_rd(g, b, j - 1 - D, r - 1 - D) + psi_rd(g, b, j - D, r - 1 - D)
              + psi_rd(g, b, j - 1 - D, r - D) + psi_rd(g, b, j - D, r - D);
        S += (0.125 * g.Gamma) * s4;
    }
    cd src = mk(0.0, 0.0);
    if (r - j >= 0) src += bar_rd(g, b, -j, r - j) - bar_rd(g, b, D - j, r - j);
    if (j >= D + 1 && r - j + D >= 0) src += bar_rd(g, b, 2 * D - j, r - j + D) - bar_rd(g, b, D - j, r - j + D);
    S -= (0.5 * g.Gamma) * src;
    if (r - j >= 0) S += b.Drv[r] * b.Phi[r - j];
    const cd bl = psi_rd(g, b, j - 1, r - 1);
    const cd br = psi_rd(g, b, j, r - 1);
    return g.cA * bl + g.cB * br + g.cinv * S;
}

__device__ inline cd cpow_int(cd x, int e)
{
    cd r = mk(1.0, 0.0);
    while (e) {
        if (e & 1) r = r * x;
        x = x * x;
        e >>= 1;
    }
    return r;
}

__device__ inline cd shfl_up_cd(cd v, int d)
{
    return mk(__shfl_up(v.re, d, 64), __shfl_up(v.im, d, 64));
}

__device__ inline cd shfl_xor_cd(cd v, int m)
{
    return mk(__shfl_xor(v.re, m, 64), __shfl_xor(v.im, m, 64));
}

__global__ __launch_bounds__(MARCH_THREADS) void k_row(Geom g, Bufs b, int64_t r, int64_t nblk)
{
    constexpr int CPT = MARCH_COLS_PER_THREAD;
    __shared__ cd wave_tot[MARCH_THREADS / 64];
    __shared__ double wave_pe[MARCH_THREADS / 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int64_t blk = blockIdx.x;
    const int64_t c0 = 1 + blk * MARCH_TX;
    const cd al = g.alpha;

    // carry into the block: psi(c0-1, r)
    cd carry0 = mk(0.0, 0.0);
    if (blk == 0) {
        carry0 = b.Phi[r] * b.Et[r];          // column 0 is exact
    } else if (wv == 0) {
        const int H = g.halo;
        cd v = mk(0.0, 0.0);
        if (lane < H) {
            const int64_t j = c0 - H + lane;
            v = cpow_int(al, H - 1 - lane) * beta_at(g, b, j, r);
        }
        for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_cd(v, m);
        carry0 = v;
    }
    if (blk != 0) {
        if (wv == 0 && lane == 0) wave_tot[0] = carry0;
        __syncthreads();
        carry0 = wave_tot[0];
        __syncthreads();
    }

    // local betas and the scan with zero carry-in
    cd u[CPT];
    const int64_t jb = c0 + (int64_t)tid * CPT;
    #pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int64_t j = jb + i;
        u[i] = (j <= g.Nx) ? beta_at(g, b, j, r) : mk(0.0, 0.0);
    }
    #pragma unroll
    for (int i = 1; i < CPT; ++i) u[i] = al * u[i - 1] + u[i];

    // inclusive scan over threads of x_t = u_last + alpha^CPT x_{t-1}
    const cd a4 = cpow_int(al, CPT);
    cd x = u[CPT - 1];
    if (tid == 0) x += a4 * carry0;
    cd m = a4;   // alpha^(CPT d)
    for (int d = 1; d < 64; d <<= 1) {
        cd y = shfl_up_cd(x, d);
        if (lane >= d) x += m * y;
        m = m * m;
    }
    // m == alpha^(CPT*64) now
    if (lane == 63) wave_tot[wv] = x;
    __syncthreads();
    // prefix over the waves (few of them: sequential)
    cd wcarry = mk(0.0, 0.0);      // x at the last thread of the previous wave
    for (int w2 = 0; w2 < wv; ++w2) wcarry = m * wcarry + wave_tot[w2];
    // the value of the previous wave's last thread includes carries from all
    // earlier waves only after this combination
    cd prevx = shfl_up_cd(x, 1);
    // inclusive value of thread t with the wave carry: x_t + alpha^(CPT(lane+1)) wcarry
    // exclusive value for thread t (the U just left of its first column):
    cd cin;
    if (lane == 0) {
        cin = (wv == 0) ? carry0 : wcarry;
    } else {
        cin = prevx + cpow_int(a4, lane) * wcarry;
    }
    if (tid == 0) cin = carry0;

    // fix up and store
    const int64_t slot = r % g.R;
    cd* __restrict__ row = b.ring + slot * g.C;
    cd ap = al;
    double pe = 0.0;
    #pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int64_t j = jb + i;
        cd v = u[i] + ap * cin;
        ap = ap * al;
        if (j <= g.Nx) {
            row[j] = v;
            double w2 = norm2(v);
            pe += (j == g.Nx) ? 0.5 * w2 : w2;
        }
    }
    if (blk == 0 && tid == 0) pe += 0.5 * norm2(carry0);
    for (int mm = 32; mm >= 1; mm >>= 1) pe += __shfl_xor(pe, mm, 64);
    __syncthreads();
    if (lane == 0) wave_pe[wv] = pe;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w2 = 0; w2 < MARCH_THREADS / 64; ++w2) s += wave_pe[w2];
        b.Ppart[r * nblk + blk] = s;
    }
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

int launch_march_rows(fdtd_ctx* c, int64_t r0, int64_t r1)
{
    for (int64_t r = r0; r <= r1; ++r) {
        hipLaunchKernelGGL(k_row, dim3((unsigned)c->nblk), dim3(MARCH_THREADS), 0, c->stream, c->g, c->b, r, c->nblk);
    }
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_EDEVICE;
}

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
